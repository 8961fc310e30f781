/*
 * Brute-force FP64 evaluator of the swap potential -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain C, OpenMP over particles, O(N^2) pair scan (no cell list, no
 * neighbour list).  Written independently of the GPU engine; shares no code
 * with it.  Build with -ffp-contract=off (no fused multiply-add) so that the
 * canonical cut/bond predicate below is evaluated with plain IEEE operations.
 *
 * What it computes (paper, Sec. 2):
 *   pair, kind 1 (swap):  v(r) = 4 eps [(sigma/r)^(2n) - (sigma/r)^n], r < r_cut   (eq. 2b)
 *   pair, kind 2 (WCA):   4 eps [(sigma/r)^12 - (sigma/r)^6] + eps,    r < r_cut
 *   switching factor:     vhat = 1 (r^2 <= r_min^2), -v/eps (inside r_cut), 0 beyond  (eq. pot)
 *   three-body:           sum_i sum_{j<k} Lambda vhat(r_ij) vhat(r_ik),  Lambda = lambda eps  (eq. 3bp)
 *                         (Lambda_ijk = sqrt(Lambda_ij Lambda_ik) when the entries differ)
 *   virial:               W_ab = sum_terms sum_m (x_m - x_centre)_a F_m,b   (eq. p3 bracket)
 *   bonds:                swap pairs with r^2 < r_min^2 = (sigma*sigma) * pow(2, 2/n)
 *
 * Canonical predicate: d = x_j - x_i folded once by +-L, r^2 = (dx*dx + dy*dy) + dz*dz.
 *
 * Parity status: pinned against the numpy evaluator, which is itself pinned by
 * closed forms and finite differences (see the tests).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

#define ORC_NONE 0
#define ORC_SWAP 1
#define ORC_WCA 2

typedef struct {
    int kind, n;
    double eps, sigma, rcut2, rmin2, Lam;
} orc_entry;

typedef struct {
    int c, p;           /* centre, partner */
    double u, u1;       /* vhat and d vhat / dr */
    double d[3];        /* x_p - x_c (minimum image) */
    double r, Lam;
} orc_edge;

static void fill_entries(int nt, const int* kind, const double* eps, const double* sigma,
                         const int* n, const double* rcut, const double* lam, orc_entry* E) {
    for (int a = 0; a < nt * nt; ++a) {
        E[a].kind = kind[a];
        E[a].n = n[a];
        E[a].eps = eps[a];
        E[a].sigma = sigma[a];
        E[a].rcut2 = rcut[a] * rcut[a];
        E[a].rmin2 = (sigma[a] * sigma[a]) * pow(2.0, 2.0 / (double)n[a]);
        E[a].Lam = lam[a] * eps[a];
    }
}

static inline double sep_r2(const double* xi, const double* xj, const double* L, double d[3]) {
    for (int a = 0; a < 3; ++a) {
        double x = xj[a] - xi[a];
        double h = 0.5 * L[a];
        if (x > h) x -= L[a];
        else if (x < -h) x += L[a];
        d[a] = x;
    }
    double s = d[0] * d[0];
    s = s + d[1] * d[1];
    s = s + d[2] * d[2];
    return s;
}

static inline double ipow(double x, int n) {
    double r = 1.0;
    for (int k = 0; k < n; ++k) r *= x;
    return r;
}

/* pair energy and d/dr for an included pair */
static inline void pair_term(const orc_entry* e, double r, double* phi, double* dphi) {
    int n = (e->kind == ORC_WCA) ? 6 : e->n;
    double s = ipow(e->sigma / r, n);
    *phi = 4.0 * e->eps * (s * s - s) + ((e->kind == ORC_WCA) ? e->eps : 0.0);
    *dphi = 4.0 * e->eps * n * (s - 2.0 * s * s) / r;
}

/* vhat and its derivative for an included swap pair */
static inline void vhat_term(const orc_entry* e, double r2, double r, double* u, double* u1) {
    if (r2 <= e->rmin2) { *u = 1.0; *u1 = 0.0; return; }
    double s = ipow(e->sigma / r, e->n);
    *u = -4.0 * (s * s - s);
    *u1 = -4.0 * e->n * (s - 2.0 * s * s) / r;
}

static inline double triplet_lam(double a, double b) { return (a == b) ? a : sqrt(a * b); }

/*
 * Full evaluation.  pos [3N] (xyz per particle), type [N], L [3].
 * Table arrays are [nt*nt] row-major.  Outputs: F [3N], pe [N],
 * out[0..8] = E, E2, E3, Wxx, Wyy, Wzz, Wxy, Wxz, Wyz; bonds; n_triplets.
 * Returns 0, or -1 on allocation failure.
 */
int orc_evaluate(int N, const double* pos, const int* type, const double* L, int nt,
                 const int* kind, const double* eps, const double* sigma, const int* n,
                 const double* rcut, const double* lam, int nthreads, double* F, double* pe,
                 double* out, long long* bonds, long long* ntrip) {
    orc_entry* E = (orc_entry*)malloc(sizeof(orc_entry) * nt * nt);
    if (!E) return -1;
    fill_entries(nt, kind, eps, sigma, n, rcut, lam, E);
    if (nthreads > 0) omp_set_num_threads(nthreads);
    int T = omp_get_max_threads();
    orc_edge** tedges = (orc_edge**)calloc(T, sizeof(orc_edge*));
    long long* tcount = (long long*)calloc(T, sizeof(long long));
    double* tred = (double*)calloc((size_t)T * 8, sizeof(double));
    long long* tbond = (long long*)calloc(T, sizeof(long long));
    int fail = 0;
    memset(F, 0, sizeof(double) * 3 * (size_t)N);
    memset(pe, 0, sizeof(double) * (size_t)N);

#pragma omp parallel
    {
        int t = omp_get_thread_num();
        long long cap = 1024, cnt = 0;
        orc_edge* buf = (orc_edge*)malloc(sizeof(orc_edge) * cap);
        double* red = tred + (size_t)t * 8;  /* E2, Wxx..Wyz */
        long long nb = 0;
        if (!buf) fail = 1;
#pragma omp for schedule(static)
        for (int i = 0; i < N; ++i) {
            if (!buf) continue;
            const double* xi = pos + 3 * (size_t)i;
            double fx = 0, fy = 0, fz = 0, ei = 0;
            for (int j = 0; j < N; ++j) {
                if (j == i) continue;
                const orc_entry* e = &E[type[i] * nt + type[j]];
                if (e->kind == ORC_NONE) continue;
                double d[3];
                double r2 = sep_r2(xi, pos + 3 * (size_t)j, L, d);
                if (!(r2 < e->rcut2)) continue;
                double r = sqrt(r2);
                double phi, dphi;
                pair_term(e, r, &phi, &dphi);
                /* force on i from the pair is +phi' rhat_ij; on j it is -phi' rhat_ij */
                double g = dphi / r;
                fx += g * d[0]; fy += g * d[1]; fz += g * d[2];
                ei += 0.5 * phi;
                red[0] += 0.5 * phi;
                double fj[3] = {-g * d[0], -g * d[1], -g * d[2]};
                red[1] += 0.5 * d[0] * fj[0];
                red[2] += 0.5 * d[1] * fj[1];
                red[3] += 0.5 * d[2] * fj[2];
                red[4] += 0.5 * d[0] * fj[1];
                red[5] += 0.5 * d[0] * fj[2];
                red[6] += 0.5 * d[1] * fj[2];
                if (e->kind == ORC_SWAP) {
                    if (j > i && r2 < e->rmin2) ++nb;
                    if (cnt == cap) {
                        cap *= 2;
                        orc_edge* nbuf = (orc_edge*)realloc(buf, sizeof(orc_edge) * cap);
                        if (!nbuf) { fail = 1; continue; }
                        buf = nbuf;
                    }
                    orc_edge* ed = &buf[cnt++];
                    ed->c = i; ed->p = j; ed->r = r; ed->Lam = e->Lam;
                    ed->d[0] = d[0]; ed->d[1] = d[1]; ed->d[2] = d[2];
                    vhat_term(e, r2, r, &ed->u, &ed->u1);
                }
            }
            F[3 * (size_t)i + 0] = fx;
            F[3 * (size_t)i + 1] = fy;
            F[3 * (size_t)i + 2] = fz;
            pe[i] = ei;
        }
        tedges[t] = buf;
        tcount[t] = cnt;
        tbond[t] = nb;
    }
    if (fail) {
        for (int t = 0; t < T; ++t) free(tedges[t]);
        free(tedges); free(tcount); free(tred); free(tbond); free(E);
        return -1;
    }
    double red[8] = {0};
    long long nbonds = 0;
    for (int t = 0; t < T; ++t) {
        for (int q = 0; q < 7; ++q) red[q] += tred[(size_t)t * 8 + q];
        nbonds += tbond[t];
    }
    /* triplets: edges of each thread are sorted by centre (static schedule) */
    double E3 = 0.0;
    long long nt3 = 0;
    for (int t = 0; t < T; ++t) {
        orc_edge* ed = tedges[t];
        long long cnt = tcount[t];
        long long s = 0;
        while (s < cnt) {
            long long e = s;
            while (e < cnt && ed[e].c == ed[s].c) ++e;
            int c = ed[s].c;
            for (long long a = s; a < e; ++a) {
                for (long long b = a + 1; b < e; ++b) {
                    double Lt = triplet_lam(ed[a].Lam, ed[b].Lam);
                    double en = Lt * ed[a].u * ed[b].u;
                    double ga = -Lt * ed[a].u1 * ed[b].u / ed[a].r;
                    double gb = -Lt * ed[a].u * ed[b].u1 / ed[b].r;
                    double Fa[3], Fb[3];
                    for (int q = 0; q < 3; ++q) {
                        Fa[q] = ga * ed[a].d[q];
                        Fb[q] = gb * ed[b].d[q];
                        F[3 * (size_t)ed[a].p + q] += Fa[q];
                        F[3 * (size_t)ed[b].p + q] += Fb[q];
                        F[3 * (size_t)c + q] -= Fa[q] + Fb[q];
                    }
                    pe[c] += en;
                    E3 += en;
                    red[1] += ed[a].d[0] * Fa[0] + ed[b].d[0] * Fb[0];
                    red[2] += ed[a].d[1] * Fa[1] + ed[b].d[1] * Fb[1];
                    red[3] += ed[a].d[2] * Fa[2] + ed[b].d[2] * Fb[2];
                    red[4] += ed[a].d[0] * Fa[1] + ed[b].d[0] * Fb[1];
                    red[5] += ed[a].d[0] * Fa[2] + ed[b].d[0] * Fb[2];
                    red[6] += ed[a].d[1] * Fa[2] + ed[b].d[1] * Fb[2];
                    ++nt3;
                }
            }
            s = e;
        }
        free(ed);
    }
    out[0] = red[0] + E3;
    out[1] = red[0];
    out[2] = E3;
    for (int q = 0; q < 6; ++q) out[3 + q] = red[1 + q];
    *bonds = nbonds;
    *ntrip = nt3;
    free(tedges); free(tcount); free(tred); free(tbond); free(E);
    return 0;
}

/* collect the swap partners of particle c (excluding 'skip'), O(N) */
static int partners_of(int c, int skip, int N, const double* pos, const int* type, const double* L,
                       int nt, const orc_entry* E, orc_edge* buf, int cap) {
    int cnt = 0;
    const double* xc = pos + 3 * (size_t)c;
    for (int k = 0; k < N; ++k) {
        if (k == c || k == skip) continue;
        const orc_entry* e = &E[type[c] * nt + type[k]];
        if (e->kind != ORC_SWAP) continue;
        double d[3];
        double r2 = sep_r2(xc, pos + 3 * (size_t)k, L, d);
        if (!(r2 < e->rcut2)) continue;
        if (cnt >= cap) return -1;
        orc_edge* ed = &buf[cnt++];
        double r = sqrt(r2);
        ed->c = c; ed->p = k; ed->r = r; ed->Lam = e->Lam;
        ed->d[0] = d[0]; ed->d[1] = d[1]; ed->d[2] = d[2];
        vhat_term(e, r2, r, &ed->u, &ed->u1);
    }
    return cnt;
}

#define ORC_CAP 256

/*
 * Forces, per-particle energies and bond degrees of M sampled particles idx[M],
 * from every pair term and every triplet term that involves them (as centre or
 * as partner).  O((1 + k) N) per sample.  Returns 0, -1 on a partner overflow.
 */
int orc_forces_subset(int N, const double* pos, const int* type, const double* L, int nt,
                      const int* kind, const double* eps, const double* sigma, const int* n,
                      const double* rcut, const double* lam, int nthreads, int M, const int* idx,
                      double* F, double* pe, int* degree) {
    orc_entry E[64 * 64];
    if (nt > 64) return -1;
    fill_entries(nt, kind, eps, sigma, n, rcut, lam, E);
    if (nthreads > 0) omp_set_num_threads(nthreads);
    int fail = 0;
#pragma omp parallel
    {
        orc_edge* mine = (orc_edge*)malloc(sizeof(orc_edge) * ORC_CAP);
        orc_edge* other = (orc_edge*)malloc(sizeof(orc_edge) * ORC_CAP);
#pragma omp for schedule(dynamic, 1)
        for (int s = 0; s < M; ++s) {
            int m = idx[s];
            const double* xm = pos + 3 * (size_t)m;
            double f[3] = {0, 0, 0}, em = 0.0;
            int deg = 0, km = 0;
            for (int j = 0; j < N; ++j) {
                if (j == m) continue;
                const orc_entry* e = &E[type[m] * nt + type[j]];
                if (e->kind == ORC_NONE) continue;
                double d[3];
                double r2 = sep_r2(xm, pos + 3 * (size_t)j, L, d);
                if (!(r2 < e->rcut2)) continue;
                double r = sqrt(r2), phi, dphi;
                pair_term(e, r, &phi, &dphi);
                double g = dphi / r;
                f[0] += g * d[0]; f[1] += g * d[1]; f[2] += g * d[2];
                em += 0.5 * phi;
                if (e->kind == ORC_SWAP) {
                    if (r2 < e->rmin2) ++deg;
                    if (km >= ORC_CAP) { fail = 1; break; }
                    orc_edge* ed = &mine[km++];
                    ed->c = m; ed->p = j; ed->r = r; ed->Lam = e->Lam;
                    ed->d[0] = d[0]; ed->d[1] = d[1]; ed->d[2] = d[2];
                    vhat_term(e, r2, r, &ed->u, &ed->u1);
                }
            }
            /* m as centre */
            for (int a = 0; a < km; ++a) {
                for (int b = a + 1; b < km; ++b) {
                    double Lt = triplet_lam(mine[a].Lam, mine[b].Lam);
                    double ga = -Lt * mine[a].u1 * mine[b].u / mine[a].r;
                    double gb = -Lt * mine[a].u * mine[b].u1 / mine[b].r;
                    for (int q = 0; q < 3; ++q) f[q] -= ga * mine[a].d[q] + gb * mine[b].d[q];
                    em += Lt * mine[a].u * mine[b].u;
                }
            }
            /* m as a partner of centre c = mine[a].p, with every other partner k of c */
            for (int a = 0; a < km; ++a) {
                int c = mine[a].p;
                int kc = partners_of(c, m, N, pos, type, L, nt, E, other, ORC_CAP);
                if (kc < 0) { fail = 1; break; }
                /* vhat(r_cm) seen from c: same distance, vector reversed */
                double ucm = mine[a].u, u1cm = mine[a].u1, rcm = mine[a].r;
                double dcm[3] = {-mine[a].d[0], -mine[a].d[1], -mine[a].d[2]};
                for (int b = 0; b < kc; ++b) {
                    double Lt = triplet_lam(mine[a].Lam, other[b].Lam);
                    double g = -Lt * u1cm * other[b].u / rcm;
                    for (int q = 0; q < 3; ++q) f[q] += g * dcm[q];
                }
            }
            F[3 * (size_t)s + 0] = f[0];
            F[3 * (size_t)s + 1] = f[1];
            F[3 * (size_t)s + 2] = f[2];
            pe[s] = em;
            degree[s] = deg;
        }
        free(mine);
        free(other);
    }
    return fail ? -1 : 0;
}
