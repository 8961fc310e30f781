// Differentiation of the swap-potential energy: Hessian-vector products and
// parameter gradients, both as atomic-free per-particle gathers.
//
// With w_ma = sqrt(Lambda_ma) vhat(r_ma) for swap partners inside r_cut and
// S_m = sum_a w_ma, the gradient of E with respect to x_m is
//     grad_m E = - sum_a rhat_ma G_ma,
//     G_ma = phi'(r_ma) + w'_ma (S_m + S_a - 2 w_ma)
// (the triplet sum of eq. 3bp over j<k regrouped per centre), so
//     (H v)_m = - sum_a [ dG_ma rhat_ma + G_ma (D_ma - dr_ma rhat_ma) / r_ma ],
//     D_ma = v_a - v_m,  dr_ma = rhat_ma . D_ma,
//     dG_ma = phi'' dr + w'' dr (S_m + S_a - 2 w) + w' (dS_m + dS_a - 2 w' dr),
//     dS_m = sum_b w'_mb dr_mb.
// A first pass stores (S, dS) of every particle; the second reads S_a and dS_a
// of a partner from there instead of walking a's list (the two-hop walk of
// the one-pass form; the values are those of the same walk, so the result is
// the same).
#include "rc_internal.h"

namespace rc {

static inline int nblk(long n, int b) { return (int)((n + b - 1) / b); }

__device__ __forceinline__ void load_table_adj(DevEntry* s_tab, const Table& t) {
    const int n = t.nt * t.nt;
    for (int q = threadIdx.x; q < n; q += blockDim.x) s_tab[q] = t.e[q];
    __syncthreads();
}

struct Deriv {  // value and first two r-derivatives of one term, plus geometry
    float r, rx, ry, rz;  // r and rhat
};

// pair: phi'(r), phi''(r)
__device__ __forceinline__ void pair_d12(const DevEntry& e, float r2, float r, float& d1, float& d2) {
    const float q = qpow(e.sig2 / r2, e.n);
    const float q2 = q * q, n = (float)e.n;
    d1 = 4.0f * e.eps * n * (q - 2.0f * q2) / r;
    d2 = 4.0f * e.eps * (2.0f * n * (2.0f * n + 1.0f) * q2 - n * (n + 1.0f) * q) / r2;
}

// w = sqrt(Lambda) vhat and its first two r-derivatives
__device__ __forceinline__ void w_d012(const DevEntry& e, bool inside, float r2, float r, float& w,
                                       float& w1, float& w2) {
    if (inside) {
        w = e.sqrt_lam;
        w1 = 0.0f;
        w2 = 0.0f;
        return;
    }
    const float q = qpow(e.sig2 / r2, e.n);
    const float q2 = q * q, n = (float)e.n;
    w = e.sqrt_lam * 4.0f * (q - q2);
    w1 = e.sqrt_lam * 4.0f * n * (2.0f * q2 - q) / r;
    w2 = -e.sqrt_lam * 4.0f * (2.0f * n * (2.0f * n + 1.0f) * q2 - n * (n + 1.0f) * q) / r2;
}

// S_c and dS_c = sum_b w'_cb rhat_cb . (v_b - v_c) over c's swap partners
__device__ __forceinline__ void centre_sums(int c, const float4& pc, const float4& vc, const int* nlist,
                                            const int* nn, int k_max, int N, const float4* pos, const float4* v,
                                            const DevEntry* tab, int nt, const Box& box, double& S,
                                            double& dS) {
    const int tc = ptype(pc.w);
    const int cnt = nn_swap(nn[c]);   // swap-kind neighbours fill the front of the column
    S = 0.0;
    dS = 0.0;
    for (int t = 0; t < cnt; ++t) {
        const int b = nlist[(size_t)t * N + c];
        const float4 pb = pos[b];
        const DevEntry& e = tab[tc * nt + ptype(pb.w)];
        if (e.kind != RC_KIND_SWAP) continue;
        double dx, dy, dz;
        const double r2d = canon_r2(pc, pb, box, dx, dy, dz);
        if (!(r2d < e.rcut2)) continue;
        const float r2 = (float)r2d, r = sqrtf(r2);
        float w, w1, w2;
        w_d012(e, r2d <= e.rmin2, r2, r, w, w1, w2);
        const float4 vb = v[b];
        const float dr = ((float)dx * (vb.x - vc.x) + (float)dy * (vb.y - vc.y) + (float)dz * (vb.z - vc.z)) / r;
        S += (double)w;
        dS += (double)(w1 * dr);
    }
}

// first pass: (S, dS) of every particle; grid row y works on vector y
__global__ __launch_bounds__(kBlock) void k_hvp_sums(HvpArgs a) {
    extern __shared__ DevEntry s_tab[];
    load_table_adj(s_tab, a.tab);
    const int m = xcd_block(gridDim.x) * blockDim.x + threadIdx.x;
    if (m >= a.N) return;
    const size_t vo = (size_t)blockIdx.y * a.N;
    const float4* v = a.v + vo;
    double S, dS;
    centre_sums(m, a.pos[m], v[m], a.nlist, a.nn, a.k_max, a.N, a.pos, v, s_tab, a.tab.nt, a.box, S, dS);
    a.sums[vo + m] = make_double2(S, dS);
}

__global__ __launch_bounds__(kBlock) void k_hvp(HvpArgs a) {
    extern __shared__ DevEntry s_tab[];
    load_table_adj(s_tab, a.tab);
    const int nt = a.tab.nt;
    const int m = xcd_block(gridDim.x) * blockDim.x + threadIdx.x;
    if (m >= a.N) return;
    const size_t vo = (size_t)blockIdx.y * a.N;
    const float4* v = a.v + vo;
    const double2* sums = a.sums + vo;
    const float4 pm = a.pos[m];
    const float4 vm = v[m];
    const int tm = ptype(pm.w);
    const int packed = a.nn[m];
    const int ns = nn_swap(packed), cnt = ns + nn_other(packed);
    const double2 sm = sums[m];
    const double Sm = sm.x, dSm = sm.y;
    float hx = 0.f, hy = 0.f, hz = 0.f;
    for (int s = 0; s < cnt; ++s) {
        const int slot = s < ns ? s : a.k_max - 1 - (s - ns);
        const int j = a.nlist[(size_t)slot * a.N + m];
        const float4 pj = a.pos[j];
        const DevEntry& e = s_tab[tm * nt + ptype(pj.w)];
        if (e.kind == RC_KIND_NONE) continue;
        double dxd, dyd, dzd;
        const double r2d = canon_r2(pm, pj, a.box, dxd, dyd, dzd);
        if (!(r2d < e.rcut2)) continue;
        const float r2 = (float)r2d, r = sqrtf(r2), ir = 1.0f / r;
        const float rx = (float)dxd * ir, ry = (float)dyd * ir, rz = (float)dzd * ir;
        const float4 vj = v[j];
        const float Dx = vj.x - vm.x, Dy = vj.y - vm.y, Dz = vj.z - vm.z;
        const float dr = rx * Dx + ry * Dy + rz * Dz;
        float G, dG;
        pair_d12(e, r2, r, G, dG);
        dG *= dr;
        if (e.kind == RC_KIND_SWAP) {
            float w, w1, w2;
            w_d012(e, r2d <= e.rmin2, r2, r, w, w1, w2);
            if (w1 != 0.0f || w2 != 0.0f) {
                const double2 sj = sums[j];
                const double Sj = sj.x, dSj = sj.y;
                const float X = (float)((Sm - (double)w) + (Sj - (double)w));
                const float dX = (float)((dSm - (double)(w1 * dr)) + (dSj - (double)(w1 * dr)));
                G += w1 * X;
                dG += w2 * dr * X + w1 * dX;
            }
        }
        const float c = G * ir;
        hx -= dG * rx + c * (Dx - dr * rx);
        hy -= dG * ry + c * (Dy - dr * ry);
        hz -= dG * rz + c * (Dz - dr * rz);
    }
    a.hv[vo + m] = make_float4(hx, hy, hz, 0.0f);
}

hipError_t launch_hvp(const HvpArgs& a, hipStream_t s) {
    if (a.nvec < 1 || a.nvec > 65535) return hipErrorInvalidValue;
    const size_t shm = sizeof(DevEntry) * a.tab.nt * a.tab.nt;
    const dim3 grid(nblk(a.N, kBlock), a.nvec);
    hipLaunchKernelGGL(k_hvp_sums, grid, dim3(kBlock), shm, s, a);
    hipLaunchKernelGGL(k_hvp, grid, dim3(kBlock), shm, s, a);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// dE / d(eps, sigma, lambda) per table entry, at fixed r_cut.
//  pair (half per list direction):  d/deps = phi/eps,  d/dsigma = 4 eps n (2q^2 - q)/sigma
//  triplets of centre m, per active partner a with entry e:
//     d/dlambda_e  = w_a (S - w_a) / (2 lambda_e)        (lambda_e > 0)
//                  = eps_e u_a (U_e - u_a) / 2            (lambda_e = 0, same-entry pairs)
//     d/deps_e     = w_a (S - w_a) / (2 eps_e)
//     d/dsigma_e   = sqrt(Lambda) du_a/dsigma (S - w_a),  du/dsigma = -4 n (2q^2 - q)/sigma beyond r_min
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_param_grad(ParamArgs a) {
    extern __shared__ __align__(16) unsigned char s_raw[];
    const int nt = a.tab.nt, ne = nt * nt;
    DevEntry* s_tab = reinterpret_cast<DevEntry*>(s_raw);
    double* s_acc = reinterpret_cast<double*>(s_raw + sizeof(DevEntry) * ne);
    for (int q = threadIdx.x; q < ne * 3; q += blockDim.x) s_acc[q] = 0.0;
    load_table_adj(s_tab, a.tab);
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m < a.N) {
        const float4 pm = a.pos[m];
        const int tm = ptype(pm.w);
        const int packed = a.nn[m];
        const int ns = nn_swap(packed), cnt = ns + nn_other(packed);
        double S = 0.0;
        for (int pass = 0; pass < 2; ++pass) {
            const int upto = pass == 0 ? cnt : ns;   // the triplet pass reads the swap range only
            for (int s = 0; s < upto; ++s) {
                const int slot = s < ns ? s : a.k_max - 1 - (s - ns);
                const int j = a.nlist[(size_t)slot * a.N + m];
                const float4 pj = a.pos[j];
                const int tj = ptype(pj.w);
                const DevEntry& e = s_tab[tm * nt + tj];
                if (e.kind == RC_KIND_NONE) continue;
                double dx, dy, dz;
                const double r2d = canon_r2(pm, pj, a.box, dx, dy, dz);
                if (!(r2d < e.rcut2)) continue;
                const int key = (tm < tj ? tm * nt + tj : tj * nt + tm) * 3;
                const float r2 = (float)r2d;
                const bool inside = r2d <= e.rmin2;
                if (pass == 0) {
                    float phi, g;
                    pair_eval(e, r2, phi, g);
                    const float q = qpow(e.sig2 / r2, e.n);
                    atomicAdd(&s_acc[key + 0], 0.5 * (double)(phi / e.eps));
                    atomicAdd(&s_acc[key + 1],
                              0.5 * (double)(4.0f * e.eps * (float)e.n * (2.0f * q * q - q) / e.sigma));
                    if (e.kind == RC_KIND_SWAP) S += (double)(e.sqrt_lam * vhat_value(e, inside, r2));
                } else {
                    if (e.kind != RC_KIND_SWAP) continue;
                    const float u = vhat_value(e, inside, r2);
                    const float w = e.sqrt_lam * u;
                    const double excl = S - (double)w;
                    if (e.lam > 0.0f) {
                        atomicAdd(&s_acc[key + 2], (double)w * excl / (2.0 * (double)e.lam));
                    } else {
                        // lambda = 0: E3 of same-entry pairs is lambda eps sum u_a u_b
                        double U = 0.0;
                        for (int t = 0; t < ns; ++t) {
                            const int k = a.nlist[(size_t)t * a.N + m];
                            const float4 pk = a.pos[k];
                            if (k == j || ptype(pk.w) != tj) continue;
                            double ex, ey, ez;
                            const double r2k = canon_r2(pm, pk, a.box, ex, ey, ez);
                            if (!(r2k < e.rcut2)) continue;
                            U += (double)vhat_value(e, r2k <= e.rmin2, (float)r2k);
                        }
                        atomicAdd(&s_acc[key + 2], 0.5 * (double)e.eps * (double)u * U);
                    }
                    atomicAdd(&s_acc[key + 0], (double)w * excl / (2.0 * (double)e.eps));
                    if (!inside) {
                        const float q = qpow(e.sig2 / r2, e.n);
                        const float du = -4.0f * (float)e.n * (2.0f * q * q - q) / e.sigma;
                        atomicAdd(&s_acc[key + 1], (double)(e.sqrt_lam * du) * excl);
                    }
                }
            }
        }
    }
    __syncthreads();
    for (int q = threadIdx.x; q < ne * 3; q += blockDim.x) a.part[(size_t)blockIdx.x * ne * 3 + q] = s_acc[q];
}

// ---------------------------------------------------------------------------
// Force-parameter VJP: out[e][w] = sum_m a_m . dF_m / dtheta_w(e), theta =
// (eps, sigma, lambda) of the unordered entry e.  With D = rhat . (a_j - a_m)
// the work of the adjoint field on a term:
//  pair (half per list direction):  a . F = -phi'(r) D, so
//     d/deps = -(phi'/eps) D,  d/dsigma = -4 eps n^2 (q - 4 q^2) / (sigma r) D
//  triplets of centre m (swap partners a inside r_cut, k_a = sqrt(lambda eps)
//  of the edge, u = vhat, u' = du/dr, D_a = rhat_a . (a_a - a_m)):
//     a . F = -T,  T = sum_{a != b} k_a k_b u_b u'_a D_a = S P - Q,
//     S = sum k u,  P = sum k u' D,  Q = sum k^2 u u' D.
//  Per partner entry e (sums restricted to partners of entry e carry the
//  subscript e; U, V, X are the unweighted sum u, sum u' D, sum u u' D):
//     dT/dlambda_e = eps_e (U V - X) + [P_e (S - S_e) + (P - P_e) S_e] / (2 lambda_e)
//     dT/deps_e    = lambda_e (U V - X) + [P_e (S - S_e) + (P - P_e) S_e] / (2 eps_e)
//     dT/dsigma_e  = A P - B + C S - G,  A = sum_e k u_s,  B = sum_e k^2 u_s u' D,
//                    C = sum_e k u'_s D,  G = sum_e k^2 u'_s D u
//  with u_s = du/dsigma = 4 n (q - 2q^2)/sigma and u'_s = 4 n^2 (4q^2 - q)/(sigma r)
//  beyond r_min (all zero inside, where u = 1).  The cross term of
//  dT/dlambda_e is taken as 0 when lambda_e = 0 (its derivative is unbounded
//  there), as in the energy gradient.
// ---------------------------------------------------------------------------
struct SwapTerms {  // u, u', du/dsigma, du'/dsigma of one swap edge
    float u, u1, us, u1s;
};

__device__ __forceinline__ SwapTerms swap_terms(const DevEntry& e, bool inside, float r2, float r) {
    SwapTerms t{1.0f, 0.0f, 0.0f, 0.0f};
    if (inside) return t;
    const float q = qpow(e.sig2 / r2, e.n);
    const float q2 = q * q, n = (float)e.n;
    t.u = 4.0f * (q - q2);
    t.u1 = 4.0f * n * (2.0f * q2 - q) / r;
    t.us = 4.0f * n * (q - 2.0f * q2) / e.sigma;
    t.u1s = 4.0f * n * n * (4.0f * q2 - q) / (e.sigma * r);
    return t;
}

__global__ __launch_bounds__(kBlock) void k_param_vjp(ParamArgs a) {
    extern __shared__ __align__(16) unsigned char s_raw[];
    const int nt = a.tab.nt, ne = nt * nt;
    DevEntry* s_tab = reinterpret_cast<DevEntry*>(s_raw);
    double* s_acc = reinterpret_cast<double*>(s_raw + sizeof(DevEntry) * ne);
    for (int q = threadIdx.x; q < ne * 3; q += blockDim.x) s_acc[q] = 0.0;
    load_table_adj(s_tab, a.tab);
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m < a.N) {
        const float4 pm = a.pos[m];
        const float4 am = a.adj[m];
        const int tm = ptype(pm.w);
        const int packed = a.nn[m];
        const int ns = nn_swap(packed), cnt = ns + nn_other(packed);
        // pass 0: pair terms (every entry) and the totals S, P over the swap partners
        double S = 0.0, P = 0.0;
        unsigned present = 0u;   // partner types met in the swap range
        for (int s = 0; s < cnt; ++s) {
            const int slot = s < ns ? s : a.k_max - 1 - (s - ns);
            const int j = a.nlist[(size_t)slot * a.N + m];
            const float4 pj = a.pos[j];
            const int tj = ptype(pj.w);
            const DevEntry& e = s_tab[tm * nt + tj];
            if (e.kind == RC_KIND_NONE) continue;
            double dx, dy, dz;
            const double r2d = canon_r2(pm, pj, a.box, dx, dy, dz);
            if (!(r2d < e.rcut2)) continue;
            const float r2 = (float)r2d, r = sqrtf(r2), ir = 1.0f / r;
            const float4 aj = a.adj[j];
            const float D = ((float)dx * (aj.x - am.x) + (float)dy * (aj.y - am.y) + (float)dz * (aj.z - am.z)) * ir;
            const float q = qpow(e.sig2 / r2, e.n), q2 = q * q, n = (float)e.n;
            const float d1 = 4.0f * e.eps * n * (q - 2.0f * q2) * ir;
            const float d1s = 4.0f * e.eps * n * n * (q - 4.0f * q2) / (e.sigma * r);
            const int key = (tm < tj ? tm * nt + tj : tj * nt + tm) * 3;
            atomicAdd(&s_acc[key + 0], -0.5 * (double)(d1 / e.eps * D));
            atomicAdd(&s_acc[key + 1], -0.5 * (double)(d1s * D));
            if (e.kind == RC_KIND_SWAP) {
                const SwapTerms t = swap_terms(e, r2d <= e.rmin2, r2, r);
                S += (double)(e.sqrt_lam * t.u);
                P += (double)(e.sqrt_lam * t.u1 * D);
                present |= 1u << tj;
            }
        }
        // pass 1: per partner entry, the restricted sums of the swap range
        for (int te = 0; te < nt; ++te) {
            if (!(present & (1u << te))) continue;
            const DevEntry& ee = s_tab[tm * nt + te];
            double U = 0, V = 0, X = 0, Se = 0, Pe = 0, A = 0, B = 0, C = 0, G = 0;
            for (int s = 0; s < ns; ++s) {
                const int j = a.nlist[(size_t)s * a.N + m];
                const float4 pj = a.pos[j];
                if (ptype(pj.w) != te) continue;
                double dx, dy, dz;
                const double r2d = canon_r2(pm, pj, a.box, dx, dy, dz);
                if (!(r2d < ee.rcut2)) continue;
                const float r2 = (float)r2d, r = sqrtf(r2);
                const float4 aj = a.adj[j];
                const float D = ((float)dx * (aj.x - am.x) + (float)dy * (aj.y - am.y) + (float)dz * (aj.z - am.z)) / r;
                const SwapTerms t = swap_terms(ee, r2d <= ee.rmin2, r2, r);
                const double k = (double)ee.sqrt_lam, k2 = k * k;
                U += t.u;
                V += (double)t.u1 * D;
                X += (double)t.u * t.u1 * D;
                Se += k * t.u;
                Pe += k * t.u1 * D;
                A += k * t.us;
                B += k2 * t.us * t.u1 * D;
                C += k * t.u1s * D;
                G += k2 * t.u1s * D * t.u;
            }
            const double same = U * V - X;
            const double cross = Pe * (S - Se) + (P - Pe) * Se;
            const double lam = (double)ee.lam, eps = (double)ee.eps;
            const double dl = eps * same + (lam > 0.0 ? cross / (2.0 * lam) : 0.0);
            const double de = lam * same + cross / (2.0 * eps);
            const double ds = A * P - B + C * S - G;
            const int key = (tm < te ? tm * nt + te : te * nt + tm) * 3;
            atomicAdd(&s_acc[key + 0], -de);
            atomicAdd(&s_acc[key + 1], -ds);
            atomicAdd(&s_acc[key + 2], -dl);
        }
    }
    __syncthreads();
    for (int q = threadIdx.x; q < ne * 3; q += blockDim.x) a.part[(size_t)blockIdx.x * ne * 3 + q] = s_acc[q];
}

__global__ __launch_bounds__(kBlock) void k_reduce_param(const double* __restrict__ part, int nblocks,
                                                        int nt, double* __restrict__ out) {
    // one block per output value (upper-triangle key), mirrored to both entries
    __shared__ double red[kBlock];
    const int q = blockIdx.x;
    const int ne3 = nt * nt * 3;
    double s = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += blockDim.x) s += part[(size_t)b * ne3 + q];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const int key = q / 3, comp = q % 3;
        const int ta = key / nt, tb = key % nt;
        if (ta <= tb) {
            out[(ta * nt + tb) * 3 + comp] = red[0];
            out[(tb * nt + ta) * 3 + comp] = red[0];
        }
    }
}

hipError_t launch_param(const ParamArgs& a, hipStream_t s) {
    const int ne = a.tab.nt * a.tab.nt;
    const size_t shm = sizeof(DevEntry) * ne + sizeof(double) * ne * 3;
    hipLaunchKernelGGL(k_param_grad, dim3(nblk(a.N, kBlock)), dim3(kBlock), shm, s, a);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Soft bond count B = sum over swap pairs i<j inside r_cut of vhat(r_ij)
// (1 for a bonded pair, r <= r_min, decaying to 0 at r_cut; eq. pot) and its
// gradient dB/dx_m = - sum_j vhat'(r_mj) rhat_mj over m's swap partners.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_soft_bonds(const float4* __restrict__ pos,
                                                      const int* __restrict__ nlist, const int* __restrict__ nn,
                                                      int k_max, int N, Table tab, Box box,
                                                      double* __restrict__ part, float4* __restrict__ grad) {
    extern __shared__ DevEntry s_tab[];
    __shared__ double s_w[kBlock / kWave];
    load_table_adj(s_tab, tab);
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    double b = 0.0;
    if (m < N) {
        const float4 pm = pos[m];
        const int tm = ptype(pm.w);
        const int ns = nn_swap(nn[m]);
        float gx = 0.f, gy = 0.f, gz = 0.f;
        for (int s = 0; s < ns; ++s) {
            const int j = nlist[(size_t)s * N + m];
            const float4 pj = pos[j];
            const DevEntry& e = s_tab[tm * tab.nt + ptype(pj.w)];
            if (e.kind != RC_KIND_SWAP) continue;
            double dx, dy, dz;
            const double r2d = canon_r2(pm, pj, box, dx, dy, dz);
            if (!(r2d < e.rcut2)) continue;
            float u, u1r;
            vhat_eval(e, r2d <= e.rmin2, (float)r2d, u, u1r);
            b += 0.5 * (double)u;
            gx -= u1r * (float)dx;
            gy -= u1r * (float)dy;
            gz -= u1r * (float)dz;
        }
        if (grad) grad[m] = make_float4(gx, gy, gz, 0.0f);
    }
    b = wave_sum(b);
    if ((threadIdx.x & (kWave - 1)) == 0) s_w[threadIdx.x / kWave] = b;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < kBlock / kWave; ++w) t += s_w[w];
        part[blockIdx.x] = t;
    }
}

__global__ __launch_bounds__(kBlock) void k_sum_doubles(const double* __restrict__ part, int nb,
                                                       double* __restrict__ out) {
    __shared__ double red[kBlock];
    double s = 0.0;
    for (int b = threadIdx.x; b < nb; b += blockDim.x) s += part[b];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = red[0];
}

hipError_t launch_soft_bonds(const float4* pos, const int* nlist, const int* nn, int k_max, int N, Table tab,
                             Box box, double* part, double* value, float4* grad, hipStream_t s) {
    const size_t shm = sizeof(DevEntry) * tab.nt * tab.nt;
    const int nb = nblk(N, kBlock);
    hipLaunchKernelGGL(k_soft_bonds, dim3(nb), dim3(kBlock), shm, s, pos, nlist, nn, k_max, N, tab, box, part, grad);
    hipLaunchKernelGGL(k_sum_doubles, dim3(1), dim3(kBlock), 0, s, part, nb, value);
    return hipGetLastError();
}

hipError_t launch_param_vjp(const ParamArgs& a, hipStream_t s) {
    const int ne = a.tab.nt * a.tab.nt;
    const size_t shm = sizeof(DevEntry) * ne + sizeof(double) * ne * 3;
    hipLaunchKernelGGL(k_param_vjp, dim3(nblk(a.N, kBlock)), dim3(kBlock), shm, s, a);
    return hipGetLastError();
}

hipError_t launch_reduce_param(const double* part, int nblocks, int nt, double* out, hipStream_t s) {
    hipLaunchKernelGGL(k_reduce_param, dim3(nt * nt * 3), dim3(kBlock), 0, s, part, nblocks, nt, out);
    return hipGetLastError();
}

}  // namespace rc
