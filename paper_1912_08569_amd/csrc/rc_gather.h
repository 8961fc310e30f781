// Device-side building blocks shared by the force, step and batch kernels:
// list walks, the two-hop partner sum, and the wavefront-cooperative gather.
//
// Notation: for a centre c and a swap partner a inside r_cut, w_ca =
// sqrt(Lambda_ca) vhat(r_ca); a triplet term is w_ca w_cb (eq. 3bp with
// Lambda_cab = sqrt(Lambda_ca Lambda_cb)); d = x_a - x_c (minimum image).
#pragma once

#include "rc_internal.h"

namespace rc {

// The system a particle belongs to: its box and its coefficient table.
// One periodic system (table staged in LDS):
struct OneSystem {
    const DevEntry* tab;
    int nt;
    Box box;
    __device__ __forceinline__ const DevEntry* table(int) const { return tab; }
    __device__ __forceinline__ const Box& boxof(int) const { return box; }
};

__device__ __forceinline__ void load_table(DevEntry* s_tab, const Table& t) {
    const int n = t.nt * t.nt;
    for (int q = threadIdx.x; q < n; q += blockDim.x) s_tab[q] = t.e[q];
    __syncthreads();
}

// Position of particle j: from the wavefront's LDS copy of the positions of
// particles [base, base + 64) when j is one of them (most list neighbours are:
// the particles are in Morton order), else from global memory.
struct PosWin {
    const float4* s;   // LDS copy, or NULL (always global)
    int base;
    __device__ __forceinline__ float4 get(const float4* pos, int j) const {
        const unsigned lj = (unsigned)(j - base);
        float4 p;
        if (s && lj < (unsigned)kWave) p = s[lj];
        else p = pos[j];
        return p;
    }
};

// Walk of particle m's list: the swap range (slots 0 .. ns-1) and, unless
// SWAP_ONLY, the other range (slots k_max-1 down to k_max-no).  For every
// neighbour j != skip inside its cutoff (canonical decision) the functor gets
// (j, pj, entry, geometry of m -> j).
template <bool SWAP_ONLY, typename F>
__device__ __forceinline__ void walk_list_w(int m, const float4& pm, int tm, const int* nlist, int packed,
                                            int k_max, int N, const float4* pos, const DevEntry* tab, int nt,
                                            const Box& box, int skip, PosWin win, F&& f) {
    auto visit = [&](int j) {
        if (j == skip) return;
        const float4 pj = win.get(pos, j);
        const DevEntry& e = tab[tm * nt + ptype(pj.w)];
        if (e.kind == RC_KIND_NONE) return;
        const PairGeom g = pair_geom(pm, pj, box, e);
        if (!g.cut) return;
        f(j, pj, e, g);
    };
    const int ns = nn_swap(packed);
    for (int s = 0; s < ns; ++s) visit(nlist[(size_t)s * N + m]);
    if (!SWAP_ONLY) {
        const int no = nn_other(packed);
        for (int s = 0; s < no; ++s) visit(nlist[(size_t)(k_max - 1 - s) * N + m]);
    }
}

template <bool SWAP_ONLY, typename F>
__device__ __forceinline__ void walk_list(int m, const float4& pm, int tm, const int* nlist, int packed,
                                          int k_max, int N, const float4* pos, const DevEntry* tab, int nt,
                                          const Box& box, int skip, F&& f) {
    walk_list_w<SWAP_ONLY>(m, pm, tm, nlist, packed, k_max, N, pos, tab, nt, box, skip, PosWin{nullptr, 0}, f);
}

// sum of w_ck over the swap partners k of centre c inside r_cut, except 'skip'
// (only c's swap range is read: for a bonded pair it usually holds skip alone)
__device__ __forceinline__ float partner_sum_excluding(int c, const float4& pc, int skip,
                                                       const int* nlist, const int* nn, int k_max, int N,
                                                       const float4* pos, const DevEntry* tab,
                                                       int nt, const Box& box, PosWin win = PosWin{nullptr, 0}) {
    float s = 0.0f;
    walk_list_w<true>(c, pc, ptype(pc.w), nlist, nn[c], k_max, N, pos, tab, nt, box, skip, win,
                    [&](int, const float4&, const DevEntry& e, const PairGeom& g) {
                        s += e.sqrt_lam * vhat_value(e, g.inside, g.r2);
                    });
    return s;
}

struct Acc {
    float fx, fy, fz, e;
    float w[6];     // xx yy zz xy xz yz
    unsigned nbond; // EV gathers: bonds (swap, canonical r^2 < r_min^2, owner < neighbour) among the
                    // entries this lane evaluated (a wavefront's sum is its particles' bond count)
};

__device__ __forceinline__ void acc_virial(Acc& a, float c, float dx, float dy, float dz) {
    // adds c * d (x) d  (a term (r)_a (F)_b with F = c d)
    a.w[0] += c * dx * dx;
    a.w[1] += c * dy * dy;
    a.w[2] += c * dz * dz;
    a.w[3] += c * dx * dy;
    a.w[4] += c * dx * dz;
    a.w[5] += c * dy * dz;
}

// ---------------------------------------------------------------------------
// Wavefront-cooperative gather (one wavefront per block).  The 64 lanes own
// 64 consecutive particles; their (particle, list slot) entries are laid out
// flat (exclusive scan of the list lengths) and every lane evaluates PL
// entries per pass, so a wave needs about (sum of list lengths)/(64 PL)
// passes instead of one pass per slot of its longest list.  Per-entry
// contributions are staged in LDS and each owner lane sums its own entries in
// slot order (deterministic, and the same for every PL).
//
// Three-body forces, two forms of the same sum (eq. 3bp; the energy of centre
// c is sum_{a<b} w_ca w_cb = (S_c^2 - sum_a w_ca^2)/2 with S_c = sum_a w_ca):
//  * walk (SF = false): an entry (m, j) inside r_cut and beyond r_min adds
//    the term centred on j by walking j's swap range for S_j - w_jm; the
//    terms centred on m are added afterwards by a walk of m's own swap range
//    (only for centres with two or more active partners).
//  * sums (SF = true): S of every particle is precomputed (swap_sums) and an
//    entry adds both parts at once with the factor (S_m - w) + (S_j - w).
// ---------------------------------------------------------------------------
template <bool EV, bool SF>
struct Stage {
    // walk: fx fy fz w active [e w0..w5];  sums: fx fy fz [e w0..w5]
    static constexpr int n = SF ? (EV ? 10 : 3) : (EV ? 12 : 5);
    static constexpr int e = SF ? 3 : 5;   // first EV column
};
// PL = flattened entries each lane evaluates per pass (the gather width).
constexpr int kDefaultWidth = 2;

// Most wavefronts one workgroup of the multi-wave (WS) gather holds.
constexpr int kGatherMaxWaves = 16;

// Barrier of the gather's LDS exchange.  With one wavefront per block (WS =
// false) it is the block barrier; with several (WS = true) the exchange stays
// inside each wavefront, whose trip counts differ, so it is a wavefront-level
// barrier with workgroup-scope fences (LDS writes complete before the reads).
template <bool WS>
__device__ __forceinline__ void gather_sync() {
    if constexpr (WS) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    } else {
        __syncthreads();
    }
}

// PK: the entries come from the packed copy of the list (pl_j, pl_o: neighbour
// and owner lane of every flattened entry, pack_wave_lists) instead of the
// owner map in LDS and a search of the list columns; same entries, same order.
template <bool EV, int kPerLane, bool SF, class Ctx, bool WS = false, bool PK = false>
__device__ __forceinline__ void wave_gather(int base_m, bool live, const float4& pm, int packed,
                                            const float4* pos, const int* nlist, const int* nn, int k_max,
                                            int N, const Ctx& ctx, Acc& acc, const float* ssum = nullptr,
                                            const int* pl_j = nullptr, const unsigned char* pl_o = nullptr) {
    const int nt = ctx.nt;
    constexpr int NC = Stage<EV, SF>::n;
    constexpr int CE = Stage<EV, SF>::e;
    constexpr int W = kPerLane * kWave;  // entries per pass
    constexpr int NW = WS ? kGatherMaxWaves : 1;  // LDS slices, one per wavefront
    __shared__ int s_off_w[NW][kWave + 1];
    __shared__ int s_ns_w[NW][kWave];
    __shared__ unsigned char s_own_w[NW][W];  // owner lane of each entry of the current pass
    __shared__ float4 s_pos_w[NW][kWave];
    __shared__ float s_S_w[NW][SF ? kWave : 1];
    __shared__ float s_c_w[NW][NC][W];
    const int lane = threadIdx.x & (kWave - 1);
    const int wv = WS ? (int)(threadIdx.x / kWave) : 0;
    int* s_off = s_off_w[wv];
    int* s_ns = s_ns_w[wv];
    unsigned char* s_own = s_own_w[wv];
    float4* s_pos = s_pos_w[wv];
    float* s_S = s_S_w[wv];
    float(*s_c)[W] = s_c_w[wv];
    const int ns = live ? nn_swap(packed) : 0;
    const int cnt = live ? ns + nn_other(packed) : 0;
    const int inc = wave_inclusive_scan(cnt);  // every lane of the wavefront is active here
    const int my_off = inc - cnt;
    if (!PK) {
        s_off[lane] = my_off;
        if (lane == kWave - 1) s_off[kWave] = inc;
        s_ns[lane] = ns;
    }
    s_pos[lane] = pm;
    if (SF) s_S[lane] = live ? ssum[base_m + lane] : 0.0f;
    gather_sync<WS>();
    const int T = PK ? __builtin_amdgcn_readlane(inc, kWave - 1) : s_off[kWave];
    const size_t pk_base = (size_t)base_m * k_max;  // the wavefront's region of the packed list
    double S = 0.0;
    int nact = 0;
    for (int base = 0; base < T; base += W) {
        if (!PK) {
            // owner map of the pass: each lane marks its own entries in the window
            const int q1 = min(my_off + cnt, base + W) - base;
            for (int q = max(my_off, base) - base; q < q1; ++q) s_own[q] = (unsigned char)lane;
            gather_sync<WS>();
        }
        // locate and load all entries of this pass first, so their memory
        // latencies overlap (list index, then neighbour position)
        int own[kPerLane], jj[kPerLane];
        bool sw[kPerLane];
        float4 pj[kPerLane];
        float sj[kPerLane];
#pragma unroll
        for (int u = 0; u < kPerLane; ++u) {
            const int e = base + u * kWave + lane;
            own[u] = -1;
            jj[u] = 0;
            sw[u] = false;
            if (e < T) {
                if (PK) {
                    own[u] = pl_o[pk_base + e];
                    jj[u] = pl_j[pk_base + e];
                    sw[u] = true;  // S_j is read for every entry and used for swap-kind ones only
                } else {
                    const int lo = s_own[e - base];
                    const int sl = e - s_off[lo], nso = s_ns[lo];
                    sw[u] = sl < nso;
                    const int slot = sw[u] ? sl : k_max - 1 - (sl - nso);
                    own[u] = lo;
                    jj[u] = nlist[(size_t)slot * N + base_m + lo];
                }
            }
        }
#pragma unroll
        for (int u = 0; u < kPerLane; ++u) {
            pj[u] = pm;
            if (own[u] >= 0) {
                // neighbours among the wave's own 64 particles come from its LDS copy
                const unsigned lj = (unsigned)(jj[u] - base_m);
                if (lj < (unsigned)kWave)
                    pj[u] = s_pos[lj];
                else
                    pj[u] = pos[jj[u]];
            }
            if (SF) {
                const unsigned lj = (unsigned)(jj[u] - base_m);
                sj[u] = sw[u] ? (lj < (unsigned)kWave ? s_S[lj] : ssum[jj[u]]) : 0.0f;
            }
        }
#pragma unroll
        for (int u = 0; u < kPerLane; ++u) {
            float c[NC];
#pragma unroll
            for (int q = 0; q < NC; ++q) c[q] = 0.0f;
            if (own[u] >= 0) {
                const int mo = base_m + own[u];
                const float4 po = s_pos[own[u]];
                const DevEntry* tab = ctx.table(own[u]);
                const Box& box = ctx.boxof(own[u]);
                const DevEntry& en = tab[ptype(po.w) * nt + ptype(pj[u].w)];
                if (en.kind != RC_KIND_NONE) {
                    const PairGeom pg = pair_geom(po, pj[u], box, en);
                    if (pg.cut) {
                        if (EV && en.kind == RC_KIND_SWAP && pg.bond && jj[u] > mo) ++acc.nbond;
                        const float r2 = pg.r2, dx = pg.dx, dy = pg.dy, dz = pg.dz;
                        float phi, g, uu, u1r;
                        pair_vhat_eval(en, en.kind == RC_KIND_SWAP, pg.inside, r2, phi, g, uu, u1r);
                        float f = g;
                        float h = -0.5f * g;     // virial weight of d (x) d
                        float e3 = 0.0f;         // triplet energy share (sums form)
                        if (en.kind == RC_KIND_SWAP) {
                            const float w = en.sqrt_lam * uu;
                            if (SF) {
                                const float so = s_S[own[u]] - w;   // S_m - w
                                if (u1r != 0.0f && en.sqrt_lam != 0.0f) {
                                    const float k1 = en.sqrt_lam * u1r;
                                    const float cc = k1 * so;       // terms centred on m
                                    f += cc + k1 * (sj[u] - w);     // and on j
                                    h -= cc;
                                }
                                e3 = 0.5f * w * so;
                            } else {
                                c[3] = w;
                                c[4] = 1.0f;
                                if (u1r != 0.0f && en.sqrt_lam != 0.0f)  // owner is a partner of centre j
                                    f += en.sqrt_lam * u1r *
                                         partner_sum_excluding(jj[u], pj[u], mo, nlist, nn, k_max, N, pos, tab, nt,
                                                               box);
                            }
                        }
                        if (EV) {
                            c[CE] = 0.5f * phi + e3;
                            c[CE + 1] = h * dx * dx; c[CE + 2] = h * dy * dy; c[CE + 3] = h * dz * dz;
                            c[CE + 4] = h * dx * dy; c[CE + 5] = h * dx * dz; c[CE + 6] = h * dy * dz;
                        }
                        c[0] = f * dx;
                        c[1] = f * dy;
                        c[2] = f * dz;
                    }
                }
            }
#pragma unroll
            for (int q = 0; q < NC; ++q) s_c[q][u * kWave + lane] = c[q];
        }
        gather_sync<WS>();
        const int lo = max(my_off, base) - base, hi = min(my_off + cnt, base + W) - base;
        for (int q = lo; q < hi; ++q) {
            acc.fx += s_c[0][q];
            acc.fy += s_c[1][q];
            acc.fz += s_c[2][q];
            if (!SF) {
                S += (double)s_c[3][q];
                nact += s_c[4][q] != 0.0f;
            }
            if (EV) {
                acc.e += s_c[CE][q];
#pragma unroll
                for (int w = 0; w < 6; ++w) acc.w[w] += s_c[CE + 1 + w][q];
            }
        }
        gather_sync<WS>();
    }
    if (!SF && live && nact >= 2) {
        const int m = base_m + lane;
        float prefix = 0.0f;
        walk_list<true>(m, pm, ptype(pm.w), nlist, packed, k_max, N, pos, ctx.table(lane), nt, ctx.boxof(lane), -1,
                        [&](int, const float4&, const DevEntry& e, const PairGeom& g) {
                            const float dx = g.dx, dy = g.dy, dz = g.dz;
                            float u, u1r;
                            vhat_eval(e, g.inside, g.r2, u, u1r);
                            const float w = e.sqrt_lam * u;
                            const float excl = (float)(S - (double)w);
                            const float c = e.sqrt_lam * u1r * excl;  // centre gets +c d
                            acc.fx += c * dx;
                            acc.fy += c * dy;
                            acc.fz += c * dz;
                            if (EV) {
                                acc.e += w * prefix;  // sum over pairs b < a of w_b w_a
                                prefix += w;
                                acc_virial(acc, -c, dx, dy, dz);  // (d) (x) (force on a = -c d)
                            }
                        });
    }
}

// First pass of the sums form for one particle m: S_m = sum of w_mj over m's
// swap range inside r_cut, in slot order (FP32).  Positions of four slots
// are requested before any is used.
__device__ __forceinline__ float swap_sum(int m, const float4& pm, int packed, const float4* pos,
                                          const int* nlist, int N, const DevEntry* tab, int nt, const Box& box) {
    const int ns = nn_swap(packed);
    const int tm = ptype(pm.w);
    float s = 0.0f;
    for (int b = 0; b < ns; b += 4) {
        int j[4];
        float4 p[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) j[u] = (b + u < ns) ? nlist[(size_t)(b + u) * N + m] : -1;
#pragma unroll
        for (int u = 0; u < 4; ++u) p[u] = j[u] >= 0 ? pos[j[u]] : pm;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            if (j[u] < 0) continue;
            const DevEntry& e = tab[tm * nt + ptype(p[u].w)];
            if (e.kind == RC_KIND_NONE) continue;
            const PairGeom g = pair_geom(pm, p[u], box, e);
            if (g.cut) s += e.sqrt_lam * vhat_value(e, g.inside, g.r2);
        }
    }
    return s;
}

// FENE springs of particle m (tag-indexed partner table, -1 = none; rtag
// maps a tag to its current index): F_m += K d / (1 - r^2/R0^2) per bond,
// d = x_j - x_m (minimum image); half the bond energy -(K R0^2/2) ln(1 -
// r^2/R0^2) and half its virial -K d d /(1 - r^2/R0^2) go to m.  A bond
// stretched to R0 or beyond yields a non-finite force.
template <bool EV>
__device__ __forceinline__ void fene_add(int tag, const float4& pm, const int2* bonds, const int* rtag,
                                         const float4* pos, const Box& box, float K, float R02, Acc& acc) {
    const int2 b = bonds[tag];
    const int part[2] = {b.x, b.y};
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        if (part[q] < 0) continue;
        const float4 pj = pos[rtag[part[q]]];
        double dxd, dyd, dzd;
        const double r2d = canon_r2(pm, pj, box, dxd, dyd, dzd);
        const float dx = (float)dxd, dy = (float)dyd, dz = (float)dzd;
        const float s = 1.0f - (float)r2d / R02;
        const float g = s > 0.0f ? K / s : __int_as_float(0x7fc00000);
        acc.fx += g * dx;
        acc.fy += g * dy;
        acc.fz += g * dz;
        if (EV) {
            acc.e += -0.25f * K * R02 * logf(s);
            acc_virial(acc, -0.5f * g, dx, dy, dz);
        }
    }
}

// A double moved across lanes by a DPP pattern with a source for every lane.
template <int CTRL>
__device__ __forceinline__ double dpp_mov(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_mov_dpp((int)b, CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xf, 0xf, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// Wavefront sums of NW <= 16 doubles (padded to 16), stored to out[0 .. NW).
// Every lane must be active.  A halving butterfly: at each of the four levels
// inside a 16-lane row a lane and its partner (lane ^ 1, ^ 2, ^ 4, ^ 8) each
// keep half of the values and add the partner's copy of that half, so one
// DPP move per kept value instead of one per value and level; then the two
// levels across rows (^ 16, ^ 32), one value each.  Value s ends in the lanes
// whose low four bits, reversed, read s.  19 moves and 17 adds of doubles
// instead of 96 of each for 16 values; a fixed order of additions.
template <int NW>
__device__ __forceinline__ void wave_sum_store(double (&v)[NW], double* out) {
    static_assert(NW <= 16, "at most 16 sums");
    const int lane = (int)(threadIdx.x & (kWave - 1));
    const bool b1 = (lane & 1) != 0, b2 = (lane & 2) != 0, b3 = (lane & 4) != 0, b4 = (lane & 8) != 0;
    double a[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) a[q] = q < NW ? v[q] : 0.0;
    double b[8], c[4], d[2];
#pragma unroll
    for (int q = 0; q < 8; ++q)   // partner lane ^ 1 (quad_perm 1, 0, 3, 2); odd lanes keep the upper half
        b[q] = (b1 ? a[q + 8] : a[q]) + dpp_mov<0xB1>(b1 ? a[q] : a[q + 8]);
#pragma unroll
    for (int q = 0; q < 4; ++q)   // lane ^ 2 (quad_perm 2, 3, 0, 1)
        c[q] = (b2 ? b[q + 4] : b[q]) + dpp_mov<0x4E>(b2 ? b[q] : b[q + 4]);
#pragma unroll
    for (int q = 0; q < 2; ++q) {   // lane ^ 4: from lane - 4 (row_ror:4) or lane + 4 (row_ror:12)
        const double send = b3 ? c[q] : c[q + 2];
        const double r4 = dpp_mov<0x124>(send), r12 = dpp_mov<0x12C>(send);
        d[q] = (b3 ? c[q + 2] : c[q]) + (b3 ? r4 : r12);
    }
    double e = (b4 ? d[1] : d[0]) + dpp_mov<0x128>(b4 ? d[0] : d[1]);   // lane ^ 8 (row_ror:8)
    e += __shfl_xor(e, 16, kWave);
    e += __shfl_xor(e, 32, kWave);
    const int q = (b1 ? 8 : 0) + (b2 ? 4 : 0) + (b3 ? 2 : 0) + (b4 ? 1 : 0);
    if (lane < 16 && q < NW) out[q] = e;
}


}  // namespace rc
