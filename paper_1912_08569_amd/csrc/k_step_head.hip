// Fused MD step for short neighbour lists (RC_FORM_HEAD).
//
// Same forces, energies, virials and integrator as the walk form of k_step
// (the three-body forces of eq. 3bp, centred on the particle itself and on
// each of its swap partners), evaluated with as few dependent memory round
// trips as the data allow.  At a mean list length near one (the 1M-particle
// self-assembly mixture) the walk form spends its time waiting on a chain of
// dependent loads rather than moving bytes; this kernel issues every load
// whose address is already known together:
//
//   level 1: own position, velocity and list count, plus the first HS swap
//            slots and the first HO other slots of the particle's own list
//            (read whether or not the list reaches them: a wave fetches those
//            list lines anyway, and an unused slot is never interpreted);
//   level 2: positions of those partners, and for swap partners their list
//            count and first two swap slots (the two-hop walk of a partner
//            beyond r_min needs them);
//   level 3: positions of the partners' other swap partners, only where a
//            partner lies between r_min and r_cut and has another partner;
//
// and the centre's own triplet terms come from registers instead of a second
// walk of the list.  Slots beyond the heads (rare at short lists) are walked
// as in the walk form.  Each particle's terms are summed in list-slot order
// with the walk form's arithmetic, so both forms give the same trajectory up
// to the contraction choices of the compiler.
#include "rc_internal.h"
#include "rc_gather.h"
#include "rc_step.h"

#ifndef HEAD_WAVES
#define HEAD_WAVES 4
#endif

namespace rc {

namespace {

// One list entry of particle m once the partner's position is known.
struct HeadEnt {
    float dx, dy, dz;   // x_j - x_m (FP32 of the canonical FP64 difference)
    float f;            // F_m += f d (pair part, plus the partner-centred triplet part)
    float phi, g;       // pair energy and phi'/r (energy and virial steps)
    float w, u1r, sl;   // swap entries: sqrt(Lambda) vhat, vhat'/r, sqrt(Lambda)
    int on;             // 0 outside the cutoff or no interaction, 1 pair only, 2 swap pair
};

__device__ __forceinline__ void head_eval(const DevEntry* trow, const float4& pm, const float4& pj, const Box& box,
                                          HeadEnt& e) {
    e.on = 0;
    const DevEntry& en = trow[ptype(pj.w)];
    if (en.kind == RC_KIND_NONE) return;
    const PairGeom pg = pair_geom(pm, pj, box, en);
    if (!pg.cut) return;
    const float r2 = pg.r2;
    e.dx = pg.dx;
    e.dy = pg.dy;
    e.dz = pg.dz;
    float uu;
    pair_vhat_eval(en, en.kind == RC_KIND_SWAP, pg.inside, r2, e.phi, e.g, uu, e.u1r);
    e.f = e.g;
    e.on = 1;
    if (en.kind == RC_KIND_SWAP) {
        e.w = en.sqrt_lam * uu;
        e.sl = en.sqrt_lam;
        e.on = 2;
    }
}

// the partner-centred triplet terms need S_j - w_jm (walk of j's swap range)
__device__ __forceinline__ bool head_needs_hop(const HeadEnt& e) {
    return e.on == 2 && e.u1r != 0.0f && e.sl != 0.0f;
}

// one term of the partner sum: w_jk of centre j (table row of j) and partner k
__device__ __forceinline__ float hop_term(const DevEntry* tab, int nt, const float4& pj, const float4& pk,
                                          const Box& box) {
    const DevEntry& e = tab[ptype(pj.w) * nt + ptype(pk.w)];
    if (e.kind == RC_KIND_NONE) return 0.0f;
    const PairGeom g = pair_geom(pj, pk, box, e);
    if (!g.cut) return 0.0f;
    return e.sqrt_lam * vhat_value(e, g.inside, g.r2);
}

// accumulation of one entry in slot order; the products are rounded before the
// sums, as where the walk form stages them
template <bool EV>
__device__ __forceinline__ void head_acc(const HeadEnt& e, Acc& acc, double& S, int& nact) {
#pragma clang fp contract(off)
    if (e.on == 0) return;
    acc.fx += e.f * e.dx;
    acc.fy += e.f * e.dy;
    acc.fz += e.f * e.dz;
    if (e.on == 2) {
        S += (double)e.w;
        ++nact;
    }
    if (EV) {
        const float h = -0.5f * e.g;
        acc.e += 0.5f * e.phi;
        acc.w[0] += h * e.dx * e.dx;
        acc.w[1] += h * e.dy * e.dy;
        acc.w[2] += h * e.dz * e.dz;
        acc.w[3] += h * e.dx * e.dy;
        acc.w[4] += h * e.dx * e.dz;
        acc.w[5] += h * e.dy * e.dz;
    }
}

// the terms centred on m for one of its active swap partners (prefix = sum of
// the w of earlier partners, for the energy)
template <bool EV>
__device__ __forceinline__ void head_centre(float w, float u1r, float sl, float dx, float dy, float dz, double S,
                                            float& prefix, Acc& acc) {
    const float excl = (float)(S - (double)w);
    const float c = sl * u1r * excl;  // centre gets +c d
    acc.fx += c * dx;
    acc.fy += c * dy;
    acc.fz += c * dz;
    if (EV) {
        acc.e += w * prefix;
        prefix += w;
        acc_virial(acc, -c, dx, dy, dz);
    }
}

}  // namespace

// contribution of an entry of the other range (no swap kind there: the list
// keeps swap-kind neighbours in the swap range), reduced as soon as the
// partner's position arrives: the rounded force products and, on energy
// steps, the energy share and virial products
template <bool EV>
struct OtherTerm {
    float c[EV ? 10 : 3];
};

template <bool EV>
__device__ __forceinline__ void other_term(const HeadEnt& e, OtherTerm<EV>& t) {
#pragma clang fp contract(off)
    t.c[0] = e.f * e.dx;
    t.c[1] = e.f * e.dy;
    t.c[2] = e.f * e.dz;
    if (EV) {
        const float h = -0.5f * e.g;
        t.c[3] = 0.5f * e.phi;
        t.c[4] = h * e.dx * e.dx;
        t.c[5] = h * e.dy * e.dy;
        t.c[6] = h * e.dz * e.dz;
        t.c[7] = h * e.dx * e.dy;
        t.c[8] = h * e.dx * e.dz;
        t.c[9] = h * e.dy * e.dz;
    }
}

template <bool EV>
__device__ __forceinline__ void other_acc(const OtherTerm<EV>& t, Acc& acc) {
#pragma clang fp contract(off)
    acc.fx += t.c[0];
    acc.fy += t.c[1];
    acc.fz += t.c[2];
    if (EV) {
        acc.e += t.c[3];
#pragma unroll
        for (int q = 0; q < 6; ++q) acc.w[q] += t.c[4 + q];
    }
}

template <bool EV, int HS, int HO>
__device__ __forceinline__ void step_head_body(const StepArgs& a) {
    extern __shared__ DevEntry s_tab[];
    const int nt = a.tab.nt;
    const int blk = xcd_block(gridDim.x);
    const int m = blk * kWave + threadIdx.x;
    const int N = a.N, K = a.k_max;
    const bool live = m < N;
    const int* __restrict__ nl = a.nlist;
    const float4* __restrict__ pos = a.pos_in;

    // ---- level 1: own position and list heads -----------------------------------
    float4 pm = make_float4(0.f, 0.f, 0.f, 0.f);
    int packed = 0;
    int hs[HS], ho[HO];
#pragma unroll
    for (int s = 0; s < HS; ++s) hs[s] = 0;
#pragma unroll
    for (int s = 0; s < HO; ++s) ho[s] = 0;
    if (live) {
        pm = pos[m];
        packed = a.nn[m];
#pragma unroll
        for (int s = 0; s < HS; ++s) hs[s] = nl[(size_t)min(s, K - 1) * N + m];
#pragma unroll
        for (int s = 0; s < HO; ++s) ho[s] = nl[(size_t)max(K - 1 - s, 0) * N + m];
    }
    load_table(s_tab, a.tab);
    const Box& box = a.box;
    const int ns = nn_swap(packed), no = nn_other(packed);
    const DevEntry* trow = s_tab + ptype(pm.w) * nt;

    // ---- level 2: partner positions; list heads of swap partners -------------------
    float4 ps[HS], po[HO];
    int pnn[HS], pk0[HS], pk1[HS];
#pragma unroll
    for (int s = 0; s < HS; ++s) {
        pnn[s] = 0;
        pk0[s] = pk1[s] = -1;
        if (s < ns) {
            const int j = hs[s];
            ps[s] = pos[j];
            pnn[s] = a.nn[j];
            pk0[s] = nl[j];
            pk1[s] = K > 1 ? nl[(size_t)N + j] : -1;
        }
    }
#pragma unroll
    for (int s = 0; s < HO; ++s)
        if (s < no) po[s] = pos[ho[s]];

    // other head entries reduce to their products at once
    OtherTerm<EV> ot[HO];
    int on_other = 0;
#pragma unroll
    for (int s = 0; s < HO; ++s) {
        if (s < no) {
            HeadEnt e;
            head_eval(trow, pm, po[s], box, e);
            if (e.on) {
                on_other |= 1 << s;
                other_term<EV>(e, ot[s]);
            }
        }
    }

    // ---- level 3: swap head entries, the partner sums they need, own velocity ------
    HeadEnt es[HS];
    float4 pk[HS][2];
#pragma unroll
    for (int s = 0; s < HS; ++s) {
        es[s].on = 0;
        if (s < ns) head_eval(trow, pm, ps[s], box, es[s]);
        if (head_needs_hop(es[s])) {
            const int nsj = nn_swap(pnn[s]);
            if (nsj > 0 && pk0[s] != m) pk[s][0] = pos[pk0[s]];
            if (nsj > 1 && pk1[s] != m) pk[s][1] = pos[pk1[s]];
        }
    }
    const float4 vm = live ? a.vel[m] : make_float4(0.f, 0.f, 0.f, 0.f);
    const uint64_t step = a.step + (a.step_base ? *a.step_base : 0ull);
#pragma unroll
    for (int s = 0; s < HS; ++s) {
        if (!head_needs_hop(es[s])) continue;
        const int nsj = nn_swap(pnn[s]);
        float psum = 0.0f;
        if (nsj > 0 && pk0[s] != m) psum += hop_term(s_tab, nt, ps[s], pk[s][0], box);
        if (nsj > 1 && pk1[s] != m) psum += hop_term(s_tab, nt, ps[s], pk[s][1], box);
        const int j = hs[s];
        for (int q = 2; q < nsj; ++q) {  // partners with more than two swap neighbours
            const int k = nl[(size_t)q * N + j];
            if (k == m) continue;
            psum += hop_term(s_tab, nt, ps[s], pos[k], box);
        }
        es[s].f += es[s].sl * es[s].u1r * psum;
    }

    // ---- accumulate in slot order: swap range, then the other range ---------------
    Acc acc = {};
    double S = 0.0;
    int nact = 0;
#pragma unroll
    for (int s = 0; s < HS; ++s)
        if (s < ns) head_acc<EV>(es[s], acc, S, nact);
    for (int s = HS; s < ns; ++s) {  // swap slots beyond the head
        const int j = nl[(size_t)s * N + m];
        const float4 pj = pos[j];
        HeadEnt e;
        head_eval(trow, pm, pj, box, e);
        if (head_needs_hop(e))
            e.f += e.sl * e.u1r * partner_sum_excluding(j, pj, m, nl, a.nn, K, N, pos, s_tab, nt, box);
        head_acc<EV>(e, acc, S, nact);
    }
#pragma unroll
    for (int s = 0; s < HO; ++s)
        if (on_other & (1 << s)) other_acc<EV>(ot[s], acc);
    for (int s = HO; s < no; ++s) {  // other slots beyond the head
        HeadEnt e;
        head_eval(trow, pm, pos[nl[(size_t)(K - 1 - s) * N + m]], box, e);
        head_acc<EV>(e, acc, S, nact);
    }

    // ---- triplet terms centred on m --------------------------------------------------
    if (live && nact >= 2) {
        float prefix = 0.0f;
        if (ns <= HS) {
#pragma unroll
            for (int s = 0; s < HS; ++s)
                if (s < ns && es[s].on == 2)
                    head_centre<EV>(es[s].w, es[s].u1r, es[s].sl, es[s].dx, es[s].dy, es[s].dz, S, prefix, acc);
        } else {
            walk_list<true>(m, pm, ptype(pm.w), nl, packed, K, N, pos, s_tab, nt, box, -1,
                            [&](int, const float4&, const DevEntry& e, const PairGeom& g) {
                                float u, u1r;
                                vhat_eval(e, g.inside, g.r2, u, u1r);
                                head_centre<EV>(e.sqrt_lam * u, u1r, e.sqrt_lam, g.dx, g.dy, g.dz, S, prefix, acc);
                            });
        }
    }
    if (a.bonds && live) fene_add<EV>(ptag(pm.w), pm, a.bonds, a.rtag, pos, box, a.fene_k, a.fene_r02, acc);
    step_finish<EV>(a, a.pos_out, m, blk, live, pm, vm, acc, box, 0, a.seed, step);
}

// list heads: two swap slots, three other slots.  The step kernel is held to
// eight waves per SIMD (64 VGPRs); the energy step (one in a log period) is
// left to the compiler.
constexpr int kHeadSwap = 2;
constexpr int kHeadOther = 3;

__global__ __launch_bounds__(kWave) __attribute__((amdgpu_waves_per_eu(HEAD_WAVES))) void k_step_head(StepArgs a) {
    step_head_body<false, kHeadSwap, kHeadOther>(a);
}
__global__ __launch_bounds__(kWave) void k_step_head_ev(StepArgs a) { step_head_body<true, kHeadSwap, kHeadOther>(a); }

const void* step_head_fn(bool ev) {
    return ev ? reinterpret_cast<const void*>(&k_step_head_ev) : reinterpret_cast<const void*>(&k_step_head);
}

}  // namespace rc
