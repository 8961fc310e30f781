// Forces, energy and virial of the swap potential; the fused MD step; bond
// counting.  gfx950, wave64.
//
// Notation: for a centre c and a swap partner a inside r_cut, w_ca =
// sqrt(Lambda_ca) vhat(r_ca) and w'_ca/r = sqrt(Lambda_ca) vhat'(r_ca)/r_ca,
// so that a triplet term is w_ca w_cb (eq. 3bp with
// Lambda_cab = sqrt(Lambda_ca Lambda_cb)).  d = x_a - x_c (minimum image).
//   force on partner a from (c; a, b):  -w'_ca/r_ca w_cb d_ca
//   force on the centre:                minus the sum of the two
#include <hip/hip_ext.h>

#include "rc_internal.h"
#include "rc_gather.h"
#include "rc_step.h"

namespace rc {

static inline int nblk(long n, int b) { return (int)((n + b - 1) / b); }

// ---------------------------------------------------------------------------
// atomic-free gather force kernel (RC_FORCE_GATHER)
// ---------------------------------------------------------------------------
template <bool EV, bool BATCH, bool SF>
__global__ __launch_bounds__(kWave) void k_forces_gather(ForceArgs a) {
    extern __shared__ DevEntry s_tab[];
    const int blk = xcd_block(gridDim.x);
    Box box_r;
    int lim = a.N;
    if constexpr (BATCH) {
        const RepDesc& d = a.rep[a.chunk_rep[blk]];
        box_r = d.box;
        lim = d.off + d.n;
        load_table(s_tab, Table{a.tab.e + d.tab, a.tab.nt});
    } else {
        box_r = a.box;
        load_table(s_tab, a.tab);
    }
    const int m = blk * kWave + threadIdx.x;
    const bool live = m < lim;
    const float4 pm = live ? a.pos[m] : make_float4(0.f, 0.f, 0.f, 0.f);
    const int packed = live ? a.nn[m] : 0;
    Acc acc = {};
    const OneSystem sys{s_tab, a.tab.nt, box_r};
    wave_gather<EV, kDefaultWidth, SF>(m - (int)threadIdx.x, live, pm, packed, a.pos, a.nlist, a.nn, a.k_max, a.N,
                                       sys, acc, a.ssum);
    if (live) {
        float4 f = make_float4(acc.fx, acc.fy, acc.fz, acc.e);
        if (a.accumulate) {
            const float4 o = a.force[m];
            f.x += o.x;
            f.y += o.y;
            f.z += o.z;
            f.w += o.w;
        }
        a.force[m] = f;
        if (a.status && !(isfinite(f.x) && isfinite(f.y) && isfinite(f.z)))
            atomicOr(&a.status[RC_ST_FLAGS], RC_FLAG_NONFINITE);
    }
    if (EV) {
        double v[7] = {acc.e, acc.w[0], acc.w[1], acc.w[2], acc.w[3], acc.w[4], acc.w[5]};
        wave_sum_store<7>(v, a.ev_part + (size_t)blk * kEvWords);
    }
}

// ---------------------------------------------------------------------------
// triplet kernel (default of rc_compute_forces): one wavefront per block.
// Pair terms per lane; the active partners of centres with two or more of
// them are staged in an LDS pool; the wave then enumerates every (j<k)
// triplet of its 64 centres across its lanes.  Forces on partners leave with
// global atomics, the centre's share is gathered in LDS first.
// ---------------------------------------------------------------------------
constexpr int kPool = 512;   // staged partners per wave and round

__global__ __launch_bounds__(kWave) void k_forces_triplet(ForceArgs a, int want_ev) {
    extern __shared__ DevEntry s_tab[];
    __shared__ int p_j[kPool];
    __shared__ float p_w[kPool], p_g[kPool], p_dx[kPool], p_dy[kPool], p_dz[kPool];
    __shared__ int l_pool[kWave], l_k[kWave], l_tri[kWave + 1];
    __shared__ float l_f[kWave][4];
    load_table(s_tab, a.tab);
    const int nt = a.tab.nt;
    const int lane = threadIdx.x;
    const int i = blockIdx.x * kWave + lane;
    const bool live = i < a.N;
    float4 pi = live ? a.pos[i] : make_float4(0.f, 0.f, 0.f, 0.f);
    const int ti = ptype(pi.w);
    const int cnt = live ? a.nn[i] : 0;
    float fx = 0.f, fy = 0.f, fz = 0.f, en = 0.f;
    float w6[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    int nact = 0;
    walk_list<false>(i, pi, ti, a.nlist, cnt, a.k_max, a.N, a.pos, s_tab, nt, a.box, -1,
                         [&](int, const float4&, const DevEntry& e, const PairGeom& pg) {
                             const float r2 = pg.r2, dx = pg.dx, dy = pg.dy, dz = pg.dz;
                             float phi, g;
                             pair_eval(e, r2, phi, g);
                             fx += g * dx;
                             fy += g * dy;
                             fz += g * dz;
                             en += 0.5f * phi;
                             const float c = -0.5f * g;
                             w6[0] += c * dx * dx; w6[1] += c * dy * dy; w6[2] += c * dz * dz;
                             w6[3] += c * dx * dy; w6[4] += c * dx * dz; w6[5] += c * dy * dz;
                             nact += (e.kind == RC_KIND_SWAP);
                         });
    // ---- wave-wide triplet stage -------------------------------------------
    const int k = (nact >= 2) ? nact : 0;
    int incl = k;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        int t = __shfl_up(incl, o, kWave);
        if (lane >= o) incl += t;
    }
    const int off = incl - k;
    const int total = __shfl(incl, kWave - 1, kWave);
    l_f[lane][0] = l_f[lane][1] = l_f[lane][2] = l_f[lane][3] = 0.f;
    int round_start = 0;
    bool done = (k == 0);
    while (round_start < total) {
        const bool mine = !done && off >= round_start && off + k <= round_start + kPool;
        // the admitted lanes form a run; the next round starts at the first lane left out
        int next = total;
        {
            int cand = (!done && !mine) ? off : total;
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) cand = min(cand, __shfl_xor(cand, o, kWave));
            next = cand;
        }
        if (mine) {
            int q = off - round_start;
            walk_list<true>(i, pi, ti, a.nlist, cnt, a.k_max, a.N, a.pos, s_tab, nt, a.box, -1,
                                 [&](int j, const float4&, const DevEntry& e, const PairGeom& pg) {
                                     const float dx = pg.dx, dy = pg.dy, dz = pg.dz;
                                     float u, u1r;
                                     vhat_eval(e, pg.inside, pg.r2, u, u1r);
                                     p_j[q] = j;
                                     p_w[q] = e.sqrt_lam * u;
                                     p_g[q] = e.sqrt_lam * u1r;
                                     p_dx[q] = dx;
                                     p_dy[q] = dy;
                                     p_dz[q] = dz;
                                     ++q;
                                 });
        }
        const int tcount = mine ? k * (k - 1) / 2 : 0;
        int tinc = tcount;
#pragma unroll
        for (int o = 1; o < kWave; o <<= 1) {
            int t = __shfl_up(tinc, o, kWave);
            if (lane >= o) tinc += t;
        }
        l_tri[lane] = tinc - tcount;
        if (lane == kWave - 1) l_tri[kWave] = tinc;
        l_pool[lane] = off - round_start;
        l_k[lane] = mine ? k : 0;
        __syncthreads();
        const int T = l_tri[kWave];
        for (int t = lane; t < T; t += kWave) {
            int lo = 0, hi = kWave - 1;  // owner: last lane with l_tri <= t
            while (lo < hi) {
                int mid = (lo + hi + 1) >> 1;
                if (l_tri[mid] <= t) lo = mid;
                else hi = mid - 1;
            }
            const int c = lo, kc = l_k[c];
            int loc = t - l_tri[c], aa = 0;
            while (loc >= kc - 1 - aa) {
                loc -= kc - 1 - aa;
                ++aa;
            }
            const int qa = l_pool[c] + aa, qb = l_pool[c] + aa + 1 + loc;
            const float wa = p_w[qa], wb = p_w[qb];
            const float ca = -p_g[qa] * wb, cb = -p_g[qb] * wa;  // force on a = ca d_a
            const float fax = ca * p_dx[qa], fay = ca * p_dy[qa], faz = ca * p_dz[qa];
            const float fbx = cb * p_dx[qb], fby = cb * p_dy[qb], fbz = cb * p_dz[qb];
            float* Fa = reinterpret_cast<float*>(a.force + p_j[qa]);
            float* Fb = reinterpret_cast<float*>(a.force + p_j[qb]);
            atomicAdd(Fa + 0, fax); atomicAdd(Fa + 1, fay); atomicAdd(Fa + 2, faz);
            atomicAdd(Fb + 0, fbx); atomicAdd(Fb + 1, fby); atomicAdd(Fb + 2, fbz);
            atomicAdd(&l_f[c][0], -(fax + fbx));
            atomicAdd(&l_f[c][1], -(fay + fby));
            atomicAdd(&l_f[c][2], -(faz + fbz));
            atomicAdd(&l_f[c][3], wa * wb);
            w6[0] += ca * p_dx[qa] * p_dx[qa] + cb * p_dx[qb] * p_dx[qb];
            w6[1] += ca * p_dy[qa] * p_dy[qa] + cb * p_dy[qb] * p_dy[qb];
            w6[2] += ca * p_dz[qa] * p_dz[qa] + cb * p_dz[qb] * p_dz[qb];
            w6[3] += ca * p_dx[qa] * p_dy[qa] + cb * p_dx[qb] * p_dy[qb];
            w6[4] += ca * p_dx[qa] * p_dz[qa] + cb * p_dx[qb] * p_dz[qb];
            w6[5] += ca * p_dy[qa] * p_dz[qa] + cb * p_dy[qb] * p_dz[qb];
        }
        __syncthreads();
        if (mine) done = true;
        round_start = next;
    }
    __syncthreads();
    fx += l_f[lane][0];
    fy += l_f[lane][1];
    fz += l_f[lane][2];
    en += l_f[lane][3];
    if (live) {
        float* Fi = reinterpret_cast<float*>(a.force + i);
        atomicAdd(Fi + 0, fx);
        atomicAdd(Fi + 1, fy);
        atomicAdd(Fi + 2, fz);
        atomicAdd(Fi + 3, en);
        if (a.status && !(isfinite(fx) && isfinite(fy) && isfinite(fz)))
            atomicOr(&a.status[RC_ST_FLAGS], RC_FLAG_NONFINITE);
    }
    if (want_ev) {
        double v[7] = {en, w6[0], w6[1], w6[2], w6[3], w6[4], w6[5]};
#pragma unroll
        for (int q = 0; q < 7; ++q) v[q] = wave_sum(v[q]);
        if (lane == 0) {
#pragma unroll
            for (int q = 0; q < 7; ++q) a.ev_part[(size_t)blockIdx.x * kEvWords + q] = v[q];
        }
    }
}

__global__ __launch_bounds__(kBlock) void k_zero_f4(float4* __restrict__ p, int n) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        p[i] = make_float4(0.f, 0.f, 0.f, 0.f);
}

hipError_t launch_forces_triplet(const ForceArgs& a, hipStream_t s) {
    if (!a.accumulate)
        hipLaunchKernelGGL(k_zero_f4, dim3(std::min(nblk(a.N, kBlock), 4096)), dim3(kBlock), 0, s,
                           a.force, a.N);
    const size_t shm = sizeof(DevEntry) * a.tab.nt * a.tab.nt;
    hipLaunchKernelGGL(k_forces_triplet, dim3(nblk(a.N, kWave)), dim3(kWave), shm, s, a,
                       a.ev_part ? 1 : 0);
    return hipGetLastError();
}

// First pass of the sums form: S_m of every particle into a.ssum (one thread
// per particle, one wavefront per block so that a batch chunk names the table).
template <bool BATCH>
__global__ __launch_bounds__(kWave) void k_swap_sums(ForceArgs a) {
    extern __shared__ DevEntry s_tab[];
    // as in k_step: xcd_block's order from N (the grid is N / 64 blocks rounded up) with selects, and the
    // particle's own data requested before the table is staged (13.27 -> 13.12 us per dumbbell step at 8192)
    const int nbl = (a.N + kWave - 1) / kWave;
    const int per = nbl / 8;
    const int bx = blockIdx.x;
    const int blk = bx < per * 8 ? (bx & 7) * per + (bx >> 3) : bx;
    const int m = blk * kWave + threadIdx.x;
    const int mc = min(m, a.N - 1);   // in bounds; lanes past the end return below
    const float4 pm = a.pos[mc];
    const int packed = a.nn[mc];
    Box box_r;
    int lim = a.N;
    if constexpr (BATCH) {
        const RepDesc& d = a.rep[a.chunk_rep[blk]];
        box_r = d.box;
        lim = d.off + d.n;
        load_table(s_tab, Table{a.tab.e + d.tab, a.tab.nt});
    } else {
        box_r = a.box;
        load_table(s_tab, a.tab);
    }
    if (m >= lim) return;
    a.ssum[m] = swap_sum(m, pm, packed, a.pos, a.nlist, a.N, s_tab, a.tab.nt, box_r);
}

void sums_kernel_info(bool batch, const void** fn) {
    *fn = batch ? reinterpret_cast<const void*>(&k_swap_sums<true>) : reinterpret_cast<const void*>(&k_swap_sums<false>);
}

static hipError_t launch_sums(const ForceArgs& a, bool batch, hipStream_t s) {
    const size_t shm = sizeof(DevEntry) * a.tab.nt * a.tab.nt;
    if (batch)
        hipLaunchKernelGGL((k_swap_sums<true>), dim3(nblk(a.N, kWave)), dim3(kWave), shm, s, a);
    else
        hipLaunchKernelGGL((k_swap_sums<false>), dim3(nblk(a.N, kWave)), dim3(kWave), shm, s, a);
    return hipGetLastError();
}

template <bool BATCH>
static hipError_t launch_gather_any(const ForceArgs& a, hipStream_t s) {
    const size_t shm = sizeof(DevEntry) * a.tab.nt * a.tab.nt;
    const dim3 g(nblk(a.N, kWave)), b(kWave);
    if (a.ssum) {
        hipError_t e = launch_sums(a, BATCH, s);
        if (e != hipSuccess) return e;
        if (a.ev_part)
            hipLaunchKernelGGL((k_forces_gather<true, BATCH, true>), g, b, shm, s, a);
        else
            hipLaunchKernelGGL((k_forces_gather<false, BATCH, true>), g, b, shm, s, a);
    } else {
        if (a.ev_part)
            hipLaunchKernelGGL((k_forces_gather<true, BATCH, false>), g, b, shm, s, a);
        else
            hipLaunchKernelGGL((k_forces_gather<false, BATCH, false>), g, b, shm, s, a);
    }
    return hipGetLastError();
}

hipError_t launch_forces_gather(const ForceArgs& a, hipStream_t s) { return launch_gather_any<false>(a, s); }
hipError_t launch_forces_gather_batch(const ForceArgs& a, hipStream_t s) { return launch_gather_any<true>(a, s); }

// ---------------------------------------------------------------------------
// fused MD step: gather forces at x_in, finish the previous step's final half
// kick, then B A O A into pos_out.  One kernel per step, no atomics on data.
// ---------------------------------------------------------------------------
// With BATCH the wave's 64-slot chunk names its replica, which supplies the
// box, the coefficient table, the slot bound and the noise key; the noise
// counter uses the tag relative to the replica's first slot, so a replica
// draws the same numbers as the same system run on its own.
// Seven wavefronts per SIMD: the walk-form kernel at width 2 then fits 72
// VGPRs without spilling (74 otherwise, six wavefronts) and runs ~2 % faster
// at 1M particles; the other instantiations are unchanged by the hint.
// The particle's own data is requested before the table is staged in LDS,
// so that the table's load and barrier overlap it instead of preceding it
// (24.9 -> 24.3 us per step at 1M particles).
template <bool EV, bool BATCH, int PL, bool SF>
__global__ __launch_bounds__(kWave) __attribute__((amdgpu_waves_per_eu(7))) void k_step(StepArgs a) {
    extern __shared__ DevEntry s_tab[];
    const int nt = a.tab.nt;
    // Wavefronts in their load and gather part run at raised issue priority and drop it for the
    // integrator, so a SIMD's newer wavefronts get their loads out ahead of older ones' arithmetic
    // (24.52-24.70 -> 24.29-24.36 us per step at 1M particles, any raised level alike).
    __builtin_amdgcn_s_setprio(2);
    // xcd_block's order, from N (every launch's grid is N / 64 blocks rounded up) and without branches,
    // so that the arguments the own data needs come in one round of scalar loads (24.84 -> 24.68 us)
    const int nbl = (a.N + kWave - 1) / kWave;
    const int per = nbl / 8;
    const int bx = blockIdx.x;
    const int blk = bx < per * 8 ? (bx & 7) * per + (bx >> 3) : bx;
    const int m = blk * kWave + threadIdx.x;
    const int mc = min(m, a.N - 1);   // in bounds; lanes past a replica's end or N are dropped below
    const float4 pm0 = a.pos_in[mc];
    const float4 vm0 = a.vel[mc];
    const int packed0 = a.nn[mc];
    Box box_r;
    int lim = a.N, tag0 = 0;
    uint64_t seed = a.seed;
    if constexpr (BATCH) {
        const int r = a.chunk_rep[blk];
        const RepDesc& d = a.rep[r];
        box_r = d.box;
        lim = d.off + d.n;
        tag0 = d.off;
        seed = a.seeds[r];
        load_table(s_tab, Table{a.tab.e + d.tab, nt});
    } else {
        box_r = a.box;
        load_table(s_tab, a.tab);
    }
    const Box& box = box_r;
    const bool live = m < lim;
    const uint64_t step = a.step + (a.step_base ? *a.step_base : 0ull);
    Acc acc = {};
    const float4 pm = live ? pm0 : make_float4(0.f, 0.f, 0.f, 0.f);
    const float4 vm = live ? vm0 : make_float4(0.f, 0.f, 0.f, 0.f);
    const int packed = live ? packed0 : 0;
    const OneSystem sys{s_tab, nt, box};
    // the entries come from the packed copy of the list
    wave_gather<EV, PL, SF, OneSystem, false, true>(m - (int)threadIdx.x, live, pm, packed, a.pos_in, a.nlist, a.nn,
                                                     a.k_max, a.N, sys, acc, a.ssum, a.pl_j, a.pl_o);
    if (!BATCH && a.bonds && live)
        fene_add<EV>(ptag(pm.w), pm, a.bonds, a.rtag, a.pos_in, box, a.fene_k, a.fene_r02, acc);
    __builtin_amdgcn_s_setprio(0);
    step_finish<EV>(a, a.pos_out, m, blk, live, pm, vm, acc, box, tag0, seed, step);
    // the chunk's reset, when this launch carries it (no kernel of the launch reads those words); at the
    // end, so that its argument's load does not hold up the start of every wavefront (25.15 -> 24.79 us)
    if (a.reset_status && blockIdx.x == 0 && threadIdx.x == 0) chunk_reset(a.reset_status, a.reset_base, a.reset_to);
}

// Step kernels by (ev, batch, width, form); log steps use the default width.
template <bool BATCH, bool SF>
static const void* step_fn_form(bool ev, int width) {
    if (ev) return reinterpret_cast<const void*>(&k_step<true, BATCH, kDefaultWidth, SF>);
    switch (width) {
        case 1: return reinterpret_cast<const void*>(&k_step<false, BATCH, 1, SF>);
        case 4: return reinterpret_cast<const void*>(&k_step<false, BATCH, 4, SF>);
        default: return reinterpret_cast<const void*>(&k_step<false, BATCH, 2, SF>);
    }
}

template <bool BATCH>
static const void* step_fn(bool ev, int width, int form) {
    return form == RC_FORM_SUMS ? step_fn_form<BATCH, true>(ev, width) : step_fn_form<BATCH, false>(ev, width);
}

// arguments of the first pass of the sums form for a step reading pos_in
static ForceArgs sums_args(const StepArgs& a) {
    ForceArgs f{};
    f.pos = a.pos_in;
    f.nlist = a.nlist;
    f.nn = a.nn;
    f.N = a.N;
    f.k_max = a.k_max;
    f.tab = a.tab;
    f.box = a.box;
    f.rep = a.rep;
    f.chunk_rep = a.chunk_rep;
    f.ssum = a.ssum;
    return f;
}

template <bool BATCH>
static hipError_t launch_step_any(const StepArgs& a, bool ev, hipStream_t s) {
    if (a.form == RC_FORM_SUMS) {
        hipError_t e = launch_sums(sums_args(a), BATCH, s);
        if (e != hipSuccess) return e;
    }
    const size_t shm = sizeof(DevEntry) * a.tab.nt * a.tab.nt;
    StepArgs arg = a;
    void* args[] = {&arg};
    return hipLaunchKernel(step_fn<BATCH>(ev, a.width, a.form), dim3(nblk(a.N, kStepBlock)), dim3(kStepBlock), args,
                           shm, s);
}

hipError_t launch_step(const StepArgs& a, bool ev, hipStream_t s) { return launch_step_any<false>(a, ev, s); }

// A plain (no ev) step launch whose kernels each run between an event pair
// (hipExtLaunchKernel records them around the kernel alone).
template <bool BATCH>
static hipError_t launch_step_timed_any(const StepArgs& a, hipStream_t s, hipEvent_t* sums, hipEvent_t* step) {
    const size_t shm = sizeof(DevEntry) * a.tab.nt * a.tab.nt;
    if (a.form == RC_FORM_SUMS) {
        ForceArgs f = sums_args(a);
        void* fargs[] = {&f};
        const void* fn = BATCH ? reinterpret_cast<const void*>(&k_swap_sums<true>)
                               : reinterpret_cast<const void*>(&k_swap_sums<false>);
        hipError_t e = sums ? hipExtLaunchKernel(fn, dim3(nblk(a.N, kWave)), dim3(kWave), fargs, shm, s, sums[0],
                                                 sums[1], 0)
                            : hipLaunchKernel(fn, dim3(nblk(a.N, kWave)), dim3(kWave), fargs, shm, s);
        if (e != hipSuccess) return e;
    }
    StepArgs arg = a;
    void* args[] = {&arg};
    return hipExtLaunchKernel(step_fn<BATCH>(false, a.width, a.form), dim3(nblk(a.N, kStepBlock)), dim3(kStepBlock),
                              args, shm, s, step[0], step[1], 0);
}

hipError_t launch_step_timed(const StepArgs& a, bool batch, hipStream_t s, hipEvent_t* sums, hipEvent_t* step) {
    return batch ? launch_step_timed_any<true>(a, s, sums, step) : launch_step_timed_any<false>(a, s, sums, step);
}

void step_kernel_info(bool ev, int width, int form, const void** fn) { *fn = step_fn<false>(ev, width, form); }

hipError_t launch_step_batch(const StepArgs& a, bool ev, hipStream_t s) { return launch_step_any<true>(a, ev, s); }

void step_batch_kernel_info(int width, int form, const void** fn) { *fn = step_fn<true>(false, width, form); }

ForceArgs step_sums_args(const StepArgs& a) { return sums_args(a); }

// ---------------------------------------------------------------------------
// bond count: swap pairs i<j with canonical r^2 < r_min^2
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_bonds(const float4* __restrict__ pos,
                                                 const int* __restrict__ nlist,
                                                 const int* __restrict__ nn, int k_max, int N, Table tab, Box box,
                                                 unsigned long long* __restrict__ part) {
    extern __shared__ DevEntry s_tab[];
    __shared__ unsigned s_w[kBlock / kWave];
    load_table(s_tab, tab);
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    unsigned c = 0;
    if (i < N) {
        const float4 pi = pos[i];
        walk_list<true>(i, pi, ptype(pi.w), nlist, nn[i], k_max, N, pos, s_tab, tab.nt, box, -1,
                        [&](int j, const float4&, const DevEntry&, const PairGeom& pg) {
                            if (j > i && pg.bond) ++c;
                        });
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, kWave);
    if ((threadIdx.x & (kWave - 1)) == 0) s_w[threadIdx.x / kWave] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long t = 0;
        for (int w = 0; w < kBlock / kWave; ++w) t += s_w[w];
        part[blockIdx.x] = t;
    }
}

// bond partner of every particle, by tag: the tag of its one bonded swap partner
// (canonical r^2 < r_min^2), -1 when it has none, -2 when it has several
__global__ __launch_bounds__(kBlock) void k_bond_partners(const float4* __restrict__ pos,
                                                         const int* __restrict__ nlist,
                                                         const int* __restrict__ nn, int k_max, int N, Table tab,
                                                         Box box, int* __restrict__ partner) {
    extern __shared__ DevEntry s_tab[];
    load_table(s_tab, tab);
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const float4 pi = pos[i];
    int p = -1;
    walk_list<true>(i, pi, ptype(pi.w), nlist, nn[i], k_max, N, pos, s_tab, tab.nt, box, -1,
                    [&](int, const float4& pj, const DevEntry&, const PairGeom& pg) {
                        if (pg.bond) p = (p == -1) ? ptag(pj.w) : -2;
                    });
    const int t = ptag(pi.w);
    if (t >= 0 && t < N) partner[t] = p;   // tags >= N have no slot (documented requirement: tags < N)
}

hipError_t launch_bond_partners(const float4* pos, const int* nlist, const int* nn, int k_max, int N, Table tab,
                                Box box, int* partner, hipStream_t s) {
    const size_t shm = sizeof(DevEntry) * tab.nt * tab.nt;
    hipLaunchKernelGGL(k_bond_partners, dim3(nblk(N, kBlock)), dim3(kBlock), shm, s, pos, nlist, nn, k_max, N, tab,
                       box, partner);
    return hipGetLastError();
}

// one block: sum nb partial counts into *out (fixed order: exact either way)
__global__ __launch_bounds__(1024) void k_sum_u64(const unsigned long long* __restrict__ part, int nb,
                                                 unsigned long long* __restrict__ out) {
    __shared__ unsigned long long red[1024];
    unsigned long long s = 0;
    for (int b = threadIdx.x; b < nb; b += blockDim.x) s += part[b];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 512; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = red[0];
}

hipError_t launch_bonds(const float4* pos, const int* nlist, const int* nn, int k_max, int N, Table tab, Box box,
                        unsigned long long* count, unsigned long long* part, hipStream_t s) {
    const size_t shm = sizeof(DevEntry) * tab.nt * tab.nt;
    const int nb = nblk(N, kBlock);
    hipLaunchKernelGGL(k_bonds, dim3(nb), dim3(kBlock), shm, s, pos, nlist, nn, k_max, N, tab, box, part);
    hipLaunchKernelGGL(k_sum_u64, dim3(1), dim3(1024), 0, s, part, nb, count);
    return hipGetLastError();
}

// FENE springs alone (one thread per particle; accumulates into force)
template <bool EV>
__global__ __launch_bounds__(kWave) void k_fene(const float4* __restrict__ pos, const int2* __restrict__ bonds,
                                               const int* __restrict__ rtag, int N, Box box, float K, float R02,
                                               float4* __restrict__ force, double* __restrict__ ev_part) {
    const int m = blockIdx.x * kWave + threadIdx.x;
    Acc acc = {};
    if (m < N) {
        const float4 pm = pos[m];
        fene_add<EV>(ptag(pm.w), pm, bonds, rtag, pos, box, K, R02, acc);
        float4 f = force[m];
        f.x += acc.fx;
        f.y += acc.fy;
        f.z += acc.fz;
        f.w += acc.e;
        force[m] = f;
    }
    if (EV) {
        double v[7] = {acc.e, acc.w[0], acc.w[1], acc.w[2], acc.w[3], acc.w[4], acc.w[5]};
        wave_sum_store<7>(v, ev_part + (size_t)blockIdx.x * kEvWords);
    }
}

hipError_t launch_fene(const float4* pos, const int2* bonds, const int* rtag, int N, Box box, float K, float R02,
                       float4* force, double* ev_part, hipStream_t s) {
    if (ev_part)
        hipLaunchKernelGGL(k_fene<true>, dim3(nblk(N, kWave)), dim3(kWave), 0, s, pos, bonds, rtag, N, box, K, R02,
                           force, ev_part);
    else
        hipLaunchKernelGGL(k_fene<false>, dim3(nblk(N, kWave)), dim3(kWave), 0, s, pos, bonds, rtag, N, box, K, R02,
                           force, ev_part);
    return hipGetLastError();
}

// Bond counts of a batch: one 64-slot chunk per block (a chunk lies in one
// replica), a count per chunk, then one exact integer sum per replica.
__global__ __launch_bounds__(kWave) void k_bonds_batch(const float4* __restrict__ pos,
                                                      const int* __restrict__ nlist, const int* __restrict__ nn,
                                                      int k_max, int N, Table tab, const RepDesc* __restrict__ rep,
                                                      const int* __restrict__ chunk_rep,
                                                      unsigned long long* __restrict__ part) {
    extern __shared__ DevEntry s_tab[];
    const RepDesc& d = rep[chunk_rep[blockIdx.x]];
    load_table(s_tab, Table{tab.e + d.tab, tab.nt});
    const int i = blockIdx.x * kWave + threadIdx.x;
    unsigned c = 0;
    if (i < d.off + d.n) {
        const float4 pi = pos[i];
        walk_list<true>(i, pi, ptype(pi.w), nlist, nn[i], k_max, N, pos, s_tab, tab.nt, d.box, -1,
                        [&](int j, const float4&, const DevEntry&, const PairGeom& pg) {
                            if (j > i && pg.bond) ++c;
                        });
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, kWave);
    if (threadIdx.x == 0) part[blockIdx.x] = c;
}

__global__ __launch_bounds__(kBlock) void k_sum_u64_batch(const unsigned long long* __restrict__ part,
                                                         const RepDesc* __restrict__ rep,
                                                         unsigned long long* __restrict__ out) {
    __shared__ unsigned long long red[kBlock];
    const RepDesc& d = rep[blockIdx.x];
    const int c0 = d.off / kWave, nc = (d.n + kWave - 1) / kWave;
    unsigned long long s = 0;
    for (int b = threadIdx.x; b < nc; b += blockDim.x) s += part[c0 + b];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[blockIdx.x] = red[0];
}

hipError_t launch_bonds_batch(const float4* pos, const int* nlist, const int* nn, int k_max, int N, Table tab,
                              const RepDesc* rep, const int* chunk_rep, int R, unsigned long long* count,
                              unsigned long long* part, hipStream_t s) {
    const size_t shm = sizeof(DevEntry) * tab.nt * tab.nt;
    hipLaunchKernelGGL(k_bonds_batch, dim3(nblk(N, kWave)), dim3(kWave), shm, s, pos, nlist, nn, k_max, N, tab,
                       rep, chunk_rep, part);
    hipLaunchKernelGGL(k_sum_u64_batch, dim3(R), dim3(kBlock), 0, s, part, rep, count);
    return hipGetLastError();
}

// Fold the per-block slots of the step kernel into the status word (OR of
// flags, min of first steps), reset the slots, and raise status[MAXPATH] to
// the largest vel.w (path lengths only grow between list builds, and a build
// zeroes the status word).  One launch per chunk; one atomic per block and word.
__global__ __launch_bounds__(kBlock) void k_fold_status(int* __restrict__ blk, int nb,
                                                       const float4* __restrict__ vel, int N,
                                                       int* __restrict__ status) {
    __shared__ int r_fl[kBlock / kWave], r_s[kBlock / kWave], r_h[kBlock / kWave];
    __shared__ float r_p[kBlock / kWave];
    const int tid = blockIdx.x * blockDim.x + threadIdx.x, stride = gridDim.x * blockDim.x;
    int fl = 0, fs = 0x7fffffff, fh = 0x7fffffff;
    for (int b = tid; b < nb; b += stride) {
        fl |= blk[3 * b];
        fs = min(fs, blk[3 * b + 1]);
        fh = min(fh, blk[3 * b + 2]);
        blk[3 * b] = 0;
        blk[3 * b + 1] = 0x7fffffff;
        blk[3 * b + 2] = 0x7fffffff;
    }
    float pm = 0.0f;
    if (vel) {   // sixteen path lengths in flight per thread (a maximum: exact in any order)
        constexpr int U = 16;
        int i = tid;
        for (; i + (U - 1) * stride < N; i += U * stride) {
            float v[U];
#pragma unroll
            for (int u = 0; u < U; ++u) v[u] = vel[i + u * stride].w;
#pragma unroll
            for (int u = 0; u < U; ++u) pm = fmaxf(pm, v[u]);
        }
        for (; i < N; i += stride) pm = fmaxf(pm, vel[i].w);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        fl |= __shfl_xor(fl, o, kWave);
        fs = min(fs, __shfl_xor(fs, o, kWave));
        fh = min(fh, __shfl_xor(fh, o, kWave));
        pm = fmaxf(pm, __shfl_xor(pm, o, kWave));
    }
    const int w = threadIdx.x / kWave;
    if ((threadIdx.x & (kWave - 1)) == 0) {
        r_fl[w] = fl;
        r_s[w] = fs;
        r_h[w] = fh;
        r_p[w] = pm;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int q = 1; q < kBlock / kWave; ++q) {
            fl |= r_fl[q];
            fs = min(fs, r_s[q]);
            fh = min(fh, r_h[q]);
            pm = fmaxf(pm, r_p[q]);
        }
        fl |= r_fl[0];
        fs = min(fs, r_s[0]);
        fh = min(fh, r_h[0]);
        pm = fmaxf(pm, r_p[0]);
        if (fl) atomicOr(&status[RC_ST_FLAGS], fl);
        if (fs != 0x7fffffff) atomicMin(&status[RC_ST_FIRST_SOFT], fs);
        if (fh != 0x7fffffff) atomicMin(&status[RC_ST_FIRST_HARD], fh);
        if (vel) atomicMax(&status[RC_ST_MAXPATH], __float_as_int(pm));
    }
}

hipError_t launch_fold_status(int* blk, int nb, const float4* vel, int N, int* status, hipStream_t s) {
    // at most 256 blocks: each ends with atomics on the same status words (2048 blocks took 26 us at 1M
    // particles against 8.5 us)
    const int work = vel ? std::max(N, nb) : nb;
    hipLaunchKernelGGL(k_fold_status, dim3(std::max(1, std::min(nblk(work, kBlock), 256))), dim3(kBlock), 0, s,
                       blk, nb, vel, N, status);
    return hipGetLastError();
}

// Per-replica fold of a batch chunk, before k_fold_status resets the block
// slots, in two launches: the largest path length of every 64-slot chunk
// (one wavefront per chunk, all chunks in parallel), then one workgroup per
// replica over its chunks' maxima and block flags, which stores the flag of
// any block that crossed the rebuild threshold and the largest path length;
// status[MAXPATH] is raised to the largest of all.  Path lengths are
// non-negative, so their float bits order like ints.
__global__ __launch_bounds__(kBlock) void k_chunk_paths(const float4* __restrict__ vel, int nb,
                                                       float* __restrict__ chunk_path) {
    const int ch = (blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    if (ch >= nb) return;   // uniform per wavefront
    const float p = wave_maxf(vel[(size_t)ch * kWave + (threadIdx.x & (kWave - 1))].w);
    if ((threadIdx.x & (kWave - 1)) == 0) chunk_path[ch] = p;
}

__global__ __launch_bounds__(kBlock) void k_fold_reps(const int* __restrict__ blk,
                                                     const float* __restrict__ chunk_path,
                                                     const RepDesc* __restrict__ rep, int* __restrict__ rep_flag,
                                                     int* __restrict__ rep_path, int* __restrict__ status) {
    __shared__ float r_p[kBlock / kWave];
    __shared__ int r_f[kBlock / kWave];
    const int r = blockIdx.x;
    const int c0 = rep[r].off / kWave, c1 = (rep[r].off + rep[r].n + kWave - 1) / kWave;
    float pm = 0.0f;
    int fl = 0;
    for (int c = c0 + (int)threadIdx.x; c < c1; c += blockDim.x) {
        pm = fmaxf(pm, chunk_path[c]);
        fl |= blk[3 * c] & RC_FLAG_REBUILD;
    }
    pm = wave_maxf(pm);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) fl |= __shfl_xor(fl, o, kWave);
    if ((threadIdx.x & (kWave - 1)) == 0) {
        r_p[threadIdx.x / kWave] = pm;
        r_f[threadIdx.x / kWave] = fl;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int q = 1; q < kBlock / kWave; ++q) {
            pm = fmaxf(pm, r_p[q]);
            fl |= r_f[q];
        }
        rep_flag[r] = fl != 0;
        rep_path[r] = __float_as_int(pm);
        atomicMax(&status[RC_ST_MAXPATH], __float_as_int(pm));
    }
}

hipError_t launch_fold_reps(const int* blk, const float4* vel, int nb, const RepDesc* rep, int R, int* out,
                            float* chunk_path, int* status, hipStream_t s) {
    hipLaunchKernelGGL(k_chunk_paths, dim3(nblk((long)nb * kWave, kBlock)), dim3(kBlock), 0, s, vel, nb, chunk_path);
    hipLaunchKernelGGL(k_fold_reps, dim3(R), dim3(kBlock), 0, s, blk, chunk_path, rep, out, out + R, status);
    return hipGetLastError();
}

// the driver's snapshot of (pos, vel, image) and its restore, in one launch
__global__ __launch_bounds__(kBlock) void k_copy_state(const float4* __restrict__ pos, const float4* __restrict__ vel,
                                                      const int4* __restrict__ image, float4* __restrict__ pos_to,
                                                      float4* __restrict__ vel_to, int4* __restrict__ image_to,
                                                      int N, int zero_path) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    pos_to[i] = pos[i];
    float4 v = vel[i];
    if (zero_path) v.w = 0.0f;
    vel_to[i] = v;
    if (image && image_to) image_to[i] = image[i];
}

hipError_t launch_copy_state(const float4* pos, const float4* vel, const int4* image, float4* pos_to, float4* vel_to,
                             int4* image_to, int N, hipStream_t s, bool zero_path) {
    hipLaunchKernelGGL(k_copy_state, dim3(nblk(N, kBlock)), dim3(kBlock), 0, s, pos, vel, image, pos_to, vel_to,
                       image_to, N, zero_path ? 1 : 0);
    return hipGetLastError();
}

__global__ __launch_bounds__(kBlock) void k_blk_reset(int* __restrict__ blk, int nb) {
    for (int b = blockIdx.x * blockDim.x + threadIdx.x; b < nb; b += gridDim.x * blockDim.x) {
        blk[3 * b] = 0;
        blk[3 * b + 1] = 0x7fffffff;
        blk[3 * b + 2] = 0x7fffffff;
    }
}

hipError_t launch_blk_reset(int* blk, int nb, hipStream_t s) {
    hipLaunchKernelGGL(k_blk_reset, dim3(std::min(nblk(nb, kBlock), 1024)), dim3(kBlock), 0, s, blk, nb);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// fixed-order FP64 reduction of block partial rows
// ---------------------------------------------------------------------------
// Thread t's slice of one word: rows t, t + 256, t + 512, ... added in that
// order; the loads of 32 rows are issued before their adds (the same sum,
// without a load round trip per row).
__device__ __forceinline__ double strided_row_sum(const double* __restrict__ p, int nblocks, int q) {
    constexpr int U = 32;
    double s = 0.0;
    int b = threadIdx.x;
    for (; b + (U - 1) * kBlock < nblocks; b += U * kBlock) {
        double v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) v[u] = p[(size_t)(b + u * kBlock) * kEvWords + q];
#pragma unroll
        for (int u = 0; u < U; ++u) s += v[u];
    }
    for (; b < nblocks; b += kBlock) s += p[(size_t)b * kEvWords + q];
    return s;
}

__global__ __launch_bounds__(kBlock) void k_reduce_rows(const double* __restrict__ part, int nblocks,
                                                       int first, int count, double* __restrict__ out) {
    // one block per output word; each thread sums a strided slice, then a tree
    __shared__ double red[kBlock];
    const int q = first + blockIdx.x;
    const double s = strided_row_sum(part, nblocks, q);
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[blockIdx.x] = red[0];
}

// The same sums in two launches, for the driver's log rows: first every
// (thread slice t, word q) sum of k_reduce_rows, one thread each, with the
// threads of a wavefront on consecutive words of consecutive rows (coalesced
// reads spread over many CUs instead of 13 CUs each reading every row), then
// per word the same tree over the 256 slices.  Bit for bit k_reduce_rows.
// With bonds, one more column sums the per-block bond counts (64-bit integers,
// exact in any order) into *bonds_out.
__global__ __launch_bounds__(kWave) void k_row_slices(const double* __restrict__ part, int nblocks, int first,
                                                     int count, double* __restrict__ slice,
                                                     const unsigned* __restrict__ bonds) {
    const int cols = count + (bonds ? 1 : 0);
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= kBlock * cols) return;
    const int t = i / cols, qc = i % cols;
    constexpr int U = 16;
    if (qc == count) {
        unsigned long long n = 0;
        int b = t;
        for (; b + (U - 1) * kBlock < nblocks; b += U * kBlock) {
            unsigned v[U];
#pragma unroll
            for (int u = 0; u < U; ++u) v[u] = bonds[b + u * kBlock];
#pragma unroll
            for (int u = 0; u < U; ++u) n += v[u];
        }
        for (; b < nblocks; b += kBlock) n += bonds[b];
        reinterpret_cast<unsigned long long*>(slice)[i] = n;
        return;
    }
    const int q = first + qc;
    double s = 0.0;
    int b = t;
    for (; b + (U - 1) * kBlock < nblocks; b += U * kBlock) {
        double v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) v[u] = part[(size_t)(b + u * kBlock) * kEvWords + q];
#pragma unroll
        for (int u = 0; u < U; ++u) s += v[u];
    }
    for (; b < nblocks; b += kBlock) s += part[(size_t)b * kEvWords + q];
    slice[i] = s;
}

__global__ __launch_bounds__(kBlock) void k_row_tree(const double* __restrict__ slice, int count,
                                                    double* __restrict__ out,
                                                    unsigned long long* __restrict__ bonds_out) {
    const int cols = count + (bonds_out ? 1 : 0);
    if ((int)blockIdx.x == count) {   // the bond column (launched with bonds_out only)
        __shared__ unsigned long long redn[kBlock];
        redn[threadIdx.x] = reinterpret_cast<const unsigned long long*>(slice)[threadIdx.x * cols + count];
        __syncthreads();
        for (int w = kBlock / 2; w > 0; w >>= 1) {
            if (threadIdx.x < w) redn[threadIdx.x] += redn[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0) *bonds_out = redn[0];
        return;
    }
    __shared__ double red[kBlock];
    red[threadIdx.x] = slice[threadIdx.x * cols + blockIdx.x];
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[blockIdx.x] = red[0];
}

hipError_t launch_reduce_rows(const double* part, int nblocks, int first, int count, double* out,
                              hipStream_t s, double* slice, const unsigned* bonds, unsigned long long* bonds_out) {
    if ((bonds != nullptr) != (bonds_out != nullptr) || (bonds && !slice)) return hipErrorInvalidValue;
    if (slice && count <= kEvWords) {
        const int cols = count + (bonds ? 1 : 0);   // kBlock * cols <= kRowSlices
        hipLaunchKernelGGL(k_row_slices, dim3(nblk((long)kBlock * cols, kWave)), dim3(kWave), 0, s, part, nblocks,
                           first, count, slice, bonds);
        hipLaunchKernelGGL(k_row_tree, dim3(cols), dim3(kBlock), 0, s, slice, count, out, bonds_out);
    } else {
        hipLaunchKernelGGL(k_reduce_rows, dim3(count), dim3(kBlock), 0, s, part, nblocks, first, count, out);
    }
    return hipGetLastError();
}

// The same fixed-order sum per replica over its own chunk rows (grid: words x
// replicas), so a replica's sums equal those of the system run on its own.
__global__ __launch_bounds__(kBlock) void k_reduce_rows_batch(const double* __restrict__ part,
                                                             const RepDesc* __restrict__ rep, int first,
                                                             double* __restrict__ out, int out_stride) {
    __shared__ double red[kBlock];
    const RepDesc& d = rep[blockIdx.y];
    const double* p = part + (size_t)(d.off / kWave) * kEvWords;
    const int nblocks = (d.n + kWave - 1) / kWave;
    const int q = first + blockIdx.x;
    const double s = strided_row_sum(p, nblocks, q);
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[(size_t)blockIdx.y * out_stride + blockIdx.x] = red[0];
}

hipError_t launch_reduce_rows_batch(const double* part, const RepDesc* rep, int R, int first, int count,
                                    double* out, int out_stride, hipStream_t s) {
    hipLaunchKernelGGL(k_reduce_rows_batch, dim3(count, R), dim3(kBlock), 0, s, part, rep, first, out, out_stride);
    return hipGetLastError();
}

__global__ void k_status_reset_chunk(int* st, unsigned long long* base, unsigned long long step) {
    chunk_reset(st, base, step);
}
hipError_t launch_status_reset_chunk(int* status, hipStream_t s, unsigned long long* step_base,
                                     unsigned long long step) {
    hipLaunchKernelGGL(k_status_reset_chunk, dim3(1), dim3(1), 0, s, status, step_base, step);
    return hipGetLastError();
}

__global__ void k_zero_words(int* p, int n) {
    for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0;
}
hipError_t launch_zero_words(int* p, int n, hipStream_t s) {
    hipLaunchKernelGGL(k_zero_words, dim3(1), dim3(64), 0, s, p, n);
    return hipGetLastError();
}

__global__ void k_add_step(unsigned long long* p, unsigned long long v) { *p += v; }
hipError_t launch_add_step(unsigned long long* p, unsigned long long v, hipStream_t s) {
    hipLaunchKernelGGL(k_add_step, dim3(1), dim3(1), 0, s, p, v);
    return hipGetLastError();
}
void add_step_kernel_info(const void** fn) { *fn = reinterpret_cast<const void*>(&k_add_step); }

__global__ void k_set_step(unsigned long long* p, unsigned long long v) { *p = v; }
hipError_t launch_set_step(unsigned long long* p, unsigned long long v, hipStream_t s) {
    hipLaunchKernelGGL(k_set_step, dim3(1), dim3(1), 0, s, p, v);
    return hipGetLastError();
}

}  // namespace rc
