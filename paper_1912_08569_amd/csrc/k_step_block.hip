// Small systems in one workgroup.  A system of at most kBlockMaxN particles
// (one per thread, key order) is advanced by G plain steps of the fused step
// in a single launch: the positions live in LDS for the whole replay (two
// buffers), the switching sums of the two-pass form too, and the steps are
// separated by workgroup barriers.  Every wavefront runs the same gather and
// integrator code as k_step on its 64 particles, with its own LDS slices and
// wavefront-level barriers inside the gather, and writes the status slot of
// its 64-particle block, so the result is the same, bit for bit, as G
// launches of k_step (and of k_swap_sums first, in the two-pass form).  At
// these sizes a step is bound by the latency of its dependent reads; LDS
// reads and workgroup barriers replace the global reads of data written by
// the previous launch on another XCD and the launches themselves.
#include "rc_step.h"

namespace rc {

__host__ __device__ static inline size_t block_tab_bytes(int nt) {
    return (sizeof(DevEntry) * (size_t)nt * nt + 15) & ~size_t(15);
}

// Dynamic LDS: the coefficient table, two position buffers and the sums.
size_t step_block_dyn_lds(int N, int nt) {
    const size_t nthr = (size_t)((N + kWave - 1) / kWave) * kWave;
    return block_tab_bytes(nt) + 2 * sizeof(float4) * nthr + sizeof(float) * nthr;
}

template <bool SF>
__global__ __launch_bounds__(kBlockMaxN) void k_step_block(StepArgs a, float4* __restrict__ pos_final,
                                                           unsigned long long* __restrict__ step_base, int G) {
    extern __shared__ __align__(16) unsigned char s_dyn[];
    const int nt = a.tab.nt;
    const int nthr = (int)blockDim.x;
    DevEntry* s_tab = reinterpret_cast<DevEntry*>(s_dyn);
    float4* s_p0 = reinterpret_cast<float4*>(s_dyn + block_tab_bytes(nt));
    float4* s_p1 = s_p0 + nthr;
    float* s_S = reinterpret_cast<float*>(s_p1 + nthr);
    load_table(s_tab, a.tab);  // ends with a workgroup barrier
    const int m = (int)threadIdx.x;
    const int lane = m & (kWave - 1);
    const int w = m / kWave;
    const bool live = m < a.N;
    const float4 zero = make_float4(0.f, 0.f, 0.f, 0.f);
    // (branches, not selects of the loaded value: a select becomes a select of addresses)
    float4 p_first = zero;
    int packed = 0;
    if (live) {
        p_first = a.pos_in[m];
        packed = a.nn[m];
    }
    s_p0[m] = p_first;
    s_p1[m] = zero;
    const uint64_t base = *step_base;
    const OneSystem sys{s_tab, nt, a.box};
    __syncthreads();
    for (int k = 0; k < G; ++k) {
        const float4* pin = (k & 1) ? s_p1 : s_p0;
        float4* pout = (k & 1) ? s_p0 : s_p1;
        const float4 pm = pin[m];
        float4 vm = zero;
        if (live) vm = a.vel[m];
        if (SF) {
            s_S[m] = live ? swap_sum(m, pm, packed, pin, a.nlist, a.N, s_tab, nt, a.box) : 0.0f;
            __syncthreads();
        }
        Acc acc = {};
        wave_gather<false, kDefaultWidth, SF, OneSystem, true, true>(m - lane, live, pm, packed, pin, a.nlist,
                                                                       a.nn, a.k_max, a.N, sys, acc, s_S, a.pl_j,
                                                                       a.pl_o);
        if (a.bonds && live)
            fene_add<false>(ptag(pm.w), pm, a.bonds, a.rtag, pin, a.box, a.fene_k, a.fene_r02, acc);
        step_finish<false>(a, pout, m, w, live, pm, vm, acc, a.box, 0, a.seed, base + (uint64_t)k);
        __syncthreads();
    }
    if (live) pos_final[m] = s_p0[m];  // G is even: the last step wrote buffer 0
    if (m == 0) *step_base = base + (uint64_t)G;
}

template <bool SF>
static const void* block_fn() {
    return reinterpret_cast<const void*>(&k_step_block<SF>);
}

// Whether a system fits: particle count, form and the LDS the kernel needs
// (its static gather slices plus the dynamic part) within one workgroup.
bool step_block_fits(int N, int nt, int form) {
    if (N < 1 || N > kBlockMaxN) return false;
    const void* fn = form == RC_FORM_SUMS ? block_fn<true>() : block_fn<false>();
    hipFuncAttributes at{};
    if (hipFuncGetAttributes(&at, fn) != hipSuccess) return false;
    int dev = 0, max_lds = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
        return false;
    return at.sharedSizeBytes + step_block_dyn_lds(N, nt) <= (size_t)max_lds;
}

hipError_t launch_step_block(const StepArgs& a, float4* pos_final, unsigned long long* step_base, int G,
                             hipStream_t s) {
    if (a.N < 1 || a.N > kBlockMaxN || (G & 1) || G < 2) return hipErrorInvalidValue;
    const void* fn = a.form == RC_FORM_SUMS ? block_fn<true>() : block_fn<false>();
    const size_t shm = step_block_dyn_lds(a.N, a.tab.nt);
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
    if (e != hipSuccess) return e;
    const int nthr = ((a.N + kWave - 1) / kWave) * kWave;
    StepArgs arg = a;
    void* args[] = {&arg, &pos_final, &step_base, &G};
    return hipLaunchKernel(fn, dim3(1), dim3(nthr), args, shm, s);
}

}  // namespace rc
