// Observables built on the step.
//
// Bond-partner statistics between two tag-indexed partner snapshots (as
// rc_bond_partners writes them): over the selected tags, the particles bonded
// at 0, those whose partner is unchanged (the numerator of the bond
// autocorrelation, Sec. 3.1 / Fig. 3) and those whose single partner is now
// another particle (a swap event).  Wavefront ballots give per-block counts;
// a second kernel adds the block counts (integers: the order does not
// matter).
//
// The stress autocorrelation G(t) (the relaxation modulus by the
// autocorrelation method, Sec. 2.2 after eq. p3) of a series of logged rows
// (E, W(6), K(6)): V/kT times the average over the off-diagonal components
// xy, xz, yz and over every time origin of sigma(t0) sigma(t0 + t), with
// sigma_ab = -(K_ab + W_ab)/V.  One block per lag, FP64, a fixed-order tree
// over the block's threads.
#include "rc_internal.h"

namespace rc {

static inline int nblk(long n, int b) { return (int)((n + b - 1) / b); }

__global__ __launch_bounds__(kBlock) void k_partner_counts(const int* __restrict__ p0, const int* __restrict__ pt,
                                                           const unsigned char* __restrict__ sel, int N,
                                                           unsigned long long* __restrict__ part) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    bool b = false, u = false, w = false;
    if (i < N && (!sel || sel[i])) {
        const int a = p0[i];
        if (a >= 0) {
            const int c = pt[i];
            b = true;
            u = c == a;
            w = c >= 0 && c != a;
        }
    }
    const unsigned long long bb = __ballot(b), bu = __ballot(u), bw = __ballot(w);
    __shared__ unsigned long long s_cnt[kBlock / kWave][3];
    const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
    if (lane == 0) {
        s_cnt[wv][0] = (unsigned long long)__popcll(bb);
        s_cnt[wv][1] = (unsigned long long)__popcll(bu);
        s_cnt[wv][2] = (unsigned long long)__popcll(bw);
    }
    __syncthreads();
    if (threadIdx.x < 3) {
        unsigned long long t = 0;
        for (int q = 0; q < kBlock / kWave; ++q) t += s_cnt[q][threadIdx.x];
        part[(size_t)blockIdx.x * 3 + threadIdx.x] = t;
    }
}

__global__ __launch_bounds__(kBlock) void k_sum_counts3(const unsigned long long* __restrict__ part, int nb,
                                                        unsigned long long* __restrict__ out) {
    __shared__ unsigned long long red[3][kBlock];
    unsigned long long s[3] = {0, 0, 0};
    for (int b = threadIdx.x; b < nb; b += blockDim.x)
        for (int q = 0; q < 3; ++q) s[q] += part[(size_t)b * 3 + q];
    for (int q = 0; q < 3; ++q) red[q][threadIdx.x] = s[q];
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w)
            for (int q = 0; q < 3; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x < 3) out[threadIdx.x] = red[threadIdx.x][0];
}

hipError_t launch_partner_counts(const int* p0, const int* pt, const unsigned char* sel, int N,
                                 unsigned long long* part, unsigned long long* out, hipStream_t s) {
    const int nb = nblk(N, kBlock);
    hipLaunchKernelGGL(k_partner_counts, dim3(nb), dim3(kBlock), 0, s, p0, pt, sel, N, part);
    hipLaunchKernelGGL(k_sum_counts3, dim3(1), dim3(kBlock), 0, s, part, nb, out);
    return hipGetLastError();
}

__global__ __launch_bounds__(kBlock) void k_stress_acf(const double* __restrict__ rows, int T, double inv_v,
                                                       double v_over_kt, double* __restrict__ G) {
    const int t = blockIdx.x;  // lag
    double acc = 0.0;
    for (int t0 = threadIdx.x; t0 < T - t; t0 += blockDim.x) {
        const double* a = rows + (size_t)t0 * kEvWords;
        const double* b = rows + (size_t)(t0 + t) * kEvWords;
        for (int c = 0; c < 3; ++c) {  // xy, xz, yz: W at 4 + c, K at 10 + c
            const double sa = -(a[10 + c] + a[4 + c]) * inv_v;
            const double sb = -(b[10 + c] + b[4 + c]) * inv_v;
            acc += sa * sb;
        }
    }
    __shared__ double red[kBlock];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) G[t] = v_over_kt * red[0] / (3.0 * (double)(T - t));
}

hipError_t launch_stress_acf(const double* rows, int T, double volume, double kT, int max_lag, double* G,
                             hipStream_t s) {
    hipLaunchKernelGGL(k_stress_acf, dim3(max_lag + 1), dim3(kBlock), 0, s, rows, T, 1.0 / volume, volume / kT, G);
    return hipGetLastError();
}

}  // namespace rc
