// Cell binning (counting sort along a Morton curve of the cell grid) and the
// full neighbour list.  gfx950, wave64.
#include "rc_internal.h"

namespace rc {

// ---------------------------------------------------------------------------
// binning
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_fill_int(int* __restrict__ p, int n, int value) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = value;
}

// cell key of every particle and its arrival rank inside the cell
__global__ __launch_bounds__(kBlock) void k_bin(const float4* __restrict__ pos, int N, Box b, Grid g,
                                               int* __restrict__ counts, int* __restrict__ keys,
                                               int* __restrict__ rank) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    float4 p = pos[i];
    int cx = cell_coord(p.x, b.hf[0], g.inv_w[0], g.nc[0]);
    int cy = cell_coord(p.y, b.hf[1], g.inv_w[1], g.nc[1]);
    int cz = cell_coord(p.z, b.hf[2], g.inv_w[2], g.nc[2]);
    int key = (int)morton3(cx, cy, cz);
    keys[i] = key;
    rank[i] = atomicAdd(&counts[key], 1);
}

// ---- three-phase exclusive scan of counts[0..n) -----------------------------
__device__ __forceinline__ int wave_incl_scan(int v) {
    const int lane = threadIdx.x & (kWave - 1);
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        int t = __shfl_up(v, o, kWave);
        if (lane >= o) v += t;
    }
    return v;
}

// exclusive block scan of one value per thread; returns the block total too
__device__ __forceinline__ int block_excl_scan(int v, int& total) {
    __shared__ int wsum[kBlock / kWave];
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    int inc = wave_incl_scan(v);
    if (lane == kWave - 1) wsum[wid] = inc;
    __syncthreads();
    int off = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < kBlock / kWave; ++w) {
        int s = wsum[w];
        off += (w < wid) ? s : 0;
        tot += s;
    }
    __syncthreads();
    total = tot;
    return off + inc - v;
}

__global__ __launch_bounds__(kBlock) void k_scan_reduce(const int* __restrict__ counts, int n,
                                                       int* __restrict__ block_sums) {
    const int base = blockIdx.x * kScanTile + threadIdx.x * kScanItems;
    int s = 0;
#pragma unroll
    for (int q = 0; q < kScanItems; ++q) s += (base + q < n) ? counts[base + q] : 0;
    int total;
    block_excl_scan(s, total);
    if (threadIdx.x == 0) block_sums[blockIdx.x] = total;
}

// one block of 1024 threads scans up to 8192 block sums; also writes start[n]
__global__ __launch_bounds__(1024) void k_scan_top(int* __restrict__ block_sums, int nb,
                                                  int* __restrict__ start, int n) {
    __shared__ int wsum[1024 / kWave];
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    int v[8];
    int s = 0;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        int idx = threadIdx.x * 8 + q;
        v[q] = idx < nb ? block_sums[idx] : 0;
        s += v[q];
    }
    int inc = wave_incl_scan(s);
    if (lane == kWave - 1) wsum[wid] = inc;
    __syncthreads();
    int off = 0, tot = 0;
    for (int w = 0; w < 1024 / kWave; ++w) {
        off += (w < wid) ? wsum[w] : 0;
        tot += wsum[w];
    }
    int run = off + inc - s;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        int idx = threadIdx.x * 8 + q;
        if (idx < nb) block_sums[idx] = run;
        run += v[q];
    }
    if (threadIdx.x == 0) start[n] = tot;
}

__global__ __launch_bounds__(kBlock) void k_scan_down(const int* __restrict__ counts, int n,
                                                     const int* __restrict__ block_off,
                                                     int* __restrict__ start) {
    const int base = blockIdx.x * kScanTile + threadIdx.x * kScanItems;
    int v[kScanItems];
    int s = 0;
#pragma unroll
    for (int q = 0; q < kScanItems; ++q) {
        v[q] = (base + q < n) ? counts[base + q] : 0;
        s += v[q];
    }
    int total;
    int run = block_excl_scan(s, total) + block_off[blockIdx.x];
#pragma unroll
    for (int q = 0; q < kScanItems; ++q) {
        if (base + q < n) start[base + q] = run;
        run += v[q];
    }
}

__global__ __launch_bounds__(kBlock) void k_scatter(const int* __restrict__ keys,
                                                   const int* __restrict__ rank,
                                                   const int* __restrict__ start, int N,
                                                   int* __restrict__ order) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    order[start[keys[i]] + rank[i]] = i;
}

// One thread per key: order the cell's entries by previous index (the
// arrival order of the binning atomics is not deterministic).  Cells hold a
// few particles; empty and single cells return at once.
__global__ __launch_bounds__(kBlock) void k_sort_cells(const int* __restrict__ start, int nkeys,
                                                      int* __restrict__ order) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nkeys) return;
    const int s = start[k], e = start[k + 1];
    for (int a = s + 1; a < e; ++a) {
        const int v = order[a];
        int b = a - 1;
        while (b >= s && order[b] > v) {
            order[b + 1] = order[b];
            --b;
        }
        order[b + 1] = v;
    }
}

// One thread per new index q: gather the particle data into key order
// (coalesced writes; the reads follow the previous order, which is close to
// the new one after the first build).
__global__ __launch_bounds__(kBlock) void k_permute(const int* __restrict__ order, int N,
                                                   const float4* __restrict__ pos,
                                                   const float4* __restrict__ vel,
                                                   const int4* __restrict__ image,
                                                   float4* __restrict__ tpos, float4* __restrict__ tvel,
                                                   int4* __restrict__ timage, int* __restrict__ rtag) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= N) return;
    const int o = order[q];
    const float4 p = pos[o];
    tpos[q] = p;
    if (vel) tvel[q] = vel[o];
    if (image) timage[q] = image[o];
    if (rtag) {
        const int tg = ptag(p.w);
        if (tg >= 0 && tg < N) rtag[tg] = q;
    }
}

static inline int nblk(long n, int b) { return (int)((n + b - 1) / b); }

hipError_t launch_cells(const CellsArgs& a, hipStream_t s) {
    const int nk = (int)a.g.nkeys;
    const int nsb = nblk(nk, kScanTile);
    if (nsb > 8192) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_fill_int, dim3(std::min(nblk(nk, kBlock), 2048)), dim3(kBlock), 0, s,
                       a.counts, nk, 0);
    hipLaunchKernelGGL(k_bin, dim3(nblk(a.N, kBlock)), dim3(kBlock), 0, s, a.pos, a.N, a.box, a.g,
                       a.counts, a.keys, a.rank);
    hipLaunchKernelGGL(k_scan_reduce, dim3(nsb), dim3(kBlock), 0, s, a.counts, nk, a.block_sums);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(1024), 0, s, a.block_sums, nsb, a.cell_start, nk);
    hipLaunchKernelGGL(k_scan_down, dim3(nsb), dim3(kBlock), 0, s, a.counts, nk, a.block_sums,
                       a.cell_start);
    hipLaunchKernelGGL(k_scatter, dim3(nblk(a.N, kBlock)), dim3(kBlock), 0, s, a.keys, a.rank,
                       a.cell_start, a.N, a.order);
    hipLaunchKernelGGL(k_sort_cells, dim3(nblk(nk, kBlock)), dim3(kBlock), 0, s, a.cell_start, nk, a.order);
    hipLaunchKernelGGL(k_permute, dim3(nblk(a.N, kBlock)), dim3(kBlock), 0, s, a.order, a.N, a.pos, a.vel, a.image,
                       a.tpos, a.tvel, a.timage, a.rtag);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = hipMemcpyAsync(a.pos, a.tpos, sizeof(float4) * (size_t)a.N, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess && a.vel)
        e = hipMemcpyAsync(a.vel, a.tvel, sizeof(float4) * (size_t)a.N, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess && a.image)
        e = hipMemcpyAsync(a.image, a.timage, sizeof(int4) * (size_t)a.N, hipMemcpyDeviceToDevice, s);
    return e;
}

// ---------------------------------------------------------------------------
// neighbour list
// ---------------------------------------------------------------------------
// One thread per particle i (key order): scan the 27 cells around i's cell and
// keep every j != i inside r_list(t_i, t_j).  Distances use FP64 differences
// folded by the box (exact image choice) and an FP32 square; the list radius
// carries a 1e-5 relative margin for that rounding.
__global__ __launch_bounds__(kBlock) void k_nlist(NlistArgs a) {
    extern __shared__ float s_rl2[];  // [nt*nt] list radii^2, then [nt*nt] swap flags
    const int nt = a.tab.nt;
    int* s_swap = reinterpret_cast<int*>(s_rl2 + nt * nt);
    for (int q = threadIdx.x; q < nt * nt; q += blockDim.x) {
        s_rl2[q] = a.tab.e[q].rlist2;
        s_swap[q] = a.tab.e[q].kind == RC_KIND_SWAP;
    }
    __syncthreads();
    const int nb = gridDim.x;
    const int i = xcd_block(nb) * blockDim.x + threadIdx.x;
    const bool live = i < a.N;
    int ns = 0, no = 0, total = 0;
    if (live) {
        const float4 pi = a.pos[i];
        const int ti = ptype(pi.w);
        const Grid& g = a.g;
        const int cx = cell_coord(pi.x, a.box.hf[0], g.inv_w[0], g.nc[0]);
        const int cy = cell_coord(pi.y, a.box.hf[1], g.inv_w[1], g.nc[1]);
        const int cz = cell_coord(pi.z, a.box.hf[2], g.inv_w[2], g.nc[2]);
        for (int oz = -1; oz <= 1; ++oz) {
            int z = cz + oz;
            z += (z < 0) ? g.nc[2] : 0;
            z -= (z >= g.nc[2]) ? g.nc[2] : 0;
            for (int oy = -1; oy <= 1; ++oy) {
                int y = cy + oy;
                y += (y < 0) ? g.nc[1] : 0;
                y -= (y >= g.nc[1]) ? g.nc[1] : 0;
                for (int ox = -1; ox <= 1; ++ox) {
                    int x = cx + ox;
                    x += (x < 0) ? g.nc[0] : 0;
                    x -= (x >= g.nc[0]) ? g.nc[0] : 0;
                    const uint32_t key = morton3(x, y, z);
                    const int s = a.cell_start[key], e = a.cell_start[key + 1];
                    for (int j = s; j < e; ++j) {
                        if (j == i) continue;
                        const float4 pj = a.pos[j];
                        float dx = (float)fold((double)pj.x - (double)pi.x, a.box.L[0], a.box.h[0]);
                        float dy = (float)fold((double)pj.y - (double)pi.y, a.box.L[1], a.box.h[1]);
                        float dz = (float)fold((double)pj.z - (double)pi.z, a.box.L[2], a.box.h[2]);
                        float r2 = dx * dx + dy * dy + dz * dz;
                        const int q = ti * nt + ptype(pj.w);
                        if (r2 < s_rl2[q]) {
                            if (s_swap[q]) {
                                if (ns + no < a.k_max) a.nlist[(size_t)ns * a.N + i] = j;
                                ++ns;
                            } else {
                                if (ns + no < a.k_max) a.nlist[(size_t)(a.k_max - 1 - no) * a.N + i] = j;
                                ++no;
                            }
                        }
                    }
                }
            }
        }
        total = ns + no;
        // on overflow the stored prefix is what fitted (the status reports it)
        if (ns + no > a.k_max) {
            const int keep_s = min(ns, a.k_max);
            ns = keep_s;
            no = a.k_max - keep_s;
        }
        a.nn[i] = ns | (no << 16);
        if (a.vel) a.vel[i].w = 0.0f;
    }
    const int cnt = total;
    // block maximum of the list length (no same-address atomics per wave)
    __shared__ int s_m[kBlock / kWave];
    int m = cnt;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) m = max(m, __shfl_xor(m, o, kWave));
    if ((threadIdx.x & (kWave - 1)) == 0) s_m[threadIdx.x / kWave] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        int t = 0;
        for (int w = 0; w < kBlock / kWave; ++w) t = max(t, s_m[w]);
        a.block_max[blockIdx.x] = t;
    }
}

// one block: fold the per-block maxima into the status word
__global__ __launch_bounds__(1024) void k_nlist_status(const int* __restrict__ block_max, int nb, int k_max,
                                                      int* __restrict__ status) {
    __shared__ int red[1024];
    int m = 0;
    for (int b = threadIdx.x; b < nb; b += blockDim.x) m = max(m, block_max[b]);
    red[threadIdx.x] = m;
    __syncthreads();
    for (int w = 512; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] = max(red[threadIdx.x], red[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        status[RC_ST_KMAX] = max(status[RC_ST_KMAX], red[0]);
        if (red[0] > k_max) status[RC_ST_FLAGS] |= RC_FLAG_NLIST_OVERFLOW;
    }
}

hipError_t launch_nlist(const NlistArgs& a, hipStream_t s) {
    const size_t shm = 2 * sizeof(float) * a.tab.nt * a.tab.nt;
    const int nb = nblk(a.N, kBlock);
    hipLaunchKernelGGL(k_nlist, dim3(nb), dim3(kBlock), shm, s, a);
    if (a.status) hipLaunchKernelGGL(k_nlist_status, dim3(1), dim3(1024), 0, s, a.block_max, nb, a.k_max, a.status);
    return hipGetLastError();
}

}  // namespace rc
