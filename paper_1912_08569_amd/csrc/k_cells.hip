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
// the new one after the first build).  The path lengths since the last list
// build (vel.w) restart at zero for the particles whose list is rebuilt; a
// batch replica that keeps its list (build[r] == 0) keeps its order
// (order[q] == q) and its path lengths.  The temporaries are the state the
// rebuild leaves, which the driver restores on a rollback.
__global__ __launch_bounds__(kBlock) void k_permute(const int* __restrict__ order, int N,
                                                   const float4* __restrict__ pos,
                                                   const float4* __restrict__ vel,
                                                   const int4* __restrict__ image,
                                                   float4* __restrict__ tpos, float4* __restrict__ tvel,
                                                   int4* __restrict__ timage, int* __restrict__ rtag,
                                                   const int* __restrict__ build, const int* __restrict__ chunk_rep) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= N) return;
    const int o = order[q];
    if (o < 0) {   // an unused slot of a batch: zeroed
        tpos[q] = make_float4(0.f, 0.f, 0.f, 0.f);
        if (vel) tvel[q] = make_float4(0.f, 0.f, 0.f, 0.f);
        if (image) timage[q] = make_int4(0, 0, 0, 0);
        return;
    }
    const bool rebuilt = !build || build[chunk_rep[q / kWave]] != 0;
    const float4 p = pos[o];
    tpos[q] = p;
    if (vel) {
        float4 v = vel[o];
        if (rebuilt) v.w = 0.0f;
        tvel[q] = v;
    }
    if (image) timage[q] = image[o];
    if (rtag) {
        const int tg = ptag(p.w);
        if (tg >= 0 && tg < N) rtag[tg] = q;
    }
}

// ---- batches: the same counting sort over the concatenated key ranges ------
// Only the replicas with build[r] != 0 (every replica when build is NULL) are
// binned and re-ordered; the others keep their order and their lists.  A
// replica's particles go to its own slots: slot = off + (the cell start of
// its key) - (the cell start of its first key) + rank, so the order does not
// depend on which other replicas take part.
__device__ __forceinline__ bool rep_builds(const int* build, int r) { return !build || build[r] != 0; }

// order[q]: -1 for unused slots, q for the slots of replicas that keep their
// order; the scatter fills the rest
__global__ __launch_bounds__(kBlock) void k_order_init_batch(CellsArgsB a) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= a.N) return;
    const int r = a.chunk_rep[q / kWave];
    const RepDesc& d = a.rep[r];
    a.order[q] = (q < d.off + d.n && !rep_builds(a.build, r)) ? q : -1;
}

__global__ __launch_bounds__(kBlock) void k_bin_batch(CellsArgsB a) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.N) return;
    const int r = a.chunk_rep[i / kWave];
    if (!rep_builds(a.build, r)) return;
    const RepDesc& d = a.rep[r];
    if (i >= d.off + d.n) return;
    const float4 p = a.pos[i];
    const int cx = cell_coord(p.x, d.box.hf[0], d.grid.inv_w[0], d.grid.nc[0]);
    const int cy = cell_coord(p.y, d.box.hf[1], d.grid.inv_w[1], d.grid.nc[1]);
    const int cz = cell_coord(p.z, d.box.hf[2], d.grid.inv_w[2], d.grid.nc[2]);
    const int key = (int)(d.key_base + morton3(cx, cy, cz));
    a.keys[i] = key;
    a.rank[i] = atomicAdd(&a.counts[key], 1);
}

// scatter into the replica's own slots
__global__ __launch_bounds__(kBlock) void k_scatter_batch(CellsArgsB a) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.N) return;
    const int r = a.chunk_rep[i / kWave];
    if (!rep_builds(a.build, r)) return;
    const RepDesc& d = a.rep[r];
    if (i >= d.off + d.n) return;
    a.order[a.cell_start[a.keys[i]] - a.cell_start[d.key_base] + a.rank[i] + d.off] = i;
}

// per key: the replica owning it (first r with key_end[r] > k), then the
// same in-cell ordering by previous index as the single-system sort
__global__ __launch_bounds__(kBlock) void k_sort_cells_batch(CellsArgsB a) {
    const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= a.nkeys) return;
    const int s0 = a.cell_start[k], e0 = a.cell_start[k + 1];
    if (e0 - s0 < 2) return;
    int lo = 0, hi = a.R - 1;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (a.key_end[mid] > k) hi = mid;
        else lo = mid + 1;
    }
    if (!rep_builds(a.build, lo)) return;
    const int sh = a.rep[lo].off - a.cell_start[a.rep[lo].key_base];
    int* order = a.order;
    const int s = s0 + sh, e = e0 + sh;
    for (int p = s + 1; p < e; ++p) {
        const int v = order[p];
        int q = p - 1;
        while (q >= s && order[q] > v) {
            order[q + 1] = order[q];
            --q;
        }
        order[q + 1] = v;
    }
}

static inline int nblk(long n, int b) { return (int)((n + b - 1) / b); }

// The permuted state back from the temporaries, in one launch (vel and image may be NULL)
__global__ __launch_bounds__(kBlock) void k_copy_back(const float4* __restrict__ tpos, const float4* __restrict__ tvel,
                                                     const int4* __restrict__ timage, float4* __restrict__ pos,
                                                     float4* __restrict__ vel, int4* __restrict__ image, int N) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    pos[i] = tpos[i];
    if (vel) vel[i] = tvel[i];
    if (image) image[i] = timage[i];
}

hipError_t launch_cells_batch(const CellsArgsB& a, hipStream_t s) {
    const int nk = (int)a.nkeys;
    const int nsb = nblk(nk, kScanTile);
    if (nsb > 8192) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_fill_int, dim3(std::min(nblk(nk, kBlock), 2048)), dim3(kBlock), 0, s, a.counts, nk, 0);
    hipLaunchKernelGGL(k_order_init_batch, dim3(nblk(a.N, kBlock)), dim3(kBlock), 0, s, a);
    hipLaunchKernelGGL(k_bin_batch, dim3(nblk(a.N, kBlock)), dim3(kBlock), 0, s, a);
    hipLaunchKernelGGL(k_scan_reduce, dim3(nsb), dim3(kBlock), 0, s, a.counts, nk, a.block_sums);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(1024), 0, s, a.block_sums, nsb, a.cell_start, nk);
    hipLaunchKernelGGL(k_scan_down, dim3(nsb), dim3(kBlock), 0, s, a.counts, nk, a.block_sums, a.cell_start);
    hipLaunchKernelGGL(k_scatter_batch, dim3(nblk(a.N, kBlock)), dim3(kBlock), 0, s, a);
    hipLaunchKernelGGL(k_sort_cells_batch, dim3(nblk(nk, kBlock)), dim3(kBlock), 0, s, a);
    hipLaunchKernelGGL(k_permute, dim3(nblk(a.N, kBlock)), dim3(kBlock), 0, s, a.order, a.N, a.pos, a.vel, a.image,
                       a.tpos, a.tvel, a.timage, a.rtag, a.build, a.chunk_rep);
    hipLaunchKernelGGL(k_copy_back, dim3(nblk(a.N, kBlock)), dim3(kBlock), 0, s, a.tpos, a.tvel, a.timage, a.pos,
                       a.vel, a.image, a.N);
    return hipGetLastError();
}

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
                       a.tpos, a.tvel, a.timage, a.rtag, nullptr, nullptr);
    hipLaunchKernelGGL(k_copy_back, dim3(nblk(a.N, kBlock)), dim3(kBlock), 0, s, a.tpos, a.tvel, a.timage, a.pos,
                       a.vel, a.image, a.N);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// neighbour list
// ---------------------------------------------------------------------------
// List of one particle i (key order): scan the 27 cells around i's cell and
// keep every j != i inside r_list(t_i, t_j).  Cells are visited in (z, y, x)
// offset order and each cell's particles in memory order, so the list order
// is fixed.  For a cell that does not wrap around the box the difference
// x_j - x_i is one FP32 subtraction (a single rounding of the exact value);
// across a periodic face it is the FP64 difference folded by the box (exact
// image choice).  The square is FP32; the list radius carries a 1e-5 relative
// margin for that rounding.  Cell k's particles sit at cell_start[key_base +
// k] + shift onwards.  rl(q, rl2, swap) gives entry q's squared list radius
// and whether it is a swap pair.  Returns the full neighbour count and stores
// nn[i] (clipped to k_max).
//
// A cell whose nearest point is farther from i than i's largest list radius
// (over all partner types) is skipped: its count is taken as zero.  The gaps
// to the cell faces are shrunk by 1e-3 cell widths, far above the FP32
// rounding of the cell coordinates, so no cell that holds a listable
// neighbour is skipped.
//
// Per z slab the nine cells' candidates are numbered t = 0 .. tot-1 in
// visiting order (exclusive prefix pre[q] of the cell counts), and candidate t
// is located without branches: the last cell q with pre[q] <= t gives
// j = t + (start_q - pre_q).  The offset and the cell's wrap flag are packed in
// one word, so a candidate costs eight compare/select pairs and a wavefront
// runs one uniform loop per slab instead of a data-dependent cursor.  The next
// candidate's position is requested before the current one is tested.
template <class Radii>
__device__ __forceinline__ int list_one(int i, const float4& pi, const Box& b, const Grid& g, uint32_t key_base,
                                        int shift, const int* __restrict__ cell_start, const float4* __restrict__ pos,
                                        int nt, int k_max, int N, int* __restrict__ nlist, int* __restrict__ nn,
                                        Radii rl) {
    int ns = 0, no = 0;
    const int ti = ptype(pi.w);
    const int cx = cell_coord(pi.x, b.hf[0], g.inv_w[0], g.nc[0]);
    const int cy = cell_coord(pi.y, b.hf[1], g.inv_w[1], g.nc[1]);
    const int cz = cell_coord(pi.z, b.hf[2], g.inv_w[2], g.nc[2]);
    float rmax2 = 0.0f;  // i's largest squared list radius
    for (int t = 0; t < nt; ++t) {
        float r2t;
        bool sw;
        rl(ti * nt + t, r2t, sw);
        rmax2 = fmaxf(rmax2, r2t);
    }
    // squared gaps from i to the cells at offsets -1, 0, +1 along an axis
    auto gaps = [&](float x, float h, float inv_w, int c, float& g0, float& g2) {
        const float f = (x + h) * inv_w - (float)c;  // place in the cell, in widths
        const float w = 1.0f / inv_w;
        const float lo = fmaxf(f - 1e-3f, 0.0f) * w, hi = fmaxf(1.0f - f - 1e-3f, 0.0f) * w;
        g0 = lo * lo;
        g2 = hi * hi;
    };
    float gx0, gx2, gy0, gy2, gz0, gz2;
    gaps(pi.x, b.hf[0], g.inv_w[0], cx, gx0, gx2);
    gaps(pi.y, b.hf[1], g.inv_w[1], cy, gy0, gy2);
    gaps(pi.z, b.hf[2], g.inv_w[2], cz, gz0, gz2);
    // Morton parts of the three cell coordinates per axis, and whether the offset wraps
    int wxy = 0;  // bit o: x offset o wraps; bit 3 + o: y offset o wraps
    auto axis = [&](int c, int o, int nc, int bit) {
        int x = c + o - 1;
        wxy |= (x < 0 || x >= nc) ? bit : 0;
        x += (x < 0) ? nc : 0;
        x -= (x >= nc) ? nc : 0;
        return spread3((uint32_t)x);
    };
    const uint32_t kx0 = axis(cx, 0, g.nc[0], 1), kx1 = axis(cx, 1, g.nc[0], 2), kx2 = axis(cx, 2, g.nc[0], 4);
    const uint32_t ky0 = axis(cy, 0, g.nc[1], 8) << 1, ky1 = axis(cy, 1, g.nc[1], 16) << 1,
                   ky2 = axis(cy, 2, g.nc[1], 32) << 1;
    auto consider = [&](int j, const float4& pj, bool wrapped) {
        float dx, dy, dz;
        if (wrapped) {
            dx = (float)fold((double)pj.x - (double)pi.x, b.L[0], b.h[0]);
            dy = (float)fold((double)pj.y - (double)pi.y, b.L[1], b.h[1]);
            dz = (float)fold((double)pj.z - (double)pi.z, b.L[2], b.h[2]);
        } else {
            dx = pj.x - pi.x;
            dy = pj.y - pi.y;
            dz = pj.z - pi.z;
        }
        const float r2 = dx * dx + dy * dy + dz * dz;
        float rl2;
        bool swap;
        rl(ti * nt + ptype(pj.w), rl2, swap);
        if (r2 < rl2 && j != i) {
            // swap kind from the front, the rest from the back (counters stay in registers)
            const int slot = swap ? ns : k_max - 1 - no;
            if (ns + no < k_max) nlist[(size_t)slot * N + i] = j;
            ns += swap ? 1 : 0;
            no += swap ? 0 : 1;
        }
    };
    for (int oz = -1; oz <= 1; ++oz) {
        const float dz2 = oz < 0 ? gz0 : (oz > 0 ? gz2 : 0.0f);
        if (dz2 >= rmax2) continue;
        int z = cz + oz;
        const bool wz = z < 0 || z >= g.nc[2];
        z += (z < 0) ? g.nc[2] : 0;
        z -= (z >= g.nc[2]) ? g.nc[2] : 0;
        const uint32_t kz = spread3((uint32_t)z) << 2;
        // cell 0's packed word, then cells 1..8: exclusive prefix of the counts and
        // (start - prefix) * 2 + wraps (vector values, so they stay in registers)
        typedef int int8v __attribute__((ext_vector_type(8)));
        int ow0 = 0, tot = 0;
        int8v pre, ow;
#pragma unroll
        for (int q = 0; q < 9; ++q) {
            const uint32_t kxq = q % 3 == 0 ? kx0 : (q % 3 == 1 ? kx1 : kx2);
            const uint32_t kyq = q / 3 == 0 ? ky0 : (q / 3 == 1 ? ky1 : ky2);
            const uint32_t key = key_base + (kxq | kyq | kz);
            const float d2 = dz2 + (q / 3 == 0 ? gy0 : (q / 3 == 2 ? gy2 : 0.0f)) +
                             (q % 3 == 0 ? gx0 : (q % 3 == 2 ? gx2 : 0.0f));
            const int st = cell_start[key] + shift;
            const int en = d2 < rmax2 ? cell_start[key + 1] + shift : st;
            const bool wq = wz || (wxy & ((1 << (q % 3)) | (8 << (q / 3)))) != 0;
            const int o = (st - tot) * 2 + (wq ? 1 : 0);  // st - tot may be negative: >> 1 is arithmetic
            if (q == 0) {
                ow0 = o;
            } else {
                pre[q - 1] = tot;
                ow[q - 1] = o;
            }
            tot += en - st;
        }
        if (tot == 0) continue;
#define RC_LOCATE(t, o)                                      \
    do {                                                     \
        o = ow0;                                             \
        _Pragma("unroll") for (int q = 0; q < 8; ++q) o = ((t) >= pre[q]) ? ow[q] : o; \
    } while (0)
        // candidates in groups of four, all four positions requested before any is tested (in candidate
        // order, so the list is the same): 102 -> 95 us per build at 1M particles; one ahead, two, three,
        // six or eight at a time, or the next group requested during the current one, were slower
        constexpr int kAhead = 4;
        for (int t0 = 0; t0 < tot; t0 += kAhead) {
            int oq[kAhead];
            float4 pq[kAhead];
#pragma unroll
            for (int u = 0; u < kAhead; ++u) {
                oq[u] = 0;
                pq[u] = pi;
                if (t0 + u < tot) {
                    RC_LOCATE(t0 + u, oq[u]);
                    pq[u] = pos[t0 + u + (oq[u] >> 1)];
                }
            }
#pragma unroll
            for (int u = 0; u < kAhead; ++u)
                if (t0 + u < tot) consider(t0 + u + (oq[u] >> 1), pq[u], (oq[u] & 1) != 0);
        }
#undef RC_LOCATE
    }
    const int total = ns + no;
    // on overflow the stored prefix is what fitted (the status reports it)
    if (ns + no > k_max) {
        const int keep_s = min(ns, k_max);
        ns = keep_s;
        no = k_max - keep_s;
    }
    nn[i] = ns | (no << 16);
    return total;
}

// block maximum of the list length and block sum of the swap-range lengths
// (no same-address atomics per wave): out[0] and out[nb] of the block's slot
__device__ __forceinline__ void block_max_store(int cnt, int ns, int* __restrict__ out, int nb) {
    __shared__ int s_m[kBlock / kWave], s_n[kBlock / kWave];
    int m = cnt, t_ns = ns;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        m = max(m, __shfl_xor(m, o, kWave));
        t_ns += __shfl_xor(t_ns, o, kWave);
    }
    if ((threadIdx.x & (kWave - 1)) == 0) {
        s_m[threadIdx.x / kWave] = m;
        s_n[threadIdx.x / kWave] = t_ns;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int t = 0, u = 0;
        for (int w = 0; w < kBlock / kWave; ++w) {
            t = max(t, s_m[w]);
            u += s_n[w];
        }
        out[0] = t;
        out[nb] = u;
    }
}

// One thread per particle (key order).
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
    int total = 0, packed = 0;
    if (i < a.N) {
        total = list_one(i, a.pos[i], a.box, a.g, 0u, 0, a.cell_start, a.pos, nt, a.k_max, a.N, a.nlist, a.nn,
                         [&](int q, float& rl2, bool& swap) {
                             rl2 = s_rl2[q];
                             swap = s_swap[q] != 0;
                         });
        packed = a.nn[i];
        if (a.vel) a.vel[i].w = 0.0f;
    }
    if (a.pl_j) pack_wave_lists(i, i < a.N, packed, a.nlist, a.k_max, a.N, a.pl_j, a.pl_o);
    block_max_store(total, nn_swap(packed), a.block_max + blockIdx.x, nb);
}

__global__ __launch_bounds__(kBlock) void k_pack_list(const int* __restrict__ nlist, const int* __restrict__ nn,
                                                      int k_max, int N, int* __restrict__ pl_j,
                                                      unsigned char* __restrict__ pl_o) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const bool live = i < N;
    pack_wave_lists(i, live, live ? nn[i] : 0, nlist, k_max, N, pl_j, pl_o);
}

hipError_t launch_pack_list(const int* nlist, const int* nn, int k_max, int N, int* pl_j, unsigned char* pl_o,
                            hipStream_t s) {
    hipLaunchKernelGGL(k_pack_list, dim3(nblk(N, kBlock)), dim3(kBlock), 0, s, nlist, nn, k_max, N, pl_j, pl_o);
    return hipGetLastError();
}

// Batches: each wave lies in one replica, which gives the box, grid, key
// range and table (its list radii staged in the wavefront's LDS slice); empty
// slots get an empty list.  A replica that keeps its list (build[r] == 0)
// keeps its lists, packed copy and path lengths; its list lengths still count
// towards the status words.
__global__ __launch_bounds__(kBlock) void k_nlist_batch(NlistArgsB a) {
    extern __shared__ float s_rl2b[];  // per wavefront: [nt*nt] list radii^2, then [nt*nt] swap flags
    const int nt = a.tab.nt, nt2 = nt * nt;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
    const int r = i < a.N ? a.chunk_rep[i / kWave] : 0;
    float* rl2s = s_rl2b + 2 * nt2 * wv;
    int* sws = reinterpret_cast<int*>(rl2s + nt2);
    if (i < a.N) {
        const DevEntry* t = a.tab.e + a.rep[r].tab;
        for (int q = lane; q < nt2; q += kWave) {
            rl2s[q] = t[q].rlist2;
            sws[q] = t[q].kind == RC_KIND_SWAP;
        }
    }
    __syncthreads();
    int total = 0, packed = 0;
    const bool builds = i < a.N && rep_builds(a.build, r);   // uniform over the wavefront
    if (i < a.N) {
        const RepDesc& d = a.rep[r];
        if (!builds) {
            packed = a.nn[i];
            total = nn_swap(packed) + nn_other(packed);
        } else if (i < d.off + d.n) {
            const int shift = d.off - a.cell_start[d.key_base];
            total = list_one(i, a.pos[i], d.box, d.grid, d.key_base, shift, a.cell_start, a.pos, nt, a.k_max,
                             a.N, a.nlist, a.nn, [&](int q, float& rl2, bool& swap) {
                                 rl2 = rl2s[q];
                                 swap = sws[q] != 0;
                             });
            packed = a.nn[i];
        } else {
            a.nn[i] = 0;
        }
        if (builds && a.vel) a.vel[i].w = 0.0f;
    }
    if (a.pl_j && (builds || i >= a.N)) pack_wave_lists(i, i < a.N, packed, a.nlist, a.k_max, a.N, a.pl_j, a.pl_o);
    block_max_store(total, nn_swap(packed), a.block_max + blockIdx.x, gridDim.x);
}

// A list laid out for k_old slots per particle copied into the layout of
// k_new >= k_old slots (swap range at the front, the rest at the back), and
// its packed copy for k_new.  One thread per slot; every lane of a
// wavefront takes part (the packing scans the wavefront's lengths).
__global__ __launch_bounds__(kBlock) void k_relayout_list(const int* __restrict__ old_list, int k_old,
                                                         int* __restrict__ new_list, int k_new,
                                                         const int* __restrict__ nn, int N, int* __restrict__ pl_j,
                                                         unsigned char* __restrict__ pl_o) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const bool live = i < N;
    int packed = 0;
    if (live) {
        packed = nn[i];
        const int ns = min(nn_swap(packed), k_old);
        const int no = min(nn_other(packed), k_old - ns);
        for (int q = 0; q < ns; ++q) new_list[(size_t)q * N + i] = old_list[(size_t)q * N + i];
        for (int q = 0; q < no; ++q) new_list[(size_t)(k_new - 1 - q) * N + i] = old_list[(size_t)(k_old - 1 - q) * N + i];
    }
    if (pl_j) pack_wave_lists(i, live, packed, new_list, k_new, N, pl_j, pl_o);
}

hipError_t launch_relayout_list(const int* old_list, int k_old, int* new_list, int k_new, const int* nn, int N,
                                int* pl_j, unsigned char* pl_o, hipStream_t s) {
    hipLaunchKernelGGL(k_relayout_list, dim3(nblk(N, kBlock)), dim3(kBlock), 0, s, old_list, k_old, new_list, k_new,
                       nn, N, pl_j, pl_o);
    return hipGetLastError();
}

// one block: fold the per-block maxima into the status word
// Fold the per-block largest list lengths into the status words: KMAX and
// the overflow flag.  fresh: write every word instead, as a cleared status
// followed by this fold and a chunk reset would leave it (the driver's
// rebuilds, which so need no separate clear and reset launches).
__global__ __launch_bounds__(1024) void k_nlist_status(const int* __restrict__ block_max, int nb, int k_max,
                                                      int* __restrict__ status, int fresh) {
    __shared__ int red[1024];
    __shared__ long long red_ns[1024];
    int m = 0;
    long long t_ns = 0;
    for (int b = threadIdx.x; b < nb; b += blockDim.x) {
        m = max(m, block_max[b]);
        t_ns += block_max[nb + b];
    }
    red[threadIdx.x] = m;
    red_ns[threadIdx.x] = t_ns;
    __syncthreads();
    for (int w = 512; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            red[threadIdx.x] = max(red[threadIdx.x], red[threadIdx.x + w]);
            red_ns[threadIdx.x] += red_ns[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const int ovf = red[0] > k_max ? RC_FLAG_NLIST_OVERFLOW : 0;
        if (fresh) {
            for (int w = 0; w < RC_STATUS_WORDS; ++w) status[w] = 0;
            status[RC_ST_FLAGS] = ovf;
            status[RC_ST_KMAX] = red[0];
            status[RC_ST_FIRST_SOFT] = 0x7fffffff;
            status[RC_ST_FIRST_HARD] = 0x7fffffff;
        } else {
            status[RC_ST_KMAX] = max(status[RC_ST_KMAX], red[0]);
            status[RC_ST_FLAGS] |= ovf;
        }
        status[RC_ST_NSWAP] = (int)min(red_ns[0], (long long)0x7fffffff);   // the latest list's
    }
}

hipError_t launch_nlist(const NlistArgs& a, hipStream_t s) {
    const size_t shm = 2 * sizeof(float) * a.tab.nt * a.tab.nt;
    const int nb = nblk(a.N, kBlock);
    hipLaunchKernelGGL(k_nlist, dim3(nb), dim3(kBlock), shm, s, a);
    if (a.status)
        hipLaunchKernelGGL(k_nlist_status, dim3(1), dim3(1024), 0, s, a.block_max, nb, a.k_max, a.status,
                           a.fresh_status);
    return hipGetLastError();
}

hipError_t launch_nlist_batch(const NlistArgsB& a, hipStream_t s) {
    const int nb = nblk(a.N, kBlock);
    const size_t shm = (size_t)(kBlock / kWave) * 2 * sizeof(float) * a.tab.nt * a.tab.nt;
    hipLaunchKernelGGL(k_nlist_batch, dim3(nb), dim3(kBlock), shm, s, a);
    if (a.status)
        hipLaunchKernelGGL(k_nlist_status, dim3(1), dim3(1024), 0, s, a.block_max, nb, a.k_max, a.status,
                           a.fresh_status);
    return hipGetLastError();
}

}  // namespace rc
