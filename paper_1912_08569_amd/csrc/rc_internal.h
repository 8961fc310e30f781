// Internal declarations of the swap-potential engine (HIP, gfx950).
//
// Device data layout and the inline device helpers shared by the kernels:
// the compiled per-type-pair table, the canonical FP64 cut predicate, the
// FP32 pair / switching-factor evaluation, Morton keys of the cell grid and
// the Philox4x32-10 thermostat noise.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/rc.h"

namespace rc {

constexpr int kBlock = 256;          // threads per block of the particle kernels
constexpr int kWave = 64;            // CDNA wavefront
constexpr int kEvWords = 13;         // E, W(6), K(6)
constexpr int kStepBlock = 64;       // one wavefront per block: the step and gather kernels
constexpr int kScanItems = 8;        // counts per thread in the scan kernels
constexpr int kScanTile = kBlock * kScanItems;

// One compiled table entry (80 bytes).  FP32 values feed the term arithmetic;
// the FP64 squares feed the canonical cut / bond decisions; the FP32 band
// edges [lo, hi] around them bracket the squares that FP32 rounding could put
// on the wrong side (see pair_geom).
struct alignas(16) DevEntry {
    int kind;          // RC_KIND_*
    int n;             // exponent (6 for WCA)
    float eps;         // epsilon
    float sig2;        // sigma^2
    float sqrt_lam;    // sqrt(lambda * eps)  (triplet weight per partner)
    float rlist2;      // (r_cut + r_buff)^2 * (1 + 1e-5), list radius
    double rcut2;      // r_cut * r_cut
    double rmin2;      // (sigma*sigma) * pow(2, 2/n)
    float inv_eps;     // 1/eps (SWAP), 0 otherwise
    float sigma;       // sigma
    float lam;         // lambda (SWAP), 0 otherwise
    float rcut2_lo, rcut2_hi;   // r_cut^2 (1 -+ 2e-6), rounded outwards
    float rmin2_lo, rmin2_hi;   // r_min^2 (1 -+ 2e-6), rounded outwards
};

struct Box {
    double L[3];
    double h[3];       // L/2
    float Lf[3];
    float hf[3];
};

// --------------------------------------------------------------------------
// neighbour-list column layout: swap-kind neighbours of i fill slots
// 0 .. ns-1 from the front, all other neighbours fill slots k_max-1 down to
// k_max-no from the back; nn[i] = ns | (no << 16).
// --------------------------------------------------------------------------
__host__ __device__ __forceinline__ int nn_swap(int packed) { return packed & 0xffff; }
__host__ __device__ __forceinline__ int nn_other(int packed) { return packed >> 16; }

// --------------------------------------------------------------------------
// particle word helpers
// --------------------------------------------------------------------------
__device__ __forceinline__ int ptype(float w) { return __float_as_int(w) & ((1 << RC_TYPE_BITS) - 1); }
__device__ __forceinline__ int ptag(float w) { return __float_as_int(w) >> RC_TYPE_BITS; }

// --------------------------------------------------------------------------
// canonical FP64 predicate: d = x_j - x_i folded once by +-L,
// r^2 = (dx*dx + dy*dy) + dz*dz with separately rounded products and sums.
// --------------------------------------------------------------------------
__device__ __forceinline__ double fold(double d, double L, double h) {
    if (d > h) d -= L;
    else if (d < -h) d += L;
    return d;
}

__device__ __forceinline__ double canon_r2(const float4& pi, const float4& pj, const Box& b,
                                           double& dx, double& dy, double& dz) {
#pragma clang fp contract(off)
    dx = fold((double)pj.x - (double)pi.x, b.L[0], b.h[0]);
    dy = fold((double)pj.y - (double)pi.y, b.L[1], b.h[1]);
    dz = fold((double)pj.z - (double)pi.z, b.L[2], b.h[2]);
    // plain operators under contract(off): each product and sum rounds separately
    const double xx = dx * dx, yy = dy * dy, zz = dz * dz;
    return (xx + yy) + zz;
}

// Geometry of one pair (i -> j) under one table entry: the FP32 minimum-image
// difference and square, and the canonical decisions.  Where x_j - x_i needs
// no periodic fold the FP32 difference is the exact difference rounded once
// (the same value as the canonical FP64 difference converted), and its FP32
// square is within 4e-7 relative of the canonical one; a decision is then
// taken in FP32 when the square lies outside the table's 2e-6 band around the
// threshold.  Pairs across a periodic face, and squares inside a band, take
// the canonical FP64 path, so every decision equals canon_r2's.
struct PairGeom {
    float dx, dy, dz;  // x_j - x_i (minimum image)
    float r2;
    bool cut;          // r^2 <  r_cut^2
    bool inside;       // r^2 <= r_min^2
    bool bond;         // r^2 <  r_min^2
};

__device__ __forceinline__ PairGeom pair_geom(const float4& pi, const float4& pj, const Box& b, const DevEntry& e) {
    PairGeom g;
    g.dx = pj.x - pi.x;
    g.dy = pj.y - pi.y;
    g.dz = pj.z - pi.z;
    const bool wrap = fabsf(g.dx) > b.hf[0] || fabsf(g.dy) > b.hf[1] || fabsf(g.dz) > b.hf[2];
    g.r2 = g.dx * g.dx + g.dy * g.dy + g.dz * g.dz;
    g.cut = g.r2 < e.rcut2_lo;
    g.inside = g.r2 < e.rmin2_lo;
    g.bond = g.inside;
    const bool sure = !wrap && (g.cut || g.r2 > e.rcut2_hi) &&
                      (e.kind != RC_KIND_SWAP || g.inside || g.r2 > e.rmin2_hi);
    if (!sure) {
        double dx, dy, dz;
        const double r2d = canon_r2(pi, pj, b, dx, dy, dz);
        g.dx = (float)dx;
        g.dy = (float)dy;
        g.dz = (float)dz;
        g.r2 = (float)r2d;
        g.cut = r2d < e.rcut2;
        g.inside = r2d <= e.rmin2;
        g.bond = r2d < e.rmin2;
    }
    return g;
}

// --------------------------------------------------------------------------
// FP32 term arithmetic
// --------------------------------------------------------------------------
// x^k by squaring; the exponents of the workloads (k = 3 for the WCA term,
// k = 5 for n = 10) are unrolled into the same products the loop forms
__device__ __forceinline__ float ipowf(float x, int k) {
    if (k == 5) {
        const float x2 = x * x;
        return x * (x2 * x2);
    }
    if (k == 3) return x * (x * x);
    float r = 1.0f;
    while (k) {
        if (k & 1) r *= x;
        x *= x;
        k >>= 1;
    }
    return r;
}

// 1/r^2 by the hardware reciprocal (1 ulp): every r^-2 factor of a term uses it
__device__ __forceinline__ float inv_r2(float r2) { return __builtin_amdgcn_rcpf(r2); }

// q = (sigma/r)^n from s2 = sigma^2 / r^2
__device__ __forceinline__ float qpow(float s2, int n) {
    float q = ipowf(s2, n >> 1);
    if (n & 1) q *= __builtin_amdgcn_sqrtf(s2);
    return q;
}

// Pair term (eq. 2b for SWAP; WCA = n 6 plus the +eps shift): energy phi and
// g = phi'(r)/r, so that the force on i from the pair is g * (x_j - x_i).
__device__ __forceinline__ void pair_eval(const DevEntry& e, float r2, float& phi, float& g) {
    const float ir2 = inv_r2(r2);
    float q = qpow(e.sig2 * ir2, e.n);
    float q2 = q * q;
    phi = 4.0f * e.eps * (q2 - q) + (e.kind == RC_KIND_WCA ? e.eps : 0.0f);
    g = 4.0f * e.eps * (float)e.n * (q - 2.0f * q2) * ir2;
}

// Switching factor of eq. (pot) inside the cutoff: u and u'(r)/r.
// 'inside' is the canonical decision r^2 <= r_min^2.
__device__ __forceinline__ void vhat_eval(const DevEntry& e, bool inside, float r2, float& u,
                                          float& u1r) {
    if (inside) {
        u = 1.0f;
        u1r = 0.0f;
        return;
    }
    const float ir2 = inv_r2(r2);
    float q = qpow(e.sig2 * ir2, e.n);
    float q2 = q * q;
    u = 4.0f * __fmaf_rn(-q, q, q);   // explicit fma: the same bits in every kernel
    u1r = 4.0f * (float)e.n * (2.0f * q2 - q) * ir2;
}

// pair_eval and vhat_eval of one entry sharing 1/r^2 and (sigma/r)^n (the
// same values as the two calls)
__device__ __forceinline__ void pair_vhat_eval(const DevEntry& e, bool swap, bool inside, float r2, float& phi,
                                               float& g, float& u, float& u1r) {
    const float ir2 = inv_r2(r2);
    const float q = qpow(e.sig2 * ir2, e.n);
    const float q2 = q * q;
    phi = 4.0f * e.eps * (q2 - q) + (e.kind == RC_KIND_WCA ? e.eps : 0.0f);
    g = 4.0f * e.eps * (float)e.n * (q - 2.0f * q2) * ir2;
    u = 0.0f;
    u1r = 0.0f;
    if (swap) {
        u = inside ? 1.0f : 4.0f * __fmaf_rn(-q, q, q);
        u1r = inside ? 0.0f : 4.0f * (float)e.n * (2.0f * q2 - q) * ir2;
    }
}

__device__ __forceinline__ float vhat_value(const DevEntry& e, bool inside, float r2) {
    if (inside) return 1.0f;
    float q = qpow(e.sig2 * inv_r2(r2), e.n);
    return 4.0f * __fmaf_rn(-q, q, q);
}

// --------------------------------------------------------------------------
// Morton keys of the cell grid (10 bits per axis)
// --------------------------------------------------------------------------
__host__ __device__ __forceinline__ uint32_t spread3(uint32_t x) {
    x &= 0x3ffu;
    x = (x | (x << 16)) & 0x030000FFu;
    x = (x | (x << 8)) & 0x0300F00Fu;
    x = (x | (x << 4)) & 0x030C30C3u;
    x = (x | (x << 2)) & 0x09249249u;
    return x;
}
__host__ __device__ __forceinline__ uint32_t morton3(uint32_t x, uint32_t y, uint32_t z) {
    return spread3(x) | (spread3(y) << 1) | (spread3(z) << 2);
}

struct Grid {
    int nc[3];
    int bits;            // Morton bits per axis
    float inv_w[3];      // nc / L
    uint32_t nkeys;      // 8^bits
};

// One replica of a batch.  Replica r owns the particle slots [off, off + n)
// with off a multiple of 64, so every wavefront of a particle kernel lies in
// one replica; the slots from off + n to the next replica's off are unused.
// Its cells own the keys [key_base, key_base + grid.nkeys) of the batch's key
// space, so the counting sort keeps every replica inside its slots.
struct RepDesc {
    Box box;
    Grid grid;
    uint32_t key_base;
    int off;       // first slot
    int n;         // particles
    int tab;       // first entry of its nt*nt table in the batch table array
    int pad;
};

__device__ __forceinline__ int cell_coord(float x, float h, float inv_w, int nc) {
    int c = (int)floorf((x + h) * inv_w);
    return c < 0 ? 0 : (c >= nc ? nc - 1 : c);
}

// --------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11) and Box-Muller normals
// --------------------------------------------------------------------------
struct U4 {
    uint32_t x, y, z, w;
};

__device__ __forceinline__ U4 philox10(U4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        // one 32x32 -> 64-bit product per multiplier (v_mad_u64_u32)
        const uint64_t p0 = (uint64_t)0xD2511F53u * c.x, p1 = (uint64_t)0xCD9E8D57u * c.z;
        const uint32_t lo0 = (uint32_t)p0, hi0 = (uint32_t)(p0 >> 32);
        const uint32_t lo1 = (uint32_t)p1, hi1 = (uint32_t)(p1 >> 32);
        c = U4{hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0};
    }
    return c;
}

__device__ __forceinline__ float u01(uint32_t x) {
    return ((float)x + 0.5f) * 2.3283064365386963e-10f;  // (x + 1/2) 2^-32
}

__device__ __forceinline__ void thermostat_normals(uint64_t seed, uint32_t tag, uint64_t step,
                                                   float& z0, float& z1, float& z2) {
    U4 w = philox10(U4{tag, (uint32_t)step, (uint32_t)(step >> 32), 0u}, (uint32_t)seed,
                    (uint32_t)(seed >> 32));
    // v_sin_f32 / v_cos_f32 take the angle in revolutions: sin(2 pi u) is one
    // instruction; the radius keeps the library logarithm (accurate near u = 1)
    const float r0 = __builtin_amdgcn_sqrtf(-2.0f * logf(u01(w.x)));
    const float r1 = __builtin_amdgcn_sqrtf(-2.0f * logf(u01(w.z)));
    const float a0 = u01(w.y), a1 = u01(w.w);
    z0 = r0 * __builtin_amdgcn_cosf(a0);
    z1 = r0 * __builtin_amdgcn_sinf(a0);
    z2 = r1 * __builtin_amdgcn_cosf(a1);
}

// --------------------------------------------------------------------------
// wave / block reductions
// --------------------------------------------------------------------------
// Inclusive prefix sum over the 64 lanes of a wavefront, all lanes active:
// shifts by 1, 2, 4, 8 inside each 16-lane row, then each row adds the last
// lane of the rows before it (row broadcasts of lanes 15 and 31).  Six DPP
// adds; no LDS round trips.
__device__ __forceinline__ int wave_inclusive_scan(int x) {
    x += __builtin_amdgcn_update_dpp(0, x, 0x111, 0xf, 0xf, false);  // row_shr:1
    x += __builtin_amdgcn_update_dpp(0, x, 0x112, 0xf, 0xf, false);  // row_shr:2
    x += __builtin_amdgcn_update_dpp(0, x, 0x114, 0xf, 0xf, false);  // row_shr:4
    x += __builtin_amdgcn_update_dpp(0, x, 0x118, 0xf, 0xf, false);  // row_shr:8
    x += __builtin_amdgcn_update_dpp(0, x, 0x142, 0xa, 0xf, false);  // row_bcast:15 into rows 1, 3
    x += __builtin_amdgcn_update_dpp(0, x, 0x143, 0xc, 0xf, false);  // row_bcast:31 into rows 2, 3
    return x;
}

// Packed copy of the lists of a wavefront's 64 particles (lanes i - lane ..
// i - lane + 63): entry e of the wavefront's region, which starts at
// (i - lane) * k_max, holds the neighbour index and the owner lane, in the
// order the gather walks them (each particle's swap range, then its other
// range; particles in lane order).  Every lane of the wavefront must be
// active; live = i < N.  The arrays hold ceil(N / 64) * 64 * k_max entries.
__device__ __forceinline__ void pack_wave_lists(int i, bool live, int packed, const int* nlist, int k_max, int N,
                                                int* pl_j, unsigned char* pl_o) {
    const int lane = (int)(threadIdx.x & (kWave - 1));
    // a built list has ns + no <= k_max; the clamp keeps every write inside the
    // wavefront's region whatever nn holds
    const int ns = live ? min(nn_swap(packed), k_max) : 0;
    const int cnt = live ? ns + min(nn_other(packed), k_max - ns) : 0;
    const int off = wave_inclusive_scan(cnt) - cnt;
    const size_t base = (size_t)(i - lane) * k_max + off;
    for (int s = 0; s < cnt; ++s) {
        const int slot = s < ns ? s : k_max - 1 - (s - ns);
        pl_j[base + s] = nlist[(size_t)slot * N + i];
        pl_o[base + s] = (unsigned char)lane;
    }
}

// One DPP step of a 64-bit scan: v plus the value of the lane ctrl selects
// (0 where the row mask or the row's edge leaves no source).
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_add(double v) {
    const long long b = __double_as_longlong(v);
    int lo, hi;
    if constexpr (ROW_MASK == 0xf) {   // every row written: lanes without a source read 0 (bound_ctrl)
        lo = __builtin_amdgcn_mov_dpp((int)b, CTRL, ROW_MASK, 0xf, true);
        hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, ROW_MASK, 0xf, true);
    } else {                           // rows left out keep the old value 0
        lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, ROW_MASK, 0xf, false);
        hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROW_MASK, 0xf, false);
    }
    return v + __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// Sum over the wavefront, returned to every lane; every lane must be active.
// The inclusive scan of wave_inclusive_scan (DPP row shifts, then the row
// broadcasts) leaves the total in lane 63, which is read back: no LDS
// permutes, and one fixed order of additions.
__device__ __forceinline__ double wave_sum(double v) {
    v = dpp_add<0x111, 0xf>(v);  // row_shr:1
    v = dpp_add<0x112, 0xf>(v);  // row_shr:2
    v = dpp_add<0x114, 0xf>(v);  // row_shr:4
    v = dpp_add<0x118, 0xf>(v);  // row_shr:8
    v = dpp_add<0x142, 0xa>(v);  // row_bcast:15 into rows 1, 3
    v = dpp_add<0x143, 0xc>(v);  // row_bcast:31 into rows 2, 3
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)b, kWave - 1);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), kWave - 1);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ float wave_maxf(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, kWave));
    return v;
}

// Sum NW doubles per thread over the block; thread 0 writes them to out[0..NW).
template <int NW>
__device__ __forceinline__ void block_sum_store(double (&v)[NW], double* out) {
    __shared__ double red[kBlock / kWave][NW];
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
#pragma unroll
    for (int q = 0; q < NW; ++q) v[q] = wave_sum(v[q]);
    if (lane == 0) {
#pragma unroll
        for (int q = 0; q < NW; ++q) red[wid][q] = v[q];
    }
    __syncthreads();
    if (threadIdx.x < NW) {
        double s = 0.0;
        for (int w = 0; w < kBlock / kWave; ++w) s += red[w][threadIdx.x];
        out[threadIdx.x] = s;
    }
}

// XCD-aware block order: consecutive dispatch slots go round-robin over the
// 8 XCDs, so hand each XCD one contiguous range of (Morton ordered) particles
// to keep neighbour gathers inside that XCD's L2.
__device__ __forceinline__ int xcd_block(int nblocks) {
    const int b = blockIdx.x;
    const int per = nblocks / 8;
    if (per == 0 || b >= per * 8) return b;
    return (b % 8) * per + b / 8;
}

// --------------------------------------------------------------------------
// argument bundles and launchers (defined in the kernel translation units)
// --------------------------------------------------------------------------
struct Table {
    const DevEntry* e;   // [nt*nt]
    int nt;
};

struct StepArgs {
    const float4* pos_in;
    float4* pos_out;
    float4* vel;
    int4* image;
    const int* nlist;
    const int* nn;
    int N;
    int mode;
    int k_max;                 // list slots allocated per particle (nlist is [k_max][N])
    Table tab;
    Box box;
    float minv[RC_MAX_TYPES];  // 1/m per type
    float c2[RC_MAX_TYPES];    // sqrt((1 - c1^2) kT / m) per type
    float dt, c1;
    int langevin;
    float noise_z;   // 1, or 0 for motion in the xy plane (no thermostat noise along z)
    float hard, soft;          // path-length thresholds (stale list, rebuild)
    uint64_t seed;
    uint64_t step;             // step index (added to *step_base if not NULL)
    const unsigned long long* step_base;
    double* ev_part;           // [nblocks*13] | NULL (row of logical block c at c*13)
    // single systems, ev steps: per logical block the number of bonds (swap pairs
    // m < j with canonical r^2 < r_min^2) among its particles' list entries | NULL
    unsigned* bond_part;
    // a chunk's reset done by this launch (thread 0 of block 0) instead of a launch of its own:
    // reset_status NULL = none; else as launch_status_reset_chunk(reset_status, reset_base, reset_to)
    int* reset_status;
    unsigned long long* reset_base;
    unsigned long long reset_to;
    int* status;
    int* blk;                  // [nblocks*3] per-block flag / first-soft / first-hard slots
    // batches only (tab.e then holds every replica's table, box is unused)
    const RepDesc* rep;        // [R]
    const int* chunk_rep;      // [N / 64] replica of each 64-slot chunk
    const uint64_t* seeds;     // [R] thermostat keys
    int width;                 // gather width of the non-logging steps: 1, 2 or 4 (read by the launcher)
    int form;                  // RC_FORM_WALK or RC_FORM_SUMS (read by the launcher)
    float* ssum;               // [N] per-particle switching sums (RC_FORM_SUMS)
    // packed list (single systems): per wavefront the flattened entries of its
    // 64 particles, neighbour index and owner lane (pack_wave_lists)
    const int* pl_j;
    const unsigned char* pl_o;
    // FENE springs (single systems; NULL bonds = none)
    const int2* bonds;         // [N] partner tags per tag, -1 = none
    const int* rtag;           // [N] tag -> index
    float fene_k, fene_r02;    // K and R0^2
};

hipError_t launch_step(const StepArgs& a, bool ev, hipStream_t s);
// a plain step launch with its kernels between event pairs (sums: [2] or NULL, step: [2])
hipError_t launch_step_timed(const StepArgs& a, bool batch, hipStream_t s, hipEvent_t* sums, hipEvent_t* step);
// Small systems (at most kBlockMaxN particles, single system, walk or sums
// form): G plain steps in one workgroup with the positions in LDS, the same
// arithmetic as G launches of the step.  pos_final receives the positions
// (the buffer a.pos_in names), *step_base is read as the first step's index
// and advanced by G.  step_block_fits says whether a system fits the kernel.
constexpr int kBlockMaxN = 1024;
bool step_block_fits(int N, int nt, int form);
hipError_t launch_step_block(const StepArgs& a, float4* pos_final, unsigned long long* step_base, int G,
                             hipStream_t s);
// the head-form step kernel (same launch shape and arguments as k_step)
void step_kernel_info(bool ev, int width, int form, const void** fn);
hipError_t launch_step_batch(const StepArgs& a, bool ev, hipStream_t s);
void step_batch_kernel_info(int width, int form, const void** fn);

struct ForceArgs {
    const float4* pos;
    const int* nlist;
    const int* nn;
    int N;
    int k_max;         // list slots allocated per particle
    Table tab;
    Box box;
    float4* force;
    double* ev_part;   // [nblocks*13] | NULL
    int accumulate;
    int* status;
    const RepDesc* rep;    // batches only
    const int* chunk_rep;
    float* ssum;           // [N] switching sums: non-NULL selects the two-pass form
};
hipError_t launch_forces_triplet(const ForceArgs& a, hipStream_t s);
hipError_t launch_forces_gather(const ForceArgs& a, hipStream_t s);
hipError_t launch_forces_gather_batch(const ForceArgs& a, hipStream_t s);
// first pass of the two-pass form: the kernel that fills ssum (for graphs)
// and its arguments for a step (positions pos_in)
void sums_kernel_info(bool batch, const void** fn);
ForceArgs step_sums_args(const StepArgs& a);

struct IntegrateArgs {
    float4* pos;
    float4* vel;
    const float4* force;
    int4* image;
    int N;
    int half;
    Box box;
    float minv[RC_MAX_TYPES];
    float c2[RC_MAX_TYPES];
    float dt, c1;
    int langevin;
    float noise_z;   // 1, or 0 for motion in the xy plane (no thermostat noise along z)
    float soft;
    uint64_t seed, step;
    double* kin_part;   // [nblocks*13] | NULL (slots 7..12 used)
    int* status;
};
hipError_t launch_integrate(const IntegrateArgs& a, hipStream_t s);
hipError_t launch_thermostat_normals(uint64_t seed, uint64_t step0, int steps, int N, float noise_z, float4* out,
                                     hipStream_t s);

struct CellsArgs {
    float4* pos;
    float4* vel;
    int4* image;
    int* rtag;
    int N;
    Box box;
    Grid g;
    // workspace
    int* counts;       // [nkeys]
    int* cell_start;   // [nkeys + 1]
    int* keys;         // [N]
    int* rank;         // [N]
    int* order;        // [N]
    int* block_sums;   // [nkeys / kScanTile + 1]
    float4* tpos;
    float4* tvel;
    int4* timage;
};
hipError_t launch_cells(const CellsArgs& a, hipStream_t s);

struct NlistArgs {
    const float4* pos;
    float4* vel;
    int N;
    Box box;
    Grid g;
    const int* cell_start;
    Table tab;
    int k_max;
    int* nlist;
    int* nn;
    int* status;
    int* block_max;    // [ceil(N / kBlock)] scratch (largest list length per block)
    int* pl_j;         // packed copy of the list (NULL: none), see pack_wave_lists
    unsigned char* pl_o;
    int fresh_status;  // 1: write every status word (see k_nlist_status); 0: fold into them
};
hipError_t launch_nlist(const NlistArgs& a, hipStream_t s);
// the packed copy of a list built elsewhere
hipError_t launch_pack_list(const int* nlist, const int* nn, int k_max, int N, int* pl_j, unsigned char* pl_o,
                            hipStream_t s);

// count: device u64 result; part: scratch of ceil(N / kBlock) u64
hipError_t launch_bonds(const float4* pos, const int* nlist, const int* nn, int k_max, int N, Table tab,
                        Box box, unsigned long long* count, unsigned long long* part, hipStream_t s);
// tag of each particle's single bonded partner (-1 none, -2 several), indexed by tag
hipError_t launch_bond_partners(const float4* pos, const int* nlist, const int* nn, int k_max, int N, Table tab,
                                Box box, int* partner, hipStream_t s);
hipError_t launch_fold_status(int* blk, int nb, const float4* vel, int N, int* status, hipStream_t s);
hipError_t launch_blk_reset(int* blk, int nb, hipStream_t s);

// reduce nblocks partial rows of 13 doubles into out[first .. first+count) (fixed order); slice:
// NULL, or scratch of kRowSlices doubles for the same sums in two launches that spread the reads.
// With slice, bonds (nblocks per-block counts) may be summed into *bonds_out by the same launches.
constexpr int kRowSlices = 256 * 14;
hipError_t launch_reduce_rows(const double* part, int nblocks, int first, int count, double* out,
                              hipStream_t s, double* slice = nullptr, const unsigned* bonds = nullptr,
                              unsigned long long* bonds_out = nullptr);
// clear the chunk-local status markers (keeping KMAX, MAXPATH and the overflow flag) and, if
// step_base is not NULL, set *step_base = step
__device__ __forceinline__ void chunk_reset(int* st, unsigned long long* base, unsigned long long step) {
    // keep KMAX, MAXPATH and the overflow flag of the current list, clear the chunk-local markers
    st[RC_ST_FLAGS] &= RC_FLAG_NLIST_OVERFLOW;
    st[RC_ST_FIRST_SOFT] = 0x7fffffff;
    st[RC_ST_FIRST_HARD] = 0x7fffffff;
    if (base) *base = step;  // the step counter of the graph replays
}
hipError_t launch_status_reset_chunk(int* status, hipStream_t s, unsigned long long* step_base = nullptr,
                                     unsigned long long step = 0);
// one launch copying pos, vel and (if both non-NULL) image: the driver's snapshot and its restore;
// zero_path writes the velocities' path lengths (w) as zero (a restore of the state a list build left)
hipError_t launch_copy_state(const float4* pos, const float4* vel, const int4* image, float4* pos_to, float4* vel_to,
                             int4* image_to, int N, hipStream_t s, bool zero_path = false);
hipError_t launch_zero_words(int* p, int n, hipStream_t s);
hipError_t launch_add_step(unsigned long long* p, unsigned long long v, hipStream_t s);
hipError_t launch_set_step(unsigned long long* p, unsigned long long v, hipStream_t s);
void add_step_kernel_info(const void** fn);

struct HvpArgs {
    const float4* pos;
    const int* nlist;
    const int* nn;
    int k_max;
    int N;
    Table tab;
    Box box;
    const float4* v;           // [nvec][N] tangent vectors
    float4* hv;                // [nvec][N] products
    double2* sums;             // [nvec][N] scratch: (S, dS) of every particle (first pass)
    int nvec;                  // vectors, one per grid row (blockIdx.y)
};
hipError_t launch_hvp(const HvpArgs& a, hipStream_t s);
// observables: partner statistics over tags (part: 3 * ceil(N/kBlock) counts of scratch; out: 3
// device counts) and the stress autocorrelation of T logged rows (G: max_lag + 1 device doubles)
hipError_t launch_partner_counts(const int* p0, const int* pt, const unsigned char* sel, int N,
                                 unsigned long long* part, unsigned long long* out, hipStream_t s);
hipError_t launch_stress_acf(const double* rows, int T, double volume, double kT, int max_lag, double* G,
                             hipStream_t s);

struct ParamArgs {
    const float4* pos;
    const int* nlist;
    const int* nn;
    int k_max;
    int N;
    Table tab;
    Box box;
    const float4* adj;     // NULL for the energy gradient
    double* part;          // [nblocks * nt*nt*3]
};
hipError_t launch_param(const ParamArgs& a, hipStream_t s);
hipError_t launch_param_vjp(const ParamArgs& a, hipStream_t s);
// FENE springs alone: force[i] += spring forces (w += half bond energies);
// ev_part: per-block rows (7 values at the head of 13-value rows) or NULL
hipError_t launch_fene(const float4* pos, const int2* bonds, const int* rtag, int N, Box box, float K, float R02,
                       float4* force, double* ev_part, hipStream_t s);
// soft bond count into *value (device double) and its gradient (float4, nullable)
hipError_t launch_soft_bonds(const float4* pos, const int* nlist, const int* nn, int k_max, int N, Table tab,
                             Box box, double* part, double* value, float4* grad, hipStream_t s);
hipError_t launch_reduce_param(const double* part, int nblocks, int nt, double* out,
                               hipStream_t s);

// ---- batches ---------------------------------------------------------------
struct CellsArgsB {
    float4* pos;
    float4* vel;
    int4* image;
    int* rtag;
    int N;                  // slots
    const RepDesc* rep;
    const int* chunk_rep;
    const uint32_t* key_end;  // [R] key_base + nkeys of each replica (ascending)
    int R;
    uint32_t nkeys;         // whole batch
    int* counts;
    int* cell_start;
    int* keys;
    int* rank;
    int* order;
    int* block_sums;
    float4* tpos;
    float4* tvel;
    int4* timage;
    const int* build;       // [R] nonzero: the replica is re-ordered (NULL: every replica)
};
hipError_t launch_cells_batch(const CellsArgsB& a, hipStream_t s);

struct NlistArgsB {
    const float4* pos;
    float4* vel;
    int N;                  // slots
    const RepDesc* rep;
    const int* chunk_rep;
    Table tab;              // every replica's table
    const int* cell_start;
    int k_max;
    int* nlist;
    int* nn;
    int* status;
    int* block_max;
    int* pl_j;              // packed copy of the list (NULL: none), see pack_wave_lists
    unsigned char* pl_o;
    int fresh_status;       // as in NlistArgs
    const int* build;       // [R] nonzero: the replica's list is rebuilt (NULL: every replica)
};
hipError_t launch_nlist_batch(const NlistArgsB& a, hipStream_t s);
// a list of k_old slots per particle copied into a layout of k_new >= k_old slots, with its packed copy
// (pl_j NULL: none)
hipError_t launch_relayout_list(const int* old_list, int k_old, int* new_list, int k_new, const int* nn, int N,
                                int* pl_j, unsigned char* pl_o, hipStream_t s);
// per-replica fold of a chunk (before launch_fold_status resets the slots), into out [2][R]:
// out[r] = 1 when a block of replica r crossed the rebuild threshold, out[R + r] = the largest path
// length of its slots (float bits); status[MAXPATH] is raised to the largest of all.  nb = slots / 64
// chunks; chunk_path: scratch of nb floats
hipError_t launch_fold_reps(const int* blk, const float4* vel, int nb, const RepDesc* rep, int R, int* out,
                            float* chunk_path, int* status, hipStream_t s);

// per-replica bond counts: part = one u64 per 64-slot chunk, count = [R]
hipError_t launch_bonds_batch(const float4* pos, const int* nlist, const int* nn, int k_max, int N, Table tab,
                              const RepDesc* rep, const int* chunk_rep, int R, unsigned long long* count,
                              unsigned long long* part, hipStream_t s);
// per-replica fixed-order sums of chunk rows: out[r * out_stride + q], q < count
hipError_t launch_reduce_rows_batch(const double* part, const RepDesc* rep, int R, int first, int count,
                                    double* out, int out_stride, hipStream_t s);

}  // namespace rc
