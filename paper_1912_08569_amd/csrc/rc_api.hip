// C ABI of the swap-potential engine for one system: validation, table
// compilation, workspace layout, launches and the chunked MD driver.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include <hip/hip_ext.h>

#include "rc_host.h"

using namespace rc;
using namespace rc::host;

// ---------------------------------------------------------------------------
// Fixed scratch of rc_compute_forces_noalloc: the per-block energy/virial rows
// of RC_NOALLOC_MAX_N particles, then their switching sums.  In host code the
// array's name is only a stand-in; its device address on each GPU is taken
// once (rc_create, with that device current) and kept in g_scratch_dev.
// ---------------------------------------------------------------------------
namespace {
constexpr size_t kNoallocRowBytes =
    sizeof(double) * kEvWords * (size_t)((RC_NOALLOC_MAX_N + kWave - 1) / kWave);
constexpr size_t kNoallocBytes = kNoallocRowBytes + sizeof(float) * (size_t)RC_NOALLOC_MAX_N;
static_assert(kNoallocRowBytes % 256 == 0, "sums must start 256-byte aligned");
static_assert(kNoallocBytes == RC_NOALLOC_SCRATCH_BYTES, "scratch size and its public value disagree");
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxDevices] = {};
}  // namespace

static __device__ __align__(256) unsigned char scratch[kNoallocBytes];

namespace {

// device address of the fixed scratch on the current device (looked up once per device)
hipError_t noalloc_scratch_here(int device, void** out) {
    *out = nullptr;
    if (device < 0 || device >= kMaxDevices) return hipSuccess;   // the entry point then reports it
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_dev[device]) {
        void* p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_dev[device] = p;
    }
    *out = g_scratch_dev[device];
    return hipSuccess;
}

int check_common(rc_ctx* c, int N, const void* pos) {
    if (!c) return RC_ERR_ARG;
    if (N < 1) return fail(c, RC_ERR_ARG, "N must be >= 1 (got %d)", N);
    if (N >= RC_MAX_TAG) return fail(c, RC_ERR_UNSUPPORTED, "N must be < 2^27");
    if (!pos) return fail(c, RC_ERR_ARG, "positions are NULL");
    if (reinterpret_cast<uintptr_t>(pos) & 15) return fail(c, RC_ERR_ARG, "positions not 16-byte aligned");
    return RC_OK;
}

int reduce_rows(rc_ctx* c, int nb, int first, int count, double* out, hipStream_t s) {
    HIP_TRY(c, launch_reduce_rows(c->d_part, nb, first, count, out, s, c->d_slices));
    return RC_OK;
}

Table dev_table(const rc_ctx* c) { return Table{c->d_tab, c->nt}; }

// rc_compute_forces on given scratch: part (per-block FP64 rows, kEvWords
// doubles per wavefront block) when ev is wanted, ssum (N floats) for the
// two-pass form.  Launches only; allocates nothing.
int forces_into(rc_ctx* c, const float* pos, const int* nlist, const int* nn, int k_max, int N, rc_box box,
                float* force, double* ev, unsigned flags, int* status, double* part, float* ssum, hipStream_t s) {
    if (!nlist || !nn || !force) return fail(c, RC_ERR_ARG, "nlist / nn / force are NULL");
    if (flags & ~(RC_FORCE_ACCUMULATE | RC_FORCE_GATHER | RC_FORCE_SUMS))
        return fail(c, RC_ERR_ARG, "unknown flags");
    Box b;
    int r;
    if ((r = make_box(c, box, b))) return r;
    if ((r = check_list(c, nlist, nn, k_max))) return r;
    const bool sums = flags & RC_FORCE_SUMS;
    const bool gather = (flags & RC_FORCE_GATHER) || sums;
    const int nb = nblocks(N, kWave);
    ForceArgs a{};
    a.pos = reinterpret_cast<const float4*>(pos);
    a.nlist = nlist;
    a.nn = nn;
    a.k_max = k_max;
    a.N = N;
    a.tab = dev_table(c);
    a.box = b;
    a.force = reinterpret_cast<float4*>(force);
    a.ev_part = ev ? part : nullptr;
    a.accumulate = (flags & RC_FORCE_ACCUMULATE) ? 1 : 0;
    a.status = status;
    a.ssum = sums ? ssum : nullptr;
    HIP_TRY(c, gather ? launch_forces_gather(a, s) : launch_forces_triplet(a, s));
    if (ev) HIP_TRY(c, launch_reduce_rows(part, nb, 0, 7, ev, s));
    return RC_OK;
}

}  // namespace

// ============================================================================
extern "C" {

int rc_version(void) { return 10000; }

const char* rc_last_error(const rc_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

int rc_create(rc_ctx** out, int ntypes, const rc_pair_coeff* table, double r_buff) {
    if (!out) return RC_ERR_ARG;
    *out = nullptr;
    if (ntypes < 1 || !table) return RC_ERR_ARG;
    if (ntypes > RC_MAX_TYPES) return RC_ERR_UNSUPPORTED;
    if (!(r_buff > 0.0) || !std::isfinite(r_buff)) return RC_ERR_ARG;
    rc_ctx* c = new (std::nothrow) rc_ctx();
    if (!c) return RC_ERR_ARG;
    c->nt = ntypes;
    c->r_buff = r_buff;
    c->table.assign(table, table + ntypes * ntypes);
    c->host_tab.resize(ntypes * ntypes);
    if (compile_table(ntypes, table, r_buff, c->host_tab.data(), &c->rlist_max, nullptr) != RC_OK) {
        delete c;
        return RC_ERR_ARG;
    }
    if (hipGetDevice(&c->device) != hipSuccess ||
        hipMalloc(&c->d_tab, sizeof(DevEntry) * ntypes * ntypes) != hipSuccess ||
        hipMemcpy(c->d_tab, c->host_tab.data(), sizeof(DevEntry) * ntypes * ntypes,
                  hipMemcpyHostToDevice) != hipSuccess ||
        hipMalloc(&c->d_step_base, sizeof(unsigned long long)) != hipSuccess ||
        hipMalloc(&c->d_slices, sizeof(double) * kRowSlices) != hipSuccess ||
        noalloc_scratch_here(c->device, &c->noalloc_scratch) != hipSuccess ||
        // the private stream the driver's rebuild graphs are recorded on: created here, as creating a
        // stream takes milliseconds (3-5 ms measured), which a run recording its first graph would pay
        hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking) != hipSuccess) {
        if (c->d_tab) (void)hipFree(c->d_tab);
        if (c->d_step_base) (void)hipFree(c->d_step_base);
        if (c->d_slices) (void)hipFree(c->d_slices);
        delete c;
        return RC_ERR_HIP;
    }
    *out = c;
    return RC_OK;
}

int rc_destroy(rc_ctx* c) {
    if (!c) return RC_ERR_ARG;
    free_ctx_buffers(c);
    delete c;
    return RC_OK;
}

int rc_set_lambda(rc_ctx* c, const double* lambda) {
    if (c) c->md.valid = false;   // a replay into the last run's steps would use other forces
    if (!c || !lambda) return RC_ERR_ARG;
    const int nt = c->nt;
    for (int a = 0; a < nt; ++a)
        for (int b = 0; b < nt; ++b)
            if (lambda[a * nt + b] != lambda[b * nt + a] || !(lambda[a * nt + b] >= 0.0))
                return fail(c, RC_ERR_ARG, "lambda table must be symmetric and >= 0");
    for (int q = 0; q < nt * nt; ++q) {
        rc_pair_coeff& p = c->table[q];
        if (p.kind != RC_KIND_SWAP) continue;
        p.lambda = lambda[q];
        c->host_tab[q].sqrt_lam = (float)std::sqrt(p.lambda * p.epsilon);
        c->host_tab[q].lam = (float)p.lambda;
    }
    HIP_TRY(c, hipDeviceSynchronize());
    HIP_TRY(c, hipMemcpy(c->d_tab, c->host_tab.data(), sizeof(DevEntry) * nt * nt, hipMemcpyHostToDevice));
    drop_graphs(c);
    return RC_OK;
}

int rc_soft_bonds(rc_ctx* c, const float* pos, const int* nlist, const int* nn, int k_max, int N, rc_box box,
                  double* value, float* grad, void* stream) {
    int r = check_common(c, N, pos);
    if (r) return r;
    if (!value) return fail(c, RC_ERR_ARG, "value is NULL");
    if (grad && (reinterpret_cast<uintptr_t>(grad) & 15)) return fail(c, RC_ERR_ARG, "grad not 16-byte aligned");
    Box b;
    if ((r = make_box(c, box, b))) return r;
    if ((r = check_list(c, nlist, nn, k_max))) return r;
    if ((r = ensure_part(c, sizeof(double) * (size_t)(nblocks(N, kBlock) + 1)))) return r;
    HIP_TRY(c, launch_soft_bonds(reinterpret_cast<const float4*>(pos), nlist, nn, k_max, N, dev_table(c), b, c->d_part,
                                 value, reinterpret_cast<float4*>(grad), S(stream)));
    return RC_OK;
}

int rc_set_bonds(rc_ctx* c, const int* bonds, const int* rtag, int N, double K, double R0) {
    if (c) c->md.valid = false;   // a replay into the last run's steps would use other forces
    if (!c) return RC_ERR_ARG;
    if (!bonds) {
        c->bonds = nullptr;
        c->bonds_rtag = nullptr;
        c->bonds_n = 0;
        drop_graphs(c);
        return RC_OK;
    }
    if (!rtag || N < 1 || N >= RC_MAX_TAG) return fail(c, RC_ERR_ARG, "rc_set_bonds: rtag NULL or bad N");
    if (reinterpret_cast<uintptr_t>(bonds) & 7) return fail(c, RC_ERR_ARG, "bond table not 8-byte aligned");
    if (!(K > 0.0) || !(R0 > 0.0) || !std::isfinite(K) || !std::isfinite(R0))
        return fail(c, RC_ERR_ARG, "FENE needs K > 0 and R0 > 0");
    c->bonds = bonds;
    c->bonds_rtag = rtag;
    c->bonds_n = N;
    c->fene_k = K;
    c->fene_r0 = R0;
    drop_graphs(c);
    return RC_OK;
}

int rc_fene_forces(rc_ctx* c, const float* pos, int N, rc_box box, float* force, double* ev, void* stream) {
    int r = check_common(c, N, pos);
    if (r) return r;
    if (!force) return fail(c, RC_ERR_ARG, "force is NULL");
    if (!c->bonds || c->bonds_n != N) return fail(c, RC_ERR_ARG, "no bond table for %d particles (rc_set_bonds)", N);
    Box b;
    if ((r = make_box(c, box, b))) return r;
    const int nb = nblocks(N, kWave);
    if (ev && (r = ensure_part(c, sizeof(double) * kEvWords * (size_t)nb))) return r;
    HIP_TRY(c, launch_fene(reinterpret_cast<const float4*>(pos), reinterpret_cast<const int2*>(c->bonds), c->bonds_rtag,
                           N, b, (float)c->fene_k, (float)(c->fene_r0 * c->fene_r0), reinterpret_cast<float4*>(force),
                           ev ? c->d_part : nullptr, S(stream)));
    if (ev && (r = reduce_rows(c, nb, 0, 7, ev, S(stream)))) return r;
    return RC_OK;
}

int rc_set_table(rc_ctx* c, const rc_pair_coeff* table) {
    if (c) c->md.valid = false;   // a replay into the last run's steps would use other forces
    if (!c || !table) return RC_ERR_ARG;
    const int nt = c->nt;
    for (int q = 0; q < nt * nt; ++q) {
        const rc_pair_coeff& o = c->table[q];
        if (table[q].kind != o.kind || table[q].n != o.n || table[q].r_cut != o.r_cut)
            return fail(c, RC_ERR_ARG, "rc_set_table: entry %d changes kind, n or r_cut", q);
    }
    std::vector<DevEntry> tab(nt * nt);
    double rl = 0.0;
    std::string why;
    if (compile_table(nt, table, c->r_buff, tab.data(), &rl, &why) != RC_OK)
        return fail(c, RC_ERR_ARG, "rc_set_table: %s", why.c_str());
    HIP_TRY(c, hipDeviceSynchronize());
    HIP_TRY(c, hipMemcpy(c->d_tab, tab.data(), sizeof(DevEntry) * nt * nt, hipMemcpyHostToDevice));
    c->table.assign(table, table + nt * nt);
    c->host_tab = tab;
    drop_graphs(c);
    return RC_OK;
}

int rc_workspace_bytes(const rc_ctx* c, int N, int k_max, int nvec, size_t* bytes) {
    if (!c || !bytes || N < 1 || k_max < 1 || k_max > 512 || nvec < 0) return RC_ERR_ARG;
    *bytes = ws_layout(plist_entries(N, k_max), (size_t)N, (size_t)N * (size_t)nvec).total;
    return RC_OK;
}

int rc_set_workspace(rc_ctx* c, void* ws, size_t bytes, int N, int k_max, int nvec) {
    if (!c) return RC_ERR_ARG;
    return set_workspace(c, ws, bytes, N, k_max, nvec);
}

int rc_ctx_device_bytes(const rc_ctx* c, size_t* bytes) {
    if (!c || !bytes) return RC_ERR_ARG;
    *bytes = ctx_device_bytes(c);
    return RC_OK;
}

int rc_set_gather_width(rc_ctx* c, int width) {
    if (!c) return RC_ERR_ARG;
    if (width != 1 && width != 2 && width != 4) return fail(c, RC_ERR_ARG, "gather width must be 1, 2 or 4");
    c->gather_width = width;
    return RC_OK;
}

int rc_set_step_form(rc_ctx* c, int form) {
    if (!c) return RC_ERR_ARG;
    if (form != RC_FORM_WALK && form != RC_FORM_SUMS)
        return fail(c, RC_ERR_ARG, "unknown step form %d", form);
    c->step_form = form;
    return RC_OK;
}

int rc_get_rlist(const rc_ctx* c, int a, int b, double* r_list) {
    if (!c || !r_list || a < 0 || b < 0 || a >= c->nt || b >= c->nt) return RC_ERR_ARG;
    const rc_pair_coeff& p = c->table[a * c->nt + b];
    *r_list = p.kind == RC_KIND_NONE ? 0.0 : p.r_cut + c->r_buff;
    return RC_OK;
}

int rc_clear_status(int* status, void* stream) {
    if (!status) return RC_ERR_ARG;
    return launch_zero_words(status, RC_STATUS_WORDS, S(stream)) == hipSuccess ? RC_OK : RC_ERR_HIP;
}

int rc_read_status(const int* status, int* out, void* stream) {
    if (!status || !out) return RC_ERR_ARG;
    if (hipMemcpyAsync(out, status, sizeof(int) * RC_STATUS_WORDS, hipMemcpyDeviceToHost, S(stream)) != hipSuccess)
        return RC_ERR_HIP;
    if (hipStreamSynchronize(S(stream)) != hipSuccess) return RC_ERR_HIP;
    const int f = out[RC_ST_FLAGS];
    if (f & RC_FLAG_LOST) return RC_ERR_LOST_PARTICLE;
    if (f & RC_FLAG_NONFINITE) return RC_ERR_NONFINITE;
    if (f & RC_FLAG_NLIST_OVERFLOW) return RC_ERR_NLIST_OVERFLOW;
    return RC_OK;
}

int rc_cells_workspace_bytes(const rc_ctx* cc, int N, rc_box box, size_t* bytes) {
    rc_ctx* c = const_cast<rc_ctx*>(cc);
    if (!c || !bytes || N < 1) return RC_ERR_ARG;
    Box b;
    Grid g;
    int r = make_box(c, box, b);
    if (r) return r;
    if ((r = make_grid(c, c->rlist_max, b, g))) return r;
    *bytes = cells_layout(N, g.nkeys).total;
    return RC_OK;
}

int rc_build_cells(rc_ctx* c, float* pos, float* vel, int* image, int* rtag, int N, rc_box box, void* ws,
                   size_t ws_bytes, void* stream) {
    if (c) c->md.valid = false;   // the state or the list changes outside the driver
    int r = check_common(c, N, pos);
    if (r) return r;
    Box b;
    Grid g;
    if ((r = make_box(c, box, b)) || (r = make_grid(c, c->rlist_max, b, g))) return r;
    const CellsLayout l = cells_layout(N, g.nkeys);
    if (!ws || ws_bytes < l.total) return fail(c, RC_ERR_WORKSPACE, "cells workspace needs %zu bytes", l.total);
    char* w = static_cast<char*>(ws);
    CellsArgs a{};
    a.pos = reinterpret_cast<float4*>(pos);
    a.vel = reinterpret_cast<float4*>(vel);
    a.image = reinterpret_cast<int4*>(image);
    a.rtag = rtag;
    a.N = N;
    a.box = b;
    a.g = g;
    a.counts = reinterpret_cast<int*>(w + l.counts);
    a.cell_start = reinterpret_cast<int*>(w + l.start);
    a.keys = reinterpret_cast<int*>(w + l.keys);
    a.rank = reinterpret_cast<int*>(w + l.rank);
    a.order = reinterpret_cast<int*>(w + l.order);
    a.block_sums = reinterpret_cast<int*>(w + l.bsums);
    a.tpos = reinterpret_cast<float4*>(w + l.tpos);
    a.tvel = reinterpret_cast<float4*>(w + l.tvel);
    a.timage = reinterpret_cast<int4*>(w + l.timage);
    HIP_TRY(c, launch_cells(a, S(stream)));
    return RC_OK;
}

// fresh: the status words are written whole (the driver's rebuilds), else folded into
static int build_nlist(rc_ctx* c, const float* pos, float* vel, int N, rc_box box, const void* ws, size_t ws_bytes,
                       int k_max, int* nlist, int* nn, int* status, bool fresh, void* stream) {
    if (c) c->md.valid = false;   // the state or the list changes outside the driver
    int r = check_common(c, N, pos);
    if (r) return r;
    if (k_max < 1 || k_max > 512) return fail(c, RC_ERR_ARG, "k_max must be in [1, 512]");
    if (!nlist || !nn) return fail(c, RC_ERR_ARG, "nlist / nn are NULL");
    Box b;
    Grid g;
    if ((r = make_box(c, box, b)) || (r = make_grid(c, c->rlist_max, b, g))) return r;
    const CellsLayout l = cells_layout(N, g.nkeys);
    if (!ws || ws_bytes < l.total) return fail(c, RC_ERR_WORKSPACE, "cells workspace needs %zu bytes", l.total);
    NlistArgs a{};
    a.pos = reinterpret_cast<const float4*>(pos);
    a.vel = reinterpret_cast<float4*>(vel);
    a.N = N;
    a.box = b;
    a.g = g;
    a.cell_start = reinterpret_cast<const int*>(static_cast<const char*>(ws) + l.start);
    a.tab = dev_table(c);
    a.k_max = k_max;
    a.nlist = nlist;
    a.nn = nn;
    a.status = status;
    a.fresh_status = fresh ? 1 : 0;
    a.block_max = reinterpret_cast<int*>(static_cast<char*>(const_cast<void*>(ws)) + l.bmax);
    if ((r = ensure_plist(c, N, k_max))) return r;
    a.pl_j = c->d_pl_j;  // the packed copy the fused step reads, made in the same launch
    a.pl_o = c->d_pl_o;
    HIP_TRY(c, launch_nlist(a, S(stream)));
    c->pl_nlist = nlist;
    c->pl_nn = nn;
    c->pl_k = k_max;
    c->pl_n = N;
    return RC_OK;
}

int rc_build_nlist(rc_ctx* c, const float* pos, float* vel, int N, rc_box box, const void* ws, size_t ws_bytes,
                   int k_max, int* nlist, int* nn, int* status, void* stream) {
    return build_nlist(c, pos, vel, N, box, ws, ws_bytes, k_max, nlist, nn, status, false, stream);
}

int rc_compute_forces(rc_ctx* c, const float* pos, const int* nlist, const int* nn, int k_max, int N, rc_box box,
                      float* force, double* ev, unsigned flags, int* status, void* stream) {
    int r = check_common(c, N, pos);
    if (r) return r;
    const int nb = nblocks(N, kWave);   // both force kernels run one wavefront per block
    if ((flags & RC_FORCE_SUMS) && (r = ensure_ssum(c, (size_t)N))) return r;
    if (ev && (r = ensure_part(c, sizeof(double) * kEvWords * (size_t)nb))) return r;
    return forces_into(c, pos, nlist, nn, k_max, N, box, force, ev, flags, status, c->d_part, c->d_ssum,
                       S(stream));
}

int rc_compute_forces_noalloc(rc_ctx* c, const float* pos, const int* nlist, const int* nn, int k_max, int N,
                              rc_box box, float* force, double* ev, unsigned flags, int* status, void* stream) {
    int r = check_common(c, N, pos);
    if (r) return r;
    if (N > RC_NOALLOC_MAX_N)
        return fail(c, RC_ERR_UNSUPPORTED,
                    "rc_compute_forces_noalloc: N = %d exceeds the fixed scratch's limit of %d particles", N,
                    RC_NOALLOC_MAX_N);
    if (!c->noalloc_scratch)
        return fail(c, RC_ERR_UNSUPPORTED, "rc_compute_forces_noalloc: no fixed scratch on device %d", c->device);
    char* base = static_cast<char*>(c->noalloc_scratch);
    double* rows = reinterpret_cast<double*>(base);
    float* sums = reinterpret_cast<float*>(base + kNoallocRowBytes);
    return forces_into(c, pos, nlist, nn, k_max, N, box, force, ev, flags, status, rows, sums, S(stream));
}

int rc_thermostat_normals(uint64_t seed, uint64_t step0, int steps, int N, int dim, float* out, void* stream) {
    if (!out || steps < 1 || N < 1 || N >= RC_MAX_TAG || (dim != 0 && dim != 2 && dim != 3)) return RC_ERR_ARG;
    if ((long)steps * (long)N > (1L << 31)) return RC_ERR_UNSUPPORTED;
    if (reinterpret_cast<uintptr_t>(out) & 15) return RC_ERR_ARG;
    return launch_thermostat_normals(seed, step0, steps, N, dim == 2 ? 0.0f : 1.0f, reinterpret_cast<float4*>(out),
                                     S(stream)) == hipSuccess
               ? RC_OK
               : RC_ERR_HIP;
}

int rc_integrate_step(rc_ctx* c, float* pos, float* vel, const float* force, int* image, int N, rc_box box,
                      const rc_integrator* cfg, uint64_t step, int half, double* kin, int* status,
                      void* stream) {
    if (c) c->md.valid = false;   // the state or the list changes outside the driver
    int r = check_common(c, N, pos);
    if (r) return r;
    if (!vel || !force) return fail(c, RC_ERR_ARG, "vel / force are NULL");
    if (half != RC_HALF_FIRST && half != RC_HALF_SECOND) return fail(c, RC_ERR_ARG, "half must be 0 or 1");
    Box b;
    if ((r = make_box(c, box, b))) return r;
    IntegrateArgs a{};
    float c1;
    int lang;
    if ((r = check_integrator(c, cfg, a.minv, a.c2, c1, lang, a.noise_z))) return r;
    const int nb = nblocks(N, kBlock);
    if (kin && (r = ensure_part(c, sizeof(double) * kEvWords * (size_t)nb))) return r;
    a.pos = reinterpret_cast<float4*>(pos);
    a.vel = reinterpret_cast<float4*>(vel);
    a.force = reinterpret_cast<const float4*>(force);
    a.image = reinterpret_cast<int4*>(image);
    a.N = N;
    a.half = half;
    a.box = b;
    a.dt = (float)cfg->dt;
    a.c1 = c1;
    a.langevin = lang;
    a.soft = (float)(0.5 * c->r_buff);
    a.seed = cfg->seed;
    a.step = step;
    a.kin_part = kin ? c->d_part : nullptr;
    a.status = status;
    HIP_TRY(c, launch_integrate(a, S(stream)));
    if (kin && (r = reduce_rows(c, nb, 7, 6, kin, S(stream)))) return r;
    return RC_OK;
}

static int fill_step_args(rc_ctx* c, StepArgs& a, const float* pos_in, float* pos_out, float* vel, int* image,
                          const int* nlist, const int* nn, int k_max, int N, const Box& b, const rc_integrator* cfg,
                          double soft_frac, int* status, hipStream_t s, bool pack = true) {
    float c1;
    int lang;
    int r = check_integrator(c, cfg, a.minv, a.c2, c1, lang, a.noise_z);
    if (r) return r;
    if ((r = check_list(c, nlist, nn, k_max))) return r;
    a.pos_in = reinterpret_cast<const float4*>(pos_in);
    a.pos_out = reinterpret_cast<float4*>(pos_out);
    a.vel = reinterpret_cast<float4*>(vel);
    a.image = reinterpret_cast<int4*>(image);
    a.nlist = nlist;
    a.nn = nn;
    a.k_max = k_max;
    a.N = N;
    a.tab = dev_table(c);
    a.box = b;
    a.dt = (float)cfg->dt;
    a.c1 = c1;
    a.langevin = lang;
    a.hard = (float)(0.5 * c->r_buff);
    a.soft = (float)(0.5 * c->r_buff * soft_frac);
    a.seed = cfg->seed;
    a.status = status;
    a.width = c->gather_width;
    a.form = c->step_form;
    a.ssum = nullptr;
    if (a.form == RC_FORM_SUMS) {
        if ((r = ensure_ssum(c, (size_t)N))) return r;
        a.ssum = c->d_ssum;
    }
    a.bonds = nullptr;
    if (c->bonds) {
        if (c->bonds_n != N) return fail(c, RC_ERR_ARG, "bond table is for %d particles, not %d", c->bonds_n, N);
        a.bonds = reinterpret_cast<const int2*>(c->bonds);
        a.rtag = c->bonds_rtag;
        a.fene_k = (float)c->fene_k;
        a.fene_r02 = (float)(c->fene_r0 * c->fene_r0);
    }
    if ((r = ensure_blk(c, nblocks(N, kStepBlock), nullptr))) return r;
    a.blk = c->d_blk;
    // the packed copy of the list (the driver's first list build makes it: pack = false)
    if ((r = pack ? packed_list_for(c, nlist, nn, k_max, N, s) : ensure_plist(c, N, k_max))) return r;
    a.pl_j = c->d_pl_j;
    a.pl_o = c->d_pl_o;
    return RC_OK;
}

int rc_step_fused(rc_ctx* c, const float* pos_in, float* pos_out, float* vel, int* image, const int* nlist,
                  const int* nn, int k_max, int N, rc_box box, const rc_integrator* cfg, uint64_t step, int mode,
                  double soft_frac, double* ev, int* status, void* stream) {
    if (c) c->md.valid = false;   // the state or the list changes outside the driver
    int r = check_common(c, N, pos_in);
    if (r) return r;
    if (!vel || !nlist || !nn || !status) return fail(c, RC_ERR_ARG, "vel / nlist / nn / status are NULL");
    if ((mode == RC_STEP_START || mode == RC_STEP_CONT) && (!pos_out || pos_out == pos_in))
        return fail(c, RC_ERR_ARG, "pos_out must be a second buffer");
    if (mode < RC_STEP_START || mode > RC_STEP_OBSERVE) return fail(c, RC_ERR_ARG, "bad mode");
    if (!(soft_frac > 0.0 && soft_frac <= 1.0)) return fail(c, RC_ERR_ARG, "soft_frac must be in (0, 1]");
    Box b;
    if ((r = make_box(c, box, b))) return r;
    StepArgs a{};
    if ((r = fill_step_args(c, a, pos_in, pos_out, vel, image, nlist, nn, k_max, N, b, cfg, soft_frac, status,
                            S(stream))))
        return r;
    const int nb = nblocks(N, kStepBlock);
    if (ev && (r = ensure_part(c, sizeof(double) * kEvWords * (size_t)nb))) return r;
    a.mode = mode;
    a.step = step;
    a.step_base = nullptr;
    a.ev_part = ev ? c->d_part : nullptr;
    HIP_TRY(c, launch_step(a, ev != nullptr, S(stream)));
    HIP_TRY(c, launch_fold_status(c->d_blk, nb, nullptr, N, status, S(stream)));
    if (ev && (r = reduce_rows(c, nb, 0, kEvWords, ev, S(stream)))) return r;
    return RC_OK;
}

int rc_time_fused_steps(rc_ctx* c, float* pos_a, float* pos_b, float* vel, const int* nlist, const int* nn,
                        int k_max, int N, rc_box box, const rc_integrator* cfg, uint64_t step0, int reps, int* status,
                        float* ms, void* stream) {
    if (c) c->md.valid = false;   // the state or the list changes outside the driver
    int r = check_common(c, N, pos_a);
    if (r) return r;
    if (!pos_b || pos_b == pos_a || !vel || !nlist || !nn || !status || !ms || reps < 1)
        return fail(c, RC_ERR_ARG, "bad arguments to rc_time_fused_steps");
    Box b;
    if ((r = make_box(c, box, b))) return r;
    StepArgs a{};
    if ((r = fill_step_args(c, a, pos_a, pos_b, vel, nullptr, nlist, nn, k_max, N, b, cfg, 0.8, status, S(stream))))
        return r;
    a.mode = RC_STEP_CONT;
    a.step_base = nullptr;
    a.ev_part = nullptr;
    hipStream_t s = S(stream);
    // every kernel launch carries its own start/stop events, which time its
    // execution alone (not the dispatch gaps between launches)
    const void* fn;
    step_kernel_info(false, a.width, a.form, &fn);
    const void* sums_fn = nullptr;
    if (a.form == RC_FORM_SUMS) sums_kernel_info(false, &sums_fn);
    const int nk = sums_fn ? 2 : 1;
    const size_t shm = sizeof(DevEntry) * a.tab.nt * a.tab.nt;
    std::vector<hipEvent_t> ev((size_t)2 * nk * reps, nullptr);
    hipError_t err = hipSuccess;
    for (size_t q = 0; q < ev.size() && err == hipSuccess; ++q) err = hipEventCreate(&ev[q]);
    float4* P[2] = {reinterpret_cast<float4*>(pos_a), reinterpret_cast<float4*>(pos_b)};
    for (int k = 0; k < reps && err == hipSuccess; ++k) {
        a.pos_in = P[k & 1];
        a.pos_out = P[(k + 1) & 1];
        a.step = step0 + (uint64_t)k;
        hipEvent_t* e = &ev[(size_t)2 * nk * k];
        if (sums_fn) {
            ForceArgs f = step_sums_args(a);
            void* args[] = {&f};
            err = hipExtLaunchKernel(sums_fn, dim3(nblocks(N, kWave)), dim3(kWave), args, shm, s, e[0], e[1], 0);
            e += 2;
        }
        if (err == hipSuccess) {
            void* args[] = {&a};
            err = hipExtLaunchKernel(fn, dim3(nblocks(N, kStepBlock)), dim3(kStepBlock), args, shm, s, e[0], e[1], 0);
        }
    }
    if (err == hipSuccess) err = launch_fold_status(c->d_blk, nblocks(N, kStepBlock), nullptr, N, status, s);
    if (err == hipSuccess) err = hipEventSynchronize(ev.back());
    double total = 0.0;
    for (size_t q = 0; q + 1 < ev.size() && err == hipSuccess; q += 2) {
        float t = 0.f;
        err = hipEventElapsedTime(&t, ev[q], ev[q + 1]);
        total += t;
    }
    *ms = (float)total;
    for (hipEvent_t e : ev)
        if (e) (void)hipEventDestroy(e);
    if (err != hipSuccess) return hip_fail(c, err, "rc_time_fused_steps");
    return RC_OK;
}

int rc_bond_count(rc_ctx* c, const float* pos, const int* nlist, const int* nn, int k_max, int N, rc_box box,
                  unsigned long long* count, void* stream) {
    int r = check_common(c, N, pos);
    if (r) return r;
    if (!nlist || !nn || !count) return fail(c, RC_ERR_ARG, "nlist / nn / count are NULL");
    Box b;
    if ((r = make_box(c, box, b))) return r;
    if ((r = ensure_part(c, sizeof(unsigned long long) * (size_t)(nblocks(N, kBlock) + 1)))) return r;
    if ((r = check_list(c, nlist, nn, k_max))) return r;
    HIP_TRY(c, launch_bonds(reinterpret_cast<const float4*>(pos), nlist, nn, k_max, N, dev_table(c), b, count,
                            reinterpret_cast<unsigned long long*>(c->d_part), S(stream)));
    return RC_OK;
}

int rc_bond_partners(rc_ctx* c, const float* pos, const int* nlist, const int* nn, int k_max, int N, rc_box box,
                     int* partner, void* stream) {
    int r = check_common(c, N, pos);
    if (r) return r;
    if (!nlist || !nn || !partner) return fail(c, RC_ERR_ARG, "nlist / nn / partner are NULL");
    if (N > RC_MAX_TAG) return fail(c, RC_ERR_ARG, "too many particles for tag-indexed output");
    Box b;
    if ((r = make_box(c, box, b))) return r;
    if ((r = check_list(c, nlist, nn, k_max))) return r;
    HIP_TRY(c, launch_bond_partners(reinterpret_cast<const float4*>(pos), nlist, nn, k_max, N, dev_table(c), b,
                                    partner, S(stream)));
    return RC_OK;
}

int rc_partner_counts(rc_ctx* c, const int* p0, const int* pt, const unsigned char* select, int N,
                      unsigned long long* counts, void* stream) {
    if (!c) return RC_ERR_ARG;
    if (!p0 || !pt || !counts) return fail(c, RC_ERR_ARG, "p0 / pt / counts are NULL");
    if (N < 1 || N > RC_MAX_TAG) return fail(c, RC_ERR_ARG, "N = %d outside [1, %d]", N, RC_MAX_TAG);
    const int nb = (N + kBlock - 1) / kBlock;
    int r = ensure_part(c, sizeof(unsigned long long) * 3 * (size_t)nb);
    if (r) return r;
    HIP_TRY(c, launch_partner_counts(p0, pt, select, N, reinterpret_cast<unsigned long long*>(c->d_part), counts,
                                     S(stream)));
    return RC_OK;
}

int rc_stress_autocorrelation(rc_ctx* c, const double* rows, int T, double volume, double kT, int max_lag,
                              double* G, void* stream) {
    if (!c) return RC_ERR_ARG;
    if (!rows || !G) return fail(c, RC_ERR_ARG, "rows / G are NULL");
    if (T < 1 || max_lag < 0 || max_lag >= T)
        return fail(c, RC_ERR_ARG, "need 0 <= max_lag < T (T = %d, max_lag = %d)", T, max_lag);
    if (!(volume > 0.0) || !(kT > 0.0)) return fail(c, RC_ERR_ARG, "volume and kT must be > 0");
    HIP_TRY(c, launch_stress_acf(rows, T, volume, kT, max_lag, G, S(stream)));
    return RC_OK;
}

int rc_force_hvp(rc_ctx* c, const float* pos, const int* nlist, const int* nn, int k_max, int N, rc_box box, const float* v,
                 float* hv, void* stream) {
    return rc_force_hvp_batch(c, pos, nlist, nn, k_max, N, box, 1, v, hv, stream);
}

int rc_force_hvp_batch(rc_ctx* c, const float* pos, const int* nlist, const int* nn, int k_max, int N, rc_box box,
                       int nvec, const float* v, float* hv, void* stream) {
    int r = check_common(c, N, pos);
    if (r) return r;
    if (!nlist || !nn || !v || !hv) return fail(c, RC_ERR_ARG, "nlist / nn / v / hv are NULL");
    if (nvec < 1 || nvec > 65535) return fail(c, RC_ERR_ARG, "nvec = %d outside [1, 65535]", nvec);
    if ((reinterpret_cast<uintptr_t>(v) | reinterpret_cast<uintptr_t>(hv)) & 15)
        return fail(c, RC_ERR_ARG, "v / hv not 16-byte aligned");
    Box b;
    if ((r = make_box(c, box, b))) return r;
    if ((r = check_list(c, nlist, nn, k_max))) return r;
    HvpArgs a{};
    a.pos = reinterpret_cast<const float4*>(pos);
    a.nlist = nlist;
    a.nn = nn;
    a.k_max = k_max;
    a.N = N;
    a.tab = dev_table(c);
    a.box = b;
    a.v = reinterpret_cast<const float4*>(v);
    a.hv = reinterpret_cast<float4*>(hv);
    a.nvec = nvec;
    if ((r = ensure_hsum(c, (size_t)N * (size_t)nvec))) return r;
    a.sums = reinterpret_cast<double2*>(c->d_hsum);
    HIP_TRY(c, launch_hvp(a, S(stream)));
    return RC_OK;
}

int rc_param_grad(rc_ctx* c, const float* pos, const int* nlist, const int* nn, int k_max, int N, rc_box box, double* grad,
                  void* stream) {
    int r = check_common(c, N, pos);
    if (r) return r;
    if (!nlist || !nn || !grad) return fail(c, RC_ERR_ARG, "nlist / nn / grad are NULL");
    Box b;
    if ((r = make_box(c, box, b))) return r;
    const int nb = nblocks(N, kBlock);
    const int nv = c->nt * c->nt * 3;
    if ((r = ensure_part(c, sizeof(double) * (size_t)nv * nb))) return r;
    if ((r = check_list(c, nlist, nn, k_max))) return r;
    ParamArgs a{};
    a.pos = reinterpret_cast<const float4*>(pos);
    a.nlist = nlist;
    a.nn = nn;
    a.k_max = k_max;
    a.N = N;
    a.tab = dev_table(c);
    a.box = b;
    a.adj = nullptr;
    a.part = c->d_part;
    HIP_TRY(c, launch_param(a, S(stream)));
    HIP_TRY(c, launch_reduce_param(c->d_part, nb, c->nt, grad, S(stream)));
    return RC_OK;
}

int rc_param_vjp(rc_ctx* c, const float* pos, const int* nlist, const int* nn, int k_max, int N, rc_box box,
                 const float* adj, double* out, void* stream) {
    int r = check_common(c, N, pos);
    if (r) return r;
    if (!nlist || !nn || !adj || !out) return fail(c, RC_ERR_ARG, "nlist / nn / adj / out are NULL");
    if (reinterpret_cast<uintptr_t>(adj) & 15) return fail(c, RC_ERR_ARG, "adj not 16-byte aligned");
    Box b;
    if ((r = make_box(c, box, b))) return r;
    const int nb = nblocks(N, kBlock);
    const int nv = c->nt * c->nt * 3;
    if ((r = ensure_part(c, sizeof(double) * (size_t)nv * nb))) return r;
    if ((r = check_list(c, nlist, nn, k_max))) return r;
    ParamArgs a{};
    a.pos = reinterpret_cast<const float4*>(pos);
    a.nlist = nlist;
    a.nn = nn;
    a.k_max = k_max;
    a.N = N;
    a.tab = dev_table(c);
    a.box = b;
    a.adj = reinterpret_cast<const float4*>(adj);
    a.part = c->d_part;
    HIP_TRY(c, launch_param_vjp(a, S(stream)));
    HIP_TRY(c, launch_reduce_param(c->d_part, nb, c->nt, out, S(stream)));
    return RC_OK;
}

// ============================================================================
// MD driver
// ============================================================================
namespace {

struct PlainOps final : DriveOps {
    rc_ctx* c;
    const rc_md_buffers* buf;
    int N;
    rc_box box;
    Box b;
    hipStream_t s;
    float* rb_pos = nullptr;   // the position buffer of the rebuild in progress
    // The cell sort and the list build of one rebuild, on stream st (direct, or being recorded)
    static int rebuild_launches(void* self, hipStream_t st) {
        PlainOps* o = static_cast<PlainOps*>(self);
        int rr = rc_build_cells(o->c, o->rb_pos, o->buf->vel, o->buf->image, o->buf->rtag, o->N, o->box,
                                o->buf->cells_ws, o->buf->cells_ws_bytes, st);
        if (rr) return rr;
        return build_nlist(o->c, o->rb_pos, o->buf->vel, o->N, o->box, o->buf->cells_ws, o->buf->cells_ws_bytes,
                           o->buf->k_max, o->buf->nlist, o->buf->nn, o->buf->status, true, st);
    }
    // Every rebuild of a run takes the same launches with the same arguments (for its position buffer),
    // so from the second one on they are replayed as one graph: the host no longer issues a dozen
    // launches while the device waits between them.
    int rebuild(float* pos, RebuildKind, float* kept_path, int64_t* rebuilt) override {
        *kept_path = 0.0f;   // every list is rebuilt
        *rebuilt = N;
        rb_pos = pos;
        if (c->ws_user == nullptr) return rebuild_launches(this, s);   // the context may still (re)allocate
        RebuildKey k;
        std::memset(&k, 0, sizeof k);
        k.pos = pos;
        k.vel = buf->vel;
        k.image = buf->image;
        k.rtag = buf->rtag;
        k.ws = buf->cells_ws;
        k.ws_bytes = buf->cells_ws_bytes;
        k.nlist = buf->nlist;
        k.nn = buf->nn;
        k.status = buf->status;
        k.pl_j = c->d_pl_j;
        k.pl_o = c->d_pl_o;
        k.tab = c->d_tab;
        k.N = N;
        k.k_max = buf->k_max;
        for (int d = 0; d < 3; ++d) k.L[d] = box.L[d];
        k.rlist_max = c->rlist_max;
        const int rr = rebuild_graphed(c, pos == buf->pos ? 0 : 1, k, &PlainOps::rebuild_launches, this, s);
        if (rr) return rr;
        // a replay skips the list build's host bookkeeping: the packed list is this list's
        c->pl_nlist = buf->nlist;
        c->pl_nn = buf->nn;
        c->pl_k = buf->k_max;
        c->pl_n = N;
        return RC_OK;
    }
    // With both logs, a row's bond count comes from the ev step that follows the bond request (the
    // driver launches one on the same positions for every row): its gather counts the bonds per block,
    // and the row's reduction sums them, instead of a list walk and a sum of their own.
    bool fused_bonds() const { return buf->ev_log != nullptr && buf->bonds_log != nullptr; }
    unsigned* bond_part() const {
        return reinterpret_cast<unsigned*>(c->d_part + (size_t)kEvWords * nblocks(N, kStepBlock));
    }
    int bonds(const float* pos, int row) override {
        if (fused_bonds()) return RC_OK;
        HIP_TRY(c, launch_bonds(reinterpret_cast<const float4*>(pos), buf->nlist, buf->nn, buf->k_max, N,
                                dev_table(c), b, buf->bonds_log + row, reinterpret_cast<unsigned long long*>(c->d_part),
                                s));
        return RC_OK;
    }
    hipError_t launch(const StepArgs& a, bool ev) override {
        if (!ev || !fused_bonds()) return launch_step(a, ev, s);
        StepArgs e = a;
        e.bond_part = bond_part();
        return launch_step(e, ev, s);
    }
    hipError_t launch_timed(const StepArgs& a, hipEvent_t* sums, hipEvent_t* step) override {
        return launch_step_timed(a, false, s, sums, step);
    }
    int reduce_ev(int row) override {
        const int nb = nblocks(N, kStepBlock);
        double* out = buf->ev_log + (size_t)row * kEvWords;
        if (!fused_bonds()) return reduce_rows(c, nb, 0, kEvWords, out, s);
        HIP_TRY(c, launch_reduce_rows(c->d_part, nb, 0, kEvWords, out, s, c->d_slices, bond_part(),
                                      buf->bonds_log + row));
        return RC_OK;
    }
    const void* graph_fn() override {
        const void* fn;
        step_kernel_info(false, c->gather_width, c->step_form, &fn);
        return fn;
    }
    const void* graph_sums_fn() override {
        if (c->step_form != RC_FORM_SUMS) return nullptr;
        const void* fn;
        sums_kernel_info(false, &fn);
        return fn;
    }
    bool block_ok() override { return step_block_fits(N, c->nt, c->step_form); }
    // the cell sort permutes pos, vel and image through the workspace's
    // temporaries and copies them back, so those hold the rebuilt state
    bool rebuild_snapshot(const float4** p, const float4** v, const int4** im) override {
        Grid g;
        if (make_grid(c, c->rlist_max, b, g)) return false;
        const CellsLayout l = cells_layout(N, g.nkeys);
        if (buf->cells_ws_bytes < l.total) return false;
        const char* w = static_cast<const char*>(buf->cells_ws);
        *p = reinterpret_cast<const float4*>(w + l.tpos);
        *v = reinterpret_cast<const float4*>(w + l.tvel);
        *im = reinterpret_cast<const int4*>(w + l.timage);
        return true;
    }
    hipError_t launch_block(const StepArgs& a, float4* pos, int G) override {
        return launch_step_block(a, pos, c->d_step_base, G, s);
    }
};

}  // namespace

int rc_md_run(rc_ctx* c, const rc_md_buffers* buf, int N, rc_box box, const rc_integrator* cfg, uint64_t step0,
              int n_steps, const rc_md_options* opt_in, rc_md_stats* stats, void* stream) {
    int r = check_common(c, N, buf ? buf->pos : nullptr);
    if (r) return r;
    if (!buf->pos_alt || !buf->vel || !buf->nlist || !buf->nn || !buf->cells_ws || !buf->status)
        return fail(c, RC_ERR_ARG, "md buffers incomplete");
    if (buf->k_max < 1 || buf->k_max > 512) return fail(c, RC_ERR_ARG, "k_max must be in [1, 512]");
    if (n_steps < 0) return fail(c, RC_ERR_ARG, "n_steps < 0");
    if (c->bonds && buf->rtag != c->bonds_rtag)
        return fail(c, RC_ERR_ARG, "with bonds, the md buffers' rtag must be the one given to rc_set_bonds");
    rc_md_options opt{1, 16, 256, 0, 0.8, 1, 1, 0, 1, 0};
    if (opt_in) opt = *opt_in;
    if (opt.graph_steps < 2 || (opt.graph_steps & 1)) opt.graph_steps = 16;
    if (opt.max_chunk < 1) opt.max_chunk = 256;
    if (!(opt.soft_frac > 0.0 && opt.soft_frac <= 1.0)) opt.soft_frac = 0.8;
    Box b;
    if ((r = make_box(c, box, b))) return r;
    hipStream_t s = S(stream);
    const int nb = nblocks(N, kStepBlock);
    // the ev steps' rows, then their per-block bond counts (PlainOps::bond_part)
    if ((r = ensure_part(c, (sizeof(double) * kEvWords + sizeof(unsigned)) * (size_t)nb))) return r;
    StepArgs tmpl{};
    if ((r = fill_step_args(c, tmpl, buf->pos, buf->pos_alt, buf->vel, buf->image, buf->nlist, buf->nn, buf->k_max, N,
                            b, cfg, opt.soft_frac, buf->status, s, false)))
        return r;
    PlainOps ops;
    ops.c = c;
    ops.buf = buf;
    ops.N = N;
    ops.box = box;
    ops.b = b;
    ops.s = s;
    return md_drive(c, ops, buf, N, tmpl, step0, n_steps, opt, stats, s);
}

}  // extern "C"
