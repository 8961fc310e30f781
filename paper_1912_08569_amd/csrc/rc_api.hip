// C ABI of the swap-potential engine: validation, table compilation,
// workspace layout, launches and the chunked MD driver.
#include <algorithm>
#include <cstdarg>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "rc_internal.h"

using namespace rc;

struct GraphCache {
    hipGraphExec_t exec[2] = {nullptr, nullptr};  // start parity 0 / 1
    hipGraph_t graph[2] = {nullptr, nullptr};
    StepArgs key{};
    int steps = 0;
    bool valid = false;
};

struct rc_ctx {
    int device = 0;
    int nt = 0;
    std::vector<rc_pair_coeff> table;
    double r_buff = 0.0;
    double rlist_max = 0.0;
    std::vector<DevEntry> host_tab;
    DevEntry* d_tab = nullptr;
    double* d_part = nullptr;        // block partial rows (13 doubles each) or param partials
    size_t part_bytes = 0;
    unsigned long long* d_step_base = nullptr;
    int* d_blk = nullptr;            // per-block status slots of the step kernel
    int blk_cap = 0;                 // slots allocated (blocks)
    GraphCache gc;
    std::string err;
};

namespace {

int fail(rc_ctx* c, int code, const char* fmt, ...) __attribute__((format(printf, 3, 4)));
int fail(rc_ctx* c, int code, const char* fmt, ...) {
    if (c) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        c->err = buf;
    }
    return code;
}

int hip_fail(rc_ctx* c, hipError_t e, const char* where) {
    return fail(c, RC_ERR_HIP, "%s: %s", where, hipGetErrorString(e));
}

#define HIP_TRY(ctx, expr)                                              \
    do {                                                                \
        hipError_t _e = (expr);                                         \
        if (_e != hipSuccess) return hip_fail((ctx), _e, #expr);        \
    } while (0)

inline hipStream_t S(void* s) { return reinterpret_cast<hipStream_t>(s); }
inline int nblocks(long n, int b) { return (int)((n + b - 1) / b); }

bool fp32_exact(double x) { return (double)(float)x == x; }

int make_box(rc_ctx* c, const rc_box& in, Box& b) {
    for (int d = 0; d < 3; ++d) {
        const double L = in.L[d];
        if (!(L > 0.0) || !std::isfinite(L)) return fail(c, RC_ERR_ARG, "box edge %d is not positive", d);
        if (!fp32_exact(L)) return fail(c, RC_ERR_ARG, "box edge %d = %.17g is not an FP32 value", d, L);
        b.L[d] = L;
        b.h[d] = 0.5 * L;
        b.Lf[d] = (float)L;
        b.hf[d] = (float)(0.5 * L);
    }
    return RC_OK;
}

int make_grid(rc_ctx* c, const Box& b, Grid& g) {
    int maxnc = 0;
    for (int d = 0; d < 3; ++d) {
        if (b.L[d] < 3.0 * c->rlist_max)
            return fail(c, RC_ERR_ARG, "box edge %.6g shorter than three list radii (%.6g)", b.L[d],
                        3.0 * c->rlist_max);
        int nc = (int)std::floor(b.L[d] / (c->rlist_max * (1.0 + 1e-5)));
        nc = std::max(3, std::min(nc, 256));
        g.nc[d] = nc;
        g.inv_w[d] = (float)(nc / b.L[d]);
        maxnc = std::max(maxnc, nc);
    }
    int bits = 0;
    while ((1 << bits) < maxnc) ++bits;
    g.bits = bits;
    g.nkeys = 1u << (3 * bits);
    return RC_OK;
}

struct CellsLayout {
    size_t counts, start, keys, rank, order, bsums, bmax, tpos, tvel, timage, total;
};

CellsLayout cells_layout(int N, const Grid& g) {
    auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
    CellsLayout l{};
    size_t o = 0;
    const size_t nk = g.nkeys;
    l.counts = o; o = al(o + 4 * nk);
    l.start = o; o = al(o + 4 * (nk + 1));
    l.keys = o; o = al(o + 4 * (size_t)N);
    l.rank = o; o = al(o + 4 * (size_t)N);
    l.order = o; o = al(o + 4 * (size_t)N);
    l.bsums = o; o = al(o + 4 * (nk / kScanTile + 2));
    l.bmax = o; o = al(o + 4 * ((size_t)N / kBlock + 2));
    l.tpos = o; o = al(o + 16 * (size_t)N);
    l.tvel = o; o = al(o + 16 * (size_t)N);
    l.timage = o; o = al(o + 16 * (size_t)N);
    l.total = o;
    return l;
}

int ensure_part(rc_ctx* c, size_t bytes) {
    if (c->part_bytes >= bytes) return RC_OK;
    if (c->d_part) (void)hipFree(c->d_part);
    c->d_part = nullptr;
    c->part_bytes = 0;
    size_t want = std::max(bytes, (size_t)1 << 20);
    HIP_TRY(c, hipMalloc(&c->d_part, want));
    c->part_bytes = want;
    return RC_OK;
}

Table dev_table(const rc_ctx* c) { return Table{c->d_tab, c->nt}; }

void drop_graphs_ns(rc_ctx* c);

// per-block status slots for nb blocks (allocated once per size, reset to neutral)
int ensure_blk(rc_ctx* c, int nb, hipStream_t s) {
    if (c->blk_cap >= nb) return RC_OK;
    drop_graphs_ns(c);   // graphs hold the old pointer
    HIP_TRY(c, hipDeviceSynchronize());
    if (c->d_blk) (void)hipFree(c->d_blk);
    c->d_blk = nullptr;
    c->blk_cap = 0;
    const int want = std::max(nb, 1024);
    HIP_TRY(c, hipMalloc(&c->d_blk, sizeof(int) * 3 * (size_t)want));
    HIP_TRY(c, launch_blk_reset(c->d_blk, want, s));
    c->blk_cap = want;
    return RC_OK;
}

int check_integrator(rc_ctx* c, const rc_integrator* cfg, float* minv, float* c2, float& c1, int& langevin) {
    if (!cfg) return fail(c, RC_ERR_ARG, "integrator is NULL");
    if (cfg->kind != RC_INTEGRATOR_NVE && cfg->kind != RC_INTEGRATOR_LANGEVIN)
        return fail(c, RC_ERR_ARG, "unknown integrator kind %d", cfg->kind);
    if (!(cfg->dt > 0.0) || !std::isfinite(cfg->dt)) return fail(c, RC_ERR_ARG, "dt must be positive");
    langevin = cfg->kind == RC_INTEGRATOR_LANGEVIN;
    if (langevin && (!(cfg->gamma >= 0.0) || !(cfg->kT >= 0.0)))
        return fail(c, RC_ERR_ARG, "Langevin needs gamma >= 0 and kT >= 0");
    const double e1 = langevin ? std::exp(-cfg->gamma * cfg->dt) : 1.0;
    c1 = (float)e1;
    for (int t = 0; t < RC_MAX_TYPES; ++t) {
        minv[t] = 0.0f;
        c2[t] = 0.0f;
    }
    for (int t = 0; t < c->nt; ++t) {
        const double m = cfg->mass[t];
        if (!(m > 0.0) || !std::isfinite(m)) return fail(c, RC_ERR_ARG, "mass of type %d must be positive", t);
        minv[t] = (float)(1.0 / m);
        c2[t] = langevin ? (float)std::sqrt((1.0 - e1 * e1) * cfg->kT / m) : 0.0f;
    }
    return RC_OK;
}

int check_common(rc_ctx* c, int N, const void* pos) {
    if (!c) return RC_ERR_ARG;
    if (N < 1) return fail(c, RC_ERR_ARG, "N must be >= 1 (got %d)", N);
    if (N >= RC_MAX_TAG) return fail(c, RC_ERR_UNSUPPORTED, "N must be < 2^27");
    if (!pos) return fail(c, RC_ERR_ARG, "positions are NULL");
    if (reinterpret_cast<uintptr_t>(pos) & 15) return fail(c, RC_ERR_ARG, "positions not 16-byte aligned");
    return RC_OK;
}

int check_list(rc_ctx* c, const int* nlist, const int* nn, int k_max) {
    if (!nlist || !nn) return fail(c, RC_ERR_ARG, "nlist / nn are NULL");
    if (k_max < 1 || k_max > 512) return fail(c, RC_ERR_ARG, "k_max must be in [1, 512]");
    return RC_OK;
}

int reduce_rows(rc_ctx* c, int nb, int first, int count, double* out, hipStream_t s) {
    HIP_TRY(c, launch_reduce_rows(c->d_part, nb, first, count, out, s));
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
    double rmax = 0.0;
    for (int a = 0; a < ntypes; ++a) {
        for (int b = 0; b < ntypes; ++b) {
            const rc_pair_coeff& p = table[a * ntypes + b];
            const rc_pair_coeff& q = table[b * ntypes + a];
            if (p.kind != q.kind || p.n != q.n || p.epsilon != q.epsilon || p.sigma != q.sigma ||
                p.r_cut != q.r_cut || (p.kind == RC_KIND_SWAP && p.lambda != q.lambda)) {
                delete c;
                return RC_ERR_ARG;
            }
            DevEntry e{};
            e.kind = p.kind;
            if (p.kind == RC_KIND_SWAP) {
                const double rmin = p.sigma * std::pow(2.0, 1.0 / p.n);
                if (!(p.epsilon > 0.0) || !(p.sigma > 0.0) || p.n < 1 || p.n > 200 || !(p.lambda >= 0.0) ||
                    !(p.r_cut > rmin) || !std::isfinite(p.r_cut)) {
                    delete c;
                    return RC_ERR_ARG;
                }
                e.n = p.n;
                e.sqrt_lam = (float)std::sqrt(p.lambda * p.epsilon);
                e.inv_eps = (float)(1.0 / p.epsilon);
                e.lam = (float)p.lambda;
            } else if (p.kind == RC_KIND_WCA) {
                if (!(p.epsilon >= 0.0) || !(p.sigma > 0.0) || !(p.r_cut > 0.0) || !std::isfinite(p.r_cut)) {
                    delete c;
                    return RC_ERR_ARG;
                }
                e.n = 6;
            } else if (p.kind != RC_KIND_NONE) {
                delete c;
                return RC_ERR_ARG;
            }
            if (p.kind != RC_KIND_NONE) {
                e.eps = (float)p.epsilon;
                e.sigma = (float)p.sigma;
                e.sig2 = (float)(p.sigma * p.sigma);
                e.rcut2 = p.r_cut * p.r_cut;
                e.rmin2 = (p.sigma * p.sigma) * std::pow(2.0, 2.0 / (double)(p.kind == RC_KIND_SWAP ? p.n : 6));
                const double rl = p.r_cut + r_buff;
                e.rlist2 = (float)(rl * rl * (1.0 + 1e-5));
                rmax = std::max(rmax, rl);
            }
            c->host_tab[a * ntypes + b] = e;
        }
    }
    if (rmax == 0.0) rmax = r_buff;
    c->rlist_max = rmax;
    if (hipGetDevice(&c->device) != hipSuccess ||
        hipMalloc(&c->d_tab, sizeof(DevEntry) * ntypes * ntypes) != hipSuccess ||
        hipMemcpy(c->d_tab, c->host_tab.data(), sizeof(DevEntry) * ntypes * ntypes,
                  hipMemcpyHostToDevice) != hipSuccess ||
        hipMalloc(&c->d_step_base, sizeof(unsigned long long)) != hipSuccess) {
        if (c->d_tab) (void)hipFree(c->d_tab);
        delete c;
        return RC_ERR_HIP;
    }
    *out = c;
    return RC_OK;
}

static void drop_graphs(rc_ctx* c);
namespace {
void drop_graphs_ns(rc_ctx* c) { drop_graphs(c); }
}
static void drop_graphs(rc_ctx* c) {
    for (int p = 0; p < 2; ++p) {
        if (c->gc.exec[p]) (void)hipGraphExecDestroy(c->gc.exec[p]);
        if (c->gc.graph[p]) (void)hipGraphDestroy(c->gc.graph[p]);
        c->gc.exec[p] = nullptr;
        c->gc.graph[p] = nullptr;
    }
    c->gc.valid = false;
}

int rc_destroy(rc_ctx* c) {
    if (!c) return RC_ERR_ARG;
    drop_graphs(c);
    if (c->d_tab) (void)hipFree(c->d_tab);
    if (c->d_part) (void)hipFree(c->d_part);
    if (c->d_step_base) (void)hipFree(c->d_step_base);
    if (c->d_blk) (void)hipFree(c->d_blk);
    delete c;
    return RC_OK;
}

int rc_set_lambda(rc_ctx* c, const double* lambda) {
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
    if ((r = make_grid(c, b, g))) return r;
    *bytes = cells_layout(N, g).total;
    return RC_OK;
}

int rc_build_cells(rc_ctx* c, float* pos, float* vel, int* image, int* rtag, int N, rc_box box, void* ws,
                   size_t ws_bytes, void* stream) {
    int r = check_common(c, N, pos);
    if (r) return r;
    Box b;
    Grid g;
    if ((r = make_box(c, box, b)) || (r = make_grid(c, b, g))) return r;
    const CellsLayout l = cells_layout(N, g);
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

int rc_build_nlist(rc_ctx* c, const float* pos, float* vel, int N, rc_box box, const void* ws, size_t ws_bytes,
                   int k_max, int* nlist, int* nn, int* status, void* stream) {
    int r = check_common(c, N, pos);
    if (r) return r;
    if (k_max < 1 || k_max > 512) return fail(c, RC_ERR_ARG, "k_max must be in [1, 512]");
    if (!nlist || !nn) return fail(c, RC_ERR_ARG, "nlist / nn are NULL");
    Box b;
    Grid g;
    if ((r = make_box(c, box, b)) || (r = make_grid(c, b, g))) return r;
    const CellsLayout l = cells_layout(N, g);
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
    a.block_max = reinterpret_cast<int*>(static_cast<char*>(const_cast<void*>(ws)) + l.bmax);
    HIP_TRY(c, launch_nlist(a, S(stream)));
    return RC_OK;
}

int rc_compute_forces(rc_ctx* c, const float* pos, const int* nlist, const int* nn, int k_max, int N, rc_box box,
                      float* force, double* ev, unsigned flags, int* status, void* stream) {
    int r = check_common(c, N, pos);
    if (r) return r;
    if (!nlist || !nn || !force) return fail(c, RC_ERR_ARG, "nlist / nn / force are NULL");
    if (flags & ~(RC_FORCE_ACCUMULATE | RC_FORCE_GATHER)) return fail(c, RC_ERR_ARG, "unknown flags");
    Box b;
    if ((r = make_box(c, box, b))) return r;
    const bool gather = flags & RC_FORCE_GATHER;
    const int nb = nblocks(N, kWave);   // both force kernels run one wavefront per block
    if (ev && (r = ensure_part(c, sizeof(double) * kEvWords * (size_t)nb))) return r;
    if ((r = check_list(c, nlist, nn, k_max))) return r;
    ForceArgs a{};
    a.pos = reinterpret_cast<const float4*>(pos);
    a.nlist = nlist;
    a.nn = nn;
    a.k_max = k_max;
    a.N = N;
    a.tab = dev_table(c);
    a.box = b;
    a.force = reinterpret_cast<float4*>(force);
    a.ev_part = ev ? c->d_part : nullptr;
    a.accumulate = (flags & RC_FORCE_ACCUMULATE) ? 1 : 0;
    a.status = status;
    HIP_TRY(c, gather ? launch_forces_gather(a, S(stream)) : launch_forces_triplet(a, S(stream)));
    if (ev && (r = reduce_rows(c, nb, 0, 7, ev, S(stream)))) return r;
    return RC_OK;
}

int rc_integrate_step(rc_ctx* c, float* pos, float* vel, const float* force, int* image, int N, rc_box box,
                      const rc_integrator* cfg, uint64_t step, int half, double* kin, int* status,
                      void* stream) {
    int r = check_common(c, N, pos);
    if (r) return r;
    if (!vel || !force) return fail(c, RC_ERR_ARG, "vel / force are NULL");
    if (half != RC_HALF_FIRST && half != RC_HALF_SECOND) return fail(c, RC_ERR_ARG, "half must be 0 or 1");
    Box b;
    if ((r = make_box(c, box, b))) return r;
    IntegrateArgs a{};
    float c1;
    int lang;
    if ((r = check_integrator(c, cfg, a.minv, a.c2, c1, lang))) return r;
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
                          double soft_frac, int* status) {
    float c1;
    int lang;
    int r = check_integrator(c, cfg, a.minv, a.c2, c1, lang);
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
    if ((r = ensure_blk(c, nblocks(N, kStepBlock), nullptr))) return r;
    a.blk = c->d_blk;
    return RC_OK;
}

int rc_step_fused(rc_ctx* c, const float* pos_in, float* pos_out, float* vel, int* image, const int* nlist,
                  const int* nn, int k_max, int N, rc_box box, const rc_integrator* cfg, uint64_t step, int mode,
                  double soft_frac, double* ev, int* status, void* stream) {
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
    if ((r = fill_step_args(c, a, pos_in, pos_out, vel, image, nlist, nn, k_max, N, b, cfg, soft_frac, status))) return r;
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
    int r = check_common(c, N, pos_a);
    if (r) return r;
    if (!pos_b || pos_b == pos_a || !vel || !nlist || !nn || !status || !ms || reps < 1)
        return fail(c, RC_ERR_ARG, "bad arguments to rc_time_fused_steps");
    Box b;
    if ((r = make_box(c, box, b))) return r;
    StepArgs a{};
    if ((r = fill_step_args(c, a, pos_a, pos_b, vel, nullptr, nlist, nn, k_max, N, b, cfg, 0.8, status))) return r;
    a.mode = RC_STEP_CONT;
    a.step_base = nullptr;
    a.ev_part = nullptr;
    hipStream_t s = S(stream);
    hipEvent_t e0, e1;
    HIP_TRY(c, hipEventCreate(&e0));
    HIP_TRY(c, hipEventCreate(&e1));
    float4* P[2] = {reinterpret_cast<float4*>(pos_a), reinterpret_cast<float4*>(pos_b)};
    hipError_t err = hipEventRecord(e0, s);
    for (int k = 0; k < reps && err == hipSuccess; ++k) {
        a.pos_in = P[k & 1];
        a.pos_out = P[(k + 1) & 1];
        a.step = step0 + (uint64_t)k;
        err = launch_step(a, false, s);
    }
    if (err == hipSuccess) err = hipEventRecord(e1, s);
    if (err == hipSuccess) err = launch_fold_status(c->d_blk, nblocks(N, kStepBlock), nullptr, N, status, s);
    if (err == hipSuccess) err = hipEventSynchronize(e1);
    if (err == hipSuccess) err = hipEventElapsedTime(ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
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

int rc_force_hvp(rc_ctx* c, const float* pos, const int* nlist, const int* nn, int k_max, int N, rc_box box, const float* v,
                 float* hv, void* stream) {
    int r = check_common(c, N, pos);
    if (r) return r;
    if (!nlist || !nn || !v || !hv) return fail(c, RC_ERR_ARG, "nlist / nn / v / hv are NULL");
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

int rc_param_vjp(rc_ctx* c, const float*, const int*, const int*, int, int, rc_box, const float*, double*, void*) {
    return fail(c, RC_ERR_UNSUPPORTED, "rc_param_vjp is not available in this build");
}

// ============================================================================
// MD driver
// ============================================================================
static int build_graphs(rc_ctx* c, const StepArgs& tmpl, int G) {
    drop_graphs(c);
    const void* fn;
    step_kernel_info(false, &fn);
    const void* add_fn;
    add_step_kernel_info(&add_fn);
    const int nb = nblocks(tmpl.N, kStepBlock);
    const size_t shm = sizeof(DevEntry) * c->nt * c->nt;
    for (int p = 0; p < 2; ++p) {
        hipGraph_t g;
        HIP_TRY(c, hipGraphCreate(&g, 0));
        hipGraphNode_t prev = nullptr;
        for (int k = 0; k < G; ++k) {
            StepArgs a = tmpl;
            const bool from_alt = ((k + p) & 1) != 0;
            const float4* A = tmpl.pos_in;                        // "pos"
            float4* B = tmpl.pos_out;                             // "pos_alt"
            a.pos_in = from_alt ? B : A;
            a.pos_out = from_alt ? const_cast<float4*>(A) : B;
            a.mode = RC_STEP_CONT;
            a.step = (uint64_t)k;
            a.step_base = c->d_step_base;
            a.ev_part = nullptr;
            void* args[] = {&a};
            hipKernelNodeParams kp{};
            kp.func = const_cast<void*>(fn);
            kp.gridDim = dim3(nb);
            kp.blockDim = dim3(kStepBlock);
            kp.sharedMemBytes = (unsigned)shm;
            kp.kernelParams = args;
            kp.extra = nullptr;
            hipGraphNode_t node;
            HIP_TRY(c, hipGraphAddKernelNode(&node, g, prev ? &prev : nullptr, prev ? 1 : 0, &kp));
            prev = node;
        }
        {
            unsigned long long* p_base = c->d_step_base;
            unsigned long long inc = (unsigned long long)G;
            void* args[] = {&p_base, &inc};
            hipKernelNodeParams kp{};
            kp.func = const_cast<void*>(add_fn);
            kp.gridDim = dim3(1);
            kp.blockDim = dim3(1);
            kp.sharedMemBytes = 0;
            kp.kernelParams = args;
            kp.extra = nullptr;
            hipGraphNode_t node;
            HIP_TRY(c, hipGraphAddKernelNode(&node, g, &prev, 1, &kp));
        }
        c->gc.graph[p] = g;
        HIP_TRY(c, hipGraphInstantiate(&c->gc.exec[p], g, nullptr, nullptr, 0));
    }
    c->gc.key = tmpl;
    c->gc.steps = G;
    c->gc.valid = true;
    return RC_OK;
}

static bool same_args(const StepArgs& x, const StepArgs& y) { return std::memcmp(&x, &y, sizeof(StepArgs)) == 0; }

int rc_md_run(rc_ctx* c, const rc_md_buffers* buf, int N, rc_box box, const rc_integrator* cfg, uint64_t step0,
              int n_steps, const rc_md_options* opt_in, rc_md_stats* stats, void* stream) {
    int r = check_common(c, N, buf ? buf->pos : nullptr);
    if (r) return r;
    if (!buf->pos_alt || !buf->vel || !buf->nlist || !buf->nn || !buf->cells_ws || !buf->status)
        return fail(c, RC_ERR_ARG, "md buffers incomplete");
    if (buf->k_max < 1 || buf->k_max > 512) return fail(c, RC_ERR_ARG, "k_max must be in [1, 512]");
    if (n_steps < 0) return fail(c, RC_ERR_ARG, "n_steps < 0");
    rc_md_options opt{1, 16, 256, 0, 0.8, 1, 0};
    if (opt_in) opt = *opt_in;
    if (opt.graph_steps < 2 || (opt.graph_steps & 1)) opt.graph_steps = 16;
    if (opt.max_chunk < 1) opt.max_chunk = 256;
    if (!(opt.soft_frac > 0.0 && opt.soft_frac <= 1.0)) opt.soft_frac = 0.8;
    const bool can_roll = buf->snap_pos && buf->snap_vel && (buf->snap_image || !buf->image);
    Box b;
    if ((r = make_box(c, box, b))) return r;
    hipStream_t s = S(stream);
    const int nb = nblocks(N, kStepBlock);
    if ((r = ensure_part(c, sizeof(double) * kEvWords * (size_t)nb))) return r;
    rc_md_stats st{};
    int hst[RC_STATUS_WORDS];

    float* P[2] = {buf->pos, buf->pos_alt};
    int cur = 0;
    StepArgs tmpl{};
    if ((r = fill_step_args(c, tmpl, buf->pos, buf->pos_alt, buf->vel, buf->image, buf->nlist, buf->nn, buf->k_max, N, b, cfg,
                            opt.soft_frac, buf->status)))
        return r;

    auto rebuild = [&](int which) -> int {
        int rr = rc_build_cells(c, P[which], buf->vel, buf->image, buf->rtag, N, box, buf->cells_ws,
                                buf->cells_ws_bytes, stream);
        if (rr) return rr;
        HIP_TRY(c, launch_zero_words(buf->status, RC_STATUS_WORDS, s));
        rr = rc_build_nlist(c, P[which], buf->vel, N, box, buf->cells_ws, buf->cells_ws_bytes, buf->k_max, buf->nlist,
                            buf->nn, buf->status, stream);
        if (rr) return rr;
        HIP_TRY(c, hipMemcpyAsync(hst, buf->status, sizeof hst, hipMemcpyDeviceToHost, s));
        HIP_TRY(c, hipStreamSynchronize(s));
        ++st.rebuilds;
        if (hst[RC_ST_FLAGS] & RC_FLAG_NLIST_OVERFLOW) {
            st.k_needed = hst[RC_ST_KMAX];
            return fail(c, RC_ERR_NLIST_OVERFLOW, "a particle has %d neighbours (k_max %d)", hst[RC_ST_KMAX],
                        buf->k_max);
        }
        return RC_OK;
    };
    auto finish = [&](int code) -> int {
        if (stats) {
            st.flags = hst[RC_ST_FLAGS];
            *stats = st;
        }
        return code;
    };

    int row = 0;
    auto log_now = [&](int which, bool ev_step) -> int {
        (void)ev_step;
        if (buf->bonds_log) {
            HIP_TRY(c, launch_bonds(reinterpret_cast<const float4*>(P[which]), buf->nlist, buf->nn, buf->k_max, N, dev_table(c), b,
                                    buf->bonds_log + row, reinterpret_cast<unsigned long long*>(c->d_part), s));
        }
        return RC_OK;
    };

    // direct launch of one step from P[cur]
    auto direct = [&](uint64_t step, int mode, bool ev) -> int {
        StepArgs a = tmpl;
        a.pos_in = reinterpret_cast<const float4*>(P[cur]);
        a.pos_out = reinterpret_cast<float4*>(P[cur ^ 1]);
        a.mode = mode;
        a.step = step;
        a.step_base = nullptr;
        a.ev_part = ev ? c->d_part : nullptr;
        HIP_TRY(c, launch_step(a, ev, s));
        if (ev && buf->ev_log) {
            int rr = reduce_rows(c, nb, 0, kEvWords, buf->ev_log + (size_t)row * kEvWords, s);
            if (rr) return rr;
        }
        return RC_OK;
    };

    if ((r = rebuild(cur))) return finish(r);
    HIP_TRY(c, launch_status_reset_chunk(buf->status, s));

    const bool logging = buf->ev_log || buf->bonds_log;
    const int lp = opt.log_period;
    bool first = true;
    int64_t done = 0;
    double rate = 0.0;           // growth of the largest path length per step
    float last_maxpath = 0.0f;
    const float hard = tmpl.hard;
    const bool graphs = opt.use_graph != 0;
    const int G = opt.graph_steps;
    if (graphs) {
        StepArgs key = tmpl;
        key.pos_in = reinterpret_cast<const float4*>(buf->pos);
        key.pos_out = reinterpret_cast<float4*>(buf->pos_alt);
        if (!c->gc.valid || c->gc.steps != G || !same_args(c->gc.key, key)) {
            if ((r = build_graphs(c, key, G))) return finish(r);
        }
    }
    uint64_t dev_base = ~0ull;   // value *d_step_base will hold once queued work ran

    while (done < n_steps) {
        // ---- plan the chunk ---------------------------------------------------
        int64_t C = std::min<int64_t>(n_steps - done, opt.max_chunk);
        if (!can_roll) C = 1;
        else if (!opt.adapt) {
            // fixed chunks: stale chunks are rolled back
        } else if (rate > 0.0) {
            const double room = (double)hard - (double)last_maxpath;
            const int64_t safe = (int64_t)std::floor(room / (1.5 * rate));
            C = std::max<int64_t>(1, std::min<int64_t>(C, safe));
        } else if (first) {
            C = std::min<int64_t>(C, 8);
        }
        const int64_t chunk_start = done;
        const int row_start = row;
        const int cur_start = cur;
        const bool first_start = first;
        if (can_roll) {
            HIP_TRY(c, hipMemcpyAsync(buf->snap_pos, P[cur], 16 * (size_t)N, hipMemcpyDeviceToDevice, s));
            HIP_TRY(c, hipMemcpyAsync(buf->snap_vel, buf->vel, 16 * (size_t)N, hipMemcpyDeviceToDevice, s));
            if (buf->image)
                HIP_TRY(c, hipMemcpyAsync(buf->snap_image, buf->image, 16 * (size_t)N, hipMemcpyDeviceToDevice, s));
        }
        HIP_TRY(c, launch_status_reset_chunk(buf->status, s));
        // ---- run it --------------------------------------------------------------
        auto run_steps = [&](int64_t from, int64_t count) -> int {
            int64_t k = 0;
            while (k < count) {
                const int64_t d = from + k;
                const uint64_t step = step0 + (uint64_t)d;
                const bool ev = logging && lp > 0 && (d % lp) == 0;
                if (ev) {
                    int rr = log_now(cur, true);
                    if (rr) return rr;
                }
                if (graphs && !first && !ev && count - k >= G) {
                    // a graph replay must not cross a logging step
                    bool clear = true;
                    if (logging && lp > 0) {
                        const int64_t next_log = ((d + lp - 1) / lp) * lp;
                        clear = next_log >= d + G || next_log == d;
                        if (next_log == d) clear = false;
                    }
                    if (clear) {
                        if (dev_base != step) HIP_TRY(c, launch_set_step(c->d_step_base, step, s));
                        HIP_TRY(c, hipGraphLaunch(c->gc.exec[cur], s));
                        dev_base = step + G;
                        k += G;
                        continue;  // G is even: cur is unchanged
                    }
                }
                int rr = direct(step, first ? RC_STEP_START : RC_STEP_CONT, ev);
                if (rr) return rr;
                if (ev) ++row;
                first = false;
                cur ^= 1;
                ++k;
            }
            return RC_OK;
        };
        if ((r = run_steps(chunk_start, C))) return finish(r);
        HIP_TRY(c, launch_fold_status(c->d_blk, nb, reinterpret_cast<const float4*>(buf->vel), N, buf->status, s));
        HIP_TRY(c, hipMemcpyAsync(hst, buf->status, sizeof hst, hipMemcpyDeviceToHost, s));
        HIP_TRY(c, hipStreamSynchronize(s));
        ++st.chunks;
        const int f = hst[RC_ST_FLAGS];
        if (f & RC_FLAG_LOST) return finish(fail(c, RC_ERR_LOST_PARTICLE, "a particle moved more than L/2 in one step"));
        if (f & RC_FLAG_NONFINITE) return finish(fail(c, RC_ERR_NONFINITE, "non-finite position or velocity"));
        float mp;
        std::memcpy(&mp, &hst[RC_ST_MAXPATH], sizeof mp);
        if (f & RC_FLAG_STALE) {
            if (!can_roll) return finish(fail(c, RC_ERR_ARG, "stale list without rollback buffers"));
            // roll back and replay up to the first soft crossing, then rebuild
            cur = cur_start;
            first = first_start;
            row = row_start;
            HIP_TRY(c, hipMemcpyAsync(P[cur], buf->snap_pos, 16 * (size_t)N, hipMemcpyDeviceToDevice, s));
            HIP_TRY(c, hipMemcpyAsync(buf->vel, buf->snap_vel, 16 * (size_t)N, hipMemcpyDeviceToDevice, s));
            if (buf->image)
                HIP_TRY(c, hipMemcpyAsync(buf->image, buf->snap_image, 16 * (size_t)N, hipMemcpyDeviceToDevice, s));
            const int64_t soft_step = (int64_t)hst[RC_ST_FIRST_SOFT];
            int64_t n_re = soft_step - (int64_t)((step0 + (uint64_t)chunk_start) & 0x7fffffff) + 1;
            n_re = std::max<int64_t>(1, std::min<int64_t>(n_re, C));
            HIP_TRY(c, launch_status_reset_chunk(buf->status, s));
            if ((r = run_steps(chunk_start, n_re))) return finish(r);
            HIP_TRY(c, launch_fold_status(c->d_blk, nb, nullptr, N, buf->status, s));  // drop replay flags
            done = chunk_start + n_re;
            ++st.rollbacks;
            if ((r = rebuild(cur))) return finish(r);
            rate = std::max(rate, (double)mp / std::max<int64_t>(1, C));
            last_maxpath = 0.0f;
            HIP_TRY(c, launch_status_reset_chunk(buf->status, s));
            continue;
        }
        done = chunk_start + C;
        rate = std::max(0.5 * rate, (double)(mp - last_maxpath) / (double)C);
        last_maxpath = mp;
        if (f & RC_FLAG_REBUILD) {
            if ((r = rebuild(cur))) return finish(r);
            last_maxpath = 0.0f;
            HIP_TRY(c, launch_status_reset_chunk(buf->status, s));
        }
    }
    // ---- final half kick (and the last log row) ------------------------------------
    {
        const bool ev = logging && buf->ev_log;
        if (logging) {
            if ((r = log_now(cur, true))) return finish(r);
        }
        if (!first) {
            if ((r = direct(step0 + (uint64_t)n_steps, RC_STEP_FINISH, ev))) return finish(r);
        } else if (ev) {
            // zero steps: report the state as it is
            if ((r = direct(step0, RC_STEP_OBSERVE, ev))) return finish(r);
        }
        if (logging) ++row;
    }
    if (cur != 0) HIP_TRY(c, hipMemcpyAsync(buf->pos, P[cur], 16 * (size_t)N, hipMemcpyDeviceToDevice, s));
    HIP_TRY(c, hipMemcpyAsync(hst, buf->status, sizeof hst, hipMemcpyDeviceToHost, s));
    HIP_TRY(c, hipStreamSynchronize(s));
    st.steps_done = done;
    st.log_rows = row;
    return finish(RC_OK);
}

}  // extern "C"
