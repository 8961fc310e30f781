// Host-side internals shared by the single-system and the batch C ABI.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>

#include "rc_host.h"

namespace rc {
namespace host {

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

static bool fp32_exact(double x) { return (double)(float)x == x; }

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

int make_grid(rc_ctx* c, double rlist_max, const Box& b, Grid& g) {
    int maxnc = 0;
    for (int d = 0; d < 3; ++d) {
        if (b.L[d] < 3.0 * rlist_max)
            return fail(c, RC_ERR_ARG, "box edge %.6g shorter than three list radii (%.6g)", b.L[d],
                        3.0 * rlist_max);
        int nc = (int)std::floor(b.L[d] / (rlist_max * (1.0 + 1e-5)));
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

CellsLayout cells_layout(int N, uint32_t nkeys) {
    auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
    CellsLayout l{};
    size_t o = 0;
    const size_t nk = nkeys;
    l.counts = o; o = al(o + 4 * nk);
    l.start = o; o = al(o + 4 * (nk + 1));
    l.keys = o; o = al(o + 4 * (size_t)N);
    l.rank = o; o = al(o + 4 * (size_t)N);
    l.order = o; o = al(o + 4 * (size_t)N);
    l.bsums = o; o = al(o + 4 * (nk / kScanTile + 2));
    l.bmax = o; o = al(o + 8 * ((size_t)N / kBlock + 2));   // per block: largest list, then swap-range sums
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

size_t plist_entries(int N, int k_max) { return (size_t)((N + kWave - 1) / kWave) * kWave * (size_t)k_max; }

WsLayout ws_layout(size_t plist, size_t n_ssum, size_t n_hsum) {
    auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
    WsLayout l{};
    size_t o = 0;
    l.pl_j = o; o = al(o + sizeof(int) * plist);
    l.pl_o = o; o = al(o + plist);
    l.ssum = o; o = al(o + sizeof(float) * n_ssum);
    l.hsum = o; o = al(o + 2 * sizeof(double) * n_hsum);
    l.total = o;
    return l;
}

int set_workspace(rc_ctx* c, void* ws, size_t bytes, int N, int k_max, int nvec) {
    if (ws && (N < 1 || k_max < 1 || k_max > 512 || nvec < 0))
        return fail(c, RC_ERR_ARG, "workspace sizes: N >= 1, 1 <= k_max <= 512, nvec >= 0");
    const size_t E = ws ? plist_entries(N, k_max) : 0;
    const WsLayout l = ws_layout(E, ws ? (size_t)N : 0, ws ? (size_t)N * (size_t)nvec : 0);
    if (ws && bytes < l.total) return fail(c, RC_ERR_WORKSPACE, "workspace needs %zu bytes (got %zu)", l.total, bytes);
    if (ws && (reinterpret_cast<uintptr_t>(ws) & 255)) return fail(c, RC_ERR_ARG, "workspace not 256-byte aligned");
    drop_graphs(c);
    c->md.valid = false;   // the packed copy of the list moves
    HIP_TRY(c, hipDeviceSynchronize());
    if (!c->ws_user) {     // the context's own buffers go
        if (c->d_pl_j) (void)hipFree(c->d_pl_j);
        if (c->d_pl_o) (void)hipFree(c->d_pl_o);
        if (c->d_ssum) (void)hipFree(c->d_ssum);
        if (c->d_hsum) (void)hipFree(c->d_hsum);
    }
    c->d_pl_j = nullptr;
    c->d_pl_o = nullptr;
    c->d_ssum = nullptr;
    c->d_hsum = nullptr;
    c->pl_cap = c->ssum_cap = c->hsum_cap = 0;
    c->pl_nlist = nullptr;
    c->ws_user = ws;
    if (ws) {
        char* w = static_cast<char*>(ws);
        c->d_pl_j = reinterpret_cast<int*>(w + l.pl_j);
        c->d_pl_o = reinterpret_cast<unsigned char*>(w + l.pl_o);
        c->d_ssum = reinterpret_cast<float*>(w + l.ssum);
        c->d_hsum = reinterpret_cast<double*>(w + l.hsum);
        c->pl_cap = E;
        c->ssum_cap = (size_t)N;
        c->hsum_cap = (size_t)N * (size_t)nvec;
    }
    return RC_OK;
}

size_t ctx_device_bytes(const rc_ctx* c) {
    size_t b = sizeof(DevEntry) * (size_t)c->nt * (size_t)c->nt + sizeof(unsigned long long) + c->part_bytes +
               sizeof(int) * 3 * (size_t)c->blk_cap + (c->d_slices ? sizeof(double) * kRowSlices : 0);
    if (!c->ws_user) b += 5 * c->pl_cap + sizeof(float) * c->ssum_cap + 2 * sizeof(double) * c->hsum_cap;
    return b;
}

int ensure_ssum(rc_ctx* c, size_t n) {
    if (c->ssum_cap >= n) return RC_OK;
    if (c->ws_user)
        return fail(c, RC_ERR_WORKSPACE, "the attached workspace holds switching sums of %zu particles, %zu needed",
                    c->ssum_cap, n);
    drop_graphs(c);
    HIP_TRY(c, hipDeviceSynchronize());
    if (c->d_ssum) (void)hipFree(c->d_ssum);
    c->d_ssum = nullptr;
    c->ssum_cap = 0;
    HIP_TRY(c, hipMalloc(&c->d_ssum, sizeof(float) * n));
    c->ssum_cap = n;
    return RC_OK;
}

int read_status_spin(rc_ctx* c, const int* d_status, int* hst, hipStream_t s) {
    if (!c->h_status) HIP_TRY(c, hipHostMalloc(reinterpret_cast<void**>(&c->h_status), sizeof(int) * RC_STATUS_WORDS));
    if (!c->ev_sync) HIP_TRY(c, hipEventCreateWithFlags(&c->ev_sync, hipEventDisableTiming));
    HIP_TRY(c, hipMemcpyAsync(c->h_status, d_status, sizeof(int) * RC_STATUS_WORDS, hipMemcpyDeviceToHost, s));
    for (const rc_ctx::StatusExtra& x : c->status_extra)
        HIP_TRY(c, hipMemcpyAsync(x.host, x.dev, x.bytes, hipMemcpyDeviceToHost, s));
    HIP_TRY(c, hipEventRecord(c->ev_sync, s));
    // a blocking synchronisation costs tens of microseconds of wake-up per call; the driver calls
    // this once per chunk, so it spins on the event instead
    hipError_t e;
    while ((e = hipEventQuery(c->ev_sync)) == hipErrorNotReady) {
    }
    if (e != hipSuccess) return hip_fail(c, e, "waiting for the status word");
    std::memcpy(hst, c->h_status, sizeof(int) * RC_STATUS_WORDS);
    return RC_OK;
}

int ensure_plist(rc_ctx* c, int N, int k_max) {
    const size_t n = plist_entries(N, k_max);
    if (c->pl_cap >= n) return RC_OK;
    if (c->ws_user)
        return fail(c, RC_ERR_WORKSPACE, "the attached workspace holds a packed list of %zu entries, %zu needed",
                    c->pl_cap, n);
    drop_graphs(c);
    HIP_TRY(c, hipDeviceSynchronize());
    if (c->d_pl_j) (void)hipFree(c->d_pl_j);
    if (c->d_pl_o) (void)hipFree(c->d_pl_o);
    c->d_pl_j = nullptr;
    c->d_pl_o = nullptr;
    c->pl_cap = 0;
    c->pl_nlist = nullptr;
    HIP_TRY(c, hipMalloc(&c->d_pl_j, sizeof(int) * n));
    HIP_TRY(c, hipMalloc(&c->d_pl_o, n));
    c->pl_cap = n;
    return RC_OK;
}

int packed_list_for(rc_ctx* c, const int* nlist, const int* nn, int k_max, int N, hipStream_t s) {
    if (c->pl_nlist == nlist && c->pl_nn == nn && c->pl_k == k_max && c->pl_n == N) return RC_OK;
    int r = ensure_plist(c, N, k_max);
    if (r) return r;
    HIP_TRY(c, launch_pack_list(nlist, nn, k_max, N, c->d_pl_j, c->d_pl_o, s));
    c->pl_nlist = nlist;
    c->pl_nn = nn;
    c->pl_k = k_max;
    c->pl_n = N;
    return RC_OK;
}

int ensure_hsum(rc_ctx* c, size_t n) {
    if (c->hsum_cap >= n) return RC_OK;
    if (c->ws_user)
        return fail(c, RC_ERR_WORKSPACE, "the attached workspace holds HVP sums for %zu particle-vectors, %zu needed",
                    c->hsum_cap, n);
    HIP_TRY(c, hipDeviceSynchronize());
    if (c->d_hsum) (void)hipFree(c->d_hsum);
    c->d_hsum = nullptr;
    c->hsum_cap = 0;
    HIP_TRY(c, hipMalloc(&c->d_hsum, 2 * sizeof(double) * n));
    c->hsum_cap = n;
    return RC_OK;
}

void free_ctx_buffers(rc_ctx* c) {
    drop_graphs(c);
    drop_rebuild_graphs(c);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    c->cap_stream = nullptr;
    for (hipEvent_t e : c->tk_events)
        if (e) (void)hipEventDestroy(e);
    c->tk_events.clear();
    c->tk_kind.clear();
    c->md.valid = false;
    if (c->d_pl_j && !c->ws_user) (void)hipFree(c->d_pl_j);
    if (c->d_pl_o && !c->ws_user) (void)hipFree(c->d_pl_o);
    c->d_pl_j = nullptr;
    c->d_pl_o = nullptr;
    c->pl_cap = 0;
    c->pl_nlist = nullptr;
    if (c->ev_sync) (void)hipEventDestroy(c->ev_sync);
    if (c->h_status) (void)hipHostFree(c->h_status);
    c->ev_sync = nullptr;
    c->h_status = nullptr;
    if (c->d_tab) (void)hipFree(c->d_tab);
    if (c->d_part) (void)hipFree(c->d_part);
    if (c->d_step_base) (void)hipFree(c->d_step_base);
    if (c->d_slices) (void)hipFree(c->d_slices);
    c->d_slices = nullptr;
    if (c->d_blk) (void)hipFree(c->d_blk);
    if (c->d_ssum && !c->ws_user) (void)hipFree(c->d_ssum);
    if (c->d_hsum && !c->ws_user) (void)hipFree(c->d_hsum);
    c->ws_user = nullptr;
    c->d_hsum = nullptr;
    c->hsum_cap = 0;
    c->d_tab = nullptr;
    c->d_part = nullptr;
    c->d_step_base = nullptr;
    c->d_blk = nullptr;
    c->d_ssum = nullptr;
}

void drop_rebuild_graphs(rc_ctx* c) {
    for (RebuildGraph& g : c->rg) {
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
        g = RebuildGraph{};
    }
}

int rebuild_graphed(rc_ctx* c, int slot, const RebuildKey& key, int (*fn)(void*, hipStream_t), void* arg,
                    hipStream_t s) {
    RebuildGraph& g = c->rg[slot];
    const bool same = g.seen && std::memcmp(&g.key, &key, sizeof key) == 0;
    if (same && g.valid) {
        HIP_TRY(c, hipGraphLaunch(g.exec, s));
        return RC_OK;
    }
    if (!same) {   // a new key: run directly (any allocation happens here), record next time
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
        g = RebuildGraph{};
        g.key = key;
        g.seen = true;
        return fn(arg, s);
    }
    if (!c->cap_stream) HIP_TRY(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
    HIP_TRY(c, hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeRelaxed));
    const int r = fn(arg, c->cap_stream);
    hipGraph_t graph = nullptr;
    const hipError_t e = hipStreamEndCapture(c->cap_stream, &graph);
    if (r != RC_OK || e != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        if (r != RC_OK) return r;
        return hip_fail(c, e, "recording the rebuild graph");
    }
    const hipError_t ei = hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ei != hipSuccess) return hip_fail(c, ei, "instantiating the rebuild graph");
    HIP_TRY(c, hipGraphUpload(g.exec, s));
    g.valid = true;
    HIP_TRY(c, hipGraphLaunch(g.exec, s));
    return RC_OK;
}

void drop_graphs(rc_ctx* c) {
    for (int p = 0; p < 2; ++p) {
        if (c->gc.exec[p]) (void)hipGraphExecDestroy(c->gc.exec[p]);
        if (c->gc.graph[p]) (void)hipGraphDestroy(c->gc.graph[p]);
        c->gc.exec[p] = nullptr;
        c->gc.graph[p] = nullptr;
    }
    c->gc.valid = false;
}

// per-block status slots for nb blocks (allocated once per size, reset to neutral)
int ensure_blk(rc_ctx* c, int nb, hipStream_t s) {
    if (c->blk_cap >= nb) return RC_OK;
    drop_graphs(c);   // graphs hold the old pointer
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

int check_integrator(rc_ctx* c, const rc_integrator* cfg, float* minv, float* c2, float& c1, int& langevin,
                     float& noise_z) {
    if (!cfg) return fail(c, RC_ERR_ARG, "integrator is NULL");
    if (cfg->dim != 0 && cfg->dim != 2 && cfg->dim != 3)
        return fail(c, RC_ERR_ARG, "integrator dim must be 2 or 3 (0 = 3), not %d", cfg->dim);
    noise_z = cfg->dim == 2 ? 0.0f : 1.0f;
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

int check_list(rc_ctx* c, const int* nlist, const int* nn, int k_max) {
    if (!nlist || !nn) return fail(c, RC_ERR_ARG, "nlist / nn are NULL");
    if (k_max < 1 || k_max > 512) return fail(c, RC_ERR_ARG, "k_max must be in [1, 512]");
    return RC_OK;
}

int compile_table(int nt, const rc_pair_coeff* table, double r_buff, DevEntry* out, double* rlist_max,
                  std::string* why) {
    auto bad = [&](const char* msg, int a, int b) {
        if (why) {
            char buf[160];
            snprintf(buf, sizeof buf, "table entry (%d, %d): %s", a, b, msg);
            *why = buf;
        }
        return RC_ERR_ARG;
    };
    double rmax = 0.0;
    for (int a = 0; a < nt; ++a) {
        for (int b = 0; b < nt; ++b) {
            const rc_pair_coeff& p = table[a * nt + b];
            const rc_pair_coeff& q = table[b * nt + a];
            if (p.kind != q.kind || p.n != q.n || p.epsilon != q.epsilon || p.sigma != q.sigma ||
                p.r_cut != q.r_cut || (p.kind == RC_KIND_SWAP && p.lambda != q.lambda))
                return bad("not symmetric", a, b);
            DevEntry e{};
            e.kind = p.kind;
            if (p.kind == RC_KIND_SWAP) {
                const double rmin = p.sigma * std::pow(2.0, 1.0 / p.n);
                if (!(p.epsilon > 0.0) || !(p.sigma > 0.0) || p.n < 1 || p.n > 200 || !(p.lambda >= 0.0) ||
                    !(p.r_cut > rmin) || !std::isfinite(p.r_cut))
                    return bad("swap entry needs eps > 0, sigma > 0, 1 <= n <= 200, lambda >= 0, r_cut > r_min",
                               a, b);
                e.n = p.n;
                e.sqrt_lam = (float)std::sqrt(p.lambda * p.epsilon);
                e.inv_eps = (float)(1.0 / p.epsilon);
                e.lam = (float)p.lambda;
            } else if (p.kind == RC_KIND_WCA) {
                if (!(p.epsilon >= 0.0) || !(p.sigma > 0.0) || !(p.r_cut > 0.0) || !std::isfinite(p.r_cut))
                    return bad("WCA entry needs eps >= 0, sigma > 0, r_cut > 0", a, b);
                e.n = 6;
            } else if (p.kind != RC_KIND_NONE) {
                return bad("unknown kind", a, b);
            }
            if (p.kind != RC_KIND_NONE) {
                e.eps = (float)p.epsilon;
                e.sigma = (float)p.sigma;
                e.sig2 = (float)(p.sigma * p.sigma);
                e.rcut2 = p.r_cut * p.r_cut;
                e.rmin2 = (p.sigma * p.sigma) * std::pow(2.0, 2.0 / (double)(p.kind == RC_KIND_SWAP ? p.n : 6));
                // guard bands of the FP32 decisions (pair_geom)
                auto band = [](double t, float& lo, float& hi) {
                    lo = std::nextafter((float)(t * (1.0 - 2e-6)), 0.0f);
                    hi = std::nextafter((float)(t * (1.0 + 2e-6)), INFINITY);
                };
                band(e.rcut2, e.rcut2_lo, e.rcut2_hi);
                band(e.rmin2, e.rmin2_lo, e.rmin2_hi);
                const double rl = p.r_cut + r_buff;
                e.rlist2 = (float)(rl * rl * (1.0 + 1e-5));
                rmax = std::max(rmax, rl);
            }
            out[a * nt + b] = e;
        }
    }
    if (rmax == 0.0) rmax = r_buff;
    *rlist_max = rmax;
    return RC_OK;
}

// ---------------------------------------------------------------------------
// step graphs: G launches of the CONT step alternating the two position
// buffers, then one add of G to the device step base; one graph per start
// parity.  Built with explicit kernel nodes (no capture, no memset nodes).
// ---------------------------------------------------------------------------
static int add_node(rc_ctx* c, hipGraph_t g, hipGraphNode_t& prev, const void* fn, void** args, int blocks,
                    int threads, size_t shm) {
    hipKernelNodeParams kp{};
    kp.func = const_cast<void*>(fn);
    kp.gridDim = dim3(blocks);
    kp.blockDim = dim3(threads);
    kp.sharedMemBytes = (unsigned)shm;
    kp.kernelParams = args;
    kp.extra = nullptr;
    hipGraphNode_t node;
    HIP_TRY(c, hipGraphAddKernelNode(&node, g, prev ? &prev : nullptr, prev ? 1 : 0, &kp));
    prev = node;
    return RC_OK;
}

static int build_graphs(rc_ctx* c, const void* fn, const void* sums_fn, const StepArgs& tmpl, int G, hipStream_t s) {
    drop_graphs(c);
    const void* add_fn;
    add_step_kernel_info(&add_fn);
    const int nb = nblocks(tmpl.N, kStepBlock);
    const size_t shm = sizeof(DevEntry) * c->nt * c->nt;
    int r;
    for (int p = 0; p < 2; ++p) {
        hipGraph_t g;
        HIP_TRY(c, hipGraphCreate(&g, 0));
        c->gc.graph[p] = g;
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
            if (sums_fn) {
                ForceArgs f = step_sums_args(a);
                void* args[] = {&f};
                if ((r = add_node(c, g, prev, sums_fn, args, nblocks(tmpl.N, kWave), kWave, shm))) return r;
            }
            void* args[] = {&a};
            if ((r = add_node(c, g, prev, fn, args, nb, kStepBlock, shm))) return r;
        }
        {
            unsigned long long* p_base = c->d_step_base;
            unsigned long long inc = (unsigned long long)G;
            void* args[] = {&p_base, &inc};
            if ((r = add_node(c, g, prev, add_fn, args, 1, 1, 0))) return r;
        }
        HIP_TRY(c, hipGraphInstantiate(&c->gc.exec[p], g, nullptr, nullptr, 0));
        // upload now: a first launch would otherwise pay it inside the run that uses the graph
        HIP_TRY(c, hipGraphUpload(c->gc.exec[p], s));
    }
    c->gc.key = tmpl;
    c->gc.fn = fn;
    c->gc.steps = G;
    c->gc.valid = true;
    return RC_OK;
}

static bool same_args(const StepArgs& x, const StepArgs& y) { return std::memcmp(&x, &y, sizeof(StepArgs)) == 0; }

}  // namespace host
}  // namespace rc

DynKey dyn_key(const rc::StepArgs& a) {
    DynKey k;
    std::memset(&k, 0, sizeof k);   // padding too: keys are compared bytewise
    std::memcpy(k.minv, a.minv, sizeof k.minv);
    std::memcpy(k.c2, a.c2, sizeof k.c2);
    k.dt = a.dt;
    k.c1 = a.c1;
    k.noise_z = a.noise_z;
    k.fene_k = a.bonds ? a.fene_k : 0.0f;
    k.fene_r02 = a.bonds ? a.fene_r02 : 0.0f;
    k.langevin = a.langevin;
    k.seed = a.seed;
    k.bonds = a.bonds;
    return k;
}

namespace rc {
namespace host {

static bool same_buffers(const rc_md_buffers& x, const rc_md_buffers& y) {
    return x.pos == y.pos && x.pos_alt == y.pos_alt && x.vel == y.vel && x.image == y.image && x.rtag == y.rtag &&
           x.nlist == y.nlist && x.nn == y.nn && x.k_max == y.k_max && x.cells_ws == y.cells_ws &&
           x.cells_ws_bytes == y.cells_ws_bytes && x.snap_pos == y.snap_pos && x.snap_vel == y.snap_vel &&
           x.snap_image == y.snap_image && x.status == y.status;
}

int md_drive(rc_ctx* c, DriveOps& ops, const rc_md_buffers* buf, int N, const StepArgs& tmpl, uint64_t step0,
             int n_steps, rc_md_options opt, rc_md_stats* stats, hipStream_t s) {
    const bool can_roll = buf->snap_pos && buf->snap_vel && (buf->snap_image || !buf->image);
    const int nb = nblocks(N, kStepBlock);
    int r;
    rc_md_stats st{};
    int hst[RC_STATUS_WORDS] = {0};
    const MdRecord prev = c->md;   // what the last run left (valid only if nothing changed the state since)
    c->md.valid = false;           // set again only by a run that returns RC_OK

    // Steps are counted absolutely: the state is at step s_cur, the run ends at s_end.
    const uint64_t s_end = step0 + (uint64_t)n_steps;
    uint64_t s_cur = step0;
    float* P[2] = {buf->pos, buf->pos_alt};
    int cur = 0;
    // Rollback state: one snapshot per list build (an epoch).  Every chunk of an epoch before the
    // last ran without a soft crossing (a soft crossing ends the epoch with a rebuild), so a chunk
    // that goes stale is replayed from the epoch's start up to its first soft crossing.
    bool need_snap = true;
    const float4 *ws_pos = nullptr, *ws_vel = nullptr;
    const int4* ws_image = nullptr;
    const bool snap_in_ws = ops.rebuild_snapshot(&ws_pos, &ws_vel, &ws_image);
    uint64_t ep_step = step0;      // the epoch's first step (may precede step0 for a kept list)
    int ep_cur = 0, ep_row = 0;
    bool ep_first = true;

    // With the rebuilt state kept in the workspace, the list's overflow check is
    // deferred to the status read that ends the next chunk (one host wait less
    // per build): an overflow there restores the epoch's start and returns.
    const bool defer_check = snap_in_ws && can_roll;
    bool check_pending = false;
    int row = 0;
    auto overflow = [&]() -> int {
        st.k_needed = hst[RC_ST_KMAX];
        return fail(c, RC_ERR_NLIST_OVERFLOW, "a particle has %d neighbours (k_max %d)", hst[RC_ST_KMAX],
                    buf->k_max);
    };
    bool first = opt.resume == 0;  // a resumed state owes its last step's final half kick
    float kept_path = 0.0f;        // largest path length of the particles the last build kept
    auto rebuild = [&](int which, RebuildKind kind) -> int {
        int64_t nre = 0;
        int rr = ops.rebuild(P[which], kind, &kept_path, &nre);
        if (rr) return rr;
        ++st.rebuilds;
        st.particles_rebuilt += nre;
        need_snap = true;
        if (defer_check) {
            check_pending = true;
            return RC_OK;
        }
        if ((rr = read_status_spin(c, buf->status, hst, s))) return rr;
        if (hst[RC_ST_FLAGS] & RC_FLAG_NLIST_OVERFLOW) return overflow();
        return RC_OK;
    };
    // every return reports the steps done: on an error the state (in buf->pos)
    // is that of step0 + steps_done with the last step's final half kick due
    auto finish = [&](int code) -> int {
        if (code != RC_OK) {
            if (cur != 0) (void)hipMemcpyAsync(buf->pos, P[cur], 16 * (size_t)N, hipMemcpyDeviceToDevice, s);
            (void)hipStreamSynchronize(s);
        }
        if (stats) {
            st.flags = hst[RC_ST_FLAGS];
            st.nswap = hst[RC_ST_NSWAP];
            st.steps_done = s_cur > step0 ? (int64_t)(s_cur - step0) : 0;
            st.log_rows = row;
            *stats = st;
        }
        return code;
    };

    // ---- per-launch timing (time_kernels) ---------------------------------------------
    const bool timing = opt.time_kernels != 0;
    size_t tk_used = 0;
    // index of a fresh (start, stop) event pair; kind 1 marks a first pass of the sums form
    auto tk_take = [&](size_t* q, int kind) -> int {
        if (c->tk_events.size() < tk_used + 2) {
            hipEvent_t e0 = nullptr, e1 = nullptr;
            HIP_TRY(c, hipEventCreate(&e0));
            HIP_TRY(c, hipEventCreate(&e1));
            c->tk_events.push_back(e0);
            c->tk_events.push_back(e1);
            c->tk_kind.push_back(0);
        }
        *q = tk_used;
        c->tk_kind[tk_used / 2] = kind;
        tk_used += 2;
        return RC_OK;
    };
    // after a status read: every timed launch of the chunk has completed
    auto tk_collect = [&]() -> int {
        for (size_t q = 0; q < tk_used; q += 2) {
            float t = 0.f;
            HIP_TRY(c, hipEventElapsedTime(&t, c->tk_events[q], c->tk_events[q + 1]));
            if (c->tk_kind[q / 2]) {
                st.sums_ms += t;
            } else {
                st.kernel_ms += t;
                ++st.kernel_launches;
            }
        }
        tk_used = 0;
        return RC_OK;
    };

    const bool logging = buf->ev_log || buf->bonds_log;
    const int lp = opt.log_period;
    // a continued run does not log its first state again when the previous run ended with a row of it
    const DynKey dyn = dyn_key(tmpl);
    const bool kept = opt.keep_list && !opt.resume && prev.valid && prev.N == N && prev.step_end == step0 &&
                      same_buffers(prev.buf, *buf) && std::memcmp(prev.L, tmpl.box.L, sizeof prev.L) == 0 &&
                      std::memcmp(&prev.dyn, &dyn, sizeof dyn) == 0;
    const bool skip_first_row = kept && prev.logged_end && lp > 0;
    auto log_at = [&](uint64_t step) -> bool {
        if (!logging || step < step0) return false;
        if (step == step0 && skip_first_row) return false;
        return lp > 0 && step % (uint64_t)lp == 0;
    };
    auto log_now = [&](int which) -> int {
        if (buf->bonds_log) return ops.bonds(P[which], row);
        return RC_OK;
    };

    // The reset the chunk being queued still owes (chunk markers cleared, replay step counter set): its
    // first direct step launch carries it, so the device starts a run's first chunk on a step instead of
    // a one-thread launch that then waits for the host's next; a graph replay is preceded by its own.
    bool reset_owed = false;
    uint64_t reset_to = 0;
    auto pay_reset = [&]() -> int {
        if (reset_owed) HIP_TRY(c, launch_status_reset_chunk(buf->status, s, c->d_step_base, reset_to));
        reset_owed = false;
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
        if (reset_owed) {
            a.reset_status = buf->status;
            a.reset_base = c->d_step_base;
            a.reset_to = reset_to;
            reset_owed = false;
        }
        if (timing && !ev && (mode == RC_STEP_START || mode == RC_STEP_CONT)) {
            // the plain step launches (log steps and the finishing kick are other work)
            const bool two = ops.graph_sums_fn() != nullptr;
            size_t qk = 0, qs = 0;
            int rr = tk_take(&qk, 0);
            if (!rr && two) rr = tk_take(&qs, 1);
            if (rr) return rr;
            HIP_TRY(c, ops.launch_timed(a, two ? &c->tk_events[qs] : nullptr, &c->tk_events[qk]));
        } else {
            HIP_TRY(c, ops.launch(a, ev));
        }
        if (ev && buf->ev_log) return ops.reduce_ev(row);
        return RC_OK;
    };

    double rate = 0.0;           // growth of the largest path length per step
    float last_maxpath = 0.0f;
    if (kept) {
        // the previous run's list, snapshot and epoch carry over; its overflow check is done
        need_snap = false;
        ep_step = prev.ep_step;
        ep_cur = prev.ep_cur;
        ep_first = prev.ep_first;
        ep_row = 0;               // rows of steps before step0 belong to the previous run
        rate = prev.rate;
        last_maxpath = prev.last_maxpath;
        st.list_kept = 1;
    } else if ((r = rebuild(cur, opt.resume ? kRebuildRetry : kRebuildAll))) {
        return finish(r);
    }

    const float hard = tmpl.hard;
    const bool graphs = opt.use_graph != 0 && !timing;
    const int G = opt.graph_steps;
    const bool blockrun = graphs && opt.one_block != 0 && ops.block_ok();
    if (graphs && !blockrun) {
        StepArgs key = tmpl;
        key.pos_in = reinterpret_cast<const float4*>(buf->pos);
        key.pos_out = reinterpret_cast<float4*>(buf->pos_alt);
        const void* fn = ops.graph_fn();
        if (!c->gc.valid || c->gc.steps != G || c->gc.fn != fn || !same_args(c->gc.key, key)) {
            if ((r = build_graphs(c, fn, ops.graph_sums_fn(), key, G, s))) return finish(r);
        }
    }
    uint64_t dev_base = ~0ull;   // value *d_step_base will hold once queued work ran

    // Graph replays pay a step-counter node and a wait at each end; direct launches cost the host
    // 7-14 us each.  A system of 2^19 particles or more takes longer per step than that, so its
    // launches keep ahead of the device, and a stretch of fewer than two replays runs directly (20-step
    // runs of 2^20 particles: 6-7 us less per run than with one replay, paired medians over 18 runs;
    // long runs and smaller systems keep the replays: 12.9 against 14.6 us per step at 2048 particles).
    const bool big = (int64_t)N >= (int64_t)1 << 19;
    // run `count` steps from the state at absolute step `from` (in P[cur])
    auto run_steps = [&](uint64_t from, int64_t count) -> int {
        const bool replays = graphs && (count >= 2 * (int64_t)G || !big);
        int64_t k = 0;
        while (k < count) {
            const uint64_t step = from + (uint64_t)k;
            const bool ev = log_at(step);
            if (ev) {
                int rr = log_now(cur);
                if (rr) return rr;
            }
            if (replays && !first && !ev && count - k >= G) {
                // a graph replay must not cross a logging step
                bool clear = true;
                for (int64_t q = 1; q < G && clear; ++q) clear = !log_at(step + (uint64_t)q);
                if (clear) {
                    int rr = pay_reset();
                    if (rr) return rr;
                    if (dev_base != step) HIP_TRY(c, launch_set_step(c->d_step_base, step, s));
                    if (blockrun) {
                        StepArgs a = tmpl;
                        a.pos_in = reinterpret_cast<const float4*>(P[cur]);
                        a.pos_out = reinterpret_cast<float4*>(P[cur ^ 1]);
                        a.mode = RC_STEP_CONT;
                        a.step = 0;
                        a.step_base = c->d_step_base;
                        a.ev_part = nullptr;
                        HIP_TRY(c, ops.launch_block(a, reinterpret_cast<float4*>(P[cur]), G));
                    } else {
                        HIP_TRY(c, hipGraphLaunch(c->gc.exec[cur], s));
                    }
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

    // The run's finishing work: the bond count of the final state, the final half kick with the last
    // log row, the positions back into buf->pos.
    auto finishing = [&]() -> int {
        const bool ev = logging && buf->ev_log;
        int rr;
        if (logging && (rr = log_now(cur))) return rr;
        if (!first) {
            if ((rr = direct(s_end, RC_STEP_FINISH, ev))) return rr;
        } else if (ev) {
            // zero steps: report the state as it is
            if ((rr = direct(step0, RC_STEP_OBSERVE, ev))) return rr;
        }
        if (logging) ++row;
        if (cur != 0) HIP_TRY(c, hipMemcpyAsync(buf->pos, P[cur], 16 * (size_t)N, hipMemcpyDeviceToDevice, s));
        return RC_OK;
    };
    bool finished = false;   // the finishing work ran with the last chunk and its status read confirmed it

    bool first_chunk = true;
    while (s_cur < s_end) {
        // ---- plan the chunk ---------------------------------------------------
        int64_t C = std::min<int64_t>((int64_t)(s_end - s_cur), opt.max_chunk);
        if (!can_roll) C = 1;
        else if (!opt.adapt) {
            // fixed chunks: stale chunks are rolled back
        } else if (rate > 0.0) {
            // end the chunk well before the stale threshold: a rollback replays the whole epoch
            // (~1.4 ms at 1M particles), far more than one more chunk's host wait; aiming the
            // end between the rebuild and stale thresholds (one chunk per epoch) rolled back
            // about once per thousand steps and was slower
            const double room = (double)hard - (double)last_maxpath;
            const int64_t safe = (int64_t)std::floor(room / (1.5 * rate));
            C = std::max<int64_t>(1, std::min<int64_t>(C, safe));
        } else if (first_chunk) {
            C = std::min<int64_t>(C, 8);
        }
        first_chunk = false;
        const uint64_t chunk_start = s_cur;
        if (can_roll && need_snap) {
            if (!snap_in_ws)
                HIP_TRY(c, launch_copy_state(reinterpret_cast<const float4*>(P[cur]),
                                             reinterpret_cast<const float4*>(buf->vel),
                                             reinterpret_cast<const int4*>(buf->image),
                                             reinterpret_cast<float4*>(buf->snap_pos),
                                             reinterpret_cast<float4*>(buf->snap_vel),
                                             reinterpret_cast<int4*>(buf->snap_image), N, s));
            ep_step = s_cur;
            ep_cur = cur;
            ep_first = first;
            ep_row = row;
            need_snap = false;
        }
        // one launch clears the chunk markers and sets the replays' step counter (to the chunk's second
        // step when its first is launched directly: a run's first step or a log step)
        const uint64_t base0 = chunk_start + ((first || log_at(chunk_start)) ? 1 : 0);
        reset_owed = true;
        reset_to = base0;
        dev_base = base0;
        // ---- run it --------------------------------------------------------------
        if ((r = run_steps(chunk_start, C))) return finish(r);
        if ((r = pay_reset())) return finish(r);
        HIP_TRY(c, ops.fold(c->d_blk, nb, reinterpret_cast<const float4*>(buf->vel), N, buf->status, s));
        // The run's last chunk queues the finishing work before its status read, so that one host wait
        // covers both.  The read confirms it when no force of the chunk or of the finishing step was
        // evaluated on a stale list (MAXPATH, the largest path length of the final state, at most the
        // stale threshold); otherwise the chunk is rolled back and replayed as below, which undoes it.
        // Only a chunk the planner expects to stay below the rebuild threshold speculates (adaptive
        // chunks with a measured growth rate), so a fallback is rare and the run's build schedule is
        // the one without speculation.
        const bool spec = can_roll && !timing && opt.adapt && rate > 0.0 && chunk_start + (uint64_t)C == s_end &&
                          (double)last_maxpath + 1.5 * rate * (double)C < (double)tmpl.soft;
        if (spec && (r = finishing())) return finish(r);
        if ((r = read_status_spin(c, buf->status, hst, s))) return finish(r);
        if (timing && (r = tk_collect())) return finish(r);
        ++st.chunks;
        const int f = hst[RC_ST_FLAGS];
        check_pending = false;
        if (f & RC_FLAG_NLIST_OVERFLOW) {
            // the epoch ran on a truncated list (it began at a build of this run, whose
            // check was deferred): back to its start, which the caller resumes
            cur = ep_cur;
            first = ep_first;
            row = ep_row;
            HIP_TRY(c, launch_copy_state(ws_pos, ws_vel, buf->image ? ws_image : nullptr,
                                         reinterpret_cast<float4*>(P[cur]), reinterpret_cast<float4*>(buf->vel),
                                         reinterpret_cast<int4*>(buf->image), N, s));
            s_cur = ep_step;
            return finish(overflow());
        }
        if (f & RC_FLAG_LOST) return finish(fail(c, RC_ERR_LOST_PARTICLE, "a particle moved more than L/2 in one step"));
        if (f & RC_FLAG_NONFINITE) return finish(fail(c, RC_ERR_NONFINITE, "non-finite position or velocity"));
        float mp;
        std::memcpy(&mp, &hst[RC_ST_MAXPATH], sizeof mp);
        if ((f & RC_FLAG_STALE) || (spec && mp > hard)) {
            if (!can_roll) return finish(fail(c, RC_ERR_ARG, "stale list without rollback buffers"));
            // roll back to the epoch's snapshot and replay up to the first soft crossing, then rebuild
            cur = ep_cur;
            first = ep_first;
            row = ep_row;
            if (snap_in_ws)   // the state the epoch's list build left (its path lengths included)
                HIP_TRY(c, launch_copy_state(ws_pos, ws_vel, buf->image ? ws_image : nullptr,
                                             reinterpret_cast<float4*>(P[cur]), reinterpret_cast<float4*>(buf->vel),
                                             reinterpret_cast<int4*>(buf->image), N, s));
            else
                HIP_TRY(c, launch_copy_state(reinterpret_cast<const float4*>(buf->snap_pos),
                                             reinterpret_cast<const float4*>(buf->snap_vel),
                                             reinterpret_cast<const int4*>(buf->snap_image),
                                             reinterpret_cast<float4*>(P[cur]), reinterpret_cast<float4*>(buf->vel),
                                             reinterpret_cast<int4*>(buf->image), N, s));
            const int64_t soft_step = (int64_t)hst[RC_ST_FIRST_SOFT];
            int64_t n_re = soft_step - (int64_t)(ep_step & 0x7fffffff) + 1;
            n_re = std::max<int64_t>(1, std::min<int64_t>(n_re, (int64_t)(chunk_start + C - ep_step)));
            HIP_TRY(c, launch_status_reset_chunk(buf->status, s, c->d_step_base, ep_step));
            dev_base = ep_step;
            if ((r = run_steps(ep_step, n_re))) return finish(r);
            if (ops.read_after_replay()) {   // the replay's own flags and path lengths choose the set
                HIP_TRY(c, ops.fold(c->d_blk, nb, reinterpret_cast<const float4*>(buf->vel), N, buf->status, s));
                if ((r = read_status_spin(c, buf->status, hst, s))) return finish(r);
            } else {
                HIP_TRY(c, launch_fold_status(c->d_blk, nb, nullptr, N, buf->status, s));  // drop replay flags
            }
            s_cur = ep_step + (uint64_t)n_re;
            ++st.rollbacks;
            if ((r = rebuild(cur, kRebuildFlagged))) return finish(r);
            rate = std::max(rate, (double)mp / std::max<int64_t>(1, C));
            last_maxpath = kept_path;
            continue;
        }
        s_cur = chunk_start + (uint64_t)C;
        double growth = 0.0;
        if (!ops.path_growth(C, &growth)) growth = (double)(mp - last_maxpath) / (double)C;
        rate = std::max(0.5 * rate, growth);
        last_maxpath = mp;
        if (spec) {   // done; a rebuild the flags ask for is left to the next run on this list
            finished = true;
            break;
        }
        if (f & RC_FLAG_REBUILD) {
            if ((r = rebuild(cur, kRebuildFlagged))) return finish(r);
            last_maxpath = kept_path;
        }
    }
    // ---- final half kick (and the last log row), unless the last chunk did it ----------
    if (!finished) {
        if (check_pending) {  // the list of the last build has not been checked yet
            if ((r = read_status_spin(c, buf->status, hst, s))) return finish(r);
            check_pending = false;
            if (hst[RC_ST_FLAGS] & RC_FLAG_NLIST_OVERFLOW)
                return finish(overflow());  // all steps done, the final half kick still due
        }
        if (need_snap) {   // a build after the last chunk: its state owes the final half kick
            ep_step = s_cur;
            ep_cur = cur;
            ep_first = false;
            need_snap = false;
        }
        if ((r = finishing())) return finish(r);
        // the status read waits for all of the run's work (pinned copy and an event, no blocking sync)
        if ((r = read_status_spin(c, buf->status, hst, s))) return finish(r);
        if (timing && (r = tk_collect())) return finish(r);
    }
    // what the next run needs to continue on this list
    c->md.valid = can_roll;
    c->md.dyn = dyn;
    c->md.buf = *buf;
    c->md.N = N;
    std::memcpy(c->md.L, tmpl.box.L, sizeof c->md.L);
    c->md.step_end = s_end;
    c->md.ep_step = ep_step;
    c->md.ep_cur = ep_cur;
    c->md.ep_first = ep_first;
    c->md.rate = rate;
    c->md.last_maxpath = last_maxpath;
    c->md.logged_end = logging;
    return finish(RC_OK);
}

}  // namespace host
}  // namespace rc
