// C ABI of the batch mode: many independent replicas (uneven size, box and
// table) behind one set of launches per step.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "rc_host.h"

using namespace rc;
using namespace rc::host;

struct rc_batch {
    rc_ctx c;                     // error text, tables, partial rows, status slots, graphs
    int R = 0;
    int n_slots = 0;
    uint32_t nkeys = 0;
    std::vector<int> counts;
    std::vector<int> offsets;     // [R + 1]
    std::vector<RepDesc> desc;
    std::vector<uint64_t> seeds;  // host copy of d_seeds
    bool seeds_set = false;
    RepDesc* d_desc = nullptr;
    int* d_chunk_rep = nullptr;
    uint32_t* d_key_end = nullptr;
    uint64_t* d_seeds = nullptr;
    // per-replica rebuilds: the fold of every chunk writes, per replica, whether a block crossed the
    // rebuild threshold and the largest path length (d_rep: [2][R] ints), which every status read
    // copies to h_rep; a build re-orders and re-lists the replicas of its set (d_build [R])
    double margin = 0.3;
    int* d_rep = nullptr;
    int* h_rep = nullptr;            // pinned [2][R]
    int* d_build = nullptr;
    float* d_chunk_path = nullptr;   // [n_slots / 64] scratch of the fold
    int* h_build[2] = {nullptr, nullptr};   // pinned [R] sets, alternating between builds
    int build_parity = 0;
    std::vector<int> last_set;       // the set of the last build of a run (a resumed run's first)
    std::vector<float> prev_path;    // per replica: its largest path length at the previous fold (0 after a build)
};

namespace {

void free_batch(rc_batch* b) {
    free_ctx_buffers(&b->c);
    if (b->d_rep) (void)hipFree(b->d_rep);
    if (b->d_build) (void)hipFree(b->d_build);
    if (b->d_chunk_path) (void)hipFree(b->d_chunk_path);
    if (b->h_rep) (void)hipHostFree(b->h_rep);
    for (int q = 0; q < 2; ++q)
        if (b->h_build[q]) (void)hipHostFree(b->h_build[q]);
    if (b->d_desc) (void)hipFree(b->d_desc);
    if (b->d_chunk_rep) (void)hipFree(b->d_chunk_rep);
    if (b->d_key_end) (void)hipFree(b->d_key_end);
    if (b->d_seeds) (void)hipFree(b->d_seeds);
    delete b;
}

int check_pos(rc_batch* b, const void* pos) {
    if (!pos) return fail(&b->c, RC_ERR_ARG, "positions are NULL");
    if (reinterpret_cast<uintptr_t>(pos) & 15) return fail(&b->c, RC_ERR_ARG, "positions not 16-byte aligned");
    return RC_OK;
}

Table all_tables(const rc_batch* b) { return Table{b->c.d_tab, b->c.nt}; }

// seeds of the next launches: the ones set, else cfg.seed + r
int ensure_seeds(rc_batch* b, const rc_integrator* cfg, hipStream_t s) {
    if (b->seeds_set) return RC_OK;
    std::vector<uint64_t> want(b->R);
    for (int r = 0; r < b->R; ++r) want[r] = cfg->seed + (uint64_t)r;
    if (want == b->seeds) return RC_OK;
    HIP_TRY(&b->c, hipStreamSynchronize(s));
    HIP_TRY(&b->c, hipMemcpy(b->d_seeds, want.data(), sizeof(uint64_t) * b->R, hipMemcpyHostToDevice));
    b->seeds = want;
    return RC_OK;
}

int fill_step_args_batch(rc_batch* b, StepArgs& a, const float* pos_in, float* pos_out, float* vel, int* image,
                         const int* nlist, const int* nn, int k_max, const rc_integrator* cfg, double soft_frac,
                         int* status, hipStream_t s, bool pack = true) {
    rc_ctx* c = &b->c;
    float c1;
    int lang;
    int r = check_integrator(c, cfg, a.minv, a.c2, c1, lang, a.noise_z);
    if (r) return r;
    if ((r = check_list(c, nlist, nn, k_max))) return r;
    if ((r = ensure_seeds(b, cfg, s))) return r;
    a.pos_in = reinterpret_cast<const float4*>(pos_in);
    a.pos_out = reinterpret_cast<float4*>(pos_out);
    a.vel = reinterpret_cast<float4*>(vel);
    a.image = reinterpret_cast<int4*>(image);
    a.nlist = nlist;
    a.nn = nn;
    a.k_max = k_max;
    a.N = b->n_slots;
    a.tab = all_tables(b);
    a.dt = (float)cfg->dt;
    a.c1 = c1;
    a.langevin = lang;
    a.hard = (float)(0.5 * c->r_buff);
    a.soft = (float)(0.5 * c->r_buff * soft_frac);
    a.seed = 0;
    a.status = status;
    a.rep = b->d_desc;
    a.chunk_rep = b->d_chunk_rep;
    a.seeds = b->d_seeds;
    a.width = c->gather_width;
    a.form = c->step_form;
    a.ssum = nullptr;
    if (a.form == RC_FORM_SUMS) {
        if ((r = ensure_ssum(c, (size_t)b->n_slots))) return r;
        a.ssum = c->d_ssum;
    }
    if ((r = ensure_blk(c, nblocks(b->n_slots, kStepBlock), nullptr))) return r;
    a.blk = c->d_blk;
    // the packed copy of the list (the driver's first list build makes it: pack = false)
    if ((r = pack ? packed_list_for(c, nlist, nn, k_max, b->n_slots, s) : ensure_plist(c, b->n_slots, k_max)))
        return r;
    a.pl_j = c->d_pl_j;
    a.pl_o = c->d_pl_o;
    return RC_OK;
}

}  // namespace

extern "C" {

int rc_batch_create(rc_batch** out, int R, int ntypes, const rc_pair_coeff* tables, const int* counts,
                    const rc_box* boxes, double r_buff) {
    if (!out) return RC_ERR_ARG;
    *out = nullptr;
    if (R < 1 || ntypes < 1 || !tables || !counts || !boxes) return RC_ERR_ARG;
    if (ntypes > RC_MAX_TYPES || R > 65535) return RC_ERR_UNSUPPORTED;
    if (!(r_buff > 0.0) || !std::isfinite(r_buff)) return RC_ERR_ARG;
    rc_batch* b = new (std::nothrow) rc_batch();
    if (!b) return RC_ERR_ARG;
    rc_ctx* c = &b->c;
    const int nt2 = ntypes * ntypes;
    c->nt = ntypes;
    c->r_buff = r_buff;
    c->host_tab.resize((size_t)R * nt2);
    b->R = R;
    b->counts.assign(counts, counts + R);
    b->offsets.resize(R + 1);
    b->desc.resize(R);
    int64_t slots = 0;
    uint64_t keys = 0;
    double rmax_all = 0.0;
    for (int r = 0; r < R; ++r) {
        double rl = 0.0;
        if (compile_table(ntypes, tables + (size_t)r * nt2, r_buff, c->host_tab.data() + (size_t)r * nt2, &rl,
                          nullptr) != RC_OK || counts[r] < 1) {
            free_batch(b);
            return RC_ERR_ARG;
        }
        rmax_all = std::max(rmax_all, rl);
        RepDesc& d = b->desc[r];
        if (make_box(c, boxes[r], d.box) || make_grid(c, rl, d.box, d.grid)) {
            free_batch(b);
            return RC_ERR_ARG;
        }
        d.key_base = (uint32_t)keys;
        d.off = (int)slots;
        d.n = counts[r];
        d.tab = r * nt2;
        b->offsets[r] = (int)slots;
        keys += d.grid.nkeys;
        slots += (int64_t)kWave * ((counts[r] + kWave - 1) / kWave);
        if (slots >= RC_MAX_TAG || keys > (uint64_t)8192 * kScanTile) {
            free_batch(b);
            return RC_ERR_UNSUPPORTED;
        }
    }
    b->offsets[R] = (int)slots;
    b->n_slots = (int)slots;
    b->nkeys = (uint32_t)keys;
    c->rlist_max = rmax_all;
    std::vector<int> chunk_rep(slots / kWave);
    std::vector<uint32_t> key_end(R);
    for (int r = 0; r < R; ++r) {
        for (int q = b->offsets[r] / kWave; q < b->offsets[r + 1] / kWave; ++q) chunk_rep[q] = r;
        key_end[r] = b->desc[r].key_base + b->desc[r].grid.nkeys;
    }
    b->seeds.assign(R, 0);
    bool ok = hipGetDevice(&c->device) == hipSuccess &&
              hipMalloc(&c->d_tab, sizeof(DevEntry) * (size_t)R * nt2) == hipSuccess &&
              hipMemcpy(c->d_tab, c->host_tab.data(), sizeof(DevEntry) * (size_t)R * nt2, hipMemcpyHostToDevice) ==
                  hipSuccess &&
              hipMalloc(&c->d_step_base, sizeof(unsigned long long)) == hipSuccess &&
              hipMalloc(&b->d_desc, sizeof(RepDesc) * R) == hipSuccess &&
              hipMemcpy(b->d_desc, b->desc.data(), sizeof(RepDesc) * R, hipMemcpyHostToDevice) == hipSuccess &&
              hipMalloc(&b->d_chunk_rep, sizeof(int) * chunk_rep.size()) == hipSuccess &&
              hipMemcpy(b->d_chunk_rep, chunk_rep.data(), sizeof(int) * chunk_rep.size(), hipMemcpyHostToDevice) ==
                  hipSuccess &&
              hipMalloc(&b->d_key_end, sizeof(uint32_t) * R) == hipSuccess &&
              hipMemcpy(b->d_key_end, key_end.data(), sizeof(uint32_t) * R, hipMemcpyHostToDevice) == hipSuccess &&
              hipMalloc(&b->d_seeds, sizeof(uint64_t) * R) == hipSuccess &&
              hipMemcpy(b->d_seeds, b->seeds.data(), sizeof(uint64_t) * R, hipMemcpyHostToDevice) == hipSuccess &&
              hipMalloc(&b->d_rep, sizeof(int) * 2 * (size_t)R) == hipSuccess &&
              hipMemset(b->d_rep, 0, sizeof(int) * 2 * (size_t)R) == hipSuccess &&
              hipMalloc(&b->d_build, sizeof(int) * (size_t)R) == hipSuccess &&
              hipMalloc(&b->d_chunk_path, sizeof(float) * (size_t)(slots / kWave)) == hipSuccess &&
              hipHostMalloc(reinterpret_cast<void**>(&b->h_rep), sizeof(int) * 2 * (size_t)R) == hipSuccess &&
              hipHostMalloc(reinterpret_cast<void**>(&b->h_build[0]), sizeof(int) * (size_t)R) == hipSuccess &&
              hipHostMalloc(reinterpret_cast<void**>(&b->h_build[1]), sizeof(int) * (size_t)R) == hipSuccess;
    if (!ok) {
        free_batch(b);
        return RC_ERR_HIP;
    }
    std::memset(b->h_rep, 0, sizeof(int) * 2 * (size_t)R);
    c->status_extra.push_back({b->h_rep, b->d_rep, sizeof(int) * 2 * (size_t)R});
    *out = b;
    return RC_OK;
}

int rc_batch_destroy(rc_batch* b) {
    if (!b) return RC_ERR_ARG;
    free_batch(b);
    return RC_OK;
}

const char* rc_batch_last_error(const rc_batch* b) { return b ? b->c.err.c_str() : "null batch"; }

int rc_batch_layout(const rc_batch* b, int* n_slots, int* offsets) {
    if (!b || !n_slots) return RC_ERR_ARG;
    *n_slots = b->n_slots;
    if (offsets) std::memcpy(offsets, b->offsets.data(), sizeof(int) * (b->R + 1));
    return RC_OK;
}

int rc_batch_set_seeds(rc_batch* b, const uint64_t* seeds) {
    if (b) b->c.md.valid = false;   // a replay into the last run's steps would use other noise
    if (!b || !seeds) return RC_ERR_ARG;
    HIP_TRY(&b->c, hipDeviceSynchronize());
    HIP_TRY(&b->c, hipMemcpy(b->d_seeds, seeds, sizeof(uint64_t) * b->R, hipMemcpyHostToDevice));
    b->seeds.assign(seeds, seeds + b->R);
    b->seeds_set = true;
    return RC_OK;
}

int rc_batch_workspace_bytes(const rc_batch* b, int k_max, size_t* bytes) {
    if (!b) return RC_ERR_ARG;
    return rc_workspace_bytes(&b->c, b->n_slots, k_max, 0, bytes);
}

int rc_batch_set_workspace(rc_batch* b, void* ws, size_t bytes, int k_max) {
    if (!b) return RC_ERR_ARG;
    return set_workspace(&b->c, ws, bytes, b->n_slots, k_max, 0);
}

int rc_batch_set_gather_width(rc_batch* b, int width) {
    if (!b) return RC_ERR_ARG;
    if (width != 1 && width != 2 && width != 4) return fail(&b->c, RC_ERR_ARG, "gather width must be 1, 2 or 4");
    b->c.gather_width = width;
    return RC_OK;
}

int rc_batch_set_step_form(rc_batch* b, int form) {
    if (!b) return RC_ERR_ARG;
    if (form != RC_FORM_WALK && form != RC_FORM_SUMS)
        return fail(&b->c, RC_ERR_ARG, "unknown step form %d", form);
    b->c.step_form = form;
    return RC_OK;
}

int rc_batch_cells_workspace_bytes(const rc_batch* b, size_t* bytes) {
    if (!b || !bytes) return RC_ERR_ARG;
    *bytes = cells_layout(b->n_slots, b->nkeys).total;
    return RC_OK;
}

static int batch_build_cells(rc_batch* b, float* pos, float* vel, int* image, int* rtag, void* ws, size_t ws_bytes,
                             const int* build, void* stream) {
    int r = check_pos(b, pos);
    if (r) return r;
    const CellsLayout l = cells_layout(b->n_slots, b->nkeys);
    if (!ws || ws_bytes < l.total) return fail(&b->c, RC_ERR_WORKSPACE, "cells workspace needs %zu bytes", l.total);
    char* w = static_cast<char*>(ws);
    CellsArgsB a{};
    a.pos = reinterpret_cast<float4*>(pos);
    a.vel = reinterpret_cast<float4*>(vel);
    a.image = reinterpret_cast<int4*>(image);
    a.rtag = rtag;
    a.N = b->n_slots;
    a.rep = b->d_desc;
    a.chunk_rep = b->d_chunk_rep;
    a.key_end = b->d_key_end;
    a.R = b->R;
    a.nkeys = b->nkeys;
    a.counts = reinterpret_cast<int*>(w + l.counts);
    a.cell_start = reinterpret_cast<int*>(w + l.start);
    a.keys = reinterpret_cast<int*>(w + l.keys);
    a.rank = reinterpret_cast<int*>(w + l.rank);
    a.order = reinterpret_cast<int*>(w + l.order);
    a.block_sums = reinterpret_cast<int*>(w + l.bsums);
    a.tpos = reinterpret_cast<float4*>(w + l.tpos);
    a.tvel = reinterpret_cast<float4*>(w + l.tvel);
    a.timage = reinterpret_cast<int4*>(w + l.timage);
    a.build = build;
    HIP_TRY(&b->c, launch_cells_batch(a, S(stream)));
    return RC_OK;
}

int rc_batch_build_cells(rc_batch* b, float* pos, float* vel, int* image, int* rtag, void* ws, size_t ws_bytes,
                         void* stream) {
    if (b) b->c.md.valid = false;   // the state or the list changes outside the driver
    if (!b) return RC_ERR_ARG;
    return batch_build_cells(b, pos, vel, image, rtag, ws, ws_bytes, nullptr, stream);
}

// fresh: the status words are written whole (the driver's rebuilds), else folded into
static int batch_build_nlist(rc_batch* b, const float* pos, float* vel, const void* ws, size_t ws_bytes, int k_max,
                             int* nlist, int* nn, int* status, bool fresh, const int* build, void* stream) {
    if (!b) return RC_ERR_ARG;
    int r = check_pos(b, pos);
    if (r) return r;
    if ((r = check_list(&b->c, nlist, nn, k_max))) return r;
    const CellsLayout l = cells_layout(b->n_slots, b->nkeys);
    if (!ws || ws_bytes < l.total) return fail(&b->c, RC_ERR_WORKSPACE, "cells workspace needs %zu bytes", l.total);
    NlistArgsB a{};
    a.pos = reinterpret_cast<const float4*>(pos);
    a.vel = reinterpret_cast<float4*>(vel);
    a.N = b->n_slots;
    a.rep = b->d_desc;
    a.chunk_rep = b->d_chunk_rep;
    a.tab = all_tables(b);
    a.cell_start = reinterpret_cast<const int*>(static_cast<const char*>(ws) + l.start);
    a.k_max = k_max;
    a.nlist = nlist;
    a.nn = nn;
    a.status = status;
    a.fresh_status = fresh ? 1 : 0;
    a.build = build;
    a.block_max = reinterpret_cast<int*>(static_cast<char*>(const_cast<void*>(ws)) + l.bmax);
    rc_ctx* c = &b->c;
    if ((r = ensure_plist(c, b->n_slots, k_max))) return r;
    a.pl_j = c->d_pl_j;  // the packed copy the fused step reads, made in the same launch
    a.pl_o = c->d_pl_o;
    HIP_TRY(c, launch_nlist_batch(a, S(stream)));
    c->pl_nlist = nlist;
    c->pl_nn = nn;
    c->pl_k = k_max;
    c->pl_n = b->n_slots;
    return RC_OK;
}

int rc_batch_build_nlist(rc_batch* b, const float* pos, float* vel, const void* ws, size_t ws_bytes, int k_max,
                         int* nlist, int* nn, int* status, void* stream) {
    if (b) b->c.md.valid = false;   // the state or the list changes outside the driver
    return batch_build_nlist(b, pos, vel, ws, ws_bytes, k_max, nlist, nn, status, false, nullptr, stream);
}

int rc_batch_set_rebuild_margin(rc_batch* b, double margin) {
    if (!b) return RC_ERR_ARG;
    if (!(margin >= 0.0 && margin <= 1.0)) return fail(&b->c, RC_ERR_ARG, "rebuild margin must be in [0, 1]");
    b->margin = margin;
    return RC_OK;
}

int rc_batch_relayout_lists(rc_batch* b, const int* old_nlist, int k_old, int* new_nlist, int k_new, const int* nn,
                            void* stream) {
    if (!b) return RC_ERR_ARG;
    rc_ctx* c = &b->c;
    int r = check_list(c, new_nlist, nn, k_new);
    if (r) return r;
    if (!old_nlist || k_old < 1 || k_old > k_new || old_nlist == new_nlist)
        return fail(c, RC_ERR_ARG, "relayout needs a distinct old list with 1 <= k_old <= k_new");
    if ((r = ensure_plist(c, b->n_slots, k_new))) return r;
    HIP_TRY(c, launch_relayout_list(old_nlist, k_old, new_nlist, k_new, nn, b->n_slots, c->d_pl_j, c->d_pl_o,
                                    S(stream)));
    c->pl_nlist = new_nlist;
    c->pl_nn = nn;
    c->pl_k = k_new;
    c->pl_n = b->n_slots;
    return RC_OK;
}

int rc_batch_compute_forces(rc_batch* b, const float* pos, const int* nlist, const int* nn, int k_max, float* force,
                            double* ev, int* status, void* stream) {
    if (!b) return RC_ERR_ARG;
    rc_ctx* c = &b->c;
    int r = check_pos(b, pos);
    if (r) return r;
    if (!force) return fail(c, RC_ERR_ARG, "force is NULL");
    if ((r = check_list(c, nlist, nn, k_max))) return r;
    const int nb = nblocks(b->n_slots, kWave);
    if (ev && (r = ensure_part(c, sizeof(double) * kEvWords * (size_t)nb))) return r;
    ForceArgs a{};
    a.pos = reinterpret_cast<const float4*>(pos);
    a.nlist = nlist;
    a.nn = nn;
    a.k_max = k_max;
    a.N = b->n_slots;
    a.tab = all_tables(b);
    a.force = reinterpret_cast<float4*>(force);
    a.ev_part = ev ? c->d_part : nullptr;
    a.accumulate = 0;
    a.status = status;
    a.rep = b->d_desc;
    a.chunk_rep = b->d_chunk_rep;
    a.ssum = nullptr;
    if (c->step_form == RC_FORM_SUMS) {
        if ((r = ensure_ssum(c, (size_t)b->n_slots))) return r;
        a.ssum = c->d_ssum;
    }
    hipStream_t s = S(stream);
    HIP_TRY(c, launch_forces_gather_batch(a, s));
    if (ev) HIP_TRY(c, launch_reduce_rows_batch(c->d_part, b->d_desc, b->R, 0, 7, ev, 7, s));
    return RC_OK;
}

int rc_batch_bond_count(rc_batch* b, const float* pos, const int* nlist, const int* nn, int k_max,
                        unsigned long long* counts, void* stream) {
    if (!b) return RC_ERR_ARG;
    rc_ctx* c = &b->c;
    int r = check_pos(b, pos);
    if (r) return r;
    if (!counts) return fail(c, RC_ERR_ARG, "counts is NULL");
    if ((r = check_list(c, nlist, nn, k_max))) return r;
    if ((r = ensure_part(c, sizeof(unsigned long long) * (size_t)nblocks(b->n_slots, kWave)))) return r;
    HIP_TRY(c, launch_bonds_batch(reinterpret_cast<const float4*>(pos), nlist, nn, k_max, b->n_slots, all_tables(b),
                                  b->d_desc, b->d_chunk_rep, b->R, counts,
                                  reinterpret_cast<unsigned long long*>(c->d_part), S(stream)));
    return RC_OK;
}

int rc_batch_step_fused(rc_batch* b, const float* pos_in, float* pos_out, float* vel, int* image, const int* nlist,
                        const int* nn, int k_max, const rc_integrator* cfg, uint64_t step, int mode, double soft_frac,
                        double* ev, int* status, void* stream) {
    if (b) b->c.md.valid = false;   // the state or the list changes outside the driver
    if (!b) return RC_ERR_ARG;
    rc_ctx* c = &b->c;
    int r = check_pos(b, pos_in);
    if (r) return r;
    if (!vel || !status) return fail(c, RC_ERR_ARG, "vel / status are NULL");
    if ((mode == RC_STEP_START || mode == RC_STEP_CONT) && (!pos_out || pos_out == pos_in))
        return fail(c, RC_ERR_ARG, "pos_out must be a second buffer");
    if (mode < RC_STEP_START || mode > RC_STEP_OBSERVE) return fail(c, RC_ERR_ARG, "bad mode");
    if (!(soft_frac > 0.0 && soft_frac <= 1.0)) return fail(c, RC_ERR_ARG, "soft_frac must be in (0, 1]");
    hipStream_t s = S(stream);
    StepArgs a{};
    if ((r = fill_step_args_batch(b, a, pos_in, pos_out, vel, image, nlist, nn, k_max, cfg, soft_frac, status, s)))
        return r;
    const int nb = nblocks(b->n_slots, kStepBlock);
    if (ev && (r = ensure_part(c, sizeof(double) * kEvWords * (size_t)nb))) return r;
    a.mode = mode;
    a.step = step;
    a.step_base = nullptr;
    a.ev_part = ev ? c->d_part : nullptr;
    HIP_TRY(c, launch_step_batch(a, ev != nullptr, s));
    HIP_TRY(c, launch_fold_status(c->d_blk, nb, nullptr, b->n_slots, status, s));
    if (ev) HIP_TRY(c, launch_reduce_rows_batch(c->d_part, b->d_desc, b->R, 0, kEvWords, ev, kEvWords, s));
    return RC_OK;
}

int rc_batch_time_fused_steps(rc_batch* b, float* pos_a, float* pos_b, float* vel, const int* nlist, const int* nn,
                              int k_max, const rc_integrator* cfg, uint64_t step0, int reps, int* status, float* ms,
                              void* stream) {
    if (b) b->c.md.valid = false;   // the state or the list changes outside the driver
    if (!b) return RC_ERR_ARG;
    rc_ctx* c = &b->c;
    int r = check_pos(b, pos_a);
    if (r) return r;
    if (!pos_b || pos_b == pos_a || !vel || !status || !ms || reps < 1)
        return fail(c, RC_ERR_ARG, "bad arguments to rc_batch_time_fused_steps");
    hipStream_t s = S(stream);
    StepArgs a{};
    if ((r = fill_step_args_batch(b, a, pos_a, pos_b, vel, nullptr, nlist, nn, k_max, cfg, 0.8, status, s))) return r;
    a.mode = RC_STEP_CONT;
    a.step_base = nullptr;
    a.ev_part = nullptr;
    hipEvent_t e0, e1;
    HIP_TRY(c, hipEventCreate(&e0));
    HIP_TRY(c, hipEventCreate(&e1));
    float4* P[2] = {reinterpret_cast<float4*>(pos_a), reinterpret_cast<float4*>(pos_b)};
    hipError_t err = hipEventRecord(e0, s);
    for (int k = 0; k < reps && err == hipSuccess; ++k) {
        a.pos_in = P[k & 1];
        a.pos_out = P[(k + 1) & 1];
        a.step = step0 + (uint64_t)k;
        err = launch_step_batch(a, false, s);
    }
    if (err == hipSuccess) err = hipEventRecord(e1, s);
    if (err == hipSuccess) err = launch_fold_status(c->d_blk, nblocks(b->n_slots, kStepBlock), nullptr, b->n_slots,
                                                    status, s);
    if (err == hipSuccess) err = hipEventSynchronize(e1);
    if (err == hipSuccess) err = hipEventElapsedTime(ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (err != hipSuccess) return hip_fail(c, err, "rc_batch_time_fused_steps");
    return RC_OK;
}

}  // extern "C"

namespace {

struct BatchOps final : DriveOps {
    rc_batch* b;
    const rc_md_buffers* buf;
    hipStream_t s;
    float soft = 0.0f;   // the rebuild threshold of the path lengths
    // The set of replicas a build re-orders and re-lists, from the last status read's per-replica
    // fold: those with a block that crossed the rebuild threshold and those whose largest path
    // length exceeds margin x that threshold.  Uploaded from a pinned buffer (the two buffers
    // alternate; a status read, which waits for the stream, separates two builds).
    int rebuild(float* pos, RebuildKind kind, float* kept_path, int64_t* rebuilt) override {
        const int R = b->R;
        int* set = b->h_build[b->build_parity];
        b->build_parity ^= 1;
        const int* flag = b->h_rep;
        const int* path = b->h_rep + R;
        float kp = 0.0f;
        int64_t nre = 0;
        const bool retry = kind == kRebuildRetry && (int)b->last_set.size() == R;
        for (int r = 0; r < R; ++r) {
            int on = 1;
            if (retry) {
                on = b->last_set[r];
            } else if (kind == kRebuildFlagged) {
                float pr;
                std::memcpy(&pr, &path[r], sizeof pr);
                on = flag[r] != 0 || pr > (float)b->margin * soft;
                if (!on) kp = std::max(kp, pr);
            }
            set[r] = on;
            if (on) nre += b->counts[r];
        }
        if (kind == kRebuildFlagged || retry) b->last_set.assign(set, set + R);
        else b->last_set.clear();   // a full build: a retry rebuilds everything
        if ((int)b->prev_path.size() != R) b->prev_path.assign(R, 0.0f);
        for (int r = 0; r < R; ++r) {
            if (set[r]) {
                b->prev_path[r] = 0.0f;
            } else {
                float pr;
                std::memcpy(&pr, &path[r], sizeof pr);
                b->prev_path[r] = pr;
            }
        }
        *kept_path = kp;
        *rebuilt = nre;
        HIP_TRY(&b->c, hipMemcpyAsync(b->d_build, set, sizeof(int) * (size_t)R, hipMemcpyHostToDevice, s));
        int rr = batch_build_cells(b, pos, buf->vel, buf->image, buf->rtag, buf->cells_ws, buf->cells_ws_bytes,
                                   b->d_build, s);
        if (rr) return rr;
        return batch_build_nlist(b, pos, buf->vel, buf->cells_ws, buf->cells_ws_bytes, buf->k_max, buf->nlist,
                                 buf->nn, buf->status, true, b->d_build, s);
    }
    hipError_t fold(int* blk, int nb, const float4* vel, int N, int* status, hipStream_t st) override {
        if (vel) {
            hipError_t e = launch_fold_reps(blk, vel, nb, b->d_desc, b->R, b->d_rep, b->d_chunk_path, status, st);
            if (e != hipSuccess) return e;
        }
        return launch_fold_status(blk, nb, nullptr, N, status, st);
    }
    bool read_after_replay() override { return true; }
    // growth of each replica's largest path length since the previous fold (or its build)
    bool path_growth(int64_t C, double* growth) override {
        const int R = b->R;
        if ((int)b->prev_path.size() != R) b->prev_path.assign(R, 0.0f);
        double g = 0.0;
        for (int r = 0; r < R; ++r) {
            float pr;
            std::memcpy(&pr, &b->h_rep[R + r], sizeof pr);
            g = std::max(g, (double)(pr - b->prev_path[r]));
            b->prev_path[r] = pr;
        }
        *growth = g / (double)std::max<int64_t>(C, 1);
        return true;
    }
    int bonds(const float* pos, int row) override {
        HIP_TRY(&b->c, launch_bonds_batch(reinterpret_cast<const float4*>(pos), buf->nlist, buf->nn, buf->k_max,
                                          b->n_slots, all_tables(b), b->d_desc, b->d_chunk_rep, b->R,
                                          buf->bonds_log + (size_t)row * b->R,
                                          reinterpret_cast<unsigned long long*>(b->c.d_part), s));
        return RC_OK;
    }
    hipError_t launch(const StepArgs& a, bool ev) override { return launch_step_batch(a, ev, s); }
    hipError_t launch_timed(const StepArgs& a, hipEvent_t* sums, hipEvent_t* step) override {
        return launch_step_timed(a, true, s, sums, step);
    }
    int reduce_ev(int row) override {
        HIP_TRY(&b->c, launch_reduce_rows_batch(b->c.d_part, b->d_desc, b->R, 0, kEvWords,
                                                buf->ev_log + (size_t)row * b->R * kEvWords, kEvWords, s));
        return RC_OK;
    }
    const void* graph_fn() override {
        const void* fn;
        step_batch_kernel_info(b->c.gather_width, b->c.step_form, &fn);
        return fn;
    }
    const void* graph_sums_fn() override {
        if (b->c.step_form != RC_FORM_SUMS) return nullptr;
        const void* fn;
        sums_kernel_info(true, &fn);
        return fn;
    }
    // the batch cell sort also permutes (pos, vel, image) of every slot through
    // the workspace's temporaries and copies them back
    bool rebuild_snapshot(const float4** p, const float4** v, const int4** im) override {
        const CellsLayout l = cells_layout(b->n_slots, b->nkeys);
        if (buf->cells_ws_bytes < l.total) return false;
        const char* w = static_cast<const char*>(buf->cells_ws);
        *p = reinterpret_cast<const float4*>(w + l.tpos);
        *v = reinterpret_cast<const float4*>(w + l.tvel);
        *im = reinterpret_cast<const int4*>(w + l.timage);
        return true;
    }
};

}  // namespace

extern "C" int rc_batch_run(rc_batch* b, const rc_md_buffers* buf, const rc_integrator* cfg, uint64_t step0,
                            int n_steps, const rc_md_options* opt_in, rc_md_stats* stats, void* stream) {
    if (!b || !buf) return RC_ERR_ARG;
    rc_ctx* c = &b->c;
    int r = check_pos(b, buf->pos);
    if (r) return r;
    if (!buf->pos_alt || !buf->vel || !buf->nlist || !buf->nn || !buf->cells_ws || !buf->status)
        return fail(c, RC_ERR_ARG, "md buffers incomplete");
    if (buf->k_max < 1 || buf->k_max > 512) return fail(c, RC_ERR_ARG, "k_max must be in [1, 512]");
    if (n_steps < 0) return fail(c, RC_ERR_ARG, "n_steps < 0");
    rc_md_options opt{1, 16, 256, 0, 0.8, 1, 0, 0, 1, 0};
    if (opt_in) opt = *opt_in;
    if (opt.graph_steps < 2 || (opt.graph_steps & 1)) opt.graph_steps = 16;
    if (opt.max_chunk < 1) opt.max_chunk = 256;
    if (!(opt.soft_frac > 0.0 && opt.soft_frac <= 1.0)) opt.soft_frac = 0.8;
    hipStream_t s = S(stream);
    const int nb = nblocks(b->n_slots, kStepBlock);
    if ((r = ensure_part(c, sizeof(double) * kEvWords * (size_t)nb))) return r;
    StepArgs tmpl{};
    if ((r = fill_step_args_batch(b, tmpl, buf->pos, buf->pos_alt, buf->vel, buf->image, buf->nlist, buf->nn,
                                  buf->k_max, cfg, opt.soft_frac, buf->status, s, false)))
        return r;
    BatchOps ops;
    ops.b = b;
    ops.buf = buf;
    ops.s = s;
    ops.soft = tmpl.soft;
    return md_drive(c, ops, buf, b->n_slots, tmpl, step0, n_steps, opt, stats, s);
}
