// Host-side internals shared by the single-system and the batch C ABI:
// the context, argument checks, workspace layout, the table compiler, step
// graphs and the chunked MD driver.
#pragma once

#include <cstddef>
#include <string>
#include <vector>

#include "rc_internal.h"

struct GraphCache {
    hipGraphExec_t exec[2] = {nullptr, nullptr};  // start parity 0 / 1
    hipGraph_t graph[2] = {nullptr, nullptr};
    rc::StepArgs key{};
    const void* fn = nullptr;
    int steps = 0;
    bool valid = false;
};

// A list rebuild of the driver (cell sort and list build) replayed as one graph:
// what its launches were recorded with.  A build with another key runs directly
// once and is recorded at its next occurrence.
struct RebuildKey {
    const void* pos;
    const void* vel;
    const void* image;
    const void* rtag;
    const void* ws;
    size_t ws_bytes;
    const void* nlist;
    const void* nn;
    const void* status;
    const void* pl_j;
    const void* pl_o;
    const void* tab;
    int N;
    int k_max;
    double L[3];
    double rlist_max;
};
struct RebuildGraph {
    hipGraphExec_t exec = nullptr;
    RebuildKey key{};
    bool seen = false;    // key ran directly once
    bool valid = false;   // exec replays key
};

// What an rc_md_run that returned RC_OK left, for a next run that continues on
// its list (rc_md_options.keep_list).  Cleared by every other call that
// changes the state or the list.
// The integrator settings a replay of earlier steps must share (compared bytewise).
struct DynKey {
    float minv[RC_MAX_TYPES], c2[RC_MAX_TYPES];
    float dt, c1, noise_z, fene_k, fene_r02;
    int langevin;
    uint64_t seed;
    const void* bonds;
};
DynKey dyn_key(const rc::StepArgs& a);

struct MdRecord {
    bool valid = false;
    DynKey dyn{};               // its integrator settings
    rc_md_buffers buf{};        // the buffers it ran on
    int N = 0;
    double L[3] = {0.0, 0.0, 0.0};
    uint64_t step_end = 0;      // step index of the state it left (on-step velocities)
    uint64_t ep_step = 0;       // step index of the state of its last list build (the snapshot)
    int ep_cur = 0;             // position buffer that state was in (0 pos, 1 pos_alt)
    bool ep_first = true;       // that state had on-step velocities (no half kick owed)
    bool logged_end = false;    // its last log row is the state it left
    double rate = 0.0;          // growth of the largest path length per step
    float last_maxpath = 0.0f;  // largest path length since the build, at the end
};

struct rc_ctx {
    int device = 0;
    int nt = 0;
    std::vector<rc_pair_coeff> table;   // as given (one table; a batch keeps its own copies)
    double r_buff = 0.0;
    double rlist_max = 0.0;
    std::vector<rc::DevEntry> host_tab;
    rc::DevEntry* d_tab = nullptr;
    double* d_part = nullptr;           // block partial rows (13 doubles each) or param partials
    size_t part_bytes = 0;
    unsigned long long* d_step_base = nullptr;
    double* d_slices = nullptr;         // kRowSlices doubles: the two-launch row reduction
    int* d_blk = nullptr;               // per-block status slots of the step kernel
    int blk_cap = 0;                    // slots allocated (blocks)
    int gather_width = 2;               // flattened list entries per lane and pass of the step kernel
    int step_form = RC_FORM_WALK;       // RC_FORM_WALK | RC_FORM_SUMS
    float* d_ssum = nullptr;            // per-particle switching sums of the sums form
    size_t ssum_cap = 0;                // floats allocated
    double* d_hsum = nullptr;           // per-particle (S, dS) of the Hessian-vector product
    size_t hsum_cap = 0;                // particles allocated
    // packed copy of the last list (pack_wave_lists), read by the single-system step kernel
    int* d_pl_j = nullptr;
    unsigned char* d_pl_o = nullptr;
    size_t pl_cap = 0;                  // entries allocated
    const int* pl_nlist = nullptr;      // the list it was made from: (nlist, nn, k_max, N)
    const int* pl_nn = nullptr;
    int pl_k = 0, pl_n = 0;
    const int* bonds = nullptr;         // FENE partner table (caller-owned, [n_bonded][2] by tag)
    const int* bonds_rtag = nullptr;    // tag -> index map the springs read (caller-owned)
    int bonds_n = 0;
    double fene_k = 0.0, fene_r0 = 0.0;
    int* h_status = nullptr;            // pinned host copy of a status word (driver waits)
    hipEvent_t ev_sync = nullptr;       // the driver's wait event (no timing)
    GraphCache gc;
    RebuildGraph rg[2];                 // the driver's rebuilds, one per position buffer
    hipStream_t cap_stream = nullptr;   // private stream the rebuild graphs are recorded on
    void* noalloc_scratch = nullptr;    // device address of the fixed scratch on this device
    MdRecord md;                        // the last run, for keep_list
    // caller-owned workspace (rc_set_workspace): when attached, the packed list, the switching sums
    // and the HVP sums live there, and the ensure_* functions never allocate them
    void* ws_user = nullptr;
    std::vector<hipEvent_t> tk_events;  // event pairs of time_kernels
    std::vector<int> tk_kind;           // per pair: 0 step kernel, 1 first pass of the sums form
    // device words copied to (pinned) host memory with every status read (a batch's per-replica fold)
    struct StatusExtra {
        void* host;
        const void* dev;
        size_t bytes;
    };
    std::vector<StatusExtra> status_extra;
    std::string err;
};

namespace rc {
namespace host {

int fail(rc_ctx* c, int code, const char* fmt, ...) __attribute__((format(printf, 3, 4)));
int hip_fail(rc_ctx* c, hipError_t e, const char* where);

#define HIP_TRY(ctx, expr)                                              \
    do {                                                                \
        hipError_t _e = (expr);                                         \
        if (_e != hipSuccess) return ::rc::host::hip_fail((ctx), _e, #expr); \
    } while (0)

inline hipStream_t S(void* s) { return reinterpret_cast<hipStream_t>(s); }
inline int nblocks(long n, int b) { return (int)((n + b - 1) / b); }

int make_box(rc_ctx* c, const rc_box& in, Box& b);
int make_grid(rc_ctx* c, double rlist_max, const Box& b, Grid& g);

struct CellsLayout {
    size_t counts, start, keys, rank, order, bsums, bmax, tpos, tvel, timage, total;
};
CellsLayout cells_layout(int N, uint32_t nkeys);

int ensure_part(rc_ctx* c, size_t bytes);
// Layout of a caller-owned workspace holding a packed list of plist entries,
// n_ssum switching sums and n_hsum HVP sums (offsets and total, 256-byte aligned).
struct WsLayout {
    size_t pl_j, pl_o, ssum, hsum, total;
};
WsLayout ws_layout(size_t plist, size_t n_ssum, size_t n_hsum);
size_t plist_entries(int N, int k_max);   // ceil(N / 64) * 64 * k_max
// attach (ws != NULL) or detach a caller-owned workspace sized for (N, k_max, nvec)
int set_workspace(rc_ctx* c, void* ws, size_t bytes, int N, int k_max, int nvec);
size_t ctx_device_bytes(const rc_ctx* c);
int ensure_ssum(rc_ctx* c, size_t n);   // d_ssum for n particles (drops graphs when it moves)
int ensure_hsum(rc_ctx* c, size_t n);   // d_hsum for n particles
// packed-list arrays for N particles and k_max slots (drops graphs when they move)
int ensure_plist(rc_ctx* c, int N, int k_max);
// the packed copy of (nlist, nn, k_max, N): made on the stream unless it is the current one
int packed_list_for(rc_ctx* c, const int* nlist, const int* nn, int k_max, int N, hipStream_t s);
void free_ctx_buffers(rc_ctx* c);       // every device buffer the context owns
// copy a device status word to the host and wait for it by spinning on an event
int read_status_spin(rc_ctx* c, const int* d_status, int* hst, hipStream_t s);
int ensure_blk(rc_ctx* c, int nb, hipStream_t s);
int check_integrator(rc_ctx* c, const rc_integrator* cfg, float* minv, float* c2, float& c1, int& langevin,
                     float& noise_z);
int check_list(rc_ctx* c, const int* nlist, const int* nn, int k_max);

// Validate one ntypes x ntypes table and compile it; returns RC_OK or
// RC_ERR_ARG with a message in *why.
int compile_table(int nt, const rc_pair_coeff* table, double r_buff, DevEntry* out, double* rlist_max,
                  std::string* why);

void drop_graphs(rc_ctx* c);
void drop_rebuild_graphs(rc_ctx* c);
// Run fn(stream) (the launches of one rebuild) as a graph replay on s when slot holds key, else run it
// directly on s (the first time for key) or record it on the private stream and replay it.
int rebuild_graphed(rc_ctx* c, int slot, const RebuildKey& key, int (*fn)(void*, hipStream_t), void* arg,
                    hipStream_t s);

// What the chunked driver needs from a system (one or a batch).
enum RebuildKind {
    kRebuildAll = 0,      // the first build of a run: every particle
    kRebuildFlagged = 1,  // a build the status flags asked for
    kRebuildRetry = 2,    // the first build of a resumed run: the set of the build that overflowed
};
struct DriveOps {
    virtual ~DriveOps() = default;
    // cell sort (permutes pos, vel, image) and list build from pos; the list
    // kernels write the status words whole: KMAX and the overflow flag of the
    // new list, MAXPATH zero and the chunk markers cleared (as a chunk reset
    // leaves them).  A system may rebuild part of its particles (a batch: the
    // replicas that need it); *kept_path receives the largest path length of
    // the particles that keep their lists (0 when every list is rebuilt) and
    // *rebuilt the number of particles whose lists were rebuilt.
    virtual int rebuild(float* pos, RebuildKind kind, float* kept_path, int64_t* rebuilt) = 0;
    // fold the step kernel's per-block status slots into the status word (and
    // reset them); vel non-NULL: also raise MAXPATH to the largest path length
    virtual hipError_t fold(int* blk, int nb, const float4* vel, int N, int* status, hipStream_t s) {
        return launch_fold_status(blk, nb, vel, N, status, s);
    }
    // whether a rollback's replay is folded and read back before its rebuild
    // (a partial rebuild takes its set from the state the replay ends in)
    virtual bool read_after_replay() { return false; }
    // after a chunk's status read: the largest growth per step of any part's
    // largest path length over the chunk's C steps, when the system keeps
    // lists of different ages (a batch after partial rebuilds); false: the
    // driver uses the growth of the overall largest path length
    virtual bool path_growth(int64_t, double*) { return false; }
    // bond count(s) of the state in pos into log row `row`
    virtual int bonds(const float* pos, int row) = 0;
    // one step launch with a filled StepArgs (ev: partial rows to ctx->d_part)
    virtual hipError_t launch(const StepArgs& a, bool ev) = 0;
    // reduce the partial rows of the last ev launch into log row `row`
    virtual int reduce_ev(int row) = 0;
    // kernel that the step graphs replay, and the first-pass kernel of the
    // sums form (NULL for the walk form)
    virtual const void* graph_fn() = 0;
    virtual const void* graph_sums_fn() = 0;
    // whether graph replays may run as one-workgroup launches of G steps, and
    // such a launch (a: launch arguments of the replay's first step)
    virtual bool block_ok() { return false; }
    // where the last rebuild left a copy of the state it produced (positions,
    // velocities with stale path lengths, images or NULL), if it does: the
    // driver then restores from there instead of taking its own snapshot
    virtual bool rebuild_snapshot(const float4**, const float4**, const int4**) { return false; }
    virtual hipError_t launch_block(const StepArgs&, float4*, int) { return hipErrorNotSupported; }
    // a plain step launch (no ev) with its kernels between event pairs: sums[0..1]
    // around the first pass of the sums form (NULL otherwise), step[0..1] around the step
    virtual hipError_t launch_timed(const StepArgs& a, hipEvent_t* sums, hipEvent_t* step) = 0;
};

// Chunked driver: speculative chunks of fused steps (graph replays where no
// log step intervenes), one status read per chunk, rollback and replay of
// stale chunks, rebuilds, the final half kick and the logs.  tmpl holds every
// launch argument except positions, mode, step and ev_part; N counts slots.
int md_drive(rc_ctx* c, DriveOps& ops, const rc_md_buffers* buf, int N, const StepArgs& tmpl, uint64_t step0,
             int n_steps, rc_md_options opt, rc_md_stats* stats, hipStream_t s);

}  // namespace host
}  // namespace rc
