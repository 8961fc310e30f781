/*
 * rc.h -- C ABI of the MI355X swap-potential engine.
 *
 * The engine evaluates, on one GPU, the associative bond-swap potential of
 * Ciarella & Ellenbroek (arXiv 1912.08569, Sec. 2):
 *
 *   pair (kind RC_KIND_SWAP):  v(r) = 4 eps [(sigma/r)^(2n) - (sigma/r)^n],  r < r_cut     eq. (2b)
 *   pair (kind RC_KIND_WCA):   4 eps [(sigma/r)^12 - (sigma/r)^6] + eps,      r < r_cut
 *   switching factor:          vhat = 1 (r <= r_min = sigma 2^(1/n)), -v/eps beyond     eq. (pot)
 *   three-body:                sum_i sum_{j<k} Lambda vhat(r_ij) vhat(r_ik),
 *                              Lambda = lambda eps                                       eq. (3bp)
 *   virial:                    W_ab = sum_terms sum_m (x_m - x_centre)_a F_m,b           eq. (p3)
 *
 * plus a BAOAB Langevin / velocity-Verlet integrator, cell-list binning with a
 * Morton-ordered counting sort, a full neighbour list, exact bond counting,
 * Hessian-vector products and parameter gradients of the energy, a batch
 * mode that advances many independent replicas in one launch per step, and
 * planar motion with rigid patchy bodies (the 2d systems of Sec. 3.2).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Memory.  Every array argument is caller-owned DEVICE memory on the device
 * that was current at rc_create, unless the comment says "host".  The library
 * allocates device memory only inside an rc_ctx / rc_batch (parameter table,
 * FP64 reduction rows, per-block status slots: O(ntypes^2 + N/64)) and, unless
 * the caller attaches a workspace (rc_set_workspace), its large scratch too;
 * it never frees caller memory.
 *
 * Streams.  Every launch is asynchronous on the caller's hipStream_t (passed
 * as void*; NULL = the null stream).  Functions that return a host value
 * (rc_read_status, rc_md_run) synchronise that stream and say so.
 *
 * Errors.  Every function returns an int status: RC_OK or a negative RC_ERR_*.
 * Argument errors are detected synchronously before any launch; nothing is
 * launched then.  Conditions found on the device (neighbour-list overflow,
 * non-finite forces, lost particles) are latched in a device status word and
 * reported by rc_read_status.  rc_last_error(ctx) returns a message for the
 * last failure of that context.  Nothing throws or aborts across the ABI.
 *
 * Particle layout (structure of float4, 16-byte aligned):
 *   pos[i]   = (x, y, z, w) with x,y,z in [-L/2, L/2) and w holding the int32
 *              bit pattern (tag << RC_TYPE_BITS) | type.  tag < 2^27.
 *   vel[i]   = (vx, vy, vz, w) with w = path length travelled since the last
 *              neighbour-list build (maintained by the library; the skin test).
 *   force[i] = (fx, fy, fz, e_i): e_i is the per-particle energy (half of each
 *              pair term, every triplet term to its centre), when requested.
 *   image[i] = int4 periodic image counters (x, y, z, unused); may be NULL.
 *   nlist/nn = the neighbour list of rc_build_nlist: nlist is [k_max][N] int32
 *              (column-major).  Swap-kind neighbours of i fill slots 0 .. ns-1
 *              from the front, all other neighbours slots k_max-1 down to
 *              k_max-no from the back; nn[i] = ns | (no << 16), ns + no <= k_max.
 *              Every consumer takes k_max.
 * Particle order is the library's: rc_build_cells re-orders particles along a
 * Morton curve of the cell grid; identity travels with the tag in pos.w.
 *
 * Boxes are orthorhombic, periodic and origin centred; every edge must be an
 * exactly representable FP32 value and at least 3 neighbour-list radii long.
 */
#ifndef RC_H
#define RC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes -------------------------------------------------------- */
#define RC_OK                  0
#define RC_ERR_ARG            -1   /* invalid argument (nothing launched)             */
#define RC_ERR_HIP            -2   /* a HIP runtime call failed                        */
#define RC_ERR_NLIST_OVERFLOW -3   /* a particle has more than k_max neighbours        */
#define RC_ERR_UNSUPPORTED    -4   /* valid but unsupported request                    */
#define RC_ERR_NONFINITE      -5   /* a force, energy or position became non-finite    */
#define RC_ERR_LOST_PARTICLE  -6   /* a particle moved more than L/2 in one step       */
#define RC_ERR_WORKSPACE      -7   /* workspace too small                              */

/* ---- pair kinds ------------------------------------------------------------ */
#define RC_KIND_NONE 0   /* no interaction                                        */
#define RC_KIND_SWAP 1   /* eq. (2b) pair term + the three-body term of eq. (3bp)  */
#define RC_KIND_WCA  2   /* purely repulsive 12-6 LJ shifted by +eps               */

#define RC_TYPE_BITS 4           /* pos.w = (tag << 4) | type                     */
#define RC_MAX_TYPES 16
#define RC_MAX_TAG   (1 << 27)

/* ---- device status word: int32[RC_STATUS_WORDS] ---------------------------- */
#define RC_STATUS_WORDS 8
#define RC_ST_FLAGS      0   /* OR of RC_FLAG_*                                      */
#define RC_ST_KMAX       1   /* largest neighbour count seen by the last list build */
#define RC_ST_MAXPATH    2   /* largest path length since the build (float bits)   */
#define RC_ST_FIRST_SOFT 3   /* first step whose new positions passed the soft skin */
#define RC_ST_FIRST_HARD 4   /* first step whose force used a stale list           */
#define RC_ST_NSWAP      5   /* swap-range entries of the last list build (sum over
                                particles, saturating at 2^31 - 1)                 */
#define RC_FLAG_NLIST_OVERFLOW 1
#define RC_FLAG_REBUILD        2   /* a path length passed the soft skin threshold     */
#define RC_FLAG_NONFINITE      4
#define RC_FLAG_LOST           8
#define RC_FLAG_STALE         16   /* a force was evaluated on a stale list           */
#define RC_FLAG_TRIPLET_POOL  32   /* internal staging overflow (recovered; info)      */

/* ---- parameters (host structs) -------------------------------------------- */
/* One entry of the symmetric ntypes x ntypes table: the per-type-pair
 * coefficients of the paper's potential (Sec. 2: sigma, n, epsilon, lambda3,
 * and the cutoff).  SWAP requires eps > 0, sigma > 0, integer n >= 1,
 * r_min = sigma 2^(1/n) < r_cut and lambda >= 0.  WCA requires eps >= 0,
 * sigma > 0, r_cut > 0 (normally 2^(1/6) sigma); n and lambda are ignored.  */
typedef struct rc_pair_coeff {
    int kind;
    int n;
    double epsilon;
    double sigma;
    double r_cut;
    double lambda;
} rc_pair_coeff;

typedef struct rc_box {
    double L[3];   /* edges, FP32-exact */
} rc_box;

#define RC_INTEGRATOR_NVE      0   /* velocity Verlet                           */
#define RC_INTEGRATOR_LANGEVIN 1   /* BAOAB (Leimkuhler-Matthews 2013)          */

typedef struct rc_integrator {
    int kind;                      /* RC_INTEGRATOR_*                            */
    int dim;                       /* 3 (or 0): 3D.  2: motion in the xy plane:
                                      the thermostat draws no z noise, so a
                                      system whose particles share one z and
                                      have vz = 0 keeps them (the z force
                                      components are then exactly zero); the
                                      box's z edge is still >= 3 list radii  */
    double dt;
    double kT;
    double gamma;                  /* friction (1/time); ignored for NVE        */
    uint64_t seed;                 /* Philox key: (seed mod 2^32, seed >> 32)   */
    double mass[RC_MAX_TYPES];     /* mass per type (> 0)                       */
} rc_integrator;

typedef struct rc_ctx rc_ctx;

/* ---- context ----------------------------------------------------------------
 * rc_create: validate the table (must be symmetric), compile it into a device
 * table on the current device and precompute r_cut^2 and the canonical
 * r_min^2 = (sigma*sigma) * pow(2, 2/n) in FP64, and the neighbour-list radii
 * r_list = r_cut + r_buff.  r_buff > 0 is the skin.  Host pointers.
 * Returns RC_ERR_ARG on an invalid table, RC_ERR_UNSUPPORTED for
 * ntypes > RC_MAX_TYPES.                                                      */
int rc_create(rc_ctx** out, int ntypes, const rc_pair_coeff* table /* host [ntypes*ntypes] */,
              double r_buff);
int rc_destroy(rc_ctx* ctx);
const char* rc_last_error(const rc_ctx* ctx);
int rc_version(void);
/* Replace lambda of every SWAP entry with table values (host, ntypes^2);
 * takes effect for launches issued after it returns.                         */
int rc_set_lambda(rc_ctx* ctx, const double* lambda /* host [ntypes*ntypes] */);
/* Neighbour-list radius actually used for type pair (a, b) (host).           */
int rc_get_rlist(const rc_ctx* ctx, int a, int b, double* r_list);
/* Gather width of the fused step kernel: the flattened (particle, list slot)
 * entries each lane of a wavefront evaluates per pass (1, 2 or 4; default 2).
 * A tuning knob only: every width sums each particle's terms in the same
 * order, so results are bit-identical.  RC_ERR_ARG for other values.        */
int rc_set_gather_width(rc_ctx* ctx, int width);
/* How the fused step (and rc_compute_forces with RC_FORCE_SUMS) evaluates
 * the three-body forces of eq. (3bp):
 *   RC_FORM_WALK (default): one pass; the part of the force on m that comes
 *     from triplets centred on a partner j is summed by walking j's list
 *     (work grows as k^2 per particle; no extra memory).
 *   RC_FORM_SUMS: two passes.  The first stores S_i = sum of w_ij over i's
 *     swap partners inside r_cut (w = sqrt(lambda eps) vhat); the second
 *     gives every (m, j) entry the factor (S_m - w) + (S_j - w), i.e. the
 *     triplet sum of eq. (3bp) rewritten as (S^2 - sum w^2)/2 per centre
 *     (linear in k; one float per particle of context-owned scratch).
 * Both are exact rewritings of the same energy; results differ by rounding
 * order only.  RC_ERR_ARG for other values.                                 */
#define RC_FORM_WALK 0
#define RC_FORM_SUMS 1
int rc_set_step_form(rc_ctx* ctx, int form);

/* ---- caller-owned workspace ---------------------------------------------------
 * The context's large scratch -- the packed copy of the list that the fused
 * step reads (5 bytes per slot, ceil(N/64) * 64 * k_max slots), the switching
 * sums of the two-pass form (4 bytes per particle) and the first-pass sums of
 * the Hessian-vector products (16 bytes per particle and tangent vector) --
 * can live in caller-owned device memory:
 * rc_workspace_bytes: the size for N particles, lists of k_max slots and up to
 *   nvec tangent vectors per rc_force_hvp_batch call (host out).
 * rc_set_workspace: attach ws (device, 256-byte aligned, at least that many
 *   bytes; the caller keeps it alive and does not touch it while attached;
 *   NULL detaches).  Synchronises the device once; the context's own copies of
 *   these buffers are freed.  While a workspace is attached the context never
 *   allocates them: a call that needs more (a larger N or k_max, more vectors)
 *   returns RC_ERR_WORKSPACE and launches nothing.  Without one, the context
 *   allocates them itself on first use (growing them synchronises the device).
 * rc_ctx_device_bytes: device memory the context itself holds (host out): the
 *   coefficient table, the FP64 reduction rows and per-block status slots
 *   (O(ntypes^2 + N/64)), plus the large scratch above when no workspace is
 *   attached.                                                                */
int rc_workspace_bytes(const rc_ctx* ctx, int N, int k_max, int nvec, size_t* bytes /* host */);
int rc_set_workspace(rc_ctx* ctx, void* ws, size_t bytes, int N, int k_max, int nvec);
int rc_ctx_device_bytes(const rc_ctx* ctx, size_t* bytes /* host */);

/* ---- status ---------------------------------------------------------------
 * rc_clear_status: zero a status word (async).  rc_read_status: synchronise
 * `stream`, copy the word to host `out` and return the matching error code:
 * RC_ERR_NLIST_OVERFLOW, RC_ERR_NONFINITE, RC_ERR_LOST_PARTICLE or RC_OK.    */
int rc_clear_status(int* status /* device [RC_STATUS_WORDS] */, void* stream);
int rc_read_status(const int* status, int* out /* host [RC_STATUS_WORDS] */, void* stream);

/* ---- cell binning (hot-path step a1) -----------------------------------------
 * Cells: nc_d = floor(L_d / r_list_max) >= 3 per axis; a particle's cell is
 * floor((x + L/2) nc / L) clamped to [0, nc); cells are keyed by the 3-D
 * Morton code of their integer coordinates.  rc_build_cells counts particles
 * per key (atomics), takes an exclusive prefix scan into cell_start, scatters
 * by (key, rank), orders each cell by previous index (deterministic), and
 * permutes pos, vel (nullable) and image (nullable) in place into key order,
 * so that a Morton walk of the grid is a walk of memory.  If rtag is not NULL
 * it receives rtag[tag] = new index (device, N ints; requires tags < N).
 * ws must hold rc_cells_workspace_bytes(ctx, N, box) bytes; it keeps the cell
 * table for rc_build_nlist and must not be touched in between.
 * Returns RC_ERR_ARG for N < 1, a non-FP32 box or a box shorter than three
 * list radii, RC_ERR_WORKSPACE if ws_bytes is too small.                     */
int rc_cells_workspace_bytes(const rc_ctx* ctx, int N, rc_box box, size_t* bytes /* host */);
int rc_build_cells(rc_ctx* ctx, float* pos /* [N*4] */, float* vel /* [N*4] | NULL */,
                   int* image /* [N*4] | NULL */, int* rtag /* [N] | NULL */, int N, rc_box box,
                   void* ws, size_t ws_bytes, void* stream);

/* ---- neighbour list (hot-path step a2) -----------------------------------------
 * Full list (i -> j and j -> i) of every pair with r < r_list(t_i, t_j) =
 * r_cut + r_buff, found by scanning the 27 cells around each particle's cell
 * (cell table from the last rc_build_cells on ws).  Column-major:
 * nlist[s * N + i] is the s-th neighbour of i, s < nn[i] <= k_max.  A
 * particle with more than k_max neighbours sets RC_FLAG_NLIST_OVERFLOW and
 * status[RC_ST_KMAX] = its count (its list is truncated).  If vel is not NULL
 * the path lengths vel[i].w are reset to 0 (the skin reference).  The list is
 * valid while every path length stays <= r_buff / 2: any pair then outside
 * the list is at least r_cut apart (the paper's three-particle neighbour
 * lists, SI "Performance").  Layout: swap-kind neighbours first, the others
 * from the back of the column (nn[i] = ns | (no << 16), see above), so that
 * the triplet walks read swap partners only.  The same launch writes a packed
 * copy of the list into the context (per wavefront of 64 particles, its
 * entries flattened in walk order: neighbour index and owner lane, 5 bytes
 * per slot), which the single-system fused step reads; a fused step given a
 * list it did not see built packs it first.  A list changed by other means
 * than rc_build_nlist under the same pointers must be rebuilt with it.       */
int rc_build_nlist(rc_ctx* ctx, const float* pos, float* vel /* NULL ok */, int N, rc_box box,
                   const void* ws, size_t ws_bytes, int k_max, int* nlist /* [k_max*N] */,
                   int* nn /* [N] */, int* status /* [RC_STATUS_WORDS] | NULL */, void* stream);

/* ---- forces, energy, virial (hot-path step a3) -------------------------------
 * F = -grad(E2 + E3) of the pair terms (eq. 2b / WCA) and the three-body term
 * (eq. 3bp with eq. pot), one term per centre i and unordered partner pair
 * {j, k}; Lambda_ijk = sqrt(Lambda_ij Lambda_ik) when the entries differ.
 * Cut decisions use the canonical FP64 predicate (minimum image
 * d = x_j - x_i folded once by +-L, r^2 = (dx*dx + dy*dy) + dz*dz, no fused
 * multiply-add, compared with r_cut*r_cut); the terms are evaluated in FP32.
 * Default algorithm (the triplet kernel): each lane owns a centre, walks its
 * list for the pair terms, stages the active swap partners of centres with two
 * or more of them in LDS, and the wavefront enumerates all (j<k) triplets of
 * its 64 centres across its lanes; forces on j and k go out with atomics, so
 * the summation order (last bits) is not deterministic.
 * flags:
 *   RC_FORCE_ACCUMULATE  add into force instead of overwriting it
 *   RC_FORCE_GATHER      atomic-free gather algorithm (each particle sums
 *                        every term that moves it; deterministic)
 *   RC_FORCE_SUMS        the gather in the two-pass form (see
 *                        rc_set_step_form; implies RC_FORCE_GATHER)
 * force[i].w receives the per-particle energy (added when accumulating).
 * ev (device, nullable) receives 7 doubles: E, Wxx, Wyy, Wzz, Wxy, Wxz, Wyz
 * with W the configurational virial of eq. (p3) (stress = -(K + W)/V),
 * reduced in FP64 in a fixed order.                                          */
#define RC_FORCE_ACCUMULATE 1u
#define RC_FORCE_GATHER     4u
#define RC_FORCE_SUMS       8u
int rc_compute_forces(rc_ctx* ctx, const float* pos, const int* nlist, const int* nn, int k_max, int N,
                      rc_box box, float* force /* [N*4] */, double* ev /* [7] | NULL */,
                      unsigned flags, int* status /* NULL ok */, void* stream);

/* ---- forces without allocation ------------------------------------------------
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.
 * rc_compute_forces_noalloc takes the arguments of rc_compute_forces, computes
 * what it computes (bit for bit with RC_FORCE_GATHER or RC_FORCE_SUMS; the
 * default triplet kernel sums with atomics, so its last bits vary from call
 * to call, as rc_compute_forces' do) and calls no hipMalloc, hipFree or other
 * allocating routine.  Its scratch -- the per-block FP64 rows of the
 * energy/virial reduction and, with RC_FORCE_SUMS, the per-particle switching
 * sums -- is a fixed device array of RC_NOALLOC_SCRATCH_BYTES that the library
 * holds on each GPU it runs on from the first rc_create there until the
 * process ends, instead of the context's growable buffers.  Every launch
 * writes all the scratch it reads, so nothing in it needs to start at zero.
 * Every call on one GPU shares that GPU's array: calls whose launches can
 * overlap on one GPU (different streams or threads) race, and the caller
 * must order them.  N > RC_NOALLOC_MAX_N returns RC_ERR_UNSUPPORTED with
 * nothing launched; other errors as rc_compute_forces.                       */
#define RC_NOALLOC_MAX_N 1048576   /* 2^20 particles */
#define RC_NOALLOC_SCRATCH_BYTES ((size_t)13 * 8 * (RC_NOALLOC_MAX_N / 64) + (size_t)4 * RC_NOALLOC_MAX_N)
int rc_compute_forces_noalloc(rc_ctx* ctx, const float* pos, const int* nlist, const int* nn, int k_max, int N,
                              rc_box box, float* force /* [N*4] */, double* ev /* [7] | NULL */,
                              unsigned flags, int* status /* NULL ok */, void* stream);

/* ---- integrator (hot-path step a5) -------------------------------------------
 * BAOAB Langevin (the paper's "canonical Langevin dynamics", Sec. 3.2; scheme
 * of Leimkuhler & Matthews 2013) or velocity Verlet (NVE):
 *   RC_HALF_FIRST : v += dt/2 F/m ; x += dt/2 v ; v = c1 v + sqrt((1-c1^2) kT/m) xi ;
 *                   x += dt/2 v ; wrap into [-L/2, L/2) (image += crossings) ;
 *                   vel.w += |x_new - x_old|   (c1 = exp(-gamma dt); NVE: c1 = 1)
 *   RC_HALF_SECOND: v += dt/2 F/m
 * xi = three normals from Philox4x32-10 (key = seed, counter = (tag, step lo,
 * step hi, 0)) by Box-Muller on u = (x + 1/2) 2^-32.  kin (nullable, device)
 * receives sum m v_a v_b (xx, yy, zz, xy, xz, yz) of the velocities after the
 * call.  A step that moves a particle by more than L/2 sets RC_FLAG_LOST; a
 * non-finite position sets RC_FLAG_NONFINITE; a path length above r_buff/2
 * sets RC_FLAG_REBUILD.                                                      */
#define RC_HALF_FIRST  0
#define RC_HALF_SECOND 1
int rc_integrate_step(rc_ctx* ctx, float* pos, float* vel, const float* force,
                      int* image /* NULL ok */, int N, rc_box box, const rc_integrator* cfg /* host */,
                      uint64_t step, int half, double* kin /* [6] | NULL */,
                      int* status /* NULL ok */, void* stream);

/* rc_thermostat_normals: the normals xi the integrators above draw (Philox4x32-10
 * keyed by seed, counter (tag, step), Box-Muller as described), for host-side
 * integrators that must follow the engine's noise (the trajectory fit):
 * out[k][t] = (xi_x, xi_y, xi_z, 0) of tag t in [0, N) at step step0 + k,
 * xi_z = 0 for dim 2 (device, 16-byte aligned, [steps][N][4] floats, steps * N
 * <= 2^31).  No context needed.                                               */
int rc_thermostat_normals(uint64_t seed, uint64_t step0, int steps, int N, int dim,
                          float* out /* [steps*N*4] */, void* stream);

/* ---- rigid planar bodies (next-4: the patchy colloids of Sec. 3.2) ----------
 * Body b is the particle with tag centre[b] (a disk; its type's mass) plus the
 * massless member particles with tags member[first[b] .. first[b+1]) held at
 * body-frame offsets (offset[2m], offset[2m+1]), turned by the angle theta[b].
 * Motion is in the xy plane: cfg->dim must be 2, and every particle keeps its
 * z.  With the forces in `force` (every particle, current positions):
 *   RC_HALF_FIRST : v += dt/2 F/M, w += dt/2 tau/I ; x += dt/2 v, theta += dt/2 w ;
 *                   v = c1 v + sqrt((1-c1^2) kT/M) (xi_x, xi_y),
 *                   w = c1 w + sqrt((1-c1^2) kT/I) xi_z ; x += dt/2 v,
 *                   theta += dt/2 w (theta folded into [-pi, pi)) ; members
 *                   placed at x + R(theta) offset, their path lengths grown
 *                   by their own moves
 *   RC_HALF_SECOND: v += dt/2 F/M, w += dt/2 tau/I
 * F and tau (about the centre, minimum image) sum the centre's and the
 * members' forces; xi are the centre's thermostat normals (tag, step).  Member
 * velocities are set to v + w x d.  rtag maps tag -> index (rc_build_cells);
 * inertia, theta and omega are [B] device arrays, first is [B+1], member [M],
 * offset [M][2].  A non-finite body state sets RC_FLAG_NONFINITE in status.  */
int rc_rigid_step(rc_ctx* ctx, float* pos, float* vel, const float* force, int* image /* NULL ok */,
                  const int* rtag, int B, const int* centre, const int* first, const int* member,
                  const float* offset, const float* inertia, float* theta, float* omega, int N, rc_box box,
                  const rc_integrator* cfg /* host */, uint64_t step, int half, int* status /* NULL ok */,
                  void* stream);

/* ---- fused step (the metric path: a3 + a5 in one kernel) ---------------------
 * One kernel per MD step.  Reads pos_in, writes pos_out (pos_in != pos_out,
 * double buffered).  Each particle m gathers every force term that moves it:
 * its pair terms, the triplets it centres, and the triplets in which it is a
 * partner of a centre c (the other partners of c are found by walking c's
 * list: a two-hop gather), so no atomics are needed and the result is
 * deterministic.  Then it integrates.  Between steps vel holds the velocity
 * after the O and second A of BAOAB (the final half kick is folded into the
 * next step):
 *   RC_STEP_START : v = vel (on-step velocity); B A O A       -> pos_out, vel
 *   RC_STEP_CONT  : v = vel + dt/2 F/m (ends the previous step); B A O A
 *   RC_STEP_FINISH: v = vel + dt/2 F/m; vel = v; pos_out untouched
 *   RC_STEP_OBSERVE: v = vel (on-step); nothing written except ev and status
 * ev (nullable, device) receives 13 doubles at x_in: E, W(6) as in
 * rc_compute_forces, K(6) = sum m v v of the on-step velocity.  The kernel
 * sets RC_FLAG_STALE (and RC_ST_FIRST_HARD = step) when an input path length
 * exceeds r_buff/2, and RC_FLAG_REBUILD (RC_ST_FIRST_SOFT = step) when an
 * output path length exceeds soft_frac * r_buff/2.                           */
#define RC_STEP_START  0
#define RC_STEP_CONT   1
#define RC_STEP_FINISH 2
#define RC_STEP_OBSERVE 3
int rc_step_fused(rc_ctx* ctx, const float* pos_in, float* pos_out, float* vel, int* image,
                  const int* nlist, const int* nn, int k_max, int N, rc_box box,
                  const rc_integrator* cfg /* host */, uint64_t step, int mode, double soft_frac,
                  double* ev /* [13] | NULL */, int* status, void* stream);

/* Measurement helper: launch `reps` RC_STEP_CONT fused steps back to back on
 * `stream` (alternating pos_a -> pos_b -> pos_a ...; status is written to
 * status), each kernel launch carrying its own start/stop hipEvents
 * (hipExtLaunchKernel); synchronises and returns in *ms (host) the sum of
 * the kernels' own execution times in milliseconds (the sums pass included
 * in the two-pass form; the dispatch gaps between launches excluded).  Used
 * to time the step kernel alone.                                            */
int rc_time_fused_steps(rc_ctx* ctx, float* pos_a, float* pos_b, float* vel, const int* nlist,
                        const int* nn, int k_max, int N, rc_box box, const rc_integrator* cfg /* host */,
                        uint64_t step0, int reps, int* status, float* ms /* host */, void* stream);

/* ---- bond partners (the bond autocorrelation of the paper's swap test) --------
 * partner (device int32 [N], indexed by TAG, overwritten): the tag of the one
 * swap partner bonded to the particle (canonical r^2 < r_min^2, as for the
 * bond count), -1 if it has no bond, -2 if it has more than one.  The bond
 * autocorrelation (Sec. 3.1: the fraction of the bonds of time 0 that are
 * still unswapped at time t) is the fraction of particles whose partner at t
 * equals their partner at 0.  Requires tags < N (as rtag does).              */
int rc_bond_partners(rc_ctx* ctx, const float* pos, const int* nlist, const int* nn, int k_max, int N,
                     rc_box box, int* partner /* [N] */, void* stream);

/* ---- observables built on the step ------------------------------------------
 * rc_partner_counts: counts[0..2] (device uint64, overwritten) = over the tags
 *   t < N with select[t] != 0 (select: device bytes by tag, NULL = all) the
 *   particles bonded at 0 (p0[t] >= 0), those with an unchanged partner
 *   (pt[t] == p0[t]) and those whose single partner is another particle
 *   (pt[t] >= 0, != p0[t]: a swap event), for two partner snapshots p0, pt
 *   (device int32 [N], as rc_bond_partners writes them).  counts[1]/counts[0]
 *   is the bond autocorrelation at the lag between them (Sec. 3.1, Fig. 3).
 *   Exact (integers).  Uses the context's scratch.
 * rc_stress_autocorrelation: G[t], t = 0 .. max_lag (device doubles,
 *   overwritten) = V/kT times the average over the off-diagonal components
 *   xy, xz, yz and over every time origin t0 < T - t of sigma(t0)
 *   sigma(t0 + t), sigma_ab = -(K_ab + W_ab)/V, for T logged rows (device
 *   doubles [T][13]: E, W(6), K(6) as rc_md_run writes ev_log); t counts rows.
 *   The relaxation modulus by the autocorrelation method (Sec. 2.2 after eq.
 *   p3).  FP64, deterministic (fixed reduction order).  0 <= max_lag < T.   */
int rc_partner_counts(rc_ctx* ctx, const int* p0, const int* pt, const unsigned char* select /* [N] | NULL */,
                      int N, unsigned long long* counts /* device [3] */, void* stream);
int rc_stress_autocorrelation(rc_ctx* ctx, const double* rows /* device [T][13] */, int T, double volume,
                              double kT, int max_lag, double* G /* device [max_lag+1] */, void* stream);

/* ---- bond count (hot-path step a4) -------------------------------------------
 * Number of swap pairs i<j with r^2 < r_min^2 (canonical FP64 predicate, the
 * bond criterion of the swap system), written to *count (device, uint64).
 * Exact; independent of list order.  Requires a list built with this ctx.    */
int rc_bond_count(rc_ctx* ctx, const float* pos, const int* nlist, const int* nn, int k_max, int N,
                  rc_box box, unsigned long long* count /* device */, void* stream);

/* ---- MD driver (hot-path step a6) --------------------------------------------
 * Advances (pos, vel) by n_steps steps of cfg, starting at step index step0,
 * on `stream`, and returns after synchronising it.  It bins and builds the
 * list at entry (unless opt->keep_list continues the previous run's list),
 * then runs chunks of fused steps, each chunk either replayed from a captured
 * hipGraph or launched directly, with one host sync per chunk.  A list
 * rebuild happens at a chunk boundary when any path length passed soft_frac *
 * r_buff/2.  If a chunk evaluated a force on a stale list (a path length
 * above r_buff/2) the state is restored from the snapshot of its list's build
 * and replayed up to the step where the soft threshold was first crossed;
 * the counter-based noise makes the replay exact.  Log rows (13 doubles: E,
 * W, K at that step, appended to ev_log, and one bond count appended to
 * bonds_log) are taken at every step index in [step0, step0 + n_steps) that
 * is a multiple of log_period (none for log_period 0) and at the end; a run
 * that continues the previous run's list (keep_list) skips the row of its
 * first state when the previous run's last row already holds it.
 * On an error return stats (if given) still holds steps_done and log_rows,
 * and pos / vel hold the state after steps_done steps; after
 * RC_ERR_NLIST_OVERFLOW with steps_done > 0 that state owes its last step's
 * final half kick, so the caller continues it (with a larger k_max) by a
 * call with resume = 1 for the remaining steps.  A single system detects an
 * overflow at the status read that ends the chunk after the build and then
 * returns the state at the build.  Buffers are caller owned: */
typedef struct rc_md_buffers {
    float* pos;        /* [N*4] state in/out                                  */
    float* pos_alt;    /* [N*4] second position buffer                        */
    float* vel;        /* [N*4] state in/out (on-step velocities)             */
    int* image;        /* [N*4] | NULL                                        */
    int* rtag;         /* [N]   | NULL (tag -> index after the last build)    */
    int* nlist;        /* [k_max*N]                                           */
    int* nn;           /* [N]                                                 */
    int k_max;
    int pad;
    void* cells_ws;    /* rc_cells_workspace_bytes                            */
    size_t cells_ws_bytes;
    float* snap_pos;   /* [N*4] | NULL (NULL disables rollback)               */
    float* snap_vel;   /* [N*4] | NULL                                        */
    int* snap_image;   /* [N*4] | NULL                                        */
    int* status;       /* [RC_STATUS_WORDS]                                   */
    double* ev_log;    /* [rows*13] | NULL, rows = n_steps/log_period + 1     */
    unsigned long long* bonds_log; /* [rows] | NULL                           */
    /* ev_log and bonds_log may be device memory or pinned host memory (the
       driver's kernels write them; the run's final status read waits for
       them); every other buffer is device memory.                          */
} rc_md_buffers;

typedef struct rc_md_options {
    int use_graph;      /* capture chunks as hipGraphs (1) or launch directly */
    int graph_steps;    /* steps per captured graph (even)                    */
    int max_chunk;      /* steps between host syncs (upper bound)             */
    int log_period;     /* rows at multiples of it and at the end; 0: the end */
    double soft_frac;   /* rebuild threshold as a fraction of r_buff/2        */
    int adapt;          /* 1: size chunks from the measured growth of the path
                           lengths so that rollbacks stay rare; 0: always
                           max_chunk steps (rollbacks repair stale chunks)    */
    int one_block;      /* 1: with use_graph, a system of at most 1024 particles
                           (walk or sums form) runs each graph_steps-step replay
                           as one launch of one workgroup that keeps the
                           positions in LDS (same results, bit for bit); 0:
                           hipGraphs only.  Ignored by rc_batch_run.          */
    int resume;         /* 1: the state owes its last step's final half kick
                           (it is what an earlier call left when it returned an
                           error after steps_done > 0): the first step applies
                           it, and n_steps = 0 applies just that kick.         */
    int keep_list;      /* 1: continue on the list of the previous run instead of
                           binning and building at entry, when the last call of
                           this context (batch) that changed the state was an
                           rc_md_run (rc_batch_run) that returned RC_OK with the
                           same buffers, N, box and k_max and ended at step
                           step0.  The caller promises that positions, images,
                           the list and the cell workspace were not changed since
                           (velocities may be).  Otherwise, and with resume = 1,
                           the run builds at entry.  A rollback into the epoch
                           the previous run began replays its steps from that
                           epoch's snapshot (same results).                    */
    int time_kernels;   /* 1: launch every step directly (no graphs, no
                           one-workgroup replays), each step kernel between its
                           own start and stop events; stats then sums their
                           execution times.  Results are the same bit for bit.
                           The defaults (opt = NULL) are
                           {1, 16, 256, 0, 0.8, 1, 1, 0, 1, 0}.                */
} rc_md_options;

typedef struct rc_md_stats {
    int64_t steps_done;
    int64_t rebuilds;
    int64_t rollbacks;
    int64_t chunks;
    int64_t log_rows;
    int32_t k_needed;   /* on RC_ERR_NLIST_OVERFLOW: the neighbour count found */
    int32_t flags;      /* last status flags                                  */
    int64_t kernel_launches; /* time_kernels: step-kernel launches timed      */
    double kernel_ms;   /* time_kernels: their summed execution time (ms)     */
    double sums_ms;     /* time_kernels, RC_FORM_SUMS: the first passes' time */
    int32_t list_kept;  /* 1: the run continued the previous run's list       */
    int32_t nswap;      /* RC_ST_NSWAP of the list in use at the end          */
    int64_t particles_rebuilt; /* summed over the run's list builds: the
                           particles whose lists each build rebuilt (every
                           particle for a single system; the replicas that
                           needed it, and those near it, for a batch)        */
} rc_md_stats;

int rc_md_run(rc_ctx* ctx, const rc_md_buffers* buf, int N, rc_box box,
              const rc_integrator* cfg /* host */, uint64_t step0, int n_steps,
              const rc_md_options* opt /* host, NULL = defaults */,
              rc_md_stats* stats /* host, NULL ok */, void* stream);

/* ---- FENE bond springs (supporting term of the bead-spring networks) -----------
 * rc_set_bonds: attach a bond table to the context (NULL bonds detaches it).
 *   bonds: device int32 [N][2], 8-byte aligned, indexed by TAG: the tags of
 *   up to two spring partners, -1 for none; every bond listed at both ends.
 *   rtag: device int32 [N], the tag -> index map that rc_build_cells keeps
 *   (pass the same array there; rc_md_run requires buf->rtag == rtag).  Both
 *   stay caller-owned and must outlive their use.  K > 0, R0 > 0: the spring
 *   U(r) = -(K R0^2 / 2) ln(1 - (r/R0)^2) of Kremer & Grest, on top of the
 *   pair table (bonded pairs keep their pair terms).  Once attached, every
 *   fused step (rc_step_fused, rc_md_run) adds the spring forces, energies and
 *   virials; a spring stretched to R0 gives a non-finite force (reported as
 *   RC_ERR_NONFINITE by the driver).  Batches take no bonds.
 * rc_fene_forces: the springs alone: force [N*4] += spring forces (w += half
 *   of each bond energy); ev (device, nullable) = 7 doubles E, W of the
 *   springs (overwritten).                                                     */
int rc_set_bonds(rc_ctx* ctx, const int* bonds /* [N*2] | NULL */, const int* rtag /* [N] */, int N, double K,
                 double R0);
int rc_fene_forces(rc_ctx* ctx, const float* pos, int N, rc_box box, float* force /* [N*4] */,
                   double* ev /* [7] | NULL */, void* stream);

/* ---- differentiation (hot-path step a7) --------------------------------------
 * rc_force_hvp: hv = H v with H = d^2 E / dx dx (FP32, per-particle float4,
 *   w ignored/zero): second derivatives of the pair terms (phi'', phi'/r) and
 *   of the triplets through vhat, vhat', vhat'' (vhat'' = -v''/eps beyond
 *   r_min, 0 inside; H is defined off the r_min and r_cut shells).  The force
 *   JVP is -hv.  Atomic-free gather (deterministic) in two passes: the first
 *   keeps every particle's switching sum and its derivative along v in
 *   context-owned scratch (16 bytes per particle), the second reads a
 *   partner's sums from there.
 * rc_param_grad: grad[(a*nt + b)*3 + {0,1,2}] = dE/d(eps, sigma, lambda) of the
 *   unordered entry {a, b} (reported on both (a,b) and (b,a)), FP64, fixed
 *   r_cut.  Device output, overwritten.
 * rc_param_vjp: out[(a*nt+b)*3 + w] = sum_m adj_m . dF_m/dtheta_w{a,b}
 *   (FP64, device, overwritten; adj is float4 with w ignored), for fitting
 *   through trajectories: closed-form derivatives of the pair force and of
 *   the three-body forces of eq. (3bp) written per centre as
 *   S P - Q (S = sum k u, P = sum k u' D, Q = sum k^2 u u' D, k = sqrt(lambda
 *   eps), D = rhat . (adj_a - adj_centre)).  At lambda_e = 0 the part of
 *   d/dlambda_e coupling entry e to other entries is reported as 0 (it is
 *   unbounded there), as in rc_param_grad.  One thread per centre; FP64
 *   partial sums per block reduced in a fixed order.
 * rc_set_table: replace eps, sigma and lambda of the table (host,
 *   ntypes^2, validated as in rc_create); kinds, exponents and r_cut must
 *   equal the current ones (RC_ERR_ARG otherwise), so list radii and cell
 *   grids stay valid.  Takes effect for launches issued after it returns.    */
int rc_force_hvp(rc_ctx* ctx, const float* pos, const int* nlist, const int* nn, int k_max, int N,
                 rc_box box, const float* v /* [N*4] */, float* hv /* [N*4] */, void* stream);
/* rc_force_hvp_batch: the products of nvec tangent vectors at once, v and hv
 *   [nvec][N*4] (device, 16-byte aligned, nvec in [1, 65535]); each product
 *   equals rc_force_hvp of that vector bit for bit.  One launch per pass
 *   covers every vector (grid rows), so small systems fill the GPU.  The
 *   context keeps 16 * N * nvec bytes of first-pass sums (grown on demand;
 *   growing synchronises the device).                                         */
int rc_force_hvp_batch(rc_ctx* ctx, const float* pos, const int* nlist, const int* nn, int k_max, int N,
                       rc_box box, int nvec, const float* v /* [nvec][N*4] */, float* hv /* [nvec][N*4] */,
                       void* stream);
int rc_param_grad(rc_ctx* ctx, const float* pos, const int* nlist, const int* nn, int k_max, int N,
                  rc_box box, double* grad /* [nt*nt*3] */, void* stream);
int rc_param_vjp(rc_ctx* ctx, const float* pos, const int* nlist, const int* nn, int k_max, int N,
                 rc_box box, const float* adj /* [N*4] */, double* out /* [nt*nt*3] */,
                 void* stream);
int rc_set_table(rc_ctx* ctx, const rc_pair_coeff* table /* host [ntypes*ntypes] */);
/* Soft bond count: value (device double, overwritten) = sum over swap pairs
 * i<j inside r_cut of vhat(r_ij) (eq. pot: 1 for a bonded pair, r <= r_min,
 * falling to 0 at r_cut), so it equals rc_bond_count whenever no swap pair
 * sits between r_min and r_cut; grad (device float4 [N], w = 0, nullable)
 * receives dvalue/dx.  A differentiable bond observable for fits.          */
int rc_soft_bonds(rc_ctx* ctx, const float* pos, const int* nlist, const int* nn, int k_max, int N,
                  rc_box box, double* value /* [1] */, float* grad /* [N*4] | NULL */, void* stream);

/* ---- batches of independent replicas (hot-path step a8) -----------------------
 * A batch holds R independent periodic systems of uneven size, box and
 * coefficient table (e.g. a lambda sweep) and advances all of them with one
 * launch per kernel: the cell sort, the list build, the fused step and the
 * bond count each cover every replica at once.
 *
 * Slots.  Replica r owns the particle slots [off_r, off_r + n_r) of every
 * per-particle array; off_0 = 0 and off_{r+1} = off_r + 64*ceil(n_r/64), so
 * each wavefront lies in one replica.  The slots between replicas are unused
 * (zeroed by rc_batch_build_cells; nn = 0 there).  n_slots = off_R is the
 * length N of every per-particle array (pos, vel, image, nlist column, nn,
 * force); rc_batch_layout reports it and the offsets.  A particle's tag is
 * its global tag, off_r + (its tag inside the replica); the thermostat noise
 * uses the tag inside the replica and the replica's seed, so replica r of a
 * batch follows the same trajectory, bit for bit, as the same system run
 * alone with rc_md_run and that seed.
 *
 * rc_batch_create: tables is host [R][ntypes][ntypes] (one table per
 *   replica, validated like rc_create's), counts host [R] (n_r >= 1), boxes
 *   host [R].  Each replica's cell grid follows its own table's largest list
 *   radius.  Fails with RC_ERR_ARG on an invalid table, count or box and with
 *   RC_ERR_UNSUPPORTED when R > 65535, n_slots >= 2^27 or the batch needs
 *   more than 2^24 cell keys.
 * rc_batch_set_seeds: host [R] thermostat keys (default: cfg.seed + r).
 * rc_batch_set_gather_width, rc_batch_set_step_form: as rc_set_gather_width
 *   and rc_set_step_form, for the batch.
 * rc_batch_compute_forces: force [n_slots*4] as rc_compute_forces with
 *   RC_FORCE_GATHER, or RC_FORCE_SUMS when the batch's step form is
 *   RC_FORM_SUMS (overwritten; unused slots untouched); ev = device
 *   [R][7] (E, W) per replica, or NULL.
 * rc_batch_bond_count: counts = device [R] u64, overwritten.
 * rc_batch_step_fused: one fused step of every replica (modes as
 *   rc_step_fused); ev = device [R][13] or NULL; status as rc_step_fused.
 * rc_batch_run: rc_md_run over the whole batch: buf arrays are n_slots long,
 *   ev_log is [rows][R][13] and bonds_log [rows][R].  A list build of the
 *   batch happens when any replica needs one, and rebuilds only the replicas
 *   whose own particles crossed the rebuild threshold plus those whose
 *   largest path length since their own last build exceeds margin x that
 *   threshold (rc_batch_set_rebuild_margin); the other replicas keep their
 *   order, lists and path lengths.  The first build of a run covers every
 *   replica; the first build of a resumed run (opt.resume = 1, after
 *   RC_ERR_NLIST_OVERFLOW) covers the replicas of the build that overflowed.
 *   stats->particles_rebuilt counts the rebuilt particles.  Synchronises the
 *   stream.
 * rc_batch_set_rebuild_margin: margin in [0, 1] (default 0.3); 0 rebuilds
 *   every replica at every build, 1 only the replicas that crossed.
 * rc_batch_relayout_lists: copies the lists of every slot from old_nlist
 *   (k_old slots per particle) into new_nlist (k_new >= k_old) and writes
 *   their packed copy for k_new into the attached workspace (which must hold
 *   k_new), so that a run resumed after RC_ERR_NLIST_OVERFLOW with larger
 *   lists keeps the lists of the replicas it does not rebuild.  nn is the
 *   count array both lists share.  Launches on the stream.
 * rc_batch_build_nlist also writes the packed copy of the lists that the
 *   batch's fused step reads (as rc_build_nlist does for one system).
 * rc_batch_time_fused_steps: as rc_time_fused_steps for the batch.
 * rc_batch_workspace_bytes / rc_batch_set_workspace: as rc_workspace_bytes /
 *   rc_set_workspace for the batch's n_slots slots (no tangent vectors).    */
typedef struct rc_batch rc_batch;

int rc_batch_create(rc_batch** out, int R, int ntypes, const rc_pair_coeff* tables /* host */,
                    const int* counts /* host [R] */, const rc_box* boxes /* host [R] */, double r_buff);
int rc_batch_destroy(rc_batch* b);
const char* rc_batch_last_error(const rc_batch* b);
int rc_batch_layout(const rc_batch* b, int* n_slots /* host */, int* offsets /* host [R+1] | NULL */);
int rc_batch_set_seeds(rc_batch* b, const uint64_t* seeds /* host [R] */);
int rc_batch_set_gather_width(rc_batch* b, int width);
int rc_batch_workspace_bytes(const rc_batch* b, int k_max, size_t* bytes /* host */);
int rc_batch_set_workspace(rc_batch* b, void* ws, size_t bytes, int k_max);
int rc_batch_set_step_form(rc_batch* b, int form);
int rc_batch_cells_workspace_bytes(const rc_batch* b, size_t* bytes /* host */);
int rc_batch_build_cells(rc_batch* b, float* pos, float* vel, int* image, int* rtag, void* ws, size_t ws_bytes,
                         void* stream);
int rc_batch_build_nlist(rc_batch* b, const float* pos, float* vel, const void* ws, size_t ws_bytes, int k_max,
                         int* nlist, int* nn, int* status, void* stream);
int rc_batch_compute_forces(rc_batch* b, const float* pos, const int* nlist, const int* nn, int k_max, float* force,
                            double* ev /* [R*7] | NULL */, int* status, void* stream);
int rc_batch_bond_count(rc_batch* b, const float* pos, const int* nlist, const int* nn, int k_max,
                        unsigned long long* counts /* [R] */, void* stream);
int rc_batch_step_fused(rc_batch* b, const float* pos_in, float* pos_out, float* vel, int* image, const int* nlist,
                        const int* nn, int k_max, const rc_integrator* cfg /* host */, uint64_t step, int mode,
                        double soft_frac, double* ev /* [R*13] | NULL */, int* status, void* stream);
int rc_batch_run(rc_batch* b, const rc_md_buffers* buf, const rc_integrator* cfg /* host */, uint64_t step0,
                 int n_steps, const rc_md_options* opt /* host, NULL = defaults */,
                 rc_md_stats* stats /* host, NULL ok */, void* stream);
int rc_batch_time_fused_steps(rc_batch* b, float* pos_a, float* pos_b, float* vel, const int* nlist, const int* nn,
                              int k_max, const rc_integrator* cfg /* host */, uint64_t step0, int reps, int* status,
                              float* ms /* host */, void* stream);
int rc_batch_set_rebuild_margin(rc_batch* b, double margin);
int rc_batch_relayout_lists(rc_batch* b, const int* old_nlist, int k_old, int* new_nlist, int k_new, const int* nn,
                            void* stream);

#ifdef __cplusplus
}
#endif

#endif /* RC_H */
