/*
 * csfmm.h -- C ABI of the cubed sphere fast multipole method (CSFMM) on one
 * AMD MI355X (gfx950).
 *
 * The library evaluates N-body sums on the unit sphere (paper §1, eq.
 * nbodysum):
 *
 *     phi(x_i) = sum_j K(x_i, y_j) w_j ,   i = 1..n_t,
 *
 * for target points x_i and source points y_j on the unit sphere with source
 * weights w_j, by the CSFMM of paper §8 (Algorithm 2): quadtrees of
 * equiangular cubed-sphere cells (§3), barycentric Lagrange interpolation at
 * tensor Chebyshev proxy points in each cell (§4), the four interactions PP,
 * PC, CP and CC (§5), the upward pass (§6), a dual tree traversal with the
 * MAC (r_t + r_s)/R < theta (§8) and the downward pass (§8.1).  The singular
 * self term is omitted (§1): a source is skipped for a target exactly when
 * their coordinates are equal.
 *
 * Conventions for every call:
 *   - Array pointers are DEVICE pointers (for example a torch tensor's
 *     data_ptr()), float64, C order.  Points are [n][3] (x, y, z).
 *   - `stream` is a hipStream_t (NULL = the null stream).  Work is ordered on
 *     that stream; only csfmm_plan waits for the device.
 *   - Inputs and outputs stay owned by the caller.  A plan owns its own device
 *     memory until csfmm_plan_destroy.
 *   - Results are in the caller's point order.
 *   - Every call returns CSFMM_OK (0) or a negative csfmm_status; no
 *     exception or abort crosses the boundary.  csfmm_last_error() then
 *     returns a message for the calling thread.
 *   - Argument errors are detected on the host before any launch.
 */
#ifndef CSFMM_H
#define CSFMM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct csfmm_plan_s* csfmm_plan_t;
typedef struct csfmm_workspace_s* csfmm_workspace_t;

enum csfmm_status {
    CSFMM_OK = 0,
    CSFMM_E_INVALID = -1,       /* bad argument (size, degree, theta, kernel, pointer) */
    CSFMM_E_NOT_ON_SPHERE = -2, /* a point is not finite or | |x| - 1 | > 1e-12 */
    CSFMM_E_OOM = -3,           /* device allocation failed */
    CSFMM_E_HIP = -4,           /* a HIP runtime call failed */
    CSFMM_E_BUSY = -5,          /* reserved */
    CSFMM_E_UNSUPPORTED = -6,   /* reserved */
    CSFMM_E_INTERNAL = -7       /* a kernel reported a broken internal bound (its result is void) */
};

/* Kernels K(x, y) for x, y on the unit sphere (paper §2). */
enum csfmm_kernel {
    CSFMM_K_POISSON_LOG = 1, /* -(1/4pi) ln(1 - x.y), eq. (G_L); one output */
    CSFMM_K_BIOT_SAVART = 2, /* -(1/4pi) (x cross y)/(1 - x.y), eq. (K_BS); three outputs */
    CSFMM_K_INV_DIST = 3,    /* 1/|x - y| = 1/gamma(x, y), the first term of eq. (G_SAL_approx) */
    CSFMM_K_BIHARMONIC = 4,  /* (1/4pi) dilog((1 + x.y)/2), eq. (G_B); one output */
    CSFMM_K_SAL = 5          /* eq. (G_SAL_approx): (3 rw/(4pi re)) ((1 - b0)/gamma
                                - (a1 - b1) ln(gamma/2 + gamma^2/4)), gamma = |x - y|,
                                a1 = -2.7, b0 = -6.21196, b1 = 6.1, rw/re = 1025/5514
                                (the ratio is named, not given, in §2.4); one output */
};

/* Precision forms, and cluster shrinking (a plan option). */
enum csfmm_flags {
    CSFMM_FP64 = 0,      /* every step in FP64 */
    CSFMM_FP32_FORM = 1, /* kernel evaluations (PP, PC, CP, CC, direct) in FP32 on
                            coordinates recentred at the target cell in FP64;
                            partial sums added into FP64; geometry, mapping,
                            interpolation and final sums in FP64 */
    CSFMM_SHRINK = 2     /* csfmm_plan only (paper §3, the remark on nonuniform
                            particles): each non-empty cluster's box -- centre,
                            radius, proxies, local coordinates -- is the smallest
                            (xi, eta) rectangle holding its points, half widths at
                            least 2^-20 of its cell's; the tree keeps its quadrants,
                            and the operators of eqs. (upwardpass2) and
                            (downward_2) become per cluster */
};

typedef struct csfmm_stats {
    int64_t n_targets, n_sources;
    int32_t same_set, kernel, p, leaf_size;
    double theta;
    uint32_t flags;
    int32_t depth_t, depth_s;              /* deepest level (roots are level 0) */
    int64_t n_cells_t, n_cells_s;          /* all levels */
    int64_t n_leaves_t, n_leaves_s;
    int64_t n_pp, n_pc, n_cp, n_cc;        /* (target cell, source cell) pairs */
    int64_t evals_pp, evals_pc, evals_cp, evals_cc; /* kernel evaluations per eval */
    int64_t device_bytes;                  /* device memory the plan holds */
    int64_t max_leaf_t;                    /* most points in a target leaf */
    int64_t pp_sym_pairs, pp_one_way;      /* same-set plans: PP entries of distinct leaves
                                              that hold both ways, counted once per pair,
                                              and those that hold one way (on the
                                              one-wave-per-leaf near field the scalar
                                              kernels evaluate a pair once for both
                                              directions); 0 otherwise */
    int64_t pp_close;                      /* FP32 form: PP entries of non-overlapping
                                              leaves whose points may come so close that
                                              the expanded squared distance would lose
                                              more than ~1e-4 of it; they take exact
                                              differences (and no symmetric pairs) */
    int64_t near_wave;                     /* 1: the near field takes one wave per target
                                              leaf (leaves of at most 64 points, at least
                                              8 leaves per compute unit); 0: one block of
                                              four waves per leaf */
} csfmm_stats;

/*
 * Build a plan: trees, cell geometry and proxy points, the fixed parent-child
 * interpolation matrices and the PP/PC/CP/CC interaction lists (paper §3, §4,
 * §8 Algorithm 2, tree and traversal; the lists depend only on the points, p,
 * theta and N0, not on the weights).
 *
 *   targets   [n_t][3] device, unit vectors; copied into the plan
 *   sources   [n_s][3] device, or NULL: the sources are the targets (one tree,
 *             i = j omitted); copied into the plan
 *   kernel_id csfmm_kernel; the default kernel of csfmm_eval
 *   p         interpolation degree n of the paper, 1..16; (p+1)^2 proxies per cell
 *   theta     MAC parameter, 0 < theta < 1
 *   leaf_size N0: a cell with more than N0 points is split (deepest level 20)
 *   flags     csfmm_flags
 *   out       receives the plan handle
 * n_t, n_s >= 1.  Waits for the device (list sizes are data dependent).
 * Errors: CSFMM_E_INVALID, CSFMM_E_NOT_ON_SPHERE, CSFMM_E_OOM, CSFMM_E_HIP.
 */
int csfmm_plan(const double* targets, int64_t n_t, const double* sources, int64_t n_s,
               int kernel_id, int p, double theta, int leaf_size, unsigned flags,
               void* stream, csfmm_plan_t* out);

/*
 * Apply a plan to source weights (§8 Algorithm 2 after the traversal): upward pass
 * (P2M, M2M), interactions (PP, PC, CP, CC), downward pass (L2L, L2P).
 *   weights [n_s] device (for a same-set plan n_s = n_t)
 *   out     [n_t] device, or [n_t][3] for Biot-Savart
 * Asynchronous on `stream`; weights must stay valid and out must not be read
 * until the stream work completes.  One eval in flight per plan.  The PP near
 * field runs on a side stream of the plan's workspace, forked from and joined
 * back into `stream` with events, so work ordered after the eval on `stream`
 * sees all of it (this also holds under stream capture).
 */
int csfmm_eval(csfmm_plan_t plan, const double* weights, double* out, void* stream);

/* As csfmm_eval, with the kernel given per call instead of the plan's
 * default (the plan is geometry only). */
int csfmm_eval_kernel(csfmm_plan_t plan, int kernel_id, const double* weights, double* out,
                      void* stream);

/*
 * Cubed sphere treecode (paper §7, Algorithm 1), the paper's O(N log N)
 * comparison method, on the plan's source tree: the upward pass (P2M, M2M)
 * as in csfmm_eval, then for every target particle x a traversal of the
 * source tree from the six roots: a cluster with r^2 < theta^2 R^2 (r its
 * radius, R the chord distance from x to its centre) and more than leaf_size
 * points interacts by PC (eq. PC, its proxies and proxy weights); a separated
 * cluster with at most leaf_size points, or a leaf that is not separated, by
 * PP (eq. PP, its particles, exact coincidences omitted); other clusters are
 * opened into their children.  Always FP64, whatever the plan's flags.
 *   weights [n_s] device, out [n_t] or [n_t][3] device (caller order).
 * Waits for `stream` before it returns: the traversal's stack (72 entries
 * per wave; 66 suffice for 20 levels) reports an overflow in a status word
 * that is read back, and the call then fails with CSFMM_E_INTERNAL instead
 * of returning a sum with clusters left out.  Uses the plan's own workspace,
 * so it must not overlap a csfmm_eval of the same plan.
 * Errors: CSFMM_E_INVALID (NULL pointer, kernel id), CSFMM_E_INTERNAL,
 * CSFMM_E_HIP.
 */
int csfmm_eval_treecode(csfmm_plan_t plan, int kernel_id, const double* weights, double* out,
                        void* stream);

/*
 * One classical 4th order Runge-Kutta step of the barotropic vorticity
 * equation on the rotating sphere by the Lagrangian vortex method (paper
 * §2.3, eqs. BVE and BVE_ODEs; §12): dx_i/dt = sum_j K_BS(x_i, x_j) zeta_j A_j
 * and dzeta_i/dt = -2 omega dz_i/dt.  Every stage builds a plan on the stage
 * positions (kernel Biot-Savart, p, theta, leaf_size, flags as in csfmm_plan)
 * and evaluates with it, or uses csfmm_direct when use_direct != 0; stage and
 * final positions are projected back onto the sphere.
 *   x [n][3] (unit vectors) and zeta [n]: device, updated in place;
 *   area [n] device (the particles' fixed areas A_i); dt > 0; omega the
 *   rotation rate (2 pi per day in the paper's units).
 * Waits for `stream` after each stage eval (plans are rebuilt per stage).
 * Errors: CSFMM_E_INVALID, CSFMM_E_NOT_ON_SPHERE, CSFMM_E_OOM, CSFMM_E_HIP.
 */
int csfmm_bve_rk4_step(double* x, double* zeta, const double* area, int64_t n, double dt,
                       double omega, int p, double theta, int leaf_size, unsigned flags,
                       int use_direct, void* stream);

/*
 * Remeshing of the vortex particles (paper §12: after every step, by local
 * biquadratic interpolation) onto the equiangular cubed-sphere grid of E cells
 * per face edge, N = 6 E^2.  The particles started the step at the cell
 * centres and ended at x.  Each cell centre y takes the vorticity that the
 * flow carried to it.  Its departure point a solves normalize(a + D(a)) = y,
 * with D the biquadratic interpolant of the displacements x - grid, by 8
 * fixed-point steps a <- normalize(y - D(a)) from a = y.  The new vorticity
 * is q(a) - 2 omega z(y), with q the interpolant of the absolute vorticities
 * zeta + 2 omega z(x).  Interpolation uses the 3 x 3 stencil of the nearest
 * node on the face of the point, with the three-point Lagrange weights in
 * the face angles.  Nodes beyond a face edge are ghosts: each lies on a node
 * line of the neighbouring face, where its value comes from a stencil
 * clamped to that face.
 *   grid [N][3] device: the cell centres.  Point f E^2 + i E + j is the
 *     centre of cell (i, j) of face f, at face angles
 *     -pi/4 + (i + 1/2) pi/(2E) along e1 and -pi/4 + (j + 1/2) pi/(2E) along
 *     e2.  The frames (n, e1, e2) of faces 0..5 are:
 *       (+x, +y, +z), (-x, +z, +y), (+y, +z, +x),
 *       (-y, +x, +z), (+z, +x, +y), (-z, +y, +x).
 *     Must not overlap x.
 *   x [N][3] device: the particles' end positions in grid order.  Set to
 *     grid on return.
 *   zeta [N] device: the particles' vorticity, replaced by the remeshed
 *     vorticity at the cell centres.
 *   omega: the rotation rate.
 * Asynchronous on `stream`; the call allocates 32 N bytes of stream-ordered
 * scratch.
 * Errors: CSFMM_E_INVALID (NULL arrays, E outside [3, 16384], a non-finite
 * omega, any two of grid, x and zeta overlapping), CSFMM_E_OOM, CSFMM_E_HIP.
 */
int csfmm_bve_remesh(const double* grid, int64_t E, double* x, double* zeta, double omega,
                     void* stream);

/*
 * Direct sum of paper eq. (nbodysum) over all pairs (the O(N^2) method of §1):
 * out[i] = sum_j K(x_i, y_j) w_j with exact coincidences omitted.
 *   targets [n_t][3], sources [n_s][3], weights [n_s], out [n_t] or [n_t][3].
 *   flags CSFMM_FP64 or CSFMM_FP32_FORM (FP32 evaluation on hi/lo split
 *   coordinates, FP64 partial sums).  Asynchronous on `stream`.
 */
int csfmm_direct(const double* targets, int64_t n_t, const double* sources, int64_t n_s,
                 const double* weights, int kernel_id, unsigned flags, double* out,
                 void* stream);

/*
 * csfmm_direct for callers that cannot allocate device memory (code under
 * HIP graph capture, serving loops that forbid hipMalloc): the same
 * arguments, kernels and result, bit for bit, with no hipMalloc, hipFree or
 * other allocating call.  The partial sums over source splits go to a static
 * scratch array of 4 Mi doubles (32 MiB) that each GPU the library runs on
 * holds until the process ends; so n_t is at most 4,194,304 (1,398,101 for
 * Biot-Savart, three outputs), and larger n_t fails with CSFMM_E_INVALID
 * before any launch.  Every call on one GPU uses that GPU's one array:
 * calls that overlap on a GPU (other streams, other host threads) race and
 * must be ordered by the caller.  The array needs no clearing (every
 * partial sum is written before it is read).  Asynchronous on `stream`.
 */
int csfmm_direct_noalloc(const double* targets, int64_t n_t, const double* sources,
                         int64_t n_s, const double* weights, int kernel_id, unsigned flags,
                         double* out, void* stream);

/*
 * Serving: several requests evaluated together (continuous batching).
 * A workspace holds one request's eval buffers (sorted weights, proxy
 * weights, proxy potentials, near field) and the side stream of its PP near
 * field (a packed eval uses the side stream of workspaces[0]) for a given
 * plan, so one resident
 * plan can serve several in-flight requests.  csfmm_eval_many runs the eval
 * phases of n_req requests with one packed launch per phase (per kernel id and
 * precision form for the near and far field): request r uses plans[r] with
 * workspaces[r] (created for that plan), kernel_ids[r] (NULL: each plan's
 * default), weights[r] [n_s] and outs[r] [n_t] or [n_t][3].  Each request's
 * arithmetic is the same as csfmm_eval's, whatever it is batched with.
 * A workspace must not be used by two evals in flight at once.
 * Signature: this adds the `workspaces` argument to the plain
 * (n_req, plans, kernel_ids, weights, outs, stream) form.  A plan's buffers
 * for one eval (proxy weights, proxy potentials, near field) cannot be shared
 * by two requests in flight, so the caller names the workspace of each
 * request; that is what lets one resident plan serve several requests at once
 * instead of allocating per call.
 */
int csfmm_workspace_create(csfmm_plan_t plan, void* stream, csfmm_workspace_t* out);
                                                        /* waits for `stream` */
int csfmm_workspace_destroy(csfmm_workspace_t ws);     /* waits for the device; NULL is OK */
int64_t csfmm_workspace_bytes(csfmm_plan_t plan);       /* device bytes of one workspace */
int64_t csfmm_workspace_device_bytes(csfmm_workspace_t ws); /* bytes this workspace holds */
int csfmm_eval_many(int n_req, const csfmm_plan_t* plans, const csfmm_workspace_t* workspaces,
                    const int* kernel_ids, const double* const* weights, double* const* outs,
                    void* stream);

/*
 * Continuous-batching scheduler (host only; it decides, the caller executes).
 * Requests are submitted with a plan key (equal keys share one resident plan),
 * the device bytes of that plan and of one workspace (csfmm_workspace_bytes)
 * and a cost estimate (>= 0, any unit, e.g. points).  csfmm_sched_step(now)
 * starts one batch of at most max_batch with the oldest waiting request
 * (t_arrival <= now) and adds, in arrival order, waiting requests whose cost
 * is within a factor 4 of its cost while their memory fits the budget
 * (others wait for a later batch, which the caller may run on another stream
 * beside this one), and reports what the caller must do before launching it:
 *   evict_keys  destroy these resident plans and their workspaces (idle, LRU)
 *   build_keys  build these plans
 *   new_ws_keys create one more workspace for each listed plan key
 *   launch_ids  run these requests now (one csfmm_eval_many)
 *   reject_ids  these requests can never fit the budget
 * A resident plan keeps a pool of workspaces as large as its peak number of
 * requests in flight; csfmm_sched_complete returns one to the pool. The oldest
 * waiting request starts every batch, and within a cost class no request
 * overtakes an older one. Every array is caller owned; cap_* is its room
 * (new_ws_keys has room for cap_launch).
 */
typedef struct csfmm_sched_s* csfmm_sched_t;
typedef struct csfmm_sched_decision {
    int64_t* launch_ids;  int cap_launch;  int n_launch;
    uint64_t* build_keys; int cap_build;   int n_build;
    uint64_t* new_ws_keys;                 int n_new_ws;
    uint64_t* evict_keys; int cap_evict;   int n_evict;
    int64_t* reject_ids;  int cap_reject;  int n_reject;
} csfmm_sched_decision;
typedef struct csfmm_sched_stats {
    int64_t submitted, launched, completed, rejected, batches;
    int64_t plan_hits, plan_misses, evictions;
    int64_t used_bytes, budget_bytes, queued, in_flight, resident_plans;
} csfmm_sched_stats;
int csfmm_sched_create(int64_t hbm_budget_bytes, int max_batch, csfmm_sched_t* out);
int csfmm_sched_destroy(csfmm_sched_t s);
int csfmm_sched_submit(csfmm_sched_t s, int64_t req_id, uint64_t plan_key, int64_t plan_bytes,
                       int64_t ws_bytes, double t_arrival, double cost);
int csfmm_sched_step(csfmm_sched_t s, double now, csfmm_sched_decision* d);
int csfmm_sched_complete(csfmm_sched_t s, int64_t req_id, double now);
int csfmm_sched_get_stats(csfmm_sched_t s, csfmm_sched_stats* out);

/* Release a plan's device memory (waits for the device first). NULL is OK.
 * Workspaces of the plan must be destroyed first. */
int csfmm_plan_destroy(csfmm_plan_t plan);

/* Sizes and interaction counts of a plan. */
int csfmm_plan_stats(csfmm_plan_t plan, csfmm_stats* s);

/*
 * Per-stage timing of csfmm_eval with HIP events recorded on the eval's
 * streams.  enable = 1 times every stage, 2 only the two interaction
 * launches, [2], [3] and [5] below (two events on the side stream around PP,
 * two on the eval stream around [3] and one after its join with PP; the other
 * sums stay 0), 0 turns timing off; turning it on resets the sums.
 * csfmm_plan_timing_read waits for the recorded events and returns the summed
 * milliseconds of the 6 stages over the timed evals (stage_ms holds 6):
 *   [0] weight gather + P2M, [1] M2M (and zeroing the proxy potentials),
 *   [2] the PP near-field launch, which runs on the workspace's side stream
 *   concurrently with [0], [1] and [3], [3] PC near field and CP + CC far
 *   field in one launch, [4] L2L + L2P + scatter in one launch, including the
 *   wait for [2], [5] the span of the two interaction launches: from the PP
 *   launch's start on the side stream to the eval stream's join with it, after
 *   both have ended (PP is queued first and starts first).
 */
int csfmm_plan_timing(csfmm_plan_t plan, int enable);
int csfmm_plan_timing_read(csfmm_plan_t plan, double* stage_ms /*[6]*/, int64_t* n_evals);

/* Upper estimate of the device bytes a plan of these sizes holds (for
 * admission control); -1 on bad arguments. */
int64_t csfmm_estimate_bytes(int64_t n_t, int64_t n_s, int p, int leaf_size, unsigned flags);

/* Message of the last error on the calling thread ("" if none). */
const char* csfmm_last_error(void);

/* ------------------------------------------------------------------------
 * Inspection calls: copy a plan's internals to HOST memory, for checking the
 * tree, geometry and lists against an independent builder.  `which` is 0 for
 * the target tree, 1 for the source tree (the same tree for a same-set plan).
 * ---------------------------------------------------------------------- */

/* Cells in breadth-first order (level by level, Morton order in a level;
 * the four children of a cell are consecutive).  Each array has n_cells
 * entries (csfmm_plan_stats); any pointer may be NULL to skip it.
 *   level, face, ci, cj: cell (face 0..5: +x, +y, -x, -y, +z, -z; index
 *     (ci, cj) in the level's 2^l x 2^l grid of local angles (xi, eta))
 *   begin, count: range of the cell's points in the plan's sorted order
 *   child0: index of the first child, -1 for a leaf
 *   center [n][3], radius [n]                                           */
int csfmm_plan_cells(csfmm_plan_t plan, int which, int32_t* level, int32_t* face, int32_t* ci,
                     int32_t* cj, int32_t* begin, int32_t* count, int32_t* child0,
                     double* center, double* radius);

/* Proxy points of every cell: [n_cells][(p+1)^2][3], proxy (k1, k2) at
 * k1*(p+1)+k2 is the image of (xi_mid + h s_k1, eta_mid + h s_k2). */
int csfmm_plan_proxies(csfmm_plan_t plan, int which, double* proxies);

/* Sorted order: perm[k] = caller index of the k-th point in sorted order. */
int csfmm_plan_permutation(csfmm_plan_t plan, int which, int64_t* perm);

/* Interaction list `kind` (0 PP, 1 PC, 2 CP, 3 CC) as (target cell, source
 * cell) pairs grouped by target cell; within a target the PP entries whose
 * cells overlap it (the only ones that can hold coincident points) come
 * first, then entries by source index; cap = room in tgt/src. */
int csfmm_plan_list(csfmm_plan_t plan, int kind, int32_t* tgt, int32_t* src, int64_t cap);

/* Eval that also copies the stage results to DEVICE buffers (NULL skips);
 * KS = (p+1)^2 rounded up to a multiple of 4 (the entries past (p+1)^2 are 0):
 *   wbar [n_cells_s][KS]        proxy weights after the upward pass
 *   psi  [vdim][n_cells_t][KS]  proxy potentials: at the target leaves after the
 *                               downward pass (eq. downward_2 through all levels),
 *                               at the other cells their own CP + CC sums
 *                               (eq. CP_CC_accumulated)
 *   near [n_t][vdim] PP+PC part of phi in the caller's order
 * where vdim = 3 for Biot-Savart, else 1. */
int csfmm_eval_stages(csfmm_plan_t plan, int kernel_id, const double* weights, double* out,
                      double* wbar, double* psi, double* near, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* CSFMM_H */
