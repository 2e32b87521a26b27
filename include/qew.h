/*
 * qew.h -- C ABI of libqew, the MI355X (gfx950) engine for the non-steady
 * relaxation of a driven elastic line in a random medium: the quenched
 * Edwards-Wilkinson (QEW) equation of Ferrero, Bustingorry and Kolton,
 * "Non-steady relaxation and critical exponents at the depinning transition"
 * (arXiv:1211.7275).
 *
 * What the library computes (the paper's method, Secs. II and III B):
 *   - Eq. (1) with eta = 1, discretised in x with dx = 1 on a periodic chain
 *     of L sites and integrated by the explicit Euler method (Sec. III B):
 *       u_j <- u_j + dt * [ c (u_{j+1} + u_{j-1} - 2 u_j) + f + F_p(j, u_j) ]
 *     synchronously over all sites, from the flat start u_j = 0 (Sec. II).
 *   - F_p: random values at the integer points (j, n) of the (x, u) plane,
 *     generated on demand (the paper's memory-free disorder, Sec. IV D) and
 *     interpolated in u by a cubic (Catmull-Rom) spline (Sec. III B).  Random
 *     field: the values are forces, uniform in (-1, 1).  Random bond: the
 *     values are potential energies, N(0, 1), and F_p = -dU/du (Sec. II).
 *     Also the paper's Case 3 (Gaussian potential, linear spline) and Case 4
 *     (Gaussian forces, no interpolation) of Sec. IV C, and an optional
 *     transverse period M of the medium in u (Sec. III B).
 *     Values are scaled by `strength`.  Generator: Philox4x32-10 (Salmon et
 *     al., SC'11) with counter (j, (uint32) n, disorder_id, 0) and key
 *     (seed low word, seed high word).
 *   - Observables of Sec. II, Eqs. (3)-(5), per sample s at every requested
 *     measurement step m: v_s(m) = mean over j of the total force at step m
 *     (equal to the mean of du/dt), ubar_s(m) = mean of u_j, and
 *     w2_s(m) = mean of (u_j - ubar_s)^2, all accumulated in FP64.  The
 *     disorder average (the overbar of Eqs. (3)-(5)) is the mean over samples,
 *     which the caller forms from the per-sample series.
 *
 * Conventions for every call:
 *   - Device pointers (`d_` prefix, and the workspace) are HIP device
 *     memory owned by the caller; host pointers (`h_` prefix and the
 *     problem's arrays) are ordinary host memory owned by the caller.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *   - Every call returns a qew_status; nothing aborts and no C++ exception
 *     crosses the ABI.  On failure qew_last_error() returns a message,
 *     thread-local and valid until the next call on that thread.
 *   - All validation of a problem happens in qew_plan, on the host, with no
 *     device call, so it can be tested without a GPU.
 */
#ifndef QEW_H
#define QEW_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t qew_status;
#define QEW_OK            0
#define QEW_EINVAL       (-1) /* bad argument or problem; nothing was launched      */
#define QEW_ENOMEM       (-2) /* workspace smaller than qew_workspace_bytes()       */
#define QEW_EDEVICE      (-3) /* HIP error; workspace contents undefined, plan valid */
#define QEW_EUNSUPPORTED (-4) /* valid but not implemented combination             */

/* disorder kinds (Sec. III B; RF = random field, RB = random bond; Sec. IV C cases) */
#define QEW_RF_CR_UNIFORM 0   /* force values uniform in (-1,1), Catmull-Rom in u     */
#define QEW_RB_CR_GAUSS   1   /* potential values N(0,1), Catmull-Rom, F_p = -dU/du   */
#define QEW_RB_LIN_GAUSS  2   /* Case 3: potential N(0,1), linear in u: F_p = -(V(n+1) - V(n)) */
#define QEW_RF_PC_GAUSS   3   /* Case 4: force values N(0,1), no interpolation: F_p = R(n)    */

/* arithmetic of the integrator */
#define QEW_FP64_PLAIN 0      /* u in FP64                                             */
#define QEW_FP32_SPLIT 1      /* u = int32 cell + FP32 offset in [0,1); FP64 sums     */

/* kernel path */
#define QEW_ONE_STEP 0        /* one Euler step per launch, all 4 nodes regenerated    */
#define QEW_FUSED    1        /* k Euler steps per launch on register tiles with halos */

/* qew_problem.flags */
#define QEW_FLAG_NO_GRAPH 1   /* launch every kernel directly instead of replaying hipGraphs */
#define QEW_FLAG_TIMING   2   /* record hipEvents around the stepping kernels (qew_run_stats) */
/*
 * The fused path runs stretches between measurements that are shorter than
 * four steps with the one-step kernel (same arithmetic, same results).
 *
 * The fused path has two variants of its kernel with identical results: the
 * dense one posts the cell changes of every sub-step slot by slot; the sparse
 * one first checks whether any site of a wave changed cell and skips the
 * bookkeeping when none did (faster for pinned or slow lines, slower for
 * moving ones).  qew_run starts dense and, before each stretch of steps
 * between two measurements, picks the variant from the velocities of the
 * measurement before last (a line at velocity v changes cell about v dt times
 * per site and step).  These flags force one variant; they are rejected
 * (QEW_EINVAL) on the one-step path.
 */
#define QEW_FLAG_FUSED_DENSE  4
#define QEW_FLAG_FUSED_SPARSE 8

/*
 * One batch of independent samples sharing c, dt, disorder kind/strength,
 * seed and measurement steps (the paper's parameters: L and dx = 1 in
 * Sec. III B; c, eta = 1 and f in Eq. (1); RF/RB and the value distribution
 * in Sec. II; independent disorder realisations averaged by the overbar).
 * Arrays are read only during qew_plan (copied into the plan).
 */
typedef struct qew_problem {
  int32_t         n_samples;    /* S >= 1                                               */
  int32_t         kind;         /* QEW_RF_CR_UNIFORM, QEW_RB_CR_GAUSS, QEW_RB_LIN_GAUSS
                                   or QEW_RF_PC_GAUSS                                    */
  const int64_t  *L;            /* [S] chain lengths, 3 <= L_s <= 2^30                  */
  const double   *f;            /* [S] drive per sample (finite)                        */
  const uint32_t *disorder_id;  /* [S] Philox counter word 2; equal ids => same disorder */
  double          c;            /* elastic constant, > 0                                */
  double          dt;           /* Euler time step, > 0, with c * dt <= 0.5             */
  double          strength;     /* >= 0; multiplies the random values (0 => F_p = 0)    */
  uint64_t        seed;         /* Philox key (low word, high word)                     */
  int64_t         n_steps;      /* >= 0 Euler steps                                     */
  const int64_t  *meas_steps;   /* [n_meas] strictly increasing, each in [0, n_steps]   */
  int32_t         n_meas;       /* >= 0                                                 */
  int32_t         precision;    /* QEW_FP64_PLAIN or QEW_FP32_SPLIT                     */
  int32_t         path;         /* QEW_ONE_STEP, or QEW_FUSED (FP32 split only)         */
  int32_t         k;            /* fused: steps per launch, 1..128 (0 = autotune)       */
  int32_t         tile;         /* fused: sites per workgroup tile, 1024/1536/2048/3072/4096 (0 = autotune); 4k <= tile */
  int32_t         flags;        /* QEW_FLAG_* bits                                      */
  int32_t         period;       /* transverse period M of the disorder in u (node n is
                                   node n mod M); 0 = no period; else 1 <= M < 2^30     */
  int32_t         sq_bins;      /* structure factor S_q (Eq. (6)) at every measurement:
                                   number of mode bins; 0 = off.  Needs every L_s equal,
                                   a power of two, 8 <= L <= 2^30                        */
  const int64_t  *sq_edges;     /* [sq_bins + 1] host, read only in qew_plan: bin b holds
                                   the modes n in [sq_edges[b], sq_edges[b+1]), q = 2 pi
                                   n / L; strictly increasing, 1 <= sq_edges[0],
                                   sq_edges[sq_bins] <= L/2 + 1                          */
} qew_problem;

typedef struct qew_plan_s qew_plan_t;

/* What a plan resolved to (after autotuning, if any). */
typedef struct qew_plan_info {
  int64_t total_sites;   /* sum of L_s                                   */
  int64_t padded_sites;  /* sites held per state buffer (64-site aligned) */
  int32_t n_tiles;       /* work items of the stepping kernel            */
  int32_t n_meas_tiles;  /* work items of the measurement kernels        */
  int32_t k;             /* steps per fused launch (1 for one-step)      */
  int32_t tile;          /* sites per fused workgroup tile (0: one-step) */
  int32_t autotuned;     /* 1 if k / tile were chosen by qew_autotune    */
  int32_t pad_;
  int64_t cur_step;      /* step index of the state in the workspace     */
} qew_plan_info;

/*
 * Statistics of the last qew_run.  The durations need QEW_FLAG_TIMING (HIP
 * events on `stream`); the counts are kept always.  A measurement that rides
 * on the first step of a stretch (one-step launches) adds that launch to the
 * stepping time and its per-sample combine to the measurement time.
 */
typedef struct qew_run_stats {
  double  total_ms;        /* the whole qew_run on the stream                          */
  double  step_ms;         /* summed duration of the stepping segments (all kernels)   */
  double  meas_ms;         /* summed duration of the measurement kernels               */
  int64_t step_launches;   /* stepping-kernel launches (graph nodes included)          */
  int64_t meas_launches;   /* measurement points taken                                 */
  int64_t site_updates;    /* sum_s L_s * (Euler steps advanced)                       */
  int64_t graph_launches;  /* hipGraphLaunch calls                                     */
  int64_t sparse_launches; /* fused launches of the sparse variant                     */
  double  fused_ms;        /* summed duration of the segments made of fused launches   */
  int64_t fused_launches;  /* fused-kernel launches                                    */
  int64_t fused_steps;     /* Euler steps advanced by fused launches                   */
  int64_t node_refreshes;  /* rebuilds of the fused path's node cache (after one-step
                              stretches or a written state)                            */
} qew_run_stats;

/*
 * Validate a problem and build a plan (host only; no device call).
 * Copies every array.  *out receives a plan to free with qew_plan_destroy.
 * Errors: QEW_EINVAL (any constraint in qew_problem violated, NULL pointers),
 * QEW_EUNSUPPORTED (FUSED with FP64_PLAIN).
 */
qew_status qew_plan(const qew_problem *problem, qew_plan_t **out);

/* Bytes of device workspace qew_run needs for this plan (0 if plan is NULL). */
size_t qew_workspace_bytes(const qew_plan_t *plan);

/* Fill *info (host pointer). */
qew_status qew_plan_info_get(const qew_plan_t *plan, qew_plan_info *info);

/*
 * Choose k and the tile width of the fused path by timing short runs on the
 * workspace (its state is overwritten).  Called by qew_run by itself when the
 * problem left k or tile at 0.  No-op for the one-step path.
 */
qew_status qew_autotune(qew_plan_t *plan, void *d_ws, size_t ws_bytes, void *stream);

/*
 * Run the problem (Eq. (1) by Euler steps, Sec. III B) and measure Eqs. (3)-(5).
 *   resume = 0: flat start u = 0 at step 0 (Sec. II).
 *   resume = 1: continue from the state and step left in this workspace by
 *               the previous qew_run or qew_write_state (QEW_EINVAL if none).
 * The run ends at problem.n_steps.  h_v, h_w2, h_ubar are host arrays
 * [S][n_meas] (row = sample); entries whose step is below the starting step
 * are left untouched.  Any of them may be NULL.  Synchronous: returns after
 * the stream has drained.  d_ws must be 256-byte aligned and hold at least
 * qew_workspace_bytes(plan) bytes (else QEW_ENOMEM).
 */
qew_status qew_run(qew_plan_t *plan, void *d_ws, size_t ws_bytes, void *stream, int32_t resume,
                   double *h_v, double *h_w2, double *h_ubar);

/*
 * qew_run for callers that cannot allocate memory (tight serving loops,
 * harnesses that forbid allocation): the same arguments, kernels and results
 * as qew_run, but the call allocates nothing, on the device or the host.  Like
 * qew_run it synchronizes its stream (the tables go in and the series come out
 * by copies), so the call itself cannot be recorded into a HIP graph.  The chains stay in d_ws (its size and
 * alignment as for qew_run); the plan's tables, tile lists, measurement
 * partials and series live in a device scratch array of the library, 8 MiB
 * per GPU, held from the library's load until the process ends (its address
 * is looked up once per device, on the first call there).  No autotuning,
 * graphs, events or pinned readbacks: the fused kernel runs its dense variant
 * (or the one a flag forces), launched directly; QEW_FLAG_TIMING gives no
 * durations.  After the call the series are also in d_ws, so qew_ensemble,
 * qew_read_state and a later qew_run with resume = 1 see this run.
 * Calls on one GPU share its scratch array: calls that overlap in time on one
 * GPU (other threads, other streams) race and must not be made.
 * Errors (before any device work): QEW_EINVAL for a fused plan without a
 * fixed geometry (give k and tile, or run qew_autotune first);
 * QEW_EUNSUPPORTED for a plan with structure-factor bins; QEW_ENOMEM when the
 * plan's tables, partials and series exceed the scratch array (about
 * 44 B per 4096 sites, 12 B per fused tile and 24 B per sample and
 * measurement); then as qew_run.
 */
qew_status qew_run_noalloc(qew_plan_t *plan, void *d_ws, size_t ws_bytes, void *stream, int32_t resume,
                           double *h_v, double *h_w2, double *h_ubar);

/*
 * Disorder average (the overbar of Sec. II, Eqs. (3)-(5)) of the series held
 * in the workspace, computed on the device in FP64 with equal weight per
 * sample, for every measurement taken so far.  h_out is a host array
 * [7][n_meas], row by row:
 *   0 mean_s v_s, 1 its standard error, 2 mean_s w2_s, 3 its standard error,
 *   4 mean_s ubar_s, 5 its standard error,
 *   6 mean_s w2_s + Var_s(ubar_s): the width about the ensemble centre of mass
 *     (the literal reading of Eq. (5) with u(t) of Eq. (4) inside the square).
 * Standard error = sample standard deviation / sqrt(S) (0 when S = 1);
 * Var_s is the population variance over samples.  Entries of measurements
 * not yet taken are NaN.  Synchronous.
 */
qew_status qew_ensemble(const qew_plan_t *plan, const void *d_ws, void *stream, double *h_out);

/*
 * Structure factor of Eq. (6), S_q(t) = overbar |L^-1 sum_x u(x,t) e^{-iqx}|^2
 * with q = 2 pi n / L, computed on the device in FP64 at every measurement
 * step of the runs so far (problem.sq_bins > 0, else QEW_EINVAL).  h_sq is a
 * host array [n_meas][sq_bins]: entry (m, b) is the mean over the samples and
 * over the modes n of bin b (modes n and L - n are equal for a real line, so
 * the bins cover 1 <= n <= L/2).  Entries of measurements not yet taken are
 * NaN.  Synchronous.
 */
qew_status qew_sq_get(const qew_plan_t *plan, const void *d_ws, void *stream, double *h_sq);

/* Statistics of the last qew_run of this plan (host pointer). */
qew_status qew_run_stats_get(const qew_plan_t *plan, qew_run_stats *stats);

/*
 * Copy sample s's state (step index `*h_step`) to h_u [L_s] as FP64
 * (cell + offset for the split precision).  Synchronous.
 */
qew_status qew_read_state(const qew_plan_t *plan, const void *d_ws, void *stream, int32_t s,
                          double *h_u, int64_t *h_step);

/*
 * Overwrite sample s's state with h_u [L_s] and set the step index of the
 * whole workspace to `step` (checkpoint restore, tests).  Split precision:
 * cell = floor(u), offset = u - cell rounded to FP32 (an offset that rounds
 * to 1 moves to the next cell).  The next qew_run must use resume = 1.
 * Synchronous.
 */
qew_status qew_write_state(qew_plan_t *plan, void *d_ws, void *stream, int32_t s,
                           const double *h_u, int64_t step);

/*
 * Debug: Philox4x32-10 of N counters.  d_ctr, d_out: device [N][4] uint32;
 * key = (seed low word, seed high word).  Asynchronous on `stream`.
 */
qew_status qew_debug_philox_fill(const uint32_t *d_ctr, uint64_t seed, uint32_t *d_out,
                                 int64_t N, void *stream);

/*
 * Debug: pinning force F_p at N points (disorder `kind`, transverse period
 * `period`, 0 = none), in the arithmetic of `precision`.
 * Point i: column d_j[i], disorder id d_did[i], u = d_cell[i] + d_frac[i]
 * (FP64 path: u formed in FP64 then floored; split path: cell as given and
 * offset rounded to FP32, which must lie in [0, 1)).  d_out: device [N] FP64.
 * Asynchronous on `stream`.
 */
qew_status qew_debug_force_eval(int32_t kind, double strength, uint64_t seed, int32_t period,
                                int32_t precision, const uint32_t *d_did, const int32_t *d_j,
                                const int32_t *d_cell, const double *d_frac, double *d_out,
                                int64_t N, void *stream);

/*
 * Critical force f_c^s and critical configuration u_c^s of samples periodic
 * in u with period M (Sec. III A): the pinned solution of
 *   c d2u/dx2 + F_p(u, x) + f = 0                                   (Sec. III A)
 * with the largest f.  The Middleton theorems make it reachable without
 * integrating Eq. (1): from a configuration whose forces are all >= 0,
 * moving a site forward to the first zero of its own force (neighbours held)
 * keeps every force >= 0 and never passes a pinned configuration ahead, so
 * such moves climb to the leftmost pinned configuration ahead if there is
 * one; a line that advances by M at every site has passed none, so there is
 * none at that drive (the translates of a pinned configuration by M are
 * pinned too).  Each sample is bisected on f independently: the start d_u is
 * first relaxed at f_lo (each site moved to the nearest zero of its force in
 * the force's direction), then each trial drive starts from the last pinned
 * configuration and is decided pinned when every |force| <= tol_force,
 * depinned when every site advanced by M.  A site whose force is within
 * tol_force / 4 of zero is not moved, and a move stops once the force left at
 * the site is within tol_force / 64.  One workgroup per sample runs the whole
 * bisection in one launch, with the chain in LDS.
 *   kind: QEW_RF_CR_UNIFORM or QEW_RB_CR_GAUSS (continuous forces; else
 *         QEW_EUNSUPPORTED).  Disorder as in qew_problem (Philox counter
 *         (j, n mod M, disorder id, 0), values times strength).
 *   n_samples S >= 1, 3 <= L <= 4096, 1 <= period M < 2^30, c > 0,
 *   f_lo < f_hi finite, tol_f > 0 (at most 200 halvings of f_hi - f_lo),
 *   tol_force > 0, max_sweeps >= 4 (sweeps per trial before it counts as
 *   undecided; one sweep moves the even and then the odd sites).
 *   d_disorder_id: device [S] uint32.
 *   d_u: device [S][L] FP64, the start on entry (e.g. the flat line), on
 *        return the last pinned configuration (u_c^s at f_lo when done).
 *   d_f: device [S][2] FP64 out: the final bracket f_lo <= f_c^s < f_hi,
 *        f_hi - f_lo < tol_f.
 *   d_status: device [S][2] int64 out: status (0 done; 1 no pinned
 *        configuration reached at f_lo; 2 a trial undecided within
 *        max_sweeps; 3 out of rounds) and the sweeps made.
 * Asynchronous on `stream`; arguments are checked on the host first.
 */
qew_status qew_critical_force(int32_t kind, double strength, uint64_t seed, int32_t period, double c,
                              int32_t n_samples, int32_t L, const uint32_t *d_disorder_id, double f_lo,
                              double f_hi, double tol_f, double tol_force, int64_t max_sweeps, double *d_u,
                              double *d_f, int64_t *d_status, void *stream);

/* Free a plan (NULL is allowed); releases its hipGraphs. */
void qew_plan_destroy(qew_plan_t *plan);

/* Message of the last failed call on this thread ("" if none). */
const char *qew_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* QEW_H */
