/*
 * am.h -- C-ABI of the MI355X batched alternating-minimization (AM) trajectory
 * optimizer of "GPU Accelerated Batch Multi-Convex Trajectory Optimization
 * for a Rectangular Holonomic Mobile Robot" (arXiv 2109.13030).
 *
 * One *problem* (Sec. II-B) is a robot modelled by m circles at offsets r_i
 * along its body axis, n axis-aligned elliptical obstacles known over the
 * horizon, and boundary conditions shared by a batch of B trajectories.  The
 * library runs the AM iteration of Sec. III-D on all B trajectories at once:
 * per iteration, xi1 and xi2 are equality-constrained QPs solved through one
 * constant KKT inverse (eqs. over_1-over_3, zeta_1_sepration_3,
 * compute_convex_surrogate), xi3/xi4 are the closed-form angle and distance
 * updates (eqs. zeta_2, alpha_v, alpha_a, compute_zeta_3, compute_dv,
 * compute_da, clipped), then the multipliers are updated (eqs.
 * update_lambda_1, update_lambda_psi).
 *
 * Conventions
 *  - Every function returns an int status: AM_OK (0) or a negative AM_ERR_*
 *    code; am_last_error() returns a thread-local message for the last
 *    failure of the calling thread.
 *  - Arrays are row-major with the time index fastest.  Array elements are
 *    float (AM_F32 handles) or double (AM_F64 handles).
 *  - "device" pointers are HIP device memory owned by the caller; the library
 *    never frees them.  "host" pointers are read during the call only.
 *  - Solves are asynchronous on the given stream (a hipStream_t passed as
 *    void*, NULL = the default stream) and allocate nothing.  am_setup is
 *    synchronous and allocates the handle's constants, released by
 *    am_destroy.
 *  - Argument checks happen on the host before anything is launched; a bad
 *    argument returns AM_ERR_INVALID and launches nothing.
 *  - Concurrent calls on one handle are allowed (the handle is read-only after
 *    am_setup) as long as their state buffers do not overlap.
 */
#ifndef AM_H
#define AM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define AM_OK             0
#define AM_ERR_INVALID   (-1)  /* bad argument (nothing launched)            */
#define AM_ERR_HIP       (-2)  /* a HIP runtime call failed                   */
#define AM_ERR_SINGULAR  (-4)  /* a KKT matrix is numerically singular        */
#define AM_ERR_NONFINITE (-5)  /* every trajectory of a served request is
                                  NaN/Inf (am_server_best)                    */
#define AM_ERR_NOMEM     (-6)  /* device allocation failed (am_setup only)    */

/* element types */
#define AM_F32 0
#define AM_F64 1

/* Readings of passages the paper leaves open (flags; 0 = default reading).
 * AM_ALPHA_LITERAL  alpha_ij = atan2(y~, x~) exactly as printed in eq. (zeta_2);
 *                   default: atan2(a y~, b x~), under which points on or
 *                   outside the ellipse are fixed points of the projection.
 * AM_XTILDE_SLACK   x~ = x + r_i c - x_j with the slack copies c, s (the
 *                   objective of eq. compute_ze_3); default: r_i cos(psi) as in
 *                   eq. (compute_zeta_33).
 * AM_PSI_NO_UNWRAP  psi_hat = atan2(s, c) in (-pi, pi]; default: the branch
 *                   nearest the current heading.
 * AM_LAMPSI_LITERAL lambda_psi update with the sign printed in eq.
 *                   (update_lambda_psi); default: the sign of eq.
 *                   (update_lambda_1).
 * AM_Q_CS_ZERO      acceleration cost on the x, y blocks of xi1 only; default:
 *                   on all four blocks (Sec. III-C, "block-diagonal stacking").
 * Precision option (not a reading; AM_F32 handles only):
 * AM_PLAIN_BF16X3   the plain path forms the stacked contraction
 *                   F^T(F xi - g) of eq. (zeta_1_sepration_3) on the matrix
 *                   cores: BF16 products, FP32 accumulation and a split
 *                   correction (a_hi b_hi + a_hi b_lo + a_lo b_hi). */
#define AM_ALPHA_LITERAL  1u
#define AM_XTILDE_SLACK   2u
#define AM_PSI_NO_UNWRAP  4u
#define AM_LAMPSI_LITERAL 8u
#define AM_Q_CS_ZERO      16u
#define AM_PLAIN_BF16X3   32u
#define AM_FLAGS_ALL      63u

/* per-trajectory residual statistics written by am_residuals */
#define AM_NRES 12
#define AM_RES_FC_MAX      0  /* max |f_c| of eq. (collision_avoidance_proposed) */
#define AM_RES_FC_RMS      1  /* RMS |f_c|                                       */
#define AM_RES_FV_MAX      2  /* max |f_v|, eq. (fv)                             */
#define AM_RES_FA_MAX      3  /* max |f_a|, eq. (fa)                             */
#define AM_RES_SLACK_MAX   4  /* max(|c - cos psi|, |s - sin psi|)               */
#define AM_RES_HEADING_MAX 5  /* max |atan2(s, c) - psi| wrapped to (-pi, pi]    */
#define AM_RES_BC_MAX      6  /* max |A c - b| over x, y, psi                    */
#define AM_RES_COST        7  /* sum_t xdd^2 + ydd^2 + psidd^2, eq. (acc_cost)   */
#define AM_RES_CLEAR_LEVEL 8  /* min sqrt(x~^2/a^2 + y~^2/b^2) - 1 (>= 0: clear) */
#define AM_RES_V_EXCESS    9  /* max_t |v| - vmax                                */
#define AM_RES_A_EXCESS   10  /* max_t |a| - amax                                */
#define AM_RES_NONFINITE  11  /* 1 if any state value is NaN/Inf, else 0        */

/* Size limits of the library (compile-time capacities of the kernels). */
#define AM_MAX_Q       128    /* timesteps                                    */
#define AM_MAX_CIRCLES 8
#define AM_MAX_OBS     64

typedef struct am_handle am_handle;

/* What fixes the constant KKT matrices (eq. over_3): one handle per shape.
 * F has 3q + m n q rows, so the matrix depends on m, n and r_i (through
 * m*n, n*sum(r_i), n*sum(r_i^2)) and on rho. */
typedef struct {
  int32_t q;            /* timesteps t_k = k tf/(q-1); 2 < q <= AM_MAX_Q       */
  int32_t nv;           /* coefficients per variable (Bernstein degree nv-1);
                           supported: 8 and 11                                 */
  double tf;            /* horizon [s] > 0                                    */
  int32_t m;            /* circles, 1..AM_MAX_CIRCLES                         */
  const double *r_off;  /* host [m] circle offsets along the body axis [m]   */
  int32_t n_obs;        /* obstacles, 0..AM_MAX_OBS                           */
  double rho;           /* penalty of eq. (reform_bergman), > 0                */
  double rho_psi;       /* step of the lambda_psi update, >= 0                 */
  int32_t dtype;        /* AM_F32 or AM_F64                                    */
  uint32_t flags;       /* AM_* readings                                       */
} am_shape;

/* One problem instance shared by the batch (Sec. II-B: all trajectories have
 * the same boundary conditions and obstacles). */
typedef struct {
  const void *obs_x;    /* device [n][q] obstacle centre x_j(t_k)             */
  const void *obs_y;    /* device [n][q] obstacle centre y_j(t_k)             */
  const void *obs_a;    /* device [n] semi-axis along x, un-inflated, > 0      */
  const void *obs_b;    /* device [n] semi-axis along y, un-inflated, > 0      */
  double r_circle;      /* circle radius; semi-axes are inflated by it, >= 0   */
  double bc_x[6];       /* (x0, vx0, ax0, xf, vxf, axf)                        */
  double bc_y[6];
  double bc_psi[6];
  double v_max, a_max;  /* bounds of eq. (acc_constraint), > 0                 */
} am_problem;

/* Per-batch state, updated in place; pass it back to warm-start. */
typedef struct {
  void *cx, *cc, *cy, *cs, *cpsi;  /* device [B][nv] Bernstein coefficients of
                                      x, c, y, s, psi (in/out)                */
  void *lam;                       /* device [B][4 nv] lambda, parts
                                      (cx, cc, cy, cs) (in/out)               */
  void *lam_psi;                   /* device [B][nv] lambda_psi (in/out)      */
  void *alpha, *d;                 /* device [B][m n][q] final alpha_ij, d_ij,
                                      row i*n + j (out; NULL = not written)   */
  void *va;                        /* device [B][4][q] final alpha_v, d_v,
                                      alpha_a, d_a (out; NULL = not written)  */
  void *traj;                      /* device [B][3][q] x, y, psi of the last
                                      iterate (out; NULL = not written)       */
  void *res;                       /* device [B][AM_NRES] residual statistics
                                      of the final state, as am_residuals
                                      writes them, formed by the solve itself
                                      (out; NULL = not written)               */
} am_state;

/* Builds the handle: the Bernstein basis, an orthonormal basis of the same
 * polynomial space (the iteration runs in it), both KKT matrices and their
 * inverses, all in FP64 on the current GPU (eqs. over_2, over_3;
 * Sec. IV "F^T F needs to be computed only once").  Synchronous.
 * Errors: AM_ERR_INVALID, AM_ERR_NOMEM, AM_ERR_SINGULAR, AM_ERR_HIP. */
int am_setup(const am_shape *shape, am_handle **out);

/* Releases the handle and its device constants (NULL is ignored). */
void am_destroy(am_handle *h);

/* Thread-local message of the last failure (never NULL). */
const char *am_last_error(void);

/* Runs the AM iteration on `batch` trajectories in one launch (Sec. III-D):
 * initial xi3, xi4 from the given cx, cy, cpsi (and cc, cs under
 * AM_XTILDE_SLACK), then `iters` iterations of xi1, xi2, xi3, xi4 and the
 * multiplier update.  With iters = 0 only the initial projection runs.
 * The state is read and written on the device; nothing is allocated.
 * batch >= 0 (0 launches nothing and reads neither st nor its arrays, which
 * may then be NULL), iters >= 0. */
int am_solve_batch(am_handle *h, const am_problem *p, int32_t batch, int32_t iters,
                   const am_state *st, void *stream);

/* Same result as am_solve_batch computed the plain way: one kernel launch
 * per sub-step per iteration, with alpha, d and the trajectories held in
 * device memory between launches as in the paper's formulation.  Needs a
 * caller-owned device workspace of am_plain_workspace_size() bytes, 16-byte
 * aligned (AM_ERR_INVALID otherwise; any hipMalloc allocation is).  Its
 * kernels read the obstacle rows and write alpha, d two or four time steps
 * at a time when q is even, so obs_x and obs_y should then be 16-byte
 * aligned too (any other alignment is slower, not wrong).  As for
 * am_solve_batch, batch 0 launches nothing and reads neither st nor the
 * workspace. */
int am_plain_workspace_size(const am_handle *h, int32_t batch, size_t *bytes);
int am_solve_batch_plain(am_handle *h, const am_problem *p, int32_t batch, int32_t iters,
                         const am_state *st, void *workspace, size_t workspace_bytes,
                         void *stream);

/* Several independent problems (possibly of different handles, batch sizes,
 * circle and obstacle counts) in one launch.  All handles must share dtype,
 * q and nv.  The launch needs a caller-owned device workspace of
 * am_multi_workspace_size(nprob) bytes for the problem table.
 * handles[nprob], problems[nprob], batch[nprob], iters[nprob], states[nprob]
 * are host arrays.  A problem with batch 0 gets no block and its state's
 * arrays may be NULL. */
int am_multi_workspace_size(int32_t nprob, size_t *bytes);
int am_solve_multi(int32_t nprob, am_handle *const *handles, const am_problem *problems,
                   const int32_t *batch, const int32_t *iters, const am_state *states,
                   void *workspace, size_t workspace_bytes, void *stream);

/* am_solve_multi for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation):
 * the same launch, with the problem table in the library's static device
 * array of AM_STATIC_MAX_PROBLEMS descriptors instead of a workspace.  Each
 * GPU holds its own copy of that array until the process ends; this call
 * allocates nothing.  nprob > AM_STATIC_MAX_PROBLEMS returns AM_ERR_INVALID
 * before any launch.  The table is written on `stream` and read by the
 * launch that follows it there: calls that overlap on one GPU (on two
 * streams, or from two threads) share the array and race, so callers
 * serialise them.  Other arguments and errors as for am_solve_multi. */
#define AM_STATIC_MAX_PROBLEMS 128
int am_solve_multi_static(int32_t nprob, am_handle *const *handles, const am_problem *problems,
                          const int32_t *batch, const int32_t *iters, const am_state *states, void *stream);

/* Launch configuration of the one-launch solve (the arithmetic, and so the
 * result, is the same for every configuration):
 * - tile: trajectories per 2*64*tile-thread block (two wavefronts per
 *   trajectory), in {1, 2, 4}; default 2;
 * - waves: register budget, the wavefronts per SIMD the kernel is built to
 *   fit, 2 (up to 256 VGPRs) or 3 (up to 168 VGPRs, reductions in two
 *   passes to halve the LDS area); default 2; FP64 handles accept 2 only.
 * A multi-problem launch uses the configuration of handles[0]. */
int am_set_tile(am_handle *h, int32_t tile);
int am_get_tile(const am_handle *h, int32_t *tile);
int am_set_waves(am_handle *h, int32_t waves);
int am_get_waves(const am_handle *h, int32_t *waves);

/* Autotuner: times am_solve_batch (one warm-up and three timed launches per
 * candidate, HIP events on `stream`) for every launch configuration on the
 * caller's scratch state -- which it overwrites -- stores the fastest in the
 * handle and returns it in *best_tile and *best_waves (either may be NULL);
 * times_ms (may be NULL) receives six mean times, tiles 1, 2, 4 at 2 waves
 * then at 3 waves (-1 where the dtype does not allow the configuration).
 * Synchronous. */
int am_autotune(am_handle *h, const am_problem *p, int32_t batch, int32_t iters, const am_state *scratch,
                void *stream, int32_t *best_tile, int32_t *best_waves, float *times_ms);
/* The same for a multi-problem launch; the chosen configuration is stored in
 * every handle of the list. */
int am_autotune_multi(int32_t nprob, am_handle *const *handles, const am_problem *problems,
                      const int32_t *batch, const int32_t *iters, const am_state *scratch,
                      void *workspace, size_t workspace_bytes, void *stream, int32_t *best_tile,
                      int32_t *best_waves, float *times_ms);

/* Residual statistics of the current state (AM_RES_* columns), written to
 * device out[batch][AM_NRES] in the handle's dtype.  alpha and d are the
 * closed-form projection of the current trajectories (what the last
 * iteration left).  Reads cx, cc, cy, cs, cpsi, lam, lam_psi of st.
 * batch 0 launches nothing (st and out may then hold NULL arrays). */
int am_residuals(am_handle *h, const am_problem *p, int32_t batch, const am_state *st,
                 void *out, void *stream);

/* Best trajectory of a batch (Fig. 1: the batch returns many locally optimal
 * trajectories and the one of least cost is used), from the rows that
 * am_residuals wrote to device `residuals` [batch][AM_NRES] (handle's dtype):
 * among trajectories with no non-finite value and max |f_c| <= fc_tol
 * (metres), the least AM_RES_COST; if none qualifies, the least max |f_c|;
 * ties go to the lower index.  Writes the index (-1 if every trajectory is
 * non-finite, or batch is 0) to device int32 *best and, when values is not NULL, (cost,
 * max |f_c|) of that trajectory to device values[2] (handle's dtype).
 * Stream-ordered, asynchronous. */
int am_select_best(const am_handle *h, int32_t batch, const void *residuals, double fc_tol, int32_t *best,
                   void *values, void *stream);

/* ---------------------------------------------------------------------------
 * Replanning server: continuous batching of independent solve requests, as a
 * model-predictive controller issues them (Sec. IV: the batch optimizer runs
 * inside an MPC loop with the multipliers warm-started from the previous
 * control loop; Fig. 1 picks the best-cost trajectory of the batch).
 *
 * Requests arrive at any time from any thread.  A scheduler thread admits
 * pending requests, in arrival order, whenever a launch slot is free and the
 * device-memory budget holds their state and problem table; all requests
 * admitted together run in one multi-problem launch, and up to `streams`
 * launches are in flight at once, so new requests start while earlier ones
 * are still on the GPU.  A request starts from its own initial coefficients
 * (fresh samples) and, when client c's previous result is still in device
 * memory with the same batch size, from that result's multipliers (else
 * from zero multipliers); a client's requests run one after another.  Idle
 * clients' kept results are dropped least recently used first when the
 * budget is short.  Latency = completion seen by the scheduler - submission.
 * ------------------------------------------------------------------------- */
typedef struct am_server am_server;

#define AM_SERVE_CONTINUOUS 0  /* batch all admissible pending requests per launch   */
#define AM_SERVE_SEQUENTIAL 1  /* one request per launch, one launch at a time       */
#define AM_SERVE_PLAIN      2  /* as SEQUENTIAL, with the plain per-sub-step path    */

typedef struct {
  size_t hbm_budget;            /* device bytes for request state and tables (> 0)      */
  int32_t streams;              /* launches in flight, 1..16 (forced to 1 unless
                                   AM_SERVE_CONTINUOUS)                                 */
  int32_t max_per_launch;       /* requests per launch, 1..256                          */
  int32_t mode;                 /* AM_SERVE_*                                           */
  int32_t dtype;                /* AM_F32 or AM_F64; every request's handle must match  */
  int32_t select_best;          /* 1: after each solve, residuals of every trajectory
                                   and the best one (am_select_best rule), read back
                                   with am_server_best; 0: off                          */
  double fc_tol;                /* collision tolerance of that rule [m], >= 0          */
  int32_t idle_spin_us;         /* 0..1000000: after its last launch or submission the
                                   scheduler keeps polling for this long before it
                                   sleeps (a woken thread adds the OS wake-up time
                                   to the next request's latency; spinning holds
                                   one host core); 0: sleep at once                     */
} am_server_config;

/* One solve request.  Host arrays are copied during am_server_submit. */
typedef struct {
  am_handle *handle;            /* shape of this request (q, nv, m, n, rho, flags), or
                                   NULL: then `shape` is used and the server takes the
                                   handle from its KKT cache (one am_setup per distinct
                                   shape, kept until am_server_destroy)                 */
  const am_shape *shape;        /* host; read when handle is NULL                       */
  int32_t client;               /* warm-start key, >= 0                                 */
  int32_t batch;                /* trajectories, >= 1                                   */
  int32_t iters;                /* AM iterations, >= 0                                  */
  const double *obs_x, *obs_y;  /* host [n][q] obstacle centres                         */
  const double *obs_a, *obs_b;  /* host [n] semi-axes, un-inflated                      */
  double r_circle, bc_x[6], bc_y[6], bc_psi[6], v_max, a_max;
  const double *init;           /* host [batch][5][nv] initial coefficients (cx, cc,
                                   cy, cs, cpsi), required                              */
} am_request;

int am_server_create(const am_server_config *cfg, am_server **out);
/* Queues a request; returns its ticket (>= 0).  Thread-safe, non-blocking.
 * AM_ERR_INVALID if the request can never fit the budget or is malformed. */
int am_server_submit(am_server *s, const am_request *r, int64_t *ticket);
/* Waits up to timeout_s (< 0: forever) for the ticket.  *done = 1 when
 * finished; then latency_s (may be NULL) receives completion - submission
 * and, when traj is not NULL, host traj [batch][3][q] (x, y, psi; in the
 * server's dtype) receives the final trajectories. */
int am_server_wait(am_server *s, int64_t ticket, double timeout_s, int32_t *done, double *latency_s,
                   void *traj);
/* Best trajectory of a finished request (server created with select_best):
 * its index in the request's batch, its cost and its max |f_c| (either may
 * be NULL).  If every trajectory is non-finite, *index = -1 and the call
 * returns AM_ERR_NONFINITE.  AM_ERR_INVALID if the request has not
 * finished. */
int am_server_best(am_server *s, int64_t ticket, int32_t *index, double *cost, double *fc_max);
/* Counters: requests completed, launches issued, peak bytes of the budget
 * in use, requests that waited for memory (any may be NULL). */
int am_server_stats(am_server *s, int64_t *completed, int64_t *launches, size_t *peak_bytes,
                    int64_t *memory_waits);
/* Finishes in-flight work, stops the scheduler, frees device memory. */
void am_server_destroy(am_server *s);

/* FP64 copies of the setup results (host buffers, any may be NULL):
 * kkt1_inv [(2nv+6)^2] and kkt2_inv [(nv+6)^2] are the inverses of the KKT
 * matrices of xi1 and xi2 in Bernstein coordinates; basis [3][q][nv] holds
 * P, Pdot, Pddot.  Synchronous. */
int am_setup_matrices(const am_handle *h, double *kkt1_inv, double *kkt2_inv, double *basis);

#ifdef __cplusplus
}
#endif
#endif /* AM_H */
