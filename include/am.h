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
#define AM_ERR_NONFINITE (-5)  /* residuals found NaN/Inf in a trajectory     */
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
 *                   on all four blocks (Sec. III-C, "block-diagonal stacking"). */
#define AM_ALPHA_LITERAL  1u
#define AM_XTILDE_SLACK   2u
#define AM_PSI_NO_UNWRAP  4u
#define AM_LAMPSI_LITERAL 8u
#define AM_Q_CS_ZERO      16u
#define AM_FLAGS_ALL      31u

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

/* Limits of this build. */
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
 * batch >= 0 (0 launches nothing), iters >= 0. */
int am_solve_batch(am_handle *h, const am_problem *p, int32_t batch, int32_t iters,
                   const am_state *st, void *stream);

/* Same result as am_solve_batch computed the plain way: one kernel launch
 * per sub-step per iteration, with alpha, d and the trajectories held in
 * device memory between launches as in the paper's formulation.  Needs a
 * caller-owned device workspace of am_plain_workspace_size() bytes. */
int am_plain_workspace_size(const am_handle *h, int32_t batch, size_t *bytes);
int am_solve_batch_plain(am_handle *h, const am_problem *p, int32_t batch, int32_t iters,
                         const am_state *st, void *workspace, size_t workspace_bytes,
                         void *stream);

/* Several independent problems (possibly of different handles, batch sizes,
 * circle and obstacle counts) in one launch.  All handles must share dtype,
 * q and nv.  The launch needs a caller-owned device workspace of
 * am_multi_workspace_size(nprob) bytes for the problem table.
 * handles[nprob], problems[nprob], batch[nprob], iters[nprob], states[nprob]
 * are host arrays. */
int am_multi_workspace_size(int32_t nprob, size_t *bytes);
int am_solve_multi(int32_t nprob, am_handle *const *handles, const am_problem *problems,
                   const int32_t *batch, const int32_t *iters, const am_state *states,
                   void *workspace, size_t workspace_bytes, void *stream);

/* Residual statistics of the current state (AM_RES_* columns), written to
 * device out[batch][AM_NRES] in the handle's dtype.  alpha and d are the
 * closed-form projection of the current trajectories (what the last
 * iteration left).  Reads cx, cc, cy, cs, cpsi, lam, lam_psi of st. */
int am_residuals(am_handle *h, const am_problem *p, int32_t batch, const am_state *st,
                 void *out, void *stream);

/* FP64 copies of the setup results (host buffers, any may be NULL):
 * kkt1_inv [(2nv+6)^2] and kkt2_inv [(nv+6)^2] are the inverses of the KKT
 * matrices of xi1 and xi2 in Bernstein coordinates; basis [3][q][nv] holds
 * P, Pdot, Pddot.  Synchronous. */
int am_setup_matrices(const am_handle *h, double *kkt1_inv, double *kkt2_inv, double *basis);

#ifdef __cplusplus
}
#endif
#endif /* AM_H */
