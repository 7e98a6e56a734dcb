/*
 * am_oracle.h -- FP64 CPU oracle for the batched alternating-minimization (AM)
 * trajectory optimizer of "GPU Accelerated Batch Multi-Convex Trajectory
 * Optimization for a Rectangular Holonomic Mobile Robot" (arXiv 2109.13030).
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the plain, slow reference that
 * the GPU path is checked against.  Only the test suite, the smoke check and
 * the CPU-baseline leg of the benchmark may load it; the product path never
 * calls it and shares no code with it.
 *
 * What it computes (paper Sec. III):
 *   problem            eqs. (acc_cost)-(coll_multiagent), reformulated as
 *                      (reform_cost)-(ine_1) with the stacked F, g of
 *                      Sec. III-C and relaxed to the augmented Lagrangian
 *                      (reform_bergman);
 *   iteration          Sec. III-D steps 1-5, in that order:
 *                      xi1 (eq. zeta_1_sepration_1 via over_2 with
 *                      zeta_1_sepration_3), xi2 (eq. compute_convex_surrogate),
 *                      xi3 (eqs. zeta_2, alpha_v, alpha_a), xi4 (eqs.
 *                      compute_zeta_3, compute_dv, compute_da, then clipping),
 *                      multipliers (eqs. update_lambda_1, update_lambda_psi).
 *
 * Every equality-constrained QP is solved by an LU factorisation (partial
 * pivoting) of its KKT matrix (eq. over_2) followed by triangular solves: no
 * explicit inverse.  All products with F are taken with the explicitly stored
 * dense F block.  Arrays are row-major, time index fastest.
 *
 * Readings where the paper is silent or inconsistent are switched by the
 * AMO_* flags below; flags = 0 is the default reading.
 */
#ifndef AM_ORACLE_H
#define AM_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

/* alpha_ij = atan2(yt, xt) exactly as printed in eq. (zeta_2); default is the
 * elliptic angle atan2(a*yt, b*xt), which makes points on or outside the
 * ellipse exact fixed points of the projection. */
#define AMO_ALPHA_LITERAL  1u
/* x~ = x + r_i*c - x_j (slack copies, as in the objective of eq. compute_ze_3)
 * instead of the default x + r_i*cos(psi) - x_j of eq. (compute_zeta_33). */
#define AMO_XTILDE_SLACK   2u
/* psi_hat = atan2(s, c) in (-pi, pi] instead of the default branch that is
 * unwrapped around the current heading. */
#define AMO_PSI_NO_UNWRAP  4u
/* lambda_psi update with the sign printed in eq. (update_lambda_psi); the
 * default uses the sign consistent with eq. (update_lambda_1). */
#define AMO_LAMPSI_LITERAL 8u
/* Acceleration cost only on the x and y blocks of xi1 (default: on all four
 * blocks, "block-diagonal stacking" read literally). */
#define AMO_Q_CS_ZERO      16u

#define AMO_OK            0
#define AMO_ERR_INVALID  (-1)
#define AMO_ERR_SINGULAR (-4)
#define AMO_ERR_NOMEM    (-6)

/* Number of per-trajectory residual statistics written by amo_residuals. */
#define AMO_NRES 12

typedef struct {
  int q;                 /* timesteps on the grid t_k = k*tf/(q-1)          */
  int nv;                /* coefficients per variable, Bernstein degree nv-1 */
  double tf;             /* horizon [s]                                     */
  int m;                 /* robot circles                                   */
  const double *r;       /* [m] circle offsets along the body axis [m]      */
  int n;                 /* obstacles                                       */
  const double *ox;      /* [n][q] obstacle centre x_j(t_k)                 */
  const double *oy;      /* [n][q] obstacle centre y_j(t_k)                 */
  const double *oa;      /* [n] semi-axis along x (un-inflated)             */
  const double *ob;      /* [n] semi-axis along y (un-inflated)             */
  double rc;             /* circle radius; semi-axes are inflated by it     */
  double bx[6], by[6], bpsi[6]; /* (p0, v0, a0, pf, vf, af), shared by the batch */
  double vmax, amax;     /* bounds of eq. (acc_constraint)                  */
  double rho, rho_psi;   /* penalty of eq. (reform_bergman); multiplier step */
  unsigned flags;        /* AMO_* readings                                  */
} amo_problem;

/* Per-batch state.  Every pointer addresses B contiguous per-trajectory rows. */
typedef struct {
  double *cx, *cc, *cy, *cs, *cpsi; /* [B][nv] coefficients (xi1, xi2)        */
  double *lam;                      /* [B][4nv] lambda: (cx, cc, cy, cs) parts */
  double *lampsi;                   /* [B][nv]  lambda_psi                     */
  double *alpha, *d;                /* [B][m*n][q] alpha_ij, d_ij; row i*n+j   */
  double *av, *dv, *aa, *da;        /* [B][q] alpha_v, d_v, alpha_a, d_a       */
  double *psihat;                   /* [B][q] psi_hat of the last xi2 step     */
} amo_state;

typedef struct amo_ctx amo_ctx;

/* Bernstein basis on the grid: P, Pdot, Pddot, each [q][nv]. */
int amo_basis(int q, int nv, double tf, double *P, double *Pd, double *Pdd);

/* Builds F, Q, the two KKT matrices and their LU factors.  On failure returns
 * NULL and writes the status to *status (may be NULL). */
amo_ctx *amo_create(const amo_problem *pb, int *status);
void amo_free(amo_ctx *ctx);

/* Copies of the setup matrices for tests: F block [(3q+mnq)][2nv], KKT of xi1
 * [(2nv+6)^2], KKT of xi2 [(nv+6)^2].  Any pointer may be NULL. */
int amo_matrices(const amo_ctx *ctx, double *F, double *kkt1, double *kkt2);

/* Individual steps on all B trajectories (for tests). */
enum { AMO_STEP_XI1 = 1, AMO_STEP_XI2 = 2, AMO_STEP_XI3 = 3, AMO_STEP_XI4 = 4,
       AMO_STEP_LAMBDA = 5 };
int amo_step(const amo_ctx *ctx, int B, int which, const amo_state *st);

/* Full solve: initialisation (xi3, xi4 from the given cx, cy, cpsi and, under
 * AMO_XTILDE_SLACK, cc, cs), then K iterations of steps xi1..lambda.
 * hist (may be NULL) receives [K][B] the collision residual after each
 * iteration.  nthreads <= 0 uses the OpenMP default. */
int amo_solve(const amo_ctx *ctx, int B, int K, const amo_state *st,
              double *hist, int nthreads);

/* Augmented Lagrangian of eq. (reform_bergman) at the current state. [B] */
int amo_lagrangian(const amo_ctx *ctx, int B, const amo_state *st, double *out);

/* Residual statistics [B][AMO_NRES]; see am_oracle.c for the list. */
int amo_residuals(const amo_ctx *ctx, int B, const amo_state *st, double *out);

#ifdef __cplusplus
}
#endif
#endif
