/*
 * am_oracle.c -- FP64 CPU oracle (test infrastructure only; see am_oracle.h).
 *
 * Plain loops, dense matrices and LU solves, written for checking by eye
 * against Sec. III of the paper.  Nothing here is blocked, fused or reordered
 * beyond what the equations state.
 */
#include "am_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

struct amo_ctx {
  amo_problem pb;        /* scalars; the pointer members are not used        */
  double *r;             /* [m]                                              */
  double *ox, *oy;       /* [n][q]                                           */
  double *a, *b;         /* [n] inflated semi-axes a_j + rc, b_j + rc        */
  double *P, *Pd, *Pdd;  /* [q][nv]                                          */
  double *A;             /* [6][nv] boundary rows                            */
  int nF;                /* rows of the F block: 3q + m*n*q                  */
  double *F;             /* [nF][2nv]                                        */
  double *Q;             /* [2nv][2nv] cost of one (position, slack) block   */
  double *K1, *K1lu;     /* [(2nv+6)^2] KKT of xi1 and its LU factors        */
  int *piv1;
  double *K2, *K2lu;     /* [(nv+6)^2] KKT of xi2 and its LU factors         */
  int *piv2;
};

/* Per-thread scratch for one trajectory. */
typedef struct {
  double *x, *xd, *xdd, *y, *yd, *ydd, *psi, *c, *s; /* [q] each */
  double *g, *Fxi;                                   /* [nF]     */
  double *rhs;                                       /* [2nv+6]  */
} scratch;

/* ------------------------------------------------------------------ */
/* small dense helpers                                                 */
/* ------------------------------------------------------------------ */

/* atan2 with the value 0 at the origin (reading: the paper does not define
 * the angle of a zero vector). */
static double atan2z(double y, double x) {
  if (x == 0.0 && y == 0.0) return 0.0;
  return atan2(y, x);
}

static double binom(int n, int k) {
  double v = 1.0;
  for (int i = 1; i <= k; ++i) v = v * (double)(n - k + i) / (double)i;
  return v;
}

/* Bernstein polynomial B_{deg,i}(tau); zero outside 0 <= i <= deg. */
static double bern(int deg, int i, double tau) {
  if (i < 0 || i > deg) return 0.0;
  return binom(deg, i) * pow(tau, i) * pow(1.0 - tau, deg - i);
}

/* LU factorisation with partial pivoting, in place; returns AMO_ERR_SINGULAR
 * when a pivot is negligible against the largest entry of the matrix. */
static int lu_factor(double *M, int *piv, int N) {
  double big = 0.0;
  for (int i = 0; i < N * N; ++i) big = fmax(big, fabs(M[i]));
  if (!(big > 0.0)) return AMO_ERR_SINGULAR;
  for (int k = 0; k < N; ++k) {
    int p = k;
    for (int i = k + 1; i < N; ++i)
      if (fabs(M[i * N + k]) > fabs(M[p * N + k])) p = i;
    if (fabs(M[p * N + k]) <= 1e-14 * big) return AMO_ERR_SINGULAR;
    piv[k] = p;
    if (p != k)
      for (int j = 0; j < N; ++j) {
        double t = M[k * N + j]; M[k * N + j] = M[p * N + j]; M[p * N + j] = t;
      }
    for (int i = k + 1; i < N; ++i) {
      M[i * N + k] /= M[k * N + k];
      for (int j = k + 1; j < N; ++j) M[i * N + j] -= M[i * N + k] * M[k * N + j];
    }
  }
  return AMO_OK;
}

static void lu_solve(const double *LU, const int *piv, int N, double *v) {
  for (int k = 0; k < N; ++k)
    if (piv[k] != k) { double t = v[k]; v[k] = v[piv[k]]; v[piv[k]] = t; }
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < i; ++j) v[i] -= LU[i * N + j] * v[j];
  for (int i = N - 1; i >= 0; --i) {
    for (int j = i + 1; j < N; ++j) v[i] -= LU[i * N + j] * v[j];
    v[i] /= LU[i * N + i];
  }
}

/* out[rows] = M[rows][cols] * v[cols] */
static void matvec(const double *M, int rows, int cols, const double *v, double *out) {
  for (int i = 0; i < rows; ++i) {
    double s = 0.0;
    for (int j = 0; j < cols; ++j) s += M[i * cols + j] * v[j];
    out[i] = s;
  }
}

/* out[cols] = M[rows][cols]^T * v[rows] */
static void matTvec(const double *M, int rows, int cols, const double *v, double *out) {
  for (int j = 0; j < cols; ++j) out[j] = 0.0;
  for (int i = 0; i < rows; ++i)
    for (int j = 0; j < cols; ++j) out[j] += M[i * cols + j] * v[i];
}

/* ------------------------------------------------------------------ */
/* setup: basis (eq. param), F and Q (Sec. III-C), KKT (eq. over_2)     */
/* ------------------------------------------------------------------ */

int amo_basis(int q, int nv, double tf, double *P, double *Pd, double *Pdd) {
  if (q < 2 || nv < 3 || !(tf > 0.0)) return AMO_ERR_INVALID;
  int N = nv - 1;
  for (int k = 0; k < q; ++k) {
    double tau = (double)k / (double)(q - 1);
    for (int i = 0; i < nv; ++i) {
      /* B'_{N,i} = N (B_{N-1,i-1} - B_{N-1,i}),
       * B''_{N,i} = N (N-1) (B_{N-2,i-2} - 2 B_{N-2,i-1} + B_{N-2,i}),
       * and d/dt = (1/tf) d/dtau on t = tau*tf. */
      P[k * nv + i] = bern(N, i, tau);
      Pd[k * nv + i] = N * (bern(N - 1, i - 1, tau) - bern(N - 1, i, tau)) / tf;
      Pdd[k * nv + i] = N * (N - 1) *
                        (bern(N - 2, i - 2, tau) - 2.0 * bern(N - 2, i - 1, tau) +
                         bern(N - 2, i, tau)) / (tf * tf);
    }
  }
  return AMO_OK;
}

void amo_free(amo_ctx *c) {
  if (!c) return;
  free(c->r); free(c->ox); free(c->oy); free(c->a); free(c->b);
  free(c->P); free(c->Pd); free(c->Pdd); free(c->A); free(c->F); free(c->Q);
  free(c->K1); free(c->K1lu); free(c->piv1); free(c->K2); free(c->K2lu); free(c->piv2);
  free(c);
}

amo_ctx *amo_create(const amo_problem *pb, int *status) {
  int st = AMO_OK;
  amo_ctx *c = NULL;
  if (!pb || pb->q < 2 || pb->nv < 3 || !(pb->tf > 0.0) || pb->m < 1 || pb->n < 0 ||
      !pb->r || (pb->n > 0 && (!pb->ox || !pb->oy || !pb->oa || !pb->ob)) ||
      !(pb->vmax > 0.0) || !(pb->amax > 0.0) || !(pb->rho > 0.0)) {
    st = AMO_ERR_INVALID;
    goto fail;
  }
  c = (amo_ctx *)calloc(1, sizeof(amo_ctx));
  if (!c) { st = AMO_ERR_NOMEM; goto fail; }
  c->pb = *pb;
  int q = pb->q, nv = pb->nv, m = pb->m, n = pb->n;
  int nF = 3 * q + m * n * q, n2 = 2 * nv, N1 = 2 * nv + 6, N2 = nv + 6;
  c->nF = nF;
  c->r = malloc(sizeof(double) * m);
  c->ox = malloc(sizeof(double) * (n * q + 1));
  c->oy = malloc(sizeof(double) * (n * q + 1));
  c->a = malloc(sizeof(double) * (n + 1));
  c->b = malloc(sizeof(double) * (n + 1));
  c->P = malloc(sizeof(double) * q * nv);
  c->Pd = malloc(sizeof(double) * q * nv);
  c->Pdd = malloc(sizeof(double) * q * nv);
  c->A = calloc(6 * nv, sizeof(double));
  c->F = calloc((size_t)nF * n2, sizeof(double));
  c->Q = calloc(n2 * n2, sizeof(double));
  c->K1 = calloc(N1 * N1, sizeof(double));
  c->K1lu = malloc(sizeof(double) * N1 * N1);
  c->piv1 = malloc(sizeof(int) * N1);
  c->K2 = calloc(N2 * N2, sizeof(double));
  c->K2lu = malloc(sizeof(double) * N2 * N2);
  c->piv2 = malloc(sizeof(int) * N2);
  if (!c->r || !c->ox || !c->oy || !c->a || !c->b || !c->P || !c->Pd || !c->Pdd || !c->A ||
      !c->F || !c->Q || !c->K1 || !c->K1lu || !c->piv1 || !c->K2 || !c->K2lu || !c->piv2) {
    st = AMO_ERR_NOMEM;
    goto fail;
  }
  memcpy(c->r, pb->r, sizeof(double) * m);
  for (int j = 0; j < n; ++j) {
    /* semi-axes inflated by the circle radius */
    c->a[j] = pb->oa[j] + pb->rc;
    c->b[j] = pb->ob[j] + pb->rc;
    if (!(c->a[j] > 0.0) || !(c->b[j] > 0.0)) { st = AMO_ERR_INVALID; goto fail; }
    for (int t = 0; t < q; ++t) {
      c->ox[j * q + t] = pb->ox[j * q + t];
      c->oy[j * q + t] = pb->oy[j * q + t];
    }
  }
  amo_basis(q, nv, pb->tf, c->P, c->Pd, c->Pdd);

  /* A: first and last rows of P, Pdot, Pddot (Sec. III-C). */
  for (int i = 0; i < nv; ++i) {
    c->A[0 * nv + i] = c->P[i];
    c->A[1 * nv + i] = c->Pd[i];
    c->A[2 * nv + i] = c->Pdd[i];
    c->A[3 * nv + i] = c->P[(q - 1) * nv + i];
    c->A[4 * nv + i] = c->Pd[(q - 1) * nv + i];
    c->A[5 * nv + i] = c->Pdd[(q - 1) * nv + i];
  }

  /* F block on (c_pos, c_slack): [A_v 0; A_a 0; A_ob; [0 P]] with
   * A_v = Pdot, A_a = Pddot and one [P, r_i P] block per (i, j). */
  for (int t = 0; t < q; ++t)
    for (int k = 0; k < nv; ++k) {
      c->F[(size_t)(t)*n2 + k] = c->Pd[t * nv + k];
      c->F[(size_t)(q + t) * n2 + k] = c->Pdd[t * nv + k];
      c->F[(size_t)(2 * q + m * n * q + t) * n2 + nv + k] = c->P[t * nv + k];
    }
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < n; ++j)
      for (int t = 0; t < q; ++t) {
        size_t row = (size_t)(2 * q + (i * n + j) * q + t);
        for (int k = 0; k < nv; ++k) {
          c->F[row * n2 + k] = c->P[t * nv + k];
          c->F[row * n2 + nv + k] = c->r[i] * c->P[t * nv + k];
        }
      }

  /* Q: block-diagonal Pddot^T Pddot on the position block and, unless
   * AMO_Q_CS_ZERO, on the slack block. */
  for (int a = 0; a < nv; ++a)
    for (int b = 0; b < nv; ++b) {
      double s = 0.0;
      for (int t = 0; t < q; ++t) s += c->Pdd[t * nv + a] * c->Pdd[t * nv + b];
      c->Q[a * n2 + b] = s;
      if (!(pb->flags & AMO_Q_CS_ZERO)) c->Q[(nv + a) * n2 + nv + b] = s;
    }

  /* KKT of xi1 (eqs. over_2, zeta_1_sepration_3): [Q + rho F^T F, A'^T; A', 0]
   * where A' = [A 0] acts on the position block only. */
  for (int a = 0; a < n2; ++a)
    for (int b = 0; b < n2; ++b) {
      double s = 0.0;
      for (int row = 0; row < nF; ++row) s += c->F[(size_t)row * n2 + a] * c->F[(size_t)row * n2 + b];
      c->K1[a * N1 + b] = c->Q[a * n2 + b] + pb->rho * s;
    }
  for (int e = 0; e < 6; ++e)
    for (int k = 0; k < nv; ++k) {
      c->K1[(n2 + e) * N1 + k] = c->A[e * nv + k];
      c->K1[k * N1 + n2 + e] = c->A[e * nv + k];
    }

  /* KKT of xi2 (eq. compute_convex_surrogate): [Pdd^T Pdd + rho P^T P, A^T; A, 0]. */
  for (int a = 0; a < nv; ++a)
    for (int b = 0; b < nv; ++b) {
      double s = 0.0;
      for (int t = 0; t < q; ++t)
        s += c->Pdd[t * nv + a] * c->Pdd[t * nv + b] + pb->rho * c->P[t * nv + a] * c->P[t * nv + b];
      c->K2[a * N2 + b] = s;
    }
  for (int e = 0; e < 6; ++e)
    for (int k = 0; k < nv; ++k) {
      c->K2[(nv + e) * N2 + k] = c->A[e * nv + k];
      c->K2[k * N2 + nv + e] = c->A[e * nv + k];
    }

  memcpy(c->K1lu, c->K1, sizeof(double) * N1 * N1);
  memcpy(c->K2lu, c->K2, sizeof(double) * N2 * N2);
  st = lu_factor(c->K1lu, c->piv1, N1);
  if (st == AMO_OK) st = lu_factor(c->K2lu, c->piv2, N2);
  if (st != AMO_OK) goto fail;
  if (status) *status = AMO_OK;
  return c;
fail:
  amo_free(c);
  if (status) *status = st;
  return NULL;
}

int amo_matrices(const amo_ctx *c, double *F, double *kkt1, double *kkt2) {
  if (!c) return AMO_ERR_INVALID;
  int nv = c->pb.nv;
  if (F) memcpy(F, c->F, sizeof(double) * (size_t)c->nF * 2 * nv);
  if (kkt1) memcpy(kkt1, c->K1, sizeof(double) * (2 * nv + 6) * (2 * nv + 6));
  if (kkt2) memcpy(kkt2, c->K2, sizeof(double) * (nv + 6) * (nv + 6));
  return AMO_OK;
}

/* ------------------------------------------------------------------ */
/* per-trajectory pieces                                               */
/* ------------------------------------------------------------------ */

static int scratch_alloc(const amo_ctx *c, scratch *w) {
  int q = c->pb.q;
  double **qs[] = {&w->x, &w->xd, &w->xdd, &w->y, &w->yd, &w->ydd, &w->psi, &w->c, &w->s};
  for (size_t i = 0; i < sizeof(qs) / sizeof(qs[0]); ++i) *qs[i] = malloc(sizeof(double) * q);
  w->g = malloc(sizeof(double) * c->nF);
  w->Fxi = malloc(sizeof(double) * c->nF);
  w->rhs = malloc(sizeof(double) * (2 * c->pb.nv + 6));
  for (size_t i = 0; i < sizeof(qs) / sizeof(qs[0]); ++i)
    if (!*qs[i]) return AMO_ERR_NOMEM;
  return (w->g && w->Fxi && w->rhs) ? AMO_OK : AMO_ERR_NOMEM;
}

static void scratch_free(scratch *w) {
  free(w->x); free(w->xd); free(w->xdd); free(w->y); free(w->yd); free(w->ydd);
  free(w->psi); free(w->c); free(w->s); free(w->g); free(w->Fxi); free(w->rhs);
}

/* Pointers to trajectory l's rows of the batch state. */
typedef struct {
  double *cx, *cc, *cy, *cs, *cpsi, *lam, *lampsi, *alpha, *d, *av, *dv, *aa, *da, *psihat;
} row;

static row row_of(const amo_ctx *c, const amo_state *st, int l) {
  int q = c->pb.q, nv = c->pb.nv;
  size_t mnq = (size_t)c->pb.m * c->pb.n * q;
  row r;
  r.cx = st->cx + (size_t)l * nv;
  r.cc = st->cc + (size_t)l * nv;
  r.cy = st->cy + (size_t)l * nv;
  r.cs = st->cs + (size_t)l * nv;
  r.cpsi = st->cpsi + (size_t)l * nv;
  r.lam = st->lam + (size_t)l * 4 * nv;
  r.lampsi = st->lampsi + (size_t)l * nv;
  r.alpha = st->alpha + (size_t)l * mnq;
  r.d = st->d + (size_t)l * mnq;
  r.av = st->av + (size_t)l * q;
  r.dv = st->dv + (size_t)l * q;
  r.aa = st->aa + (size_t)l * q;
  r.da = st->da + (size_t)l * q;
  r.psihat = st->psihat + (size_t)l * q;
  return r;
}

/* Trajectories from the coefficients (eq. param): positions, derivatives,
 * heading and the slack copies c(t), s(t). */
static void evaluate(const amo_ctx *c, const row *r, scratch *w) {
  int q = c->pb.q, nv = c->pb.nv;
  matvec(c->P, q, nv, r->cx, w->x);
  matvec(c->Pd, q, nv, r->cx, w->xd);
  matvec(c->Pdd, q, nv, r->cx, w->xdd);
  matvec(c->P, q, nv, r->cy, w->y);
  matvec(c->Pd, q, nv, r->cy, w->yd);
  matvec(c->Pdd, q, nv, r->cy, w->ydd);
  matvec(c->P, q, nv, r->cpsi, w->psi);
  matvec(c->P, q, nv, r->cc, w->c);
  matvec(c->P, q, nv, r->cs, w->s);
}

/* Offset of circle i from the robot centre along the body axis, as it enters
 * x~ and y~: (cos psi, sin psi) of eq. (compute_zeta_33), or the slack copies
 * (c, s) under AMO_XTILDE_SLACK. */
static void circle_dir(const amo_ctx *c, const scratch *w, int t, double *ux, double *uy) {
  if (c->pb.flags & AMO_XTILDE_SLACK) { *ux = w->c[t]; *uy = w->s[t]; }
  else { *ux = cos(w->psi[t]); *uy = sin(w->psi[t]); }
}

/* Target vector g of Sec. III-C for one axis (0 = x, 1 = y), built from the
 * current xi2 (heading), xi3 (angles) and xi4 (distances). */
static void build_g(const amo_ctx *c, const row *r, const scratch *w, int axis, double *g) {
  int q = c->pb.q, m = c->pb.m, n = c->pb.n;
  for (int t = 0; t < q; ++t) {
    double fv = axis == 0 ? cos(r->av[t]) : sin(r->av[t]);
    double fa = axis == 0 ? cos(r->aa[t]) : sin(r->aa[t]);
    g[t] = c->pb.vmax * r->dv[t] * fv;
    g[q + t] = c->pb.amax * r->da[t] * fa;
    g[2 * q + m * n * q + t] = axis == 0 ? cos(w->psi[t]) : sin(w->psi[t]);
  }
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < n; ++j)
      for (int t = 0; t < q; ++t) {
        int e = (i * n + j) * q + t;
        double al = r->alpha[e];
        g[2 * q + e] = axis == 0 ? c->ox[j * q + t] + c->a[j] * r->d[e] * cos(al)
                                 : c->oy[j * q + t] + c->b[j] * r->d[e] * sin(al);
      }
}

/* Step 2: xi1 from the QP (zeta_1_sepration_1); KKT right-hand side
 * [lambda + rho F^T g; b] (stationarity of eq. over_1 with the q-bar of
 * eq. zeta_1_sepration_3). */
static void step_xi1(const amo_ctx *c, const row *r, scratch *w) {
  int nv = c->pb.nv, n2 = 2 * nv;
  evaluate(c, r, w);
  for (int axis = 0; axis < 2; ++axis) {
    double Ftg[64];
    build_g(c, r, w, axis, w->g);
    matTvec(c->F, c->nF, n2, w->g, Ftg);
    const double *lam = r->lam + axis * n2;
    const double *bb = axis == 0 ? c->pb.bx : c->pb.by;
    for (int k = 0; k < n2; ++k) w->rhs[k] = lam[k] + c->pb.rho * Ftg[k];
    for (int e = 0; e < 6; ++e) w->rhs[n2 + e] = bb[e];
    lu_solve(c->K1lu, c->piv1, n2 + 6, w->rhs);
    double *cp = axis == 0 ? r->cx : r->cy;
    double *cs = axis == 0 ? r->cc : r->cs;
    for (int k = 0; k < nv; ++k) { cp[k] = w->rhs[k]; cs[k] = w->rhs[nv + k]; }
  }
}

/* Step 3: xi2 from the convex surrogate (compute_convex_surrogate).  By
 * default psi_hat = atan2(s, c) is taken on the branch nearest the current
 * heading psi^k. */
static void step_xi2(const amo_ctx *c, const row *r, scratch *w) {
  int q = c->pb.q, nv = c->pb.nv;
  evaluate(c, r, w);
  for (int t = 0; t < q; ++t) {
    double cc = w->c[t], ss = w->s[t], p = w->psi[t];
    if (c->pb.flags & AMO_PSI_NO_UNWRAP) r->psihat[t] = atan2z(ss, cc);
    else r->psihat[t] = p + atan2z(ss * cos(p) - cc * sin(p), cc * cos(p) + ss * sin(p));
  }
  double Ptp[64];
  matTvec(c->P, q, nv, r->psihat, Ptp);
  for (int k = 0; k < nv; ++k) w->rhs[k] = r->lampsi[k] + c->pb.rho * Ptp[k];
  for (int e = 0; e < 6; ++e) w->rhs[nv + e] = c->pb.bpsi[e];
  lu_solve(c->K2lu, c->piv2, nv + 6, w->rhs);
  for (int k = 0; k < nv; ++k) r->cpsi[k] = w->rhs[k];
}

/* Step 4: xi3 closed forms (zeta_2, alpha_v, alpha_a). */
static void step_xi3(const amo_ctx *c, const row *r, scratch *w) {
  int q = c->pb.q, m = c->pb.m, n = c->pb.n;
  evaluate(c, r, w);
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < n; ++j)
      for (int t = 0; t < q; ++t) {
        double ux, uy;
        circle_dir(c, w, t, &ux, &uy);
        double xt = w->x[t] + c->r[i] * ux - c->ox[j * q + t];
        double yt = w->y[t] + c->r[i] * uy - c->oy[j * q + t];
        int e = (i * n + j) * q + t;
        if (c->pb.flags & AMO_ALPHA_LITERAL) r->alpha[e] = atan2z(yt, xt);
        else r->alpha[e] = atan2z(c->a[j] * yt, c->b[j] * xt);
      }
  for (int t = 0; t < q; ++t) {
    r->av[t] = atan2z(w->yd[t], w->xd[t]);
    r->aa[t] = atan2z(w->ydd[t], w->xdd[t]);
  }
}

/* Step 5: xi4 closed forms (compute_zeta_3, compute_dv, compute_da): the
 * unconstrained minimiser of each single-variable QP, then d_ij >= 1 and
 * d_v, d_a clipped to [0, 1]. */
static void step_xi4(const amo_ctx *c, const row *r, scratch *w) {
  int q = c->pb.q, m = c->pb.m, n = c->pb.n;
  evaluate(c, r, w);
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < n; ++j)
      for (int t = 0; t < q; ++t) {
        double ux, uy;
        circle_dir(c, w, t, &ux, &uy);
        double xt = w->x[t] + c->r[i] * ux - c->ox[j * q + t];
        double yt = w->y[t] + c->r[i] * uy - c->oy[j * q + t];
        int e = (i * n + j) * q + t;
        double ca = cos(r->alpha[e]), sa = sin(r->alpha[e]);
        double a = c->a[j], b = c->b[j];
        double dd = (a * xt * ca + b * yt * sa) / (a * a * ca * ca + b * b * sa * sa);
        r->d[e] = dd > 1.0 ? dd : 1.0;
      }
  for (int t = 0; t < q; ++t) {
    double dv = (w->xd[t] * cos(r->av[t]) + w->yd[t] * sin(r->av[t])) / c->pb.vmax;
    double da = (w->xdd[t] * cos(r->aa[t]) + w->ydd[t] * sin(r->aa[t])) / c->pb.amax;
    r->dv[t] = dv < 0.0 ? 0.0 : (dv > 1.0 ? 1.0 : dv);
    r->da[t] = da < 0.0 ? 0.0 : (da > 1.0 ? 1.0 : da);
  }
}

/* Step 5 of the AM list: lambda <- lambda - rho F^T (F xi1 - g)
 * (update_lambda_1), lambda_psi <- lambda_psi - rho_psi P^T (P c_psi - psi_hat)
 * (update_lambda_psi; the printed sign under AMO_LAMPSI_LITERAL). */
static void step_lambda(const amo_ctx *c, const row *r, scratch *w) {
  int q = c->pb.q, nv = c->pb.nv, n2 = 2 * nv;
  evaluate(c, r, w);
  for (int axis = 0; axis < 2; ++axis) {
    double xi[64], Ftr[64];
    const double *cp = axis == 0 ? r->cx : r->cy;
    const double *cs = axis == 0 ? r->cc : r->cs;
    for (int k = 0; k < nv; ++k) { xi[k] = cp[k]; xi[nv + k] = cs[k]; }
    build_g(c, r, w, axis, w->g);
    matvec(c->F, c->nF, n2, xi, w->Fxi);
    for (int row = 0; row < c->nF; ++row) w->Fxi[row] -= w->g[row];
    matTvec(c->F, c->nF, n2, w->Fxi, Ftr);
    double *lam = r->lam + axis * n2;
    for (int k = 0; k < n2; ++k) lam[k] -= c->pb.rho * Ftr[k];
  }
  double diff[4096], Ptd[64];
  for (int t = 0; t < q; ++t)
    diff[t] = (c->pb.flags & AMO_LAMPSI_LITERAL) ? r->psihat[t] - w->psi[t]
                                                  : w->psi[t] - r->psihat[t];
  matTvec(c->P, q, nv, diff, Ptd);
  for (int k = 0; k < nv; ++k) r->lampsi[k] -= c->pb.rho_psi * Ptd[k];
}

/* max over (i, j, t) of |f_c| (eq. collision_avoidance_proposed). */
static double collision_residual(const amo_ctx *c, const row *r, scratch *w) {
  int q = c->pb.q, m = c->pb.m, n = c->pb.n;
  double worst = 0.0;
  evaluate(c, r, w);
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < n; ++j)
      for (int t = 0; t < q; ++t) {
        int e = (i * n + j) * q + t;
        double fx = w->x[t] + c->r[i] * cos(w->psi[t]) - c->ox[j * q + t] -
                    c->a[j] * r->d[e] * cos(r->alpha[e]);
        double fy = w->y[t] + c->r[i] * sin(w->psi[t]) - c->oy[j * q + t] -
                    c->b[j] * r->d[e] * sin(r->alpha[e]);
        worst = fmax(worst, sqrt(fx * fx + fy * fy));
      }
  return worst;
}

static int check_state(const amo_ctx *c, int B, const amo_state *st) {
  if (!c || B < 0 || !st) return AMO_ERR_INVALID;
  if (!st->cx || !st->cc || !st->cy || !st->cs || !st->cpsi || !st->lam || !st->lampsi ||
      !st->alpha || !st->d || !st->av || !st->dv || !st->aa || !st->da || !st->psihat)
    return AMO_ERR_INVALID;
  if (c->pb.q > 4096 || 2 * c->pb.nv > 64) return AMO_ERR_INVALID;
  return AMO_OK;
}

int amo_step(const amo_ctx *c, int B, int which, const amo_state *st) {
  int s = check_state(c, B, st);
  if (s != AMO_OK) return s;
  if (which < AMO_STEP_XI1 || which > AMO_STEP_LAMBDA) return AMO_ERR_INVALID;
  scratch w;
  if (scratch_alloc(c, &w) != AMO_OK) { scratch_free(&w); return AMO_ERR_NOMEM; }
  for (int l = 0; l < B; ++l) {
    row r = row_of(c, st, l);
    switch (which) {
      case AMO_STEP_XI1: step_xi1(c, &r, &w); break;
      case AMO_STEP_XI2: step_xi2(c, &r, &w); break;
      case AMO_STEP_XI3: step_xi3(c, &r, &w); break;
      case AMO_STEP_XI4: step_xi4(c, &r, &w); break;
      default: step_lambda(c, &r, &w); break;
    }
  }
  scratch_free(&w);
  return AMO_OK;
}

int amo_solve(const amo_ctx *c, int B, int K, const amo_state *st, double *hist, int nthreads) {
  int s = check_state(c, B, st);
  if (s != AMO_OK) return s;
  if (K < 0) return AMO_ERR_INVALID;
  int failed = 0;
#ifdef _OPENMP
  if (nthreads <= 0) nthreads = omp_get_max_threads();
#pragma omp parallel num_threads(nthreads) reduction(| : failed)
#endif
  {
    scratch w;
    if (scratch_alloc(c, &w) != AMO_OK) failed = 1;
    else {
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 1)
#endif
      for (int l = 0; l < B; ++l) {
        row r = row_of(c, st, l);
        /* Step 1: initial xi3, xi4 from the given trajectory. */
        step_xi3(c, &r, &w);
        step_xi4(c, &r, &w);
        for (int k = 0; k < K; ++k) {
          step_xi1(c, &r, &w);
          step_xi2(c, &r, &w);
          step_xi3(c, &r, &w);
          step_xi4(c, &r, &w);
          step_lambda(c, &r, &w);
          if (hist) hist[(size_t)k * B + l] = collision_residual(c, &r, &w);
        }
      }
    }
    scratch_free(&w);
  }
  (void)nthreads;
  return failed ? AMO_ERR_NOMEM : AMO_OK;
}

int amo_lagrangian(const amo_ctx *c, int B, const amo_state *st, double *out) {
  int s = check_state(c, B, st);
  if (s != AMO_OK || !out) return s != AMO_OK ? s : AMO_ERR_INVALID;
  int q = c->pb.q, nv = c->pb.nv, n2 = 2 * nv;
  scratch w;
  if (scratch_alloc(c, &w) != AMO_OK) { scratch_free(&w); return AMO_ERR_NOMEM; }
  for (int l = 0; l < B; ++l) {
    row r = row_of(c, st, l);
    evaluate(c, &r, &w);
    double L = 0.0;
    for (int axis = 0; axis < 2; ++axis) {
      double xi[64], Qxi[64];
      const double *cp = axis == 0 ? r.cx : r.cy;
      const double *cs = axis == 0 ? r.cc : r.cs;
      for (int k = 0; k < nv; ++k) { xi[k] = cp[k]; xi[nv + k] = cs[k]; }
      matvec(c->Q, n2, n2, xi, Qxi);
      const double *lam = r.lam + axis * n2;
      for (int k = 0; k < n2; ++k) L += 0.5 * xi[k] * Qxi[k] - lam[k] * xi[k];
      build_g(c, &r, &w, axis, w.g);
      matvec(c->F, c->nF, n2, xi, w.Fxi);
      for (int row = 0; row < c->nF; ++row) {
        double e = w.Fxi[row] - w.g[row];
        L += 0.5 * c->pb.rho * e * e;
      }
    }
    double acc[4096];
    matvec(c->Pdd, q, nv, r.cpsi, acc);
    for (int t = 0; t < q; ++t) L += 0.5 * acc[t] * acc[t];
    for (int k = 0; k < nv; ++k) L -= r.lampsi[k] * r.cpsi[k];
    out[l] = L;
  }
  scratch_free(&w);
  return AMO_OK;
}

/* Residual statistics per trajectory (columns of out):
 *  0 max |f_c|  (eq. collision_avoidance_proposed, stored alpha and d)
 *  1 RMS |f_c|
 *  2 max |f_v|  (eq. fv)           3 max |f_a|  (eq. fa)
 *  4 max(|c - cos psi|, |s - sin psi|)  (eqs. cos_ref, sin_ref)
 *  5 max |atan2(s, c) - psi| wrapped to (-pi, pi]
 *  6 max boundary violation |A c - b| over x, y, psi  (eq. reform_eq)
 *  7 cost sum_t (xdd^2 + ydd^2 + psidd^2)  (eq. acc_cost)
 *  8 min over (i, j, t) of sqrt(xt^2/a^2 + yt^2/b^2) - 1 with the physical
 *    heading (>= 0: every circle centre outside every inflated ellipse)
 *  9 max_t |v| - vmax   10 max_t |a| - amax   (eq. acc_constraint)
 * 11 1 if any state value of the trajectory is not finite, else 0 */
int amo_residuals(const amo_ctx *c, int B, const amo_state *st, double *out) {
  int s = check_state(c, B, st);
  if (s != AMO_OK || !out) return s != AMO_OK ? s : AMO_ERR_INVALID;
  int q = c->pb.q, nv = c->pb.nv, m = c->pb.m, n = c->pb.n;
  const double pi = acos(-1.0);
  scratch w;
  if (scratch_alloc(c, &w) != AMO_OK) { scratch_free(&w); return AMO_ERR_NOMEM; }
  for (int l = 0; l < B; ++l) {
    row r = row_of(c, st, l);
    double *o = out + (size_t)l * AMO_NRES;
    evaluate(c, &r, &w);
    double fcmax = 0.0, fcsq = 0.0, level = INFINITY;
    for (int i = 0; i < m; ++i)
      for (int j = 0; j < n; ++j)
        for (int t = 0; t < q; ++t) {
          int e = (i * n + j) * q + t;
          double xt = w.x[t] + c->r[i] * cos(w.psi[t]) - c->ox[j * q + t];
          double yt = w.y[t] + c->r[i] * sin(w.psi[t]) - c->oy[j * q + t];
          double fx = xt - c->a[j] * r.d[e] * cos(r.alpha[e]);
          double fy = yt - c->b[j] * r.d[e] * sin(r.alpha[e]);
          double f2 = fx * fx + fy * fy;
          fcmax = fmax(fcmax, sqrt(f2));
          fcsq += f2;
          level = fmin(level, sqrt(xt * xt / (c->a[j] * c->a[j]) + yt * yt / (c->b[j] * c->b[j])) - 1.0);
        }
    double fv = 0.0, fa = 0.0, slack = 0.0, head = 0.0, cost = 0.0, vex = -INFINITY, aex = -INFINITY;
    double psidd[4096];
    matvec(c->Pdd, q, nv, r.cpsi, psidd);
    for (int t = 0; t < q; ++t) {
      double vx = w.xd[t] - c->pb.vmax * r.dv[t] * cos(r.av[t]);
      double vy = w.yd[t] - c->pb.vmax * r.dv[t] * sin(r.av[t]);
      double ax = w.xdd[t] - c->pb.amax * r.da[t] * cos(r.aa[t]);
      double ay = w.ydd[t] - c->pb.amax * r.da[t] * sin(r.aa[t]);
      fv = fmax(fv, sqrt(vx * vx + vy * vy));
      fa = fmax(fa, sqrt(ax * ax + ay * ay));
      slack = fmax(slack, fmax(fabs(w.c[t] - cos(w.psi[t])), fabs(w.s[t] - sin(w.psi[t]))));
      double dh = atan2z(w.s[t], w.c[t]) - w.psi[t];
      dh = dh - 2.0 * pi * floor((dh + pi) / (2.0 * pi));
      head = fmax(head, fabs(dh));
      cost += w.xdd[t] * w.xdd[t] + w.ydd[t] * w.ydd[t] + psidd[t] * psidd[t];
      vex = fmax(vex, sqrt(w.xd[t] * w.xd[t] + w.yd[t] * w.yd[t]) - c->pb.vmax);
      aex = fmax(aex, sqrt(w.xdd[t] * w.xdd[t] + w.ydd[t] * w.ydd[t]) - c->pb.amax);
    }
    double bc = 0.0, Ac[6];
    const double *cs3[3] = {r.cx, r.cy, r.cpsi};
    const double *bs3[3] = {c->pb.bx, c->pb.by, c->pb.bpsi};
    for (int v = 0; v < 3; ++v) {
      matvec(c->A, 6, nv, cs3[v], Ac);
      for (int e = 0; e < 6; ++e) bc = fmax(bc, fabs(Ac[e] - bs3[v][e]));
    }
    int bad = 0;
    for (int k = 0; k < nv; ++k)
      bad |= !isfinite(r.cx[k]) || !isfinite(r.cy[k]) || !isfinite(r.cc[k]) ||
             !isfinite(r.cs[k]) || !isfinite(r.cpsi[k]) || !isfinite(r.lampsi[k]);
    for (int k = 0; k < 4 * nv; ++k) bad |= !isfinite(r.lam[k]);
    size_t mnq = (size_t)m * n * q;
    for (size_t e = 0; e < mnq; ++e) bad |= !isfinite(r.alpha[e]) || !isfinite(r.d[e]);
    o[0] = fcmax;
    o[1] = mnq ? sqrt(fcsq / (double)mnq) : 0.0;
    o[2] = fv;
    o[3] = fa;
    o[4] = slack;
    o[5] = head;
    o[6] = bc;
    o[7] = cost;
    o[8] = mnq ? level : INFINITY;
    o[9] = vex;
    o[10] = aex;
    o[11] = bad ? 1.0 : 0.0;
  }
  scratch_free(&w);
  return AMO_OK;
}
