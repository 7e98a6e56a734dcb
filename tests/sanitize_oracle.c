/* Drives every entry point of the FP64 oracle on small problems, for a build
 * with AddressSanitizer and UndefinedBehaviorSanitizer (tests/test_oracle_sanitize.py):
 * a stray read or write, an overflow or another undefined operation aborts
 * the run.  Prints one line per case and "ok" at the end. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "am_oracle.h"

static double *zeros(size_t n) {
  double *p = (double *)calloc(n ? n : 1, sizeof(double));
  if (!p) exit(3);
  return p;
}

static int run_case(int q, int nv, int m, int n, int B, unsigned flags, int nthreads) {
  double r[8], *ox = zeros((size_t)n * q), *oy = zeros((size_t)n * q), oa[8], ob[8];
  for (int i = 0; i < m; ++i) r[i] = 0.3 * (i - 0.5 * (m - 1));
  for (int j = 0; j < n; ++j) {
    oa[j] = 0.3 + 0.1 * j;
    ob[j] = 0.5 - 0.05 * j;
    for (int k = 0; k < q; ++k) {
      ox[j * q + k] = 3.0 + 1.5 * j + 0.02 * k;
      oy[j * q + k] = 5.0 - 0.5 * j + 0.01 * k;
    }
  }
  amo_problem pb;
  memset(&pb, 0, sizeof pb);
  pb.q = q; pb.nv = nv; pb.tf = 20.0; pb.m = m; pb.r = r; pb.n = n;
  pb.ox = ox; pb.oy = oy; pb.oa = oa; pb.ob = ob; pb.rc = 0.25;
  const double bx[6] = {1, 0, 0, 9, 0, 0}, by[6] = {1, 0, 0, 9, 0, 0}, bp[6] = {0, 0, 0, 0, 0, 0};
  memcpy(pb.bx, bx, sizeof bx); memcpy(pb.by, by, sizeof by); memcpy(pb.bpsi, bp, sizeof bp);
  pb.vmax = 1.5; pb.amax = 1.5; pb.rho = 1.0; pb.rho_psi = 1.0; pb.flags = flags;
  int status = 0;
  amo_ctx *ctx = amo_create(&pb, &status);
  if (!ctx) { printf("create failed %d\n", status); return 1; }
  const size_t mn = (size_t)m * n;
  amo_state st;
  st.cx = zeros((size_t)B * nv); st.cc = zeros((size_t)B * nv); st.cy = zeros((size_t)B * nv);
  st.cs = zeros((size_t)B * nv); st.cpsi = zeros((size_t)B * nv); st.lam = zeros((size_t)B * 4 * nv);
  st.lampsi = zeros((size_t)B * nv); st.alpha = zeros((size_t)B * mn * q); st.d = zeros((size_t)B * mn * q);
  st.av = zeros((size_t)B * q); st.dv = zeros((size_t)B * q); st.aa = zeros((size_t)B * q);
  st.da = zeros((size_t)B * q); st.psihat = zeros((size_t)B * q);
  for (int l = 0; l < B; ++l)
    for (int k = 0; k < nv; ++k) {   /* a straight line with a bend per sample */
      const double s = (double)k / (nv - 1);
      st.cx[l * nv + k] = 1 + 8 * s + (k > 0 && k < nv - 1 ? 0.3 * (l - 1) : 0.0);
      st.cy[l * nv + k] = 1 + 8 * s - (k > 0 && k < nv - 1 ? 0.2 * l : 0.0);
      st.cc[l * nv + k] = 1.0;
    }
  double *P = zeros((size_t)q * nv), *Pd = zeros((size_t)q * nv), *Pdd = zeros((size_t)q * nv);
  double *F = zeros((size_t)(3 * q + mn * q) * 2 * nv);
  double *K1 = zeros((size_t)(2 * nv + 6) * (2 * nv + 6)), *K2 = zeros((size_t)(nv + 6) * (nv + 6));
  double *hist = zeros((size_t)8 * B), *lag = zeros((size_t)B), *res = zeros((size_t)B * AMO_NRES);
  int rc = amo_basis(q, nv, pb.tf, P, Pd, Pdd);
  rc |= amo_matrices(ctx, F, K1, K2);
  for (int w = AMO_STEP_XI3; w <= AMO_STEP_XI4; ++w) rc |= amo_step(ctx, B, w, &st);
  for (int w = AMO_STEP_XI1; w <= AMO_STEP_LAMBDA; ++w) rc |= amo_step(ctx, B, w, &st);
  rc |= amo_solve(ctx, B, 8, &st, hist, nthreads);
  rc |= amo_lagrangian(ctx, B, &st, lag);
  rc |= amo_residuals(ctx, B, &st, res);
  double sum = 0.0;
  for (int l = 0; l < B; ++l) {
    sum += lag[l];
    for (int c = 0; c < AMO_NRES; ++c)
      if (isfinite(res[l * AMO_NRES + c])) sum += res[l * AMO_NRES + c];
  }
  printf("q=%d nv=%d m=%d n=%d B=%d flags=%u threads=%d rc=%d finite=%d\n", q, nv, m, n, B, flags, nthreads, rc,
         isfinite(sum) ? 1 : 0);
  amo_free(ctx);
  free(ox); free(oy); free(P); free(Pd); free(Pdd); free(F); free(K1); free(K2); free(hist); free(lag); free(res);
  free(st.cx); free(st.cc); free(st.cy); free(st.cs); free(st.cpsi); free(st.lam); free(st.lampsi);
  free(st.alpha); free(st.d); free(st.av); free(st.dv); free(st.aa); free(st.da); free(st.psihat);
  return rc != 0 || !isfinite(sum);
}

int main(void) {
  int bad = 0;
  bad |= run_case(24, 8, 3, 3, 4, 0u, 1);
  bad |= run_case(24, 8, 3, 3, 4, 0u, 2);
  bad |= run_case(17, 6, 1, 0, 2, 0u, 1);   /* no obstacles, one circle, odd q */
  bad |= run_case(30, 11, 5, 4, 3, AMO_ALPHA_LITERAL | AMO_XTILDE_SLACK | AMO_PSI_NO_UNWRAP | AMO_LAMPSI_LITERAL, 1);
  bad |= run_case(20, 7, 2, 2, 1, AMO_Q_CS_ZERO, 1);
  /* invalid arguments are refused without touching memory */
  amo_problem pb;
  memset(&pb, 0, sizeof pb);
  pb.q = 1; pb.nv = 11;
  int status = 0;
  amo_ctx *ctx = amo_create(&pb, &status);
  printf("invalid create -> %s, status %d\n", ctx ? "ctx" : "NULL", status);
  bad |= ctx != NULL || status == 0;
  bad |= amo_basis(0, 11, 1.0, NULL, NULL, NULL) == 0;
  printf(bad ? "FAILED\n" : "ok\n");
  return bad;
}
