// am_setup.hip -- one-time FP64 construction of the constant operators of the
// batched AM iteration (Sec. III-A eqs. over_2/over_3; Sec. IV: F^T F is
// formed once), on the GPU in a single workgroup.
//
// The Bernstein basis P (eq. param) is factored P = U R with U orthonormal on
// the time grid.  The iteration runs on z = R c: x = U z, xdot = V z,
// xddot = W z with V = Pdot R^-1, W = Pddot R^-1.  In these coordinates the
// Gram matrix of the position rows is the identity, so the xi1 KKT matrix is
// well conditioned and its FP32 application does not amplify rounding the way
// the Bernstein-coordinate inverse does.  The KKT matrices are assembled in z
// coordinates and inverted by Gauss-Jordan elimination with partial pivoting.
#include <hip/hip_runtime.h>

#include "am_internal.h"

namespace amk {
namespace {

constexpr int kSetupThreads = 256;

__device__ double bernstein(int deg, int i, double tau) {
  if (i < 0 || i > deg) return 0.0;
  // C(deg, i) tau^i (1 - tau)^(deg - i), binomial built multiplicatively
  double c = 1.0;
  for (int k = 1; k <= i; ++k) c = c * double(deg - i + k) / double(k);
  double v = c;
  for (int k = 0; k < i; ++k) v *= tau;
  for (int k = 0; k < deg - i; ++k) v *= (1.0 - tau);
  return v;
}

// Block-wide sum of one value per thread.
__device__ double block_sum(double v, double *sh) {
  const int tid = threadIdx.x;
  sh[tid] = v;
  __syncthreads();
  for (int s = kSetupThreads / 2; s > 0; s >>= 1) {
    if (tid < s) sh[tid] += sh[tid + s];
    __syncthreads();
  }
  double r = sh[0];
  __syncthreads();
  return r;
}

// In-place Gauss-Jordan inverse of the N x N matrix stored in the left half
// of aug [N][2N] (right half is set to I here).  Returns false if a pivot is
// below tol * max|K|.
__device__ bool gauss_jordan(double *aug, int N, double *sh, int *ish) {
  const int tid = threadIdx.x, W2 = 2 * N;
  for (int idx = tid; idx < N * N; idx += kSetupThreads) {
    int r = idx / N, c = idx % N;
    aug[r * W2 + N + c] = (r == c) ? 1.0 : 0.0;
  }
  double big = 0.0;
  for (int idx = tid; idx < N * N; idx += kSetupThreads)
    big = fmax(big, fabs(aug[(idx / N) * W2 + idx % N]));
  sh[tid] = big;
  __syncthreads();
  for (int s = kSetupThreads / 2; s > 0; s >>= 1) {
    if (tid < s) sh[tid] = fmax(sh[tid], sh[tid + s]);
    __syncthreads();
  }
  const double tol = 1e-13 * sh[0];
  __syncthreads();
  bool ok = sh[0] > 0.0;
  for (int col = 0; col < N && ok; ++col) {
    if (tid == 0) {
      int p = col;
      for (int r = col + 1; r < N; ++r)
        if (fabs(aug[r * W2 + col]) > fabs(aug[p * W2 + col])) p = r;
      ish[0] = p;
      ish[1] = fabs(aug[p * W2 + col]) > tol;
    }
    __syncthreads();
    const int p = ish[0];
    ok = ish[1] != 0;
    if (!ok) break;
    if (p != col)
      for (int c = tid; c < W2; c += kSetupThreads) {
        double t = aug[col * W2 + c];
        aug[col * W2 + c] = aug[p * W2 + c];
        aug[p * W2 + c] = t;
      }
    __syncthreads();
    const double inv = 1.0 / aug[col * W2 + col];
    __syncthreads();
    for (int c = tid; c < W2; c += kSetupThreads) aug[col * W2 + c] *= inv;
    // elimination factors of column `col`, read before any row is updated
    double *fac = sh;
    for (int r = tid; r < N; r += kSetupThreads) fac[r] = (r == col) ? 0.0 : aug[r * W2 + col];
    __syncthreads();
    for (int idx = tid; idx < N * W2; idx += kSetupThreads) {
      const int r = idx / W2, c = idx % W2;
      if (r != col) aug[r * W2 + c] -= fac[r] * aug[col * W2 + c];
    }
    __syncthreads();
  }
  return ok;
}

template <typename T>
__device__ void to_typed(const double *src, void *dst, int count) {
  T *d = static_cast<T *>(dst);
  for (int i = threadIdx.x; i < count; i += kSetupThreads) d[i] = T(src[i]);
}

struct SetupArgs {
  int q, nv, m, n, flags, f64;
  double tf, rho;
  const double *r;
  Consts c;
};

__global__ __launch_bounds__(kSetupThreads) void setup_kernel(SetupArgs a) {
  __shared__ double sh[kSetupThreads];
  __shared__ int ish[2];
  const int tid = threadIdx.x;
  const int q = a.q, nv = a.nv, N = nv - 1, n2 = 2 * nv, N1 = n2 + 6, N2 = nv + 6;
  const Consts &c = a.c;

  // 1. Bernstein basis and its time derivatives on t_k = k tf/(q-1).
  for (int idx = tid; idx < q * nv; idx += kSetupThreads) {
    const int t = idx / nv, i = idx % nv;
    const double tau = double(t) / double(q - 1);
    c.P[idx] = bernstein(N, i, tau);
    c.Pd[idx] = double(N) * (bernstein(N - 1, i - 1, tau) - bernstein(N - 1, i, tau)) / a.tf;
    c.Pdd[idx] = double(N) * double(N - 1) *
                 (bernstein(N - 2, i - 2, tau) - 2.0 * bernstein(N - 2, i - 1, tau) +
                  bernstein(N - 2, i, tau)) / (a.tf * a.tf);
  }
  for (int idx = tid; idx < nv * nv; idx += kSetupThreads) c.R[idx] = 0.0;
  __syncthreads();

  // 2. Thin QR, P = U R, by Gram-Schmidt with one re-orthogonalisation pass.
  for (int k = 0; k < nv; ++k) {
    for (int t = tid; t < q; t += kSetupThreads) c.U[t * nv + k] = c.P[t * nv + k];
    __syncthreads();
    for (int pass = 0; pass < 2; ++pass)
      for (int j = 0; j < k; ++j) {
        double part = 0.0;
        for (int t = tid; t < q; t += kSetupThreads) part += c.U[t * nv + j] * c.U[t * nv + k];
        const double rj = block_sum(part, sh);
        for (int t = tid; t < q; t += kSetupThreads) c.U[t * nv + k] -= rj * c.U[t * nv + j];
        if (tid == 0) c.R[j * nv + k] += rj;
        __syncthreads();
      }
    double part = 0.0;
    for (int t = tid; t < q; t += kSetupThreads) part += c.U[t * nv + k] * c.U[t * nv + k];
    const double nrm = sqrt(block_sum(part, sh));
    for (int t = tid; t < q; t += kSetupThreads) c.U[t * nv + k] /= nrm;
    if (tid == 0) c.R[k * nv + k] = nrm;
    __syncthreads();
  }

  // 3. R^-1 (upper triangular), column by column.
  if (tid < nv) {
    const int col = tid;
    for (int i = nv - 1; i >= 0; --i) {
      double s = (i == col) ? 1.0 : 0.0;
      for (int j = i + 1; j < nv; ++j) s -= c.R[i * nv + j] * c.Rinv[j * nv + col];
      c.Rinv[i * nv + col] = (i > col) ? 0.0 : s / c.R[i * nv + i];
    }
  }
  __syncthreads();

  // 4. V = Pdot R^-1, W = Pddot R^-1.
  for (int idx = tid; idx < q * nv; idx += kSetupThreads) {
    const int t = idx / nv, k = idx % nv;
    double v = 0.0, w = 0.0;
    for (int j = 0; j < nv; ++j) {
      v += c.Pd[t * nv + j] * c.Rinv[j * nv + k];
      w += c.Pdd[t * nv + j] * c.Rinv[j * nv + k];
    }
    c.V[idx] = v;
    c.W[idx] = w;
  }
  __syncthreads();

  // 5. Gram matrices G_UU, G_VV, G_WW.
  double *GUU = c.G, *GVV = c.G + nv * nv, *GWW = c.G + 2 * nv * nv;
  for (int idx = tid; idx < 3 * nv * nv; idx += kSetupThreads) {
    const int which = idx / (nv * nv), e = idx % (nv * nv), i = e / nv, j = e % nv;
    const double *X = which == 0 ? c.U : (which == 1 ? c.V : c.W);
    double s = 0.0;
    for (int t = 0; t < q; ++t) s += X[t * nv + i] * X[t * nv + j];
    c.G[idx] = s;
  }
  __syncthreads();

  // 6. F^T F of one axis and the two KKT matrices in z coordinates.
  //    F rows: [V 0], [W 0], [U r_i U] per (i, j), [0 U]  (Sec. III-C).
  double sr = 0.0, sr2 = 0.0;
  for (int i = 0; i < a.m; ++i) { sr += a.r[i]; sr2 += a.r[i] * a.r[i]; }
  const double mn = double(a.m) * double(a.n), nsr = double(a.n) * sr, nsr2 = double(a.n) * sr2;
  const bool q_cs = !(a.flags & AM_Q_CS_ZERO);
  for (int idx = tid; idx < n2 * n2; idx += kSetupThreads) {
    const int I = idx / n2, J = idx % n2, i = I % nv, j = J % nv;
    const int bi = I / nv, bj = J / nv;
    double f, qc;
    if (bi == 0 && bj == 0) {
      f = GVV[i * nv + j] + GWW[i * nv + j] + mn * GUU[i * nv + j];
      qc = GWW[i * nv + j];
    } else if (bi == 1 && bj == 1) {
      f = (nsr2 + 1.0) * GUU[i * nv + j];
      qc = q_cs ? GWW[i * nv + j] : 0.0;
    } else {
      f = nsr * GUU[i * nv + j];
      qc = 0.0;
    }
    c.GF[idx] = f;
    c.A1[I * 2 * N1 + J] = qc + a.rho * f;
  }
  // boundary rows: U, V, W at t = 0 and t = q-1 on the position block
  for (int idx = tid; idx < 6 * N1; idx += kSetupThreads) {
    const int e = idx / N1, J = idx % N1;
    double v = 0.0;
    if (J < nv) {
      const int t = e < 3 ? 0 : q - 1;
      const double *X = (e % 3 == 0) ? c.U : ((e % 3 == 1) ? c.V : c.W);
      v = X[t * nv + J];
    }
    c.A1[(n2 + e) * 2 * N1 + J] = v;   // row block  A'
    c.A1[J * 2 * N1 + n2 + e] = v;     // column block A'^T
  }
  for (int idx = tid; idx < 36; idx += kSetupThreads)
    c.A1[(n2 + idx / 6) * 2 * N1 + n2 + idx % 6] = 0.0;
  // xi2: [W^T W + rho U^T U, A^T; A, 0]
  for (int idx = tid; idx < N2 * N2; idx += kSetupThreads) {
    const int I = idx / N2, J = idx % N2;
    double v = 0.0;
    if (I < nv && J < nv) v = GWW[I * nv + J] + a.rho * GUU[I * nv + J];
    else if (I < nv || J < nv) {
      const int e = (I < nv) ? J - nv : I - nv, k = (I < nv) ? I : J;
      const int t = e < 3 ? 0 : q - 1;
      const double *X = (e % 3 == 0) ? c.U : ((e % 3 == 1) ? c.V : c.W);
      v = X[t * nv + k];
    }
    c.A2[I * 2 * N2 + J] = v;
  }
  __syncthreads();
  for (int idx = tid; idx < N1 * N1; idx += kSetupThreads)
    c.K1[idx] = c.A1[(idx / N1) * 2 * N1 + idx % N1];
  for (int idx = tid; idx < N2 * N2; idx += kSetupThreads)
    c.K2[idx] = c.A2[(idx / N2) * 2 * N2 + idx % N2];
  __syncthreads();

  // 7. Inverses.
  const bool ok1 = gauss_jordan(c.A1, N1, sh, ish);
  const bool ok2 = gauss_jordan(c.A2, N2, sh, ish);
  if (tid == 0) c.status[0] = !ok1 ? 1.0 : (!ok2 ? 2.0 : 0.0);
  __syncthreads();
  if (!ok1 || !ok2) return;

  // 8. Blocks used by the iteration: [z; mu] = Kinv [rhs; b].
  for (int idx = tid; idx < n2 * n2; idx += kSetupThreads)
    c.M1[idx] = c.A1[(idx / n2) * 2 * N1 + N1 + idx % n2];
  for (int idx = tid; idx < n2 * 6; idx += kSetupThreads)
    c.H1[idx] = c.A1[(idx / 6) * 2 * N1 + N1 + n2 + idx % 6];
  for (int idx = tid; idx < nv * nv; idx += kSetupThreads)
    c.M2[idx] = c.A2[(idx / nv) * 2 * N2 + N2 + idx % nv];
  for (int idx = tid; idx < nv * 6; idx += kSetupThreads)
    c.H2[idx] = c.A2[(idx / 6) * 2 * N2 + N2 + nv + idx % 6];
  // Bernstein-coordinate inverses T Kinv T^T with T = blkdiag(R^-1, ..., I6).
  for (int idx = tid; idx < N1 * N1; idx += kSetupThreads) {
    const int I = idx / N1, J = idx % N1;
    double s = 0.0;
    for (int k = 0; k < N1; ++k) {
      const double tik = (I < n2) ? ((k < n2 && k / nv == I / nv) ? c.Rinv[(I % nv) * nv + k % nv] : 0.0)
                                  : (k == I ? 1.0 : 0.0);
      if (tik == 0.0) continue;
      for (int l = 0; l < N1; ++l) {
        const double tjl = (J < n2) ? ((l < n2 && l / nv == J / nv) ? c.Rinv[(J % nv) * nv + l % nv] : 0.0)
                                    : (l == J ? 1.0 : 0.0);
        if (tjl != 0.0) s += tik * c.A1[k * 2 * N1 + N1 + l] * tjl;
      }
    }
    c.K1b_inv[idx] = s;
  }
  for (int idx = tid; idx < N2 * N2; idx += kSetupThreads) {
    const int I = idx / N2, J = idx % N2;
    double s = 0.0;
    for (int k = 0; k < N2; ++k) {
      const double tik = (I < nv) ? (k < nv ? c.Rinv[I * nv + k] : 0.0) : (k == I ? 1.0 : 0.0);
      if (tik == 0.0) continue;
      for (int l = 0; l < N2; ++l) {
        const double tjl = (J < nv) ? (l < nv ? c.Rinv[J * nv + l] : 0.0) : (l == J ? 1.0 : 0.0);
        if (tjl != 0.0) s += tik * c.A2[k * 2 * N2 + N2 + l] * tjl;
      }
    }
    c.K2b_inv[idx] = s;
  }
  __syncthreads();

  // N = M1 Q with Q the smoothness block of the xi1 objective (the same
  // blocks as in A1); boundary rows of the position block in the z basis
  for (int idx = tid; idx < n2 * n2; idx += kSetupThreads) {
    const int I = idx / n2, J = idx % n2, bj = J / nv, j = J % nv;
    double v = 0.0;
    if (bj == 0 || q_cs)
      for (int k = 0; k < nv; ++k) v += c.M1[I * n2 + bj * nv + k] * GWW[k * nv + j];
    c.N[idx] = v;
  }
  for (int idx = tid; idx < 6 * nv; idx += kSetupThreads) {
    const int e = idx / nv, k = idx % nv, t = e < 3 ? 0 : q - 1;
    const double *X = (e % 3 == 0) ? c.U : ((e % 3 == 1) ? c.V : c.W);
    c.Abc[idx] = X[t * nv + k];
  }
  // U~ = U M2^T: the heading step's rows premultiplied by M2
  for (int idx = tid; idx < q * nv; idx += kSetupThreads) {
    const int t = idx / nv, k = idx % nv;
    double v = 0.0;
    for (int j = 0; j < nv; ++j) v += c.U[t * nv + j] * c.M2[k * nv + j];
    c.Ut[idx] = v;
  }
  __syncthreads();

  // 9. Typed copies for the iteration kernels.
  if (a.f64) {
    to_typed<double>(c.U, c.tU, q * nv); to_typed<double>(c.V, c.tV, q * nv);
    to_typed<double>(c.W, c.tW, q * nv); to_typed<double>(c.M1, c.tM1, n2 * n2);
    to_typed<double>(c.H1, c.tH1, n2 * 6); to_typed<double>(c.M2, c.tM2, nv * nv);
    to_typed<double>(c.H2, c.tH2, nv * 6); to_typed<double>(c.GF, c.tGF, n2 * n2);
    to_typed<double>(c.P, c.tP, q * nv); to_typed<double>(c.Pd, c.tPd, q * nv);
    to_typed<double>(c.Pdd, c.tPdd, q * nv); to_typed<double>(c.Ut, c.tUt, q * nv);
    to_typed<double>(c.N, c.tN, n2 * n2);
  } else {
    to_typed<float>(c.U, c.tU, q * nv); to_typed<float>(c.V, c.tV, q * nv);
    to_typed<float>(c.W, c.tW, q * nv); to_typed<float>(c.M1, c.tM1, n2 * n2);
    to_typed<float>(c.H1, c.tH1, n2 * 6); to_typed<float>(c.M2, c.tM2, nv * nv);
    to_typed<float>(c.H2, c.tH2, nv * 6); to_typed<float>(c.GF, c.tGF, n2 * n2);
    to_typed<float>(c.P, c.tP, q * nv); to_typed<float>(c.Pd, c.tPd, q * nv);
    to_typed<float>(c.Pdd, c.tPdd, q * nv); to_typed<float>(c.Ut, c.tUt, q * nv);
    to_typed<float>(c.N, c.tN, n2 * n2);
  }
}

}  // namespace

hipError_t launch_setup(const am_shape &s, const double *r_dev, const Consts &c, bool f64,
                        hipStream_t st) {
  SetupArgs a;
  a.q = s.q; a.nv = s.nv; a.m = s.m; a.n = s.n_obs; a.flags = int(s.flags); a.f64 = f64 ? 1 : 0;
  a.tf = s.tf; a.rho = s.rho; a.r = r_dev; a.c = c;
  hipLaunchKernelGGL(setup_kernel, dim3(1), dim3(kSetupThreads), 0, st, a);
  return hipGetLastError();
}

}  // namespace amk
