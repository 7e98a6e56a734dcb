// am_plain.hip -- the AM iteration computed the plain way: one kernel launch
// per sub-step per iteration, with the method's per-(circle, obstacle, t)
// state (alpha_ij, d_ij of xi3/xi4, Sec. III-C) and the trajectories held in
// device memory between launches.  It computes the same iteration as the
// fused kernel (same basis, same readings) and exists as the reference point
// for the one-launch form; its projection and target kernels are the
// bandwidth-bound elementwise part of the method.
//
// Per iteration:  xi1 -> evaluate -> xi2 -> project (alpha, d) ->
//                 targets/residual channels -> reduce + multipliers.
//
// The xi1 step is the update form of the fused kernel,
// z' = z - H1 (A z - b) + M1 (lambda - rho F^T (F xi - g)) - N z with N = M1 Q
// (eq. over_3 and the identity M1 (Q + rho F^T F) + H1 A = I), and the
// coefficients, multipliers and positions are kept in FP64 as there.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "am_device.h"
#include "am_internal.h"

namespace amk {
namespace {

constexpr int kThreads = 256;

inline int blocks_for(size_t work) { return int((work + kThreads - 1) / kThreads); }

// Workspace carve-up (elements of T; dw elements of T per FP64 value).
struct PlainWs {
  size_t wd, zd, zdn, lamd, xyd, z, zpsi, lampsi, traj8, psi3, psih, alpha, d, va4, chan, tot, total;
};

__host__ __device__ inline PlainWs plain_layout(int B, int q, int nv, int m, int n, int dw) {
  PlainWs w;
  size_t o = 0;
  auto take = [&](size_t cnt) {
    const size_t at = o;
    o += (cnt + 63) / 64 * 64;
    return at;
  };
  w.wd = take(size_t(B) * 4 * nv * dw);     // lambda - rho F^T (F xi - g)
  w.zd = take(size_t(B) * 4 * nv * dw);     // coefficients z (current) ...
  w.zdn = take(size_t(B) * 4 * nv * dw);    // ... and after the next update
  w.lamd = take(size_t(B) * 4 * nv * dw);   // multipliers
  w.xyd = take(size_t(B) * 2 * q * dw);     // absolute positions x, y
  w.z = take(size_t(B) * 4 * nv);           // T copy of z
  w.zpsi = take(size_t(B) * nv);
  w.lampsi = take(size_t(B) * nv);
  w.traj8 = take(size_t(B) * 8 * q);
  w.psi3 = take(size_t(B) * 3 * q);
  w.psih = take(size_t(B) * q);
  w.alpha = take(size_t(B) * m * n * q);
  w.d = take(size_t(B) * m * n * q);
  w.va4 = take(size_t(B) * 4 * q);
  w.chan = take(size_t(B) * 9 * q);
  w.tot = take(size_t(B) * 5 * nv);
  w.total = o;
  return w;
}

template <typename T>
struct Ptrs {
  double *wd, *zd, *zdn, *lamd, *xyd;
  T *z, *zpsi, *lampsi, *traj8, *psi3, *psih, *alpha, *d, *va4, *chan, *tot;
};

template <typename T>
Ptrs<T> ptrs_of(void *ws, const PlainWs &w) {
  T *b = static_cast<T *>(ws);
  auto dp = [&](size_t o) { return reinterpret_cast<double *>(b + o); };
  return Ptrs<T>{dp(w.wd), dp(w.zd), dp(w.zdn), dp(w.lamd), dp(w.xyd), b + w.z, b + w.zpsi, b + w.lampsi,
                 b + w.traj8, b + w.psi3, b + w.psih, b + w.alpha, b + w.d, b + w.va4, b + w.chan, b + w.tot};
}

template <typename T>
__device__ __forceinline__ T wsum(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// ---- entry: Bernstein coefficients -> z = R (c - offset), lambda -> R^-T lambda
template <typename T, int NV>
__global__ void k_enter(Desc D, Ptrs<T> w) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= D.B * 5 * NV) return;
  const int l = g / (5 * NV), k = g % (5 * NV), b = k / NV, kk = k % NV;
  const double *R = D.R, *Ri = D.Rinv;
  const T *src = static_cast<const T *>(b == 0 ? D.cx : b == 1 ? D.cc : b == 2 ? D.cy : b == 3 ? D.cs : D.cpsi);
  const double off = b == 0 ? D.offx : (b == 2 ? D.offy : 0.0);
  double z = 0.0, lz = 0.0;
  for (int j = kk; j < NV; ++j) z += R[kk * NV + j] * (double(src[size_t(l) * NV + j]) - off);
  if (b < 4) {
    const T *gl = static_cast<const T *>(D.lam) + size_t(l) * 4 * NV + b * NV;
    for (int j = 0; j <= kk; ++j) lz += Ri[j * NV + kk] * double(gl[j]);
    w.zd[size_t(l) * 4 * NV + b * NV + kk] = z;
    w.z[size_t(l) * 4 * NV + b * NV + kk] = T(z);
    w.lamd[size_t(l) * 4 * NV + b * NV + kk] = lz;
  } else {
    const T *gl = static_cast<const T *>(D.lampsi) + size_t(l) * NV;
    for (int j = 0; j <= kk; ++j) lz += Ri[j * NV + kk] * double(gl[j]);
    w.zpsi[size_t(l) * NV + kk] = T(z);
    w.lampsi[size_t(l) * NV + kk] = T(lz);
  }
}

// ---- xi1 for both axes, as an update of z (read from zd, written to zdn):
// z' = z - H1 (A z - b) + M1 w - N z, the boundary term on the first update
// only (afterwards A z = b holds)
template <typename T, int NV>
__global__ void k_xi1(Desc D, Ptrs<T> w, int first) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= D.B * 4 * NV) return;
  const int l = g / (4 * NV), k = g % (4 * NV), b = k / NV, kk = k % NV, axis = b >> 1;
  const int I = (b & 1) * NV + kk;
  const T *M1 = static_cast<const T *>(D.M1), *NQ = static_cast<const T *>(D.N);
  const double *r = w.wd + size_t(l) * 4 * NV + axis * 2 * NV;
  const double *z = w.zd + size_t(l) * 4 * NV + axis * 2 * NV;
  double acc = 0.0;
  for (int J = 0; J < 2 * NV; ++J)
    acc += double(M1[I * 2 * NV + J]) * r[J] - double(NQ[I * 2 * NV + J]) * z[J];
  if (first) {
    const double *bb = axis == 0 ? D.bx : D.by;
    const double off = axis == 0 ? D.offx : D.offy;
    for (int e = 0; e < 6; ++e) {
      double ae = 0.0;
      for (int j = 0; j < NV; ++j) ae += D.Abc[e * NV + j] * z[j];
      acc -= D.H1d[I * 6 + e] * (ae - ((e == 0 || e == 3) ? bb[e] - off : bb[e]));
    }
  }
  const double zn = z[I] + acc;
  w.zdn[size_t(l) * 4 * NV + k] = zn;
  w.z[size_t(l) * 4 * NV + k] = T(zn);
}

// ---- trajectories on the grid: absolute positions x, y in FP64 (xyd) and
// xdot, xddot, c, ydot, yddot, s in T (traj8 channels 1-3, 5-7)
template <typename T, int NV>
__global__ void k_eval(Desc D, Ptrs<T> w) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= D.B * D.q) return;
  const int l = g / D.q, t = g % D.q, q = D.q;
  const T *U = static_cast<const T *>(D.U) + t * NV, *V = static_cast<const T *>(D.V) + t * NV,
          *W = static_cast<const T *>(D.W) + t * NV;
  const double *Ud = D.Ud + t * NV;
  const T *z = w.z + size_t(l) * 4 * NV;
  const double *zd = w.zd + size_t(l) * 4 * NV;
  T v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  double x = 0.0, y = 0.0;
  for (int k = 0; k < NV; ++k) {
    x += Ud[k] * zd[k]; y += Ud[k] * zd[2 * NV + k];
    v[1] += V[k] * z[k]; v[2] += W[k] * z[k]; v[3] += U[k] * z[NV + k];
    v[5] += V[k] * z[2 * NV + k]; v[6] += W[k] * z[2 * NV + k]; v[7] += U[k] * z[3 * NV + k];
  }
  w.xyd[size_t(l) * 2 * q + t] = x + D.offx;
  w.xyd[size_t(l) * 2 * q + q + t] = y + D.offy;
  T *o = w.traj8 + size_t(l) * 8 * q + t;
  for (int c = 0; c < 8; ++c)
    if (c != 0 && c != 4) o[c * q] = v[c];
}

// ---- heading trajectory psi = U z_psi with cos, sin
template <typename T, int NV>
__global__ void k_eval_psi(Desc D, Ptrs<T> w) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= D.B * D.q) return;
  const int l = g / D.q, t = g % D.q, q = D.q;
  const T *U = static_cast<const T *>(D.U) + t * NV;
  T p = T(0);
  for (int k = 0; k < NV; ++k) p += U[k] * w.zpsi[size_t(l) * NV + k];
  T s, c;
  Num<T>::sincos_(p, &s, &c);
  T *o = w.psi3 + size_t(l) * 3 * q + t;
  o[0] = p;
  o[q] = c;
  o[2 * q] = s;
  w.psih[size_t(l) * q + t] = p;
}

// ---- xi2 (one wavefront per trajectory): psi_hat, heading QP, psi
template <typename T, int NV>
__global__ void k_xi2(Desc D, Ptrs<T> w) {
  const int lane = threadIdx.x & 63;
  const int l = blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64;
  if (l >= D.B) return;
  const int q = D.q;
  const bool unwrap = !(D.flags & AM_PSI_NO_UNWRAP);
  const T *U = static_cast<const T *>(D.U), *M2 = static_cast<const T *>(D.M2),
          *H2 = static_cast<const T *>(D.H2);
  const T *tr = w.traj8 + size_t(l) * 8 * q;
  T *p3 = w.psi3 + size_t(l) * 3 * q, *ph = w.psih + size_t(l) * q;
  T part[NV];
  for (int k = 0; k < NV; ++k) part[k] = T(0);
  for (int t = lane; t < q; t += 64) {
    const T c = tr[3 * q + t], s = tr[7 * q + t], p = p3[t], cp = p3[q + t], sp = p3[2 * q + t];
    const T h = unwrap ? p + atan2z(s * cp - c * sp, c * cp + s * sp) : atan2z(s, c);
    ph[t] = h;
    for (int k = 0; k < NV; ++k) part[k] += U[t * NV + k] * h;
  }
  T rhs[NV];
  for (int k = 0; k < NV; ++k) rhs[k] = w.lampsi[size_t(l) * NV + k] + T(D.rho) * wsum(part[k]);
  T zp[NV];
  for (int k = 0; k < NV; ++k) {
    T acc = T(0);
    for (int e = 0; e < 6; ++e) acc += H2[k * 6 + e] * T(D.bpsi[e]);
    for (int j = 0; j < NV; ++j) acc += M2[k * NV + j] * rhs[j];
    zp[k] = acc;
  }
  if (lane < NV) w.zpsi[size_t(l) * NV + lane] = zp[lane];
  for (int t = lane; t < q; t += 64) {
    T p = T(0);
    for (int k = 0; k < NV; ++k) p += U[t * NV + k] * zp[k];
    T s, c;
    Num<T>::sincos_(p, &s, &c);
    p3[t] = p;
    p3[q + t] = c;
    p3[2 * q + t] = s;
  }
}

// The projection and target kernels work on "items" of a trajectory l: the
// pairs (i, t) = (k / q, k % q) for k < m q, each looping over the n
// obstacles.  The trajectory's values at t are loaded once for n outputs,
// consecutive lanes touch consecutive t of a row of alpha or d, and a thread
// keeps several independent row accesses in flight.
constexpr int kItemThreads = 512;
inline int item_threads(int items) { return std::min(kItemThreads, (items + 63) / 64 * 64); }

// V consecutive values of a row as one aligned load or store
template <typename T, int V>
struct alignas(V * sizeof(T)) Vec {
  T v[V];
};
template <typename T, int V>
__device__ __forceinline__ Vec<T, V> ldv(const T *p) {
  return *reinterpret_cast<const Vec<T, V> *>(p);
}
// V consecutive FP64 values in loads of at most 16 bytes (the workspace is
// only 16-byte aligned)
template <int V>
__device__ __forceinline__ Vec<double, V> ldd(const double *p) {
  Vec<double, V> r;
  if constexpr (V == 1) {
    r.v[0] = p[0];
  } else {
#pragma unroll
    for (int e = 0; e < V; e += 2) {
      const Vec<double, 2> h = *reinterpret_cast<const Vec<double, 2> *>(p + e);
      r.v[e] = h.v[0];
      r.v[e + 1] = h.v[1];
    }
  }
  return r;
}
template <typename T, int V>
__device__ __forceinline__ void stv(T *p, const Vec<T, V> &x) {
  *reinterpret_cast<Vec<T, V> *>(p) = x;
}

// ---- xi3/xi4: alpha_ij, d_ij for every (l, i, j, t); items (i, t) with
// i = m are the velocity/acceleration pairs alpha_v, d_v, alpha_a, d_a.
// An item covers V consecutive time steps (V = 2 when q is even: aligned
// 8- or 16-byte loads and stores, and half the wavefronts, so that one round
// of them fills the GPU).  The items of all trajectories form one flat range
// over small blocks, so the last blocks of a launch are short.
// rows per chunk of loads (fewer for FP64 and for two steps per item)
template <typename T, int V> constexpr int kProjChunk = (sizeof(T) == 4 ? 8 : 4) / V;

template <typename T, int V, bool LITERAL>
__global__ __launch_bounds__(kThreads) void k_project(Desc D, Ptrs<T> w) {
  __shared__ T ell[4][AM_MAX_OBS];  // a_j, b_j (grown by the circle radius), 1/a_j^2, 1/b_j^2
  const int q = D.q, m = D.m, n = D.n;
  const int qv = q / V;   // items per row; V divides q
  const int per = (m + 1) * qv;
  const int g = int(blockIdx.x) * kThreads + int(threadIdx.x);
  const bool slack = D.flags & AM_XTILDE_SLACK;
  for (int j = threadIdx.x; j < n; j += blockDim.x) {
    const T a = static_cast<const T *>(D.oa)[j] + T(D.rc), b = static_cast<const T *>(D.ob)[j] + T(D.rc);
    ell[0][j] = a;
    ell[1][j] = b;
    ell[2][j] = T(1) / (a * a);
    ell[3][j] = T(1) / (b * b);
  }
  __syncthreads();
  if (g >= D.B * per) return;
  const int l = g / per, k = g - l * per;
  const int i = k / qv, t = (k - i * qv) * V;
  const T *tr = w.traj8 + size_t(l) * 8 * q, *p3 = w.psi3 + size_t(l) * 3 * q;
  if (i < m) {
    const T ri = T(D.r[i]);
    const double *xyl = w.xyd + size_t(l) * 2 * q;
    const Vec<double, V> xv = ldd<V>(xyl + t), yv = ldd<V>(xyl + q + t);
    const Vec<T, V> uxv = slack ? ldv<T, V>(tr + 3 * q + t) : ldv<T, V>(p3 + q + t);
    const Vec<T, V> uyv = slack ? ldv<T, V>(tr + 7 * q + t) : ldv<T, V>(p3 + 2 * q + t);
    T rx[V], ry[V];
#pragma unroll
    for (int e = 0; e < V; ++e) {
      rx[e] = ri * uxv.v[e];
      ry[e] = ri * uyv.v[e];
    }
    const size_t row0 = (size_t(l) * m + i) * n;
    T *oal = w.alpha + row0 * q + t, *od = w.d + row0 * q + t;
    const T *oxt = static_cast<const T *>(D.ox) + t, *oyt = static_cast<const T *>(D.oy) + t;
    // obstacle positions are loaded a chunk at a time, so one memory
    // latency covers a chunk of outputs
    constexpr int CH = kProjChunk<T, V>;
    for (int j0 = 0; j0 < n; j0 += CH) {
      Vec<T, V> gx[CH], gy[CH];
#pragma unroll
      for (int u = 0; u < CH; ++u) {
        const int j = j0 + u < n ? j0 + u : n - 1;
        gx[u] = ldv<T, V>(oxt + size_t(j) * q);
        gy[u] = ldv<T, V>(oyt + size_t(j) * q);
      }
#pragma unroll
      for (int u = 0; u < CH; ++u) {
        const int j = j0 + u;
        if (j >= n) break;
        const T a = ell[0][j], b = ell[1][j], ia2 = ell[2][j], ib2 = ell[3][j];
        Vec<T, V> al, dd;
#pragma unroll
        for (int e = 0; e < V; ++e) {
          // offset of the robot centre from the obstacle centre in FP64,
          // rounded once
          const T xt = T(xv.v[e] - double(gx[u].v[e])) + rx[e], yt = T(yv.v[e] - double(gy[u].v[e])) + ry[e];
          if constexpr (!LITERAL) {
            // elliptic angle: the point (a d cos al, b d sin al) is (xt, yt)
            // itself, so d = sqrt(xt^2/a^2 + yt^2/b^2) (eq. compute_zeta_3)
            al.v[e] = atan2z(a * yt, b * xt);
            dd.v[e] = fmax(T(1), Num<T>::sqrt_fast(xt * xt * ia2 + yt * yt * ib2));
          } else {
            al.v[e] = atan2z(yt, xt);
            T sa, ca;
            Num<T>::sincos_(al.v[e], &sa, &ca);
            dd.v[e] = fmax(T(1), (a * xt * ca + b * yt * sa) / (a * a * ca * ca + b * b * sa * sa));
          }
        }
        stv<T, V>(oal + size_t(j) * q, al);
        stv<T, V>(od + size_t(j) * q, dd);
      }
    }
  } else {
    T *o = w.va4 + size_t(l) * 4 * q;
    const Vec<T, V> xdv = ldv<T, V>(tr + q + t), ydv = ldv<T, V>(tr + 5 * q + t);
    const Vec<T, V> xddv = ldv<T, V>(tr + 2 * q + t), yddv = ldv<T, V>(tr + 6 * q + t);
    Vec<T, V> av, dv, aa, da;
    const T ivmax = T(1) / T(D.vmax), iamax = T(1) / T(D.amax);
#pragma unroll
    for (int e = 0; e < V; ++e) {
      const T xd = xdv.v[e], yd = ydv.v[e], xdd = xddv.v[e], ydd = yddv.v[e];
      // with alpha_v = atan2(ydot, xdot), xdot cos alpha_v + ydot sin alpha_v
      // is the speed itself, so d_v = min(1, |v| / v_max) (eq. compute_dv
      // clipped to [0, 1]); likewise d_a
      av.v[e] = atan2z(yd, xd);
      aa.v[e] = atan2z(ydd, xdd);
      dv.v[e] = fmin(T(1), Num<T>::sqrt_(xd * xd + yd * yd) * ivmax);
      da.v[e] = fmin(T(1), Num<T>::sqrt_(xdd * xdd + ydd * ydd) * iamax);
    }
    stv<T, V>(o + t, av);
    stv<T, V>(o + q + t, dv);
    stv<T, V>(o + 2 * q + t, aa);
    stv<T, V>(o + 3 * q + t, da);
  }
}

// Projection launch: two time steps per item when q is even.
template <typename T>
void project(const Desc &D, const Ptrs<T> &w, hipStream_t st) {
  const size_t rows = size_t(D.B) * (D.m + 1);
  const bool lit = D.flags & AM_ALPHA_LITERAL;
  if (D.q % 2 == 0)
    hipLaunchKernelGGL((lit ? k_project<T, 2, true> : k_project<T, 2, false>), dim3(blocks_for(rows * (D.q / 2))),
                       dim3(kThreads), 0, st, D, w);
  else
    hipLaunchKernelGGL((lit ? k_project<T, 1, true> : k_project<T, 1, false>), dim3(blocks_for(rows * D.q)),
                       dim3(kThreads), 0, st, D, w);
}

// ---- residual channels of F xi - g per (l, t), reading alpha and d.  Item
// (i, t) sums circle i's deviations over the obstacles; the m partial sums
// of a t meet in LDS and one thread per t forms the channels.
template <typename T> constexpr int kTgtChunk = sizeof(T) == 4 ? 8 : 4;  // d_ij loads issued together


template <typename T, int V>
__global__ __launch_bounds__(kItemThreads) void k_targets(Desc D, Ptrs<T> w) {
  __shared__ T part[2][AM_MAX_CIRCLES * AM_MAX_Q];
  __shared__ T ell[2][AM_MAX_OBS];
  const int l = blockIdx.x;
  const int q = D.q, m = D.m, n = D.n;
  const bool slack = D.flags & AM_XTILDE_SLACK, literal = D.flags & AM_ALPHA_LITERAL;
  for (int j = threadIdx.x; j < n; j += blockDim.x) {
    ell[0][j] = static_cast<const T *>(D.oa)[j] + T(D.rc);
    ell[1][j] = static_cast<const T *>(D.ob)[j] + T(D.rc);
  }
  __syncthreads();
  const T *tr = w.traj8 + size_t(l) * 8 * q, *p3 = w.psi3 + size_t(l) * 3 * q;
  const T *va = w.va4 + size_t(l) * 4 * q;
  const T *ox = static_cast<const T *>(D.ox), *oy = static_cast<const T *>(D.oy);
  // V consecutive time steps per item (V = 2 when q is even: every row
  // offset is then even, so the pairs are aligned vector loads)
  const int qv = q / V;
  const double *xyl = w.xyd + size_t(l) * 2 * q;
  for (int k = threadIdx.x; k < m * qv; k += blockDim.x) {
    const int i = k / qv, t = (k - i * qv) * V;
    const Vec<T, V> cv = ldv<T, V>(tr + 3 * q + t), sv = ldv<T, V>(tr + 7 * q + t);
    const Vec<double, V> xv = ldd<V>(xyl + t), yv = ldd<V>(xyl + q + t);
    const Vec<T, V> uxv = slack ? cv : ldv<T, V>(p3 + q + t), uyv = slack ? sv : ldv<T, V>(p3 + 2 * q + t);
    const T ri = T(D.r[i]);
    const size_t base = (size_t(l) * m + i) * n * q + t;
    const T *al = w.alpha + base, *dd = w.d + base;
    // circle i: sum over obstacles of the deviation of the target from the
    // circle centre.  Under the elliptic angle a point with d > 1 lies
    // outside the ellipse and is its own target (eqs. zeta_2,
    // compute_zeta_3), so the deviation is exactly zero; the literal angle
    // has no such fixed points.
    T sx[V], sy[V];
#pragma unroll
    for (int e = 0; e < V; ++e) sx[e] = sy[e] = T(0);
    const T *oxt = ox + t, *oyt = oy + t;
    // a chunk of d_ij in one memory latency; colliding rows (d_ij <= 1, a
    // few percent) then load their angle and obstacle position
    for (int j0 = 0; j0 < n; j0 += kTgtChunk<T>) {
      Vec<T, V> dv[kTgtChunk<T>];
#pragma unroll
      for (int u = 0; u < kTgtChunk<T>; ++u) {
        if (j0 + u < n) {
          dv[u] = ldv<T, V>(dd + size_t(j0 + u) * q);
        } else {
#pragma unroll
          for (int e = 0; e < V; ++e) dv[u].v[e] = T(2);
        }
      }
#pragma unroll
      for (int u = 0; u < kTgtChunk<T>; ++u) {
        const int j = j0 + u;
        bool hit = literal;
#pragma unroll
        for (int e = 0; e < V; ++e) hit |= dv[u].v[e] <= T(1);
        if (j < n && hit) {
          const Vec<T, V> av = ldv<T, V>(al + size_t(j) * q), gx = ldv<T, V>(oxt + j * q),
                          gy = ldv<T, V>(oyt + j * q);
#pragma unroll
          for (int e = 0; e < V; ++e) {
            if (literal || dv[u].v[e] <= T(1)) {
              const T xt = T(xv.v[e] - double(gx.v[e])) + ri * uxv.v[e];
              const T yt = T(yv.v[e] - double(gy.v[e])) + ri * uyv.v[e];
              T sa, ca;
              Num<T>::sincos_(av.v[e], &sa, &ca);
              sx[e] += ell[0][j] * dv[u].v[e] * ca - xt;
              sy[e] += ell[1][j] * dv[u].v[e] * sa - yt;
            }
          }
        }
      }
    }
#pragma unroll
    for (int e = 0; e < V; ++e) {
      part[0][i * q + t + e] = sx[e];
      part[1][i * q + t + e] = sy[e];
    }
  }
  // inputs of the channels at t = threadIdx.x, loaded before the barrier so
  // that their latency overlaps the wait (q <= blockDim.x whenever m q fits
  // one block; otherwise the channel loop below loads them itself)
  T pre[14];
  const int t0 = threadIdx.x;
  if (t0 < q) {
    pre[0] = tr[q + t0]; pre[1] = tr[2 * q + t0]; pre[2] = tr[3 * q + t0]; pre[3] = tr[5 * q + t0];
    pre[4] = tr[6 * q + t0]; pre[5] = tr[7 * q + t0]; pre[6] = p3[t0]; pre[7] = p3[q + t0];
    pre[8] = p3[2 * q + t0]; pre[9] = w.psih[size_t(l) * q + t0];
    pre[10] = va[t0]; pre[11] = va[2 * q + t0]; pre[12] = va[q + t0]; pre[13] = va[3 * q + t0];
  }
  __syncthreads();
  for (int t = threadIdx.x; t < q; t += blockDim.x) {
    if (t != t0) {
      pre[0] = tr[q + t]; pre[1] = tr[2 * q + t]; pre[2] = tr[3 * q + t]; pre[3] = tr[5 * q + t];
      pre[4] = tr[6 * q + t]; pre[5] = tr[7 * q + t]; pre[6] = p3[t]; pre[7] = p3[q + t];
      pre[8] = p3[2 * q + t]; pre[9] = w.psih[size_t(l) * q + t];
      pre[10] = va[t]; pre[11] = va[2 * q + t]; pre[12] = va[q + t]; pre[13] = va[3 * q + t];
    }
    const T c = pre[2], s = pre[5];
    const T cp = pre[7], sp = pre[8];
    T Dx = 0, Dy = 0, DRx = 0, DRy = 0, s1 = 0, s2 = 0;
    for (int i = 0; i < m; ++i) {
      const T ri = T(D.r[i]), px = part[0][i * q + t], py = part[1][i * q + t];
      Dx += px; Dy += py; DRx += ri * px; DRy += ri * py;
      s1 += ri; s2 += ri * ri;
    }
    s1 *= T(n);
    s2 *= T(n);
    T sv, cv, sa, ca;
    Num<T>::sincos_(pre[10], &sv, &cv);
    Num<T>::sincos_(pre[11], &sa, &ca);
    const T vm = T(D.vmax), am = T(D.amax);
    const T dc = c - cp, ds = s - sp;
    const T k1 = slack ? T(0) : s1, k2 = (slack ? T(0) : s2) + T(1);
    T *ch = w.chan + size_t(l) * 9 * q + t;
    // inside the disc (d_v < 1) the velocity is its own target
    const bool vin = pre[12] < T(1), ain = pre[13] < T(1);
    ch[0] = vin ? T(0) : pre[0] - vm * pre[12] * cv;  // xdot - g_v
    ch[q] = ain ? T(0) : pre[1] - am * pre[13] * ca;  // xddot - g_a
    ch[2 * q] = k1 * dc - Dx;                         // sum_ij (x + r_i c - g_ob)
    ch[3 * q] = k2 * dc - DRx;                        // sum_ij r_i (...) + (c - cos psi)
    ch[4 * q] = vin ? T(0) : pre[3] - vm * pre[12] * sv;
    ch[5 * q] = ain ? T(0) : pre[4] - am * pre[13] * sa;
    ch[6 * q] = k1 * ds - Dy;
    ch[7 * q] = k2 * ds - DRy;
    const T psi_sign = (D.flags & AM_LAMPSI_LITERAL) ? T(-1) : T(1);
    ch[8 * q] = psi_sign * (pre[6] - pre[9]);
  }
}

// ---- F^T (F xi - g), multipliers and the next right-hand side (one wave
// per trajectory).  mode 0: initial right-hand side only.
template <typename T, int NV>
__global__ void k_contract(Desc D, Ptrs<T> w, int update) {
  const int lane = threadIdx.x & 63;
  const int l = blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64;
  if (l >= D.B) return;
  const int q = D.q;
  const T *U = static_cast<const T *>(D.U), *V = static_cast<const T *>(D.V), *W = static_cast<const T *>(D.W);
  const T *ch = w.chan + size_t(l) * 9 * q;
  T part[5 * NV];
  for (int k = 0; k < 5 * NV; ++k) part[k] = T(0);
  for (int t = lane; t < q; t += 64) {
    for (int k = 0; k < NV; ++k) {
      const T u = U[t * NV + k], v = V[t * NV + k], wv = W[t * NV + k];
      part[k] += v * ch[t] + wv * ch[q + t] + u * ch[2 * q + t];
      part[NV + k] += u * ch[3 * q + t];
      part[2 * NV + k] += v * ch[4 * q + t] + wv * ch[5 * q + t] + u * ch[6 * q + t];
      part[3 * NV + k] += u * ch[7 * q + t];
      part[4 * NV + k] += u * ch[8 * q + t];
    }
  }
  T tot[5 * NV];
  for (int k = 0; k < 5 * NV; ++k) tot[k] = wsum(part[k]);
  double *lam = w.lamd + size_t(l) * 4 * NV;
  if (lane < 4 * NV) {
    const int k = lane;
    T trv = T(0);
    for (int c = 0; c < 4 * NV; ++c)
      if (c == k) trv = tot[c];
    double lv = lam[k];
    if (update) lv -= D.rho * double(trv);
    lam[k] = lv;
    w.wd[size_t(l) * 4 * NV + k] = lv - D.rho * double(trv);
  } else if (update && lane < 5 * NV) {
    const int kk = lane - 4 * NV;
    T tp = T(0);
    for (int c = 0; c < NV; ++c)
      if (c == kk) tp = tot[4 * NV + c];
    w.lampsi[size_t(l) * NV + kk] -= T(D.rho_psi) * tp;
  }
}

// ---- the same contraction on the matrix cores: BF16 operands split into
// high and low parts (x = hi + lo, both BF16), three products per step
// (hi*hi + hi*lo + lo*hi) accumulated in FP32.  One wavefront computes a
// tile of 16 trajectories x 16 outputs of one group with
// v_mfma_f32_16x16x16_bf16; lane L supplies A[traj L%16][k 4(L/16)..+3],
// B[k 4(L/16)..+3][out L%16] and receives D[traj 4(L/16)..+3][out L%16].
typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ short bf16_bits(float x) {
  // round to nearest even (inputs are finite)
  uint32_t u = __builtin_bit_cast(uint32_t, x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return short(u >> 16);
}
__device__ __forceinline__ float bf16_value(short h) {
  return __builtin_bit_cast(float, uint32_t(uint16_t(h)) << 16);
}
__device__ __forceinline__ void split_bf16(const float (&v)[4], bf16x4 &hi, bf16x4 &lo) {
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const short h = bf16_bits(v[i]);
    hi[i] = h;
    lo[i] = bf16_bits(v[i] - bf16_value(h));
  }
}

// Block (x, g) holds four tiles of 16 trajectories and output group g
// (0: x position rows [V W U], 1: x slack rows U, 2, 3: the same for y, 4:
// heading rows U); the group's basis fragments, split once per block, are
// shared by the four wavefronts through LDS.
constexpr int kMfmaMaxK = (AM_MAX_Q + 15) / 16;   // K steps of 16 time steps

template <int NV>
__global__ __launch_bounds__(256) void k_contract_mfma(Desc D, Ptrs<float> w) {
  static_assert(NV <= 16, "one 16-wide output tile per group");
  __shared__ bf16x4 frag[3][kMfmaMaxK][64][2];   // [basis of the group][k step][lane][hi, lo]
  const int lane = threadIdx.x & 63, g = blockIdx.y;
  const int q = D.q, B = D.B;
  const int r = lane & 15, kq = lane >> 4;     // A row / B column; k quad
  const int ksteps = (q + 15) / 16;
  const float *U = static_cast<const float *>(D.U), *V = static_cast<const float *>(D.V),
              *W = static_cast<const float *>(D.W);
  // (channel, basis) pairs of the group, basis 0 = U, 1 = V, 2 = W
  const int g_ch[5][3] = {{0, 1, 2}, {3, -1, -1}, {4, 5, 6}, {7, -1, -1}, {8, -1, -1}};
  const int g_bs[5][3] = {{1, 2, 0}, {0, -1, -1}, {1, 2, 0}, {0, -1, -1}, {0, -1, -1}};
  const int ne = g_ch[g][1] < 0 ? 1 : 3;
  // B fragments: lane L holds B[k 4(L/16)..+3][out L%16] of every k step;
  // a thread's entries (at most kFragPer) are all loaded before any is
  // split, so one memory latency covers them
  constexpr int kFragPer = (3 * kMfmaMaxK * 64 + 255) / 256;
  {
    const int total = ne * ksteps * 64;
    float bv[kFragPer][4];
#pragma unroll
    for (int u = 0; u < kFragPer; ++u) {
      const int i = threadIdx.x + u * 256;
      const int e = i / (ksteps * 64), rem = i % (ksteps * 64), ks = rem / 64, ln = rem % 64;
      const float *basis = g_bs[g][e < ne ? e : 0] == 0 ? U : (g_bs[g][e < ne ? e : 0] == 1 ? V : W);
      const int rr = ln & 15, t0 = ks * 16 + (ln >> 4) * 4;
#pragma unroll
      for (int j = 0; j < 4; ++j)
        bv[u][j] = (i < total && rr < NV && t0 + j < q) ? basis[(t0 + j) * NV + rr] : 0.f;
    }
#pragma unroll
    for (int u = 0; u < kFragPer; ++u) {
      const int i = threadIdx.x + u * 256;
      if (i < total) {
        const int e = i / (ksteps * 64), rem = i % (ksteps * 64), ks = rem / 64, ln = rem % 64;
        split_bf16(bv[u], frag[e][ks][ln][0], frag[e][ks][ln][1]);
      }
    }
  }
  __syncthreads();
  const int l0 = (blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64) * 16;
  if (l0 >= B) return;
  const int la = l0 + r;                        // trajectory of this lane's A row
  const bool vec = (q % 4) == 0;                // rows of 4 time steps are 16-byte aligned
  f32x4 acc = {0.f, 0.f, 0.f, 0.f};
  for (int e = 0; e < ne; ++e) {
    const float *ch = w.chan + size_t(la < B ? la : 0) * 9 * q + size_t(g_ch[g][e]) * q;
    for (int ks = 0; ks < ksteps; ++ks) {
      const int t0 = ks * 16 + kq * 4;
      float av[4];
      if (vec && t0 < q) {
        const float4 v4 = *reinterpret_cast<const float4 *>(ch + t0);
        av[0] = v4.x; av[1] = v4.y; av[2] = v4.z; av[3] = v4.w;
      } else {
#pragma unroll
        for (int i = 0; i < 4; ++i) av[i] = t0 + i < q ? ch[t0 + i] : 0.f;
      }
      if (la >= B) av[0] = av[1] = av[2] = av[3] = 0.f;
      bf16x4 ah, al;
      split_bf16(av, ah, al);
      const bf16x4 bh = frag[e][ks][lane][0], bl = frag[e][ks][lane][1];
      acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bh, acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bl, acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(al, bh, acc, 0, 0, 0);
    }
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int lt = l0 + kq * 4 + i;
    if (lt < B && r < NV) w.tot[size_t(lt) * 5 * NV + g * NV + r] = acc[i];
  }
}

// ---- multipliers and the next xi1 right-hand side from the contraction totals
template <typename T, int NV>
__global__ void k_update(Desc D, Ptrs<T> w, int update) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= D.B * 5 * NV) return;
  const int l = g / (5 * NV), k = g % (5 * NV);
  const T trv = w.tot[size_t(l) * 5 * NV + k];
  if (k < 4 * NV) {
    double lv = w.lamd[size_t(l) * 4 * NV + k];
    if (update) lv -= D.rho * double(trv);
    w.lamd[size_t(l) * 4 * NV + k] = lv;
    w.wd[size_t(l) * 4 * NV + k] = lv - D.rho * double(trv);
  } else if (update) {
    w.lampsi[size_t(l) * NV + (k - 4 * NV)] -= T(D.rho_psi) * trv;
  }
}

// ---- exit: back to Bernstein coordinates, optional outputs
template <typename T, int NV>
__global__ void k_exit(Desc D, Ptrs<T> w) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g < D.B * 5 * NV) {
    const int l = g / (5 * NV), k = g % (5 * NV), b = k / NV, kk = k % NV;
    const double *R = D.R, *Ri = D.Rinv;
    double c = 0.0, lc = 0.0;
    if (b < 4) {
      const double *zs = w.zd + size_t(l) * 4 * NV + b * NV, *ls = w.lamd + size_t(l) * 4 * NV + b * NV;
      for (int j = kk; j < NV; ++j) c += Ri[kk * NV + j] * zs[j];
      for (int j = 0; j <= kk; ++j) lc += R[j * NV + kk] * ls[j];
    } else {
      const T *zs = w.zpsi + size_t(l) * NV, *ls = w.lampsi + size_t(l) * NV;
      for (int j = kk; j < NV; ++j) c += Ri[kk * NV + j] * double(zs[j]);
      for (int j = 0; j <= kk; ++j) lc += R[j * NV + kk] * double(ls[j]);
    }
    const double off = b == 0 ? D.offx : (b == 2 ? D.offy : 0.0);
    T *dst = static_cast<T *>(b == 0 ? D.cx : b == 1 ? D.cc : b == 2 ? D.cy : b == 3 ? D.cs : D.cpsi);
    dst[size_t(l) * NV + kk] = T(c + off);
    if (b < 4) static_cast<T *>(D.lam)[size_t(l) * 4 * NV + b * NV + kk] = T(lc);
    else static_cast<T *>(D.lampsi)[size_t(l) * NV + kk] = T(lc);
  }
  const int q = D.q;
  if (g < D.B * q) {
    const int l = g / q, t = g % q;
    const T *p3 = w.psi3 + size_t(l) * 3 * q;
    if (D.traj) {
      T *o = static_cast<T *>(D.traj) + size_t(l) * 3 * q;
      o[t] = T(w.xyd[size_t(l) * 2 * q + t]);
      o[q + t] = T(w.xyd[size_t(l) * 2 * q + q + t]);
      o[2 * q + t] = p3[t];
    }
    if (D.va) {
      T *o = static_cast<T *>(D.va) + size_t(l) * 4 * q;
      const T *v = w.va4 + size_t(l) * 4 * q;
      for (int c = 0; c < 4; ++c) o[c * q + t] = v[c * q + t];
    }
    const size_t mnq = size_t(D.m) * D.n * q;
    for (int ij = 0; ij < D.m * D.n; ++ij) {
      const size_t e = size_t(l) * mnq + size_t(ij) * q + t;
      if (D.alpha) static_cast<T *>(D.alpha)[e] = w.alpha[e];
      if (D.d) static_cast<T *>(D.d)[e] = w.d[e];
    }
  }
}

template <typename T, int NV>
void contract(const Desc &D, const Ptrs<T> &w, hipStream_t st, int update) {
  const int wave_blocks = (D.B + 3) / 4;
  if constexpr (sizeof(T) == 4) {
    if (D.flags & AM_PLAIN_BF16X3) {
      const int tiles = (D.B + 15) / 16;
      hipLaunchKernelGGL((k_contract_mfma<NV>), dim3((tiles + 3) / 4, 5), dim3(256), 0, st, D, w);
      hipLaunchKernelGGL((k_update<T, NV>), dim3(blocks_for(size_t(D.B) * 5 * NV)), dim3(kThreads), 0, st, D, w,
                         update);
      return;
    }
  }
  hipLaunchKernelGGL((k_contract<T, NV>), dim3(wave_blocks), dim3(kThreads), 0, st, D, w, update);
}

// The update reads zd and writes zdn; the two buffers then swap.
template <typename T, int NV>
void xi1(const Desc &D, Ptrs<T> &w, hipStream_t st, int first) {
  hipLaunchKernelGGL((k_xi1<T, NV>), dim3(blocks_for(size_t(D.B) * 4 * NV)), dim3(kThreads), 0, st, D, w, first);
  double *t = w.zd;
  w.zd = w.zdn;
  w.zdn = t;
}

// Four time steps per item once the batch gives every SIMD about four
// wavefronts of them (fewer, wider loads); two below that, where more
// wavefronts hide more latency.
constexpr size_t kWideItems = size_t(256) * 4 * 64 * 4;

template <typename T>
void targets(const Desc &D, const Ptrs<T> &w, hipStream_t st) {
  if (D.q % 4 == 0 && sizeof(T) == 4 && size_t(D.B) * D.m * D.q / 4 >= kWideItems)
    hipLaunchKernelGGL((k_targets<T, 4>), dim3(D.B), dim3(item_threads(D.m * D.q / 4)), 0, st, D, w);
  else if (D.q % 2 == 0)
    hipLaunchKernelGGL((k_targets<T, 2>), dim3(D.B), dim3(item_threads(D.m * D.q / 2)), 0, st, D, w);
  else
    hipLaunchKernelGGL((k_targets<T, 1>), dim3(D.B), dim3(item_threads(D.m * D.q)), 0, st, D, w);
}

template <typename T, int NV>
hipError_t run(const Desc &D, void *ws, hipStream_t st) {
  const PlainWs L = plain_layout(D.B, D.q, NV, D.m, D.n, int(sizeof(double) / sizeof(T)));
  Ptrs<T> w = ptrs_of<T>(ws, L);
  const int B = D.B, q = D.q;
  const int wave_blocks = (B + 3) / 4;
  hipLaunchKernelGGL((k_enter<T, NV>), dim3(blocks_for(size_t(B) * 5 * NV)), dim3(kThreads), 0, st, D, w);
  // step 1: initial xi3, xi4 from the given trajectories
  hipLaunchKernelGGL((k_eval<T, NV>), dim3(blocks_for(size_t(B) * q)), dim3(kThreads), 0, st, D, w);
  hipLaunchKernelGGL((k_eval_psi<T, NV>), dim3(blocks_for(size_t(B) * q)), dim3(kThreads), 0, st, D, w);
  project<T>(D, w, st);
  targets<T>(D, w, st);
  contract<T, NV>(D, w, st, 0);
  for (int it = 0; it < D.K; ++it) {
    xi1<T, NV>(D, w, st, it == 0);
    hipLaunchKernelGGL((k_eval<T, NV>), dim3(blocks_for(size_t(B) * q)), dim3(kThreads), 0, st, D, w);
    hipLaunchKernelGGL((k_xi2<T, NV>), dim3(wave_blocks), dim3(kThreads), 0, st, D, w);
    project<T>(D, w, st);
    targets<T>(D, w, st);
    contract<T, NV>(D, w, st, 1);
  }
  const size_t exit_work = std::max(size_t(B) * 5 * NV, size_t(B) * q);
  hipLaunchKernelGGL((k_exit<T, NV>), dim3(blocks_for(exit_work)), dim3(kThreads), 0, st, D, w);
  return hipGetLastError();
}

}  // namespace

size_t plain_workspace_bytes(int B, int q, int nv, int m, int n, bool f64) {
  return plain_layout(B, q, nv, m, n, f64 ? 1 : 2).total * (f64 ? 8 : 4);
}

hipError_t launch_plain(const Desc &d, void *ws, size_t, bool f64, int nv, hipStream_t st) {
  if (d.B <= 0) return hipSuccess;
  if (f64) {
    if (nv == 11) return run<double, 11>(d, ws, st);
    if (nv == 8) return run<double, 8>(d, ws, st);
  } else {
    if (nv == 11) return run<float, 11>(d, ws, st);
    if (nv == 8) return run<float, 8>(d, ws, st);
  }
  return hipErrorInvalidValue;
}

}  // namespace amk
