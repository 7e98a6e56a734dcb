// am_residuals.hip -- per-trajectory residual statistics of the current state
// (two wavefronts per trajectory), plus the small kernel that fills the
// problem table of multi-problem launches.
//
// The angles and distances are recomputed by the closed forms of eqs.
// (zeta_2, alpha_v, alpha_a, compute_zeta_3, compute_dv, compute_da) from the
// current trajectories, which is exactly what the last xi3/xi4 step produced;
// under the elliptic angle and for the velocity/acceleration discs the
// residual follows from those forms without evaluating the angle.
#include <hip/hip_runtime.h>

#include "am_device.h"
#include "am_internal.h"

namespace amk {
namespace {

template <typename T>
__device__ __forceinline__ T wave_max(T v) {   // v >= 0
  return wave_all(v, T(0), [](T a, T b) { return fmax(a, b); });
}
template <typename T>
__device__ __forceinline__ T wave_min(T v) {
  return wave_all(v, T(INFINITY), [](T a, T b) { return fmin(a, b); });
}
template <typename T>
__device__ __forceinline__ T wave_add(T v) {
  return wave_all(v, T(0), [](T a, T b) { return a + b; });
}

struct ResArgs {
  Desc d;
  const void *P, *Pd, *Pdd;
  void *out;
};

template <typename T>
constexpr T kMinNormal = sizeof(T) == 4 ? T(1.17549435082228750797e-38) : T(2.22507385850720138309e-308);

constexpr int kTrajPerResBlock = kWavesPerBlock / 2;
constexpr int kResChunk = 4;    // obstacle positions loaded together
constexpr int kResStats = 10;   // per-wave statistics combined across the pair

template <typename T, int NV>
__global__ __launch_bounds__(kWave *kWavesPerBlock) void residual_kernel(ResArgs A) {
  // per-obstacle constants of the inflated ellipses: a, b, ab, 1/a^2, 1/b^2
  __shared__ T ell[5][AM_MAX_OBS];
  const Desc &D = A.d;
  const int q = D.q, m = D.m, n = D.n;
  const T rc = T(D.rc);
  for (int j = threadIdx.x; j < n; j += blockDim.x) {
    const T a = static_cast<const T *>(D.oa)[j] + rc, b = static_cast<const T *>(D.ob)[j] + rc;
    ell[0][j] = a;
    ell[1][j] = b;
    ell[2][j] = a * b;
    ell[3][j] = T(1) / (a * a);
    ell[4][j] = T(1) / (b * b);
  }
  __syncthreads();
  // two wavefronts per trajectory, taking alternate time steps
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  const int half = wave & 1, slot = wave >> 1;
  const int l = blockIdx.x * kTrajPerResBlock + slot;
  const bool live = l < D.B;
  const bool slack = D.flags & AM_XTILDE_SLACK, literal = D.flags & AM_ALPHA_LITERAL;
  const T *P = static_cast<const T *>(A.P), *Pd = static_cast<const T *>(A.Pd),
          *Pdd = static_cast<const T *>(A.Pdd);
  const int lc = live ? l : 0;
  const T *cx = static_cast<const T *>(D.cx) + size_t(lc) * NV, *cc = static_cast<const T *>(D.cc) + size_t(lc) * NV;
  const T *cy = static_cast<const T *>(D.cy) + size_t(lc) * NV, *cs = static_cast<const T *>(D.cs) + size_t(lc) * NV;
  const T *cp = static_cast<const T *>(D.cpsi) + size_t(lc) * NV;
  const T *gox = static_cast<const T *>(D.ox), *goy = static_cast<const T *>(D.oy);
  const T vmax = T(D.vmax), amax = T(D.amax);
  const T pi = T(3.14159265358979323846);

  T rr[AM_MAX_CIRCLES];
#pragma unroll
  for (int i = 0; i < AM_MAX_CIRCLES; ++i) rr[i] = i < m ? T(D.r[i]) : T(0);

  // squared maxima and minima are tracked, one square root at the end
  T fc2max = 0, fcsq = 0, lvl2 = T(INFINITY), slk = 0, head = 0, bc = 0, cost = 0;
  T v2max = 0, a2max = 0;
  for (int t = half + 2 * lane; live && t < q; t += 2 * kWave) {
    T x = 0, xd = 0, xdd = 0, y = 0, yd = 0, ydd = 0, c = 0, s = 0, psi = 0, psidd = 0;
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      const T p = P[t * NV + k], pd = Pd[t * NV + k], pdd = Pdd[t * NV + k];
      x += p * cx[k]; xd += pd * cx[k]; xdd += pdd * cx[k];
      y += p * cy[k]; yd += pd * cy[k]; ydd += pdd * cy[k];
      c += p * cc[k]; s += p * cs[k]; psi += p * cp[k]; psidd += pdd * cp[k];
    }
    T spsi, cpsi;
    Num<T>::sincos_(psi, &spsi, &cpsi);
    // obstacles outermost, their positions at t loaded a chunk at a time
    for (int j0 = 0; j0 < n; j0 += kResChunk) {
      T gx[kResChunk], gy[kResChunk];
#pragma unroll
      for (int u = 0; u < kResChunk; ++u) {
        const int j = j0 + u < n ? j0 + u : n - 1;
        gx[u] = gox[j * q + t];
        gy[u] = goy[j * q + t];
      }
#pragma unroll
      for (int u = 0; u < kResChunk; ++u) {
        const int j = j0 + u;
        if (j >= n) break;
        const T a = ell[0][j], b = ell[1][j], ab = ell[2][j], a2 = a * a, b2 = b * b;
        const T ia2 = ell[3][j], ib2 = ell[4][j];
#pragma unroll
        for (int i = 0; i < AM_MAX_CIRCLES; ++i) {
          if (i >= m) break;
          const T ri = rr[i];
          const T px = x + ri * cpsi - gx[u], py = y + ri * spsi - gy[u];   // circle centre - obstacle
          const T xt = slack ? x + ri * c - gx[u] : px, yt = slack ? y + ri * s - gy[u] : py;
          T fx, fy;
          if (!literal) {
            // elliptic angle: (a d cos al, b d sin al) = (xt, yt) max(1, ab/r),
            // r = |(b xt, a yt)| (eqs. zeta_2, compute_zeta_3); al = 0, d = 1
            // at the zero vector.  A centre offset whose r^2 is zero or below
            // the smallest normal number (|offset| ~ 1e-19 m in FP32) counts
            // as the zero vector: the hardware 1/sqrt is not defined there.
            const T r2 = b2 * xt * xt + a2 * yt * yt;
            const T g = fmax(T(1), ab * Num<T>::rsqrt_fast(r2));
            const bool zero = !(r2 >= kMinNormal<T>);
            fx = zero ? px - a : px - xt * g;
            fy = zero ? py : py - yt * g;
          } else {
            const T al = atan2z(yt, xt);
            T sa, ca;
            Num<T>::sincos_(al, &sa, &ca);
            const T dd = fmax(T(1), (a * xt * ca + b * yt * sa) / (a * a * ca * ca + b * b * sa * sa));
            fx = px - a * dd * ca;
            fy = py - b * dd * sa;
          }
          const T f2 = fx * fx + fy * fy;
          fc2max = fmax(fc2max, f2);
          fcsq += f2;
          lvl2 = fmin(lvl2, px * px * ia2 + py * py * ib2);
        }
      }
    }
    // velocity and acceleration: the projection onto the disc of radius
    // v_max leaves a residual of length max(0, |v| - v_max) (eqs. alpha_v,
    // compute_dv; likewise for a)
    v2max = fmax(v2max, xd * xd + yd * yd);
    a2max = fmax(a2max, xdd * xdd + ydd * ydd);
    slk = fmax(slk, fmax(fabs(c - cpsi), fabs(s - spsi)));
    T dh = atan2z(s, c) - psi;
    dh = dh - T(2) * pi * floor((dh + pi) / (T(2) * pi));
    head = fmax(head, fabs(dh));
    cost += xdd * xdd + ydd * ydd + psidd * psidd;
    if (t == 0 || t == q - 1) {
      const int o = (t == 0) ? 0 : 3;
      const T vals[9] = {x, xd, xdd, y, yd, ydd, psi, T(0), T(0)};
      T psid = 0;
#pragma unroll
      for (int k = 0; k < NV; ++k) psid += Pd[t * NV + k] * cp[k];
      const T ps3[3] = {psi, psid, psidd};
      for (int e = 0; e < 3; ++e) {
        bc = fmax(bc, fabs(vals[e] - T(D.bx[o + e])));
        bc = fmax(bc, fabs(vals[3 + e] - T(D.by[o + e])));
        bc = fmax(bc, fabs(ps3[e] - T(D.bpsi[o + e])));
      }
    }
  }
  // non-finite state values (coefficients and multipliers)
  int bad = 0;
  const T *lam = static_cast<const T *>(D.lam) + size_t(lc) * 4 * NV;
  const T *lp = static_cast<const T *>(D.lampsi) + size_t(lc) * NV;
  if (live && lane < NV)
    bad = !isfinite(cx[lane]) || !isfinite(cc[lane]) || !isfinite(cy[lane]) || !isfinite(cs[lane]) ||
          !isfinite(cp[lane]) || !isfinite(lp[lane]);
  if (live && lane < 4 * NV) bad |= !isfinite(lam[lane]);
  // per-wave totals, then the second wave's handed to the first through LDS
  T st[kResStats] = {wave_max(T(bad ? 1 : 0)), wave_max(fc2max), wave_add(fcsq), wave_min(lvl2),
                     wave_max(v2max), wave_max(a2max), wave_max(slk), wave_max(head), wave_max(bc),
                     wave_add(cost)};
  __shared__ T other[kTrajPerResBlock][kResStats];
  if (half == 1 && lane == 0) {
#pragma unroll
    for (int k = 0; k < kResStats; ++k) other[slot][k] = st[k];
  }
  __syncthreads();
  if (!live || half != 0) return;
  {
    const T *o = other[slot];
    st[0] = fmax(st[0], o[0]); st[1] = fmax(st[1], o[1]); st[2] += o[2]; st[3] = fmin(st[3], o[3]);
    st[4] = fmax(st[4], o[4]); st[5] = fmax(st[5], o[5]); st[6] = fmax(st[6], o[6]);
    st[7] = fmax(st[7], o[7]); st[8] = fmax(st[8], o[8]); st[9] += o[9];
  }
  const T fbad = st[0], fcmax = Num<T>::sqrt_(st[1]);
  fcsq = st[2];
  const T level = Num<T>::sqrt_(st[3]) - T(1);
  const T vex = Num<T>::sqrt_(st[4]) - vmax, aex = Num<T>::sqrt_(st[5]) - amax;
  const T fvmax = fmax(T(0), vex), famax = fmax(T(0), aex);
  slk = st[6];
  head = st[7];
  bc = st[8];
  cost = st[9];
  if (lane == 0) {
    T *o = static_cast<T *>(A.out) + size_t(l) * AM_NRES;
    const int mnq = m * n * q;
    o[AM_RES_FC_MAX] = fcmax;
    o[AM_RES_FC_RMS] = mnq ? Num<T>::sqrt_(fcsq / T(mnq)) : T(0);
    o[AM_RES_FV_MAX] = fvmax;
    o[AM_RES_FA_MAX] = famax;
    o[AM_RES_SLACK_MAX] = slk;
    o[AM_RES_HEADING_MAX] = head;
    o[AM_RES_BC_MAX] = bc;
    o[AM_RES_COST] = cost;
    o[AM_RES_CLEAR_LEVEL] = mnq ? level : T(INFINITY);
    o[AM_RES_V_EXCESS] = vex;
    o[AM_RES_A_EXCESS] = aex;
    o[AM_RES_NONFINITE] = fbad;
  }
}

template <typename T, int NV>
hipError_t res_t(const ResArgs &a, hipStream_t st) {
  const int blocks = (a.d.B + kTrajPerResBlock - 1) / kTrajPerResBlock;
  hipLaunchKernelGGL((residual_kernel<T, NV>), dim3(blocks), dim3(kWave * kWavesPerBlock), 0, st, a);
  return hipGetLastError();
}

// Best trajectory of a batch from its residual rows: the least cost
// (AM_RES_COST) among finite trajectories whose collision residual max |f_c|
// is at most tol; when none qualifies, the least max |f_c| among finite ones;
// when none is finite, index -1.  Ties go to the lower index, so the choice
// is a pure function of the residual values.  One 256-thread block.
constexpr int kSelThreads = 256;

template <typename T>
__device__ __forceinline__ bool sel_better(int ca, T va, int ia, int cb, T vb, int ib) {
  if (ca != cb) return ca < cb;
  if (va != vb) return va < vb;
  return ia < ib;
}

template <typename T>
__global__ __launch_bounds__(kSelThreads) void select_best_kernel(const T *res, int B, T tol, int32_t *out_idx,
                                                                 T *out_vals) {
  __shared__ int s_c[kSelThreads], s_i[kSelThreads];
  __shared__ T s_v[kSelThreads];
  int bc = 3, bi = -1;   // class 0: qualifies, 1: finite only, 3: none yet
  T bv = T(0);
  for (int l = threadIdx.x; l < B; l += kSelThreads) {
    const T *r = res + size_t(l) * AM_NRES;
    if (r[AM_RES_NONFINITE] != T(0)) continue;
    const T fc = r[AM_RES_FC_MAX], cost = r[AM_RES_COST];
    const int c = fc <= tol ? 0 : 1;
    const T v = c == 0 ? cost : fc;
    if (sel_better(c, v, l, bc, bv, bi)) { bc = c; bv = v; bi = l; }
  }
  s_c[threadIdx.x] = bc; s_v[threadIdx.x] = bv; s_i[threadIdx.x] = bi;
  __syncthreads();
  for (int w = kSelThreads / 2; w > 0; w >>= 1) {
    if (int(threadIdx.x) < w) {
      const int o = threadIdx.x + w;
      if (sel_better(s_c[o], s_v[o], s_i[o], s_c[threadIdx.x], s_v[threadIdx.x], s_i[threadIdx.x])) {
        s_c[threadIdx.x] = s_c[o]; s_v[threadIdx.x] = s_v[o]; s_i[threadIdx.x] = s_i[o];
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const int b = s_i[0];
    out_idx[0] = b;
    if (out_vals) {
      out_vals[0] = b >= 0 ? res[size_t(b) * AM_NRES + AM_RES_COST] : T(0);
      out_vals[1] = b >= 0 ? res[size_t(b) * AM_NRES + AM_RES_FC_MAX] : T(0);
    }
  }
}

// Problem-table fill: descriptors travel as kernel arguments (no host staging
// buffer, nothing to keep alive after the call, capture-safe).
constexpr int kDescPerCopy = 6;
struct DescChunk {
  Desc d[kDescPerCopy];
  int count;
  Desc *dst;
};

__global__ void desc_copy_kernel(DescChunk c) {
  const int words = int(sizeof(Desc) / sizeof(uint32_t));
  for (int k = 0; k < c.count; ++k) {
    const uint32_t *src = reinterpret_cast<const uint32_t *>(&c.d[k]);
    uint32_t *dst = reinterpret_cast<uint32_t *>(c.dst + k);
    for (int w = threadIdx.x; w < words; w += blockDim.x) dst[w] = src[w];
  }
}

}  // namespace

hipError_t launch_residuals(const Desc &d, const void *P, const void *Pd, const void *Pdd, void *out,
                            bool f64, int nv, hipStream_t st) {
  if (d.B <= 0) return hipSuccess;
  ResArgs a{d, P, Pd, Pdd, out};
  if (f64) {
    if (nv == 11) return res_t<double, 11>(a, st);
    if (nv == 8) return res_t<double, 8>(a, st);
  } else {
    if (nv == 11) return res_t<float, 11>(a, st);
    if (nv == 8) return res_t<float, 8>(a, st);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_select_best(const void *res, int B, double tol, int32_t *idx, void *vals, bool f64,
                              hipStream_t st) {
  if (f64)
    hipLaunchKernelGGL(select_best_kernel<double>, dim3(1), dim3(kSelThreads), 0, st,
                       static_cast<const double *>(res), B, tol, idx, static_cast<double *>(vals));
  else
    hipLaunchKernelGGL(select_best_kernel<float>, dim3(1), dim3(kSelThreads), 0, st,
                       static_cast<const float *>(res), B, float(tol), idx, static_cast<float *>(vals));
  return hipGetLastError();
}

hipError_t preload_kernels() {
  // HIP loads a source file's kernels on the first use of any of them; the
  // attribute query loads this file's (descriptor copy, selection, residuals)
  // at set-up instead of inside a later, latency-sensitive launch
  hipFuncAttributes attr;
  return hipFuncGetAttributes(&attr, reinterpret_cast<const void *>(&desc_copy_kernel));
}

hipError_t launch_desc_copy(const Desc *host_descs, int count, Desc *dev_dst, hipStream_t st) {
  static_assert(sizeof(Desc) % sizeof(uint32_t) == 0, "descriptor is word aligned");
  for (int base = 0; base < count; base += kDescPerCopy) {
    DescChunk c;
    c.count = count - base < kDescPerCopy ? count - base : kDescPerCopy;
    for (int k = 0; k < c.count; ++k) c.d[k] = host_descs[base + k];
    c.dst = dev_dst + base;
    hipLaunchKernelGGL(desc_copy_kernel, dim3(1), dim3(64), 0, st, c);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace amk
