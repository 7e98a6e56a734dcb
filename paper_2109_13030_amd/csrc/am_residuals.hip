// am_residuals.hip -- per-trajectory residual statistics of the current state
// (one wavefront per trajectory), plus the small kernel that fills the
// problem table of multi-problem launches.
//
// The angles and distances are recomputed by the closed forms of eqs.
// (zeta_2, alpha_v, alpha_a, compute_zeta_3, compute_dv, compute_da) from the
// current trajectories, which is exactly what the last xi3/xi4 step produced.
#include <hip/hip_runtime.h>

#include "am_device.h"
#include "am_internal.h"

namespace amk {
namespace {

template <typename T>
__device__ __forceinline__ T wave_max(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
  return v;
}
template <typename T>
__device__ __forceinline__ T wave_min(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o));
  return v;
}
template <typename T>
__device__ __forceinline__ T wave_add(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

struct ResArgs {
  Desc d;
  const void *P, *Pd, *Pdd;
  void *out;
};

template <typename T, int NV>
__global__ __launch_bounds__(kWave *kWavesPerBlock) void residual_kernel(ResArgs A) {
  const Desc &D = A.d;
  const int lane = threadIdx.x & (kWave - 1);
  const int l = blockIdx.x * kWavesPerBlock + threadIdx.x / kWave;
  if (l >= D.B) return;
  const int q = D.q, m = D.m, n = D.n;
  const bool slack = D.flags & AM_XTILDE_SLACK, literal = D.flags & AM_ALPHA_LITERAL;
  const T *P = static_cast<const T *>(A.P), *Pd = static_cast<const T *>(A.Pd),
          *Pdd = static_cast<const T *>(A.Pdd);
  const T *cx = static_cast<const T *>(D.cx) + size_t(l) * NV, *cc = static_cast<const T *>(D.cc) + size_t(l) * NV;
  const T *cy = static_cast<const T *>(D.cy) + size_t(l) * NV, *cs = static_cast<const T *>(D.cs) + size_t(l) * NV;
  const T *cp = static_cast<const T *>(D.cpsi) + size_t(l) * NV;
  const T *gox = static_cast<const T *>(D.ox), *goy = static_cast<const T *>(D.oy);
  const T *goa = static_cast<const T *>(D.oa), *gob = static_cast<const T *>(D.ob);
  const T vmax = T(D.vmax), amax = T(D.amax), rc = T(D.rc);
  const T pi = T(3.14159265358979323846);

  T fcmax = 0, fcsq = 0, level = T(INFINITY), fvmax = 0, famax = 0, slk = 0, head = 0, bc = 0, cost = 0;
  T vex = T(-INFINITY), aex = T(-INFINITY);
  for (int t = lane; t < q; t += kWave) {
    T x = 0, xd = 0, xdd = 0, y = 0, yd = 0, ydd = 0, c = 0, s = 0, psi = 0, psidd = 0;
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      const T p = P[t * NV + k], pd = Pd[t * NV + k], pdd = Pdd[t * NV + k];
      x += p * cx[k]; xd += pd * cx[k]; xdd += pdd * cx[k];
      y += p * cy[k]; yd += pd * cy[k]; ydd += pdd * cy[k];
      c += p * cc[k]; s += p * cs[k]; psi += p * cp[k]; psidd += pdd * cp[k];
    }
    const T cpsi = Num<T>::cos_(psi), spsi = Num<T>::sin_(psi);
    for (int i = 0; i < m; ++i) {
      const T ri = T(D.r[i]);
      for (int j = 0; j < n; ++j) {
        const T a = goa[j] + rc, b = gob[j] + rc;
        const T px = x + ri * cpsi - gox[j * q + t], py = y + ri * spsi - goy[j * q + t];
        const T xt = slack ? x + ri * c - gox[j * q + t] : px;
        const T yt = slack ? y + ri * s - goy[j * q + t] : py;
        const T al = literal ? atan2z(yt, xt) : atan2z(a * yt, b * xt);
        const T ca = Num<T>::cos_(al), sa = Num<T>::sin_(al);
        const T dd = fmax(T(1), (a * xt * ca + b * yt * sa) / (a * a * ca * ca + b * b * sa * sa));
        const T fx = px - a * dd * ca, fy = py - b * dd * sa;
        const T f2 = fx * fx + fy * fy;
        fcmax = fmax(fcmax, Num<T>::sqrt_(f2));
        fcsq += f2;
        level = fmin(level, Num<T>::sqrt_(px * px / (a * a) + py * py / (b * b)) - T(1));
      }
    }
    const T av = atan2z(yd, xd), aa = atan2z(ydd, xdd);
    const T dv = fmin(T(1), fmax(T(0), (xd * Num<T>::cos_(av) + yd * Num<T>::sin_(av)) / vmax));
    const T da = fmin(T(1), fmax(T(0), (xdd * Num<T>::cos_(aa) + ydd * Num<T>::sin_(aa)) / amax));
    const T vx = xd - vmax * dv * Num<T>::cos_(av), vy = yd - vmax * dv * Num<T>::sin_(av);
    const T ax = xdd - amax * da * Num<T>::cos_(aa), ay = ydd - amax * da * Num<T>::sin_(aa);
    fvmax = fmax(fvmax, Num<T>::sqrt_(vx * vx + vy * vy));
    famax = fmax(famax, Num<T>::sqrt_(ax * ax + ay * ay));
    slk = fmax(slk, fmax(fabs(c - cpsi), fabs(s - spsi)));
    T dh = atan2z(s, c) - psi;
    dh = dh - T(2) * pi * floor((dh + pi) / (T(2) * pi));
    head = fmax(head, fabs(dh));
    cost += xdd * xdd + ydd * ydd + psidd * psidd;
    vex = fmax(vex, Num<T>::sqrt_(xd * xd + yd * yd) - vmax);
    aex = fmax(aex, Num<T>::sqrt_(xdd * xdd + ydd * ydd) - amax);
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
  const T *lam = static_cast<const T *>(D.lam) + size_t(l) * 4 * NV;
  const T *lp = static_cast<const T *>(D.lampsi) + size_t(l) * NV;
  if (lane < NV)
    bad = !isfinite(cx[lane]) || !isfinite(cc[lane]) || !isfinite(cy[lane]) || !isfinite(cs[lane]) ||
          !isfinite(cp[lane]) || !isfinite(lp[lane]);
  if (lane < 4 * NV) bad |= !isfinite(lam[lane]);
  const T fbad = wave_max(T(bad ? 1 : 0));
  fcmax = wave_max(fcmax);
  fcsq = wave_add(fcsq);
  level = wave_min(level);
  fvmax = wave_max(fvmax);
  famax = wave_max(famax);
  slk = wave_max(slk);
  head = wave_max(head);
  bc = wave_max(bc);
  cost = wave_add(cost);
  vex = wave_max(vex);
  aex = wave_max(aex);
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
  const int blocks = (a.d.B + kWavesPerBlock - 1) / kWavesPerBlock;
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
