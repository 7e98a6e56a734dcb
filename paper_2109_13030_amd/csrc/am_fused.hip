// am_fused.hip -- the whole batched AM iteration (Sec. III-D) in one launch.
//
// One wavefront owns one trajectory for all K iterations; its lanes own the
// time steps t = lane and t = lane + 64.  Everything the iteration carries
// (multipliers, coefficients, targets) stays in registers and LDS; global
// memory is touched only to load the initial state and to store the final
// one.  The four waves of a 256-thread block share the LDS copy of the
// problem's obstacle table and KKT operators.
//
// Algebra used (identical to the paper's steps in exact arithmetic):
//  * Coefficients live in the orthonormal basis z = R c (P = U R), so
//    x = U z, xdot = V z, xddot = W z and F^T v is formed with U^T, V^T, W^T.
//  * The xi3/xi4 closed forms are never evaluated through angles inside the
//    loop.  With the elliptic angle alpha = atan2(a y~, b x~) the target of a
//    collision row is g = (x_j, y_j) + (x~, y~) max(1, ab / sqrt(b^2 x~^2 +
//    a^2 y~^2)) (eqs. zeta_2, compute_zeta_3 with d >= 1), and the velocity
//    target is the projection of (xdot, ydot) on the disc of radius vmax
//    (eqs. alpha_v, compute_dv clipped to [0, 1]).  Only the deviation of g
//    from the current point is accumulated, so residuals are formed without
//    cancellation.
//  * lambda <- lambda - rho F^T (F xi - g) (eq. update_lambda_1) and the next
//    right-hand side lambda + rho F^T g = lambda + rho (F^T F xi - F^T(F xi - g))
//    share the single reduction F^T (F xi - g).
//  * Positions are shifted by the midpoint of start and goal on entry and back
//    on exit (exact: the basis reproduces constants, P 1 = 1, Pdot 1 = 0).
#include <hip/hip_runtime.h>

#include "am_device.h"
#include "am_internal.h"

namespace amk {
namespace {

constexpr int kMaxC = AM_MAX_CIRCLES;

template <typename T, int NV>
struct Wave {
  static constexpr int NVP = pad4(NV);
  T *z, *rhs, *lam, *tr, *h, *zpsi, *lampsi, *tpsi, *tmp, *red;
};

// Sum over the 64 lanes of G <= 16 per-lane partials.  On return lane k
// (k < G) holds the sum of partial k (lanes k+16, k+32, k+48 hold it too).
template <typename T, int G>
__device__ __forceinline__ T wave_sum_rows(const T (&p)[G], T *red, int lane) {
  static_assert(G <= 16, "at most 16 rows per call");
#pragma unroll
  for (int k = 0; k < G; ++k) red[k * kRedStride + lane] = p[k];
  wave_sync();
  const int row = lane & 15, quarter = lane >> 4;
  T s = T(0);
  if (row < G) {
    const T *src = red + row * kRedStride + quarter * 16;
#pragma unroll
    for (int c = 0; c < 16; ++c) s += src[c];
  }
  s += __shfl_xor(s, 16);
  s += __shfl_xor(s, 32);
  wave_sync();
  return s;
}

template <typename T, int NV>
__device__ void fused_body(const Desc &D, int l, T *lds, const FusedLds &L, int lane, int wave) {
  constexpr int NVP = pad4(NV);
  const int q = D.q, m = D.m, n = D.n, flags = D.flags;
  const T rho = T(D.rho), rhop = T(D.rho_psi), vmax = T(D.vmax), amax = T(D.amax);
  const bool slack = flags & AM_XTILDE_SLACK;
  const bool literal_alpha = flags & AM_ALPHA_LITERAL;
  const bool unwrap = !(flags & AM_PSI_NO_UNWRAP);
  const T psi_sign = (flags & AM_LAMPSI_LITERAL) ? T(-1) : T(1);

  const T *ox = lds + L.ox, *oy = lds + L.oy, *op = lds + L.op;
  const T *M1 = lds + L.m1, *M2 = lds + L.m2, *GF = lds + L.gf;
  const WaveLds wl = wave_layout(NV);
  T *wb = lds + L.wave0 + wave * L.wave_stride;
  T *vz = wb + wl.z, *vrhs = wb + wl.rhs, *vlam = wb + wl.lam, *vtr = wb + wl.tr, *vh = wb + wl.h;
  T *vzpsi = wb + wl.zpsi, *vlampsi = wb + wl.lampsi, *vtpsi = wb + wl.tpsi, *vtmp = wb + wl.tmp;
  T *red = wb + wl.red;

  T rr[kMaxC];
  T s1 = T(0), s2 = T(0);
#pragma unroll
  for (int i = 0; i < kMaxC; ++i) {
    rr[i] = i < m ? T(D.r[i]) : T(0);
    s1 += rr[i];
    s2 += rr[i] * rr[i];
  }
  s1 *= T(n);   // n sum r_i
  s2 *= T(n);   // n sum r_i^2

  // ---- per-lane basis rows (constant for the whole solve)
  const T *gU = static_cast<const T *>(D.U), *gV = static_cast<const T *>(D.V),
          *gW = static_cast<const T *>(D.W);
  T Ub[kSlots][NV], Vb[kSlots][NV], Wb[kSlots][NV];
  bool tv[kSlots];
#pragma unroll
  for (int s = 0; s < kSlots; ++s) {
    const int t = lane + kWave * s;
    tv[s] = t < q;
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      Ub[s][k] = tv[s] ? gU[t * NV + k] : T(0);
      Vb[s][k] = tv[s] ? gV[t * NV + k] : T(0);
      Wb[s][k] = tv[s] ? gW[t * NV + k] : T(0);
    }
  }

  // ---- boundary terms h = H b (centred positions) and the initial state
  const double *R = D.R, *Rinv = D.Rinv;
  if (lane < 4 * NV) {
    const int b = lane / NV, kk = lane % NV, axis = b >> 1;
    const double *bb = axis == 0 ? D.bx : D.by;
    const double off = axis == 0 ? D.offx : D.offy;
    const T *H1 = static_cast<const T *>(D.H1);
    const int I = (b & 1) * NV + kk;
    double hsum = 0.0;
    for (int e = 0; e < 6; ++e) {
      const double be = (e == 0 || e == 3) ? bb[e] - off : bb[e];
      hsum += double(H1[I * 6 + e]) * be;
    }
    vh[b * NVP + kk] = T(hsum);
    // z = R (c - off): the basis reproduces constants, so shifting all
    // coefficients of a position shifts its curve
    const T *src = static_cast<const T *>(b == 0 ? D.cx : (b == 1 ? D.cc : (b == 2 ? D.cy : D.cs)));
    const double coff = (b == 0) ? D.offx : ((b == 2) ? D.offy : 0.0);
    double zz = 0.0;
    for (int j = kk; j < NV; ++j) zz += R[kk * NV + j] * (double(src[size_t(l) * NV + j]) - coff);
    vz[b * NVP + kk] = T(zz);
    // lambda_z = R^-T lambda
    const T *glam = static_cast<const T *>(D.lam);
    double lz = 0.0;
    for (int j = 0; j <= kk; ++j) lz += Rinv[j * NV + kk] * double(glam[size_t(l) * 4 * NV + b * NV + j]);
    vlam[b * NVP + kk] = T(lz);
  } else if (lane < 5 * NV) {
    const int kk = lane - 4 * NV;
    const T *H2 = static_cast<const T *>(D.H2);
    double hsum = 0.0;
    for (int e = 0; e < 6; ++e) hsum += double(H2[kk * 6 + e]) * D.bpsi[e];
    vh[4 * NVP + kk] = T(hsum);
    const T *src = static_cast<const T *>(D.cpsi);
    double zz = 0.0;
    for (int j = kk; j < NV; ++j) zz += R[kk * NV + j] * double(src[size_t(l) * NV + j]);
    vzpsi[kk] = T(zz);
    const T *glp = static_cast<const T *>(D.lampsi);
    double lz = 0.0;
    for (int j = 0; j <= kk; ++j) lz += Rinv[j * NV + kk] * double(glp[size_t(l) * NV + j]);
    vlampsi[kk] = T(lz);
  }
  wave_sync();

  // ---- per-slot trajectory values
  T x[kSlots], xd[kSlots], xdd[kSlots], cc[kSlots], y[kSlots], yd[kSlots], ydd[kSlots], ss[kSlots];
  T psi[kSlots], cps[kSlots], sps[kSlots], psih[kSlots];

  auto eval_xy = [&]() {
#pragma unroll
    for (int s = 0; s < kSlots; ++s) {
      T a0 = 0, a1 = 0, a2 = 0, a3 = 0, b0 = 0, b1 = 0, b2 = 0, b3 = 0;
#pragma unroll
      for (int k = 0; k < NV; ++k) {
        const T zx = vz[k], zc = vz[NVP + k], zy = vz[2 * NVP + k], zs = vz[3 * NVP + k];
        a0 += Ub[s][k] * zx; a1 += Vb[s][k] * zx; a2 += Wb[s][k] * zx; a3 += Ub[s][k] * zc;
        b0 += Ub[s][k] * zy; b1 += Vb[s][k] * zy; b2 += Wb[s][k] * zy; b3 += Ub[s][k] * zs;
      }
      x[s] = a0; xd[s] = a1; xdd[s] = a2; cc[s] = a3;
      y[s] = b0; yd[s] = b1; ydd[s] = b2; ss[s] = b3;
    }
  };
  auto eval_psi = [&]() {
#pragma unroll
    for (int s = 0; s < kSlots; ++s) {
      T p = 0;
#pragma unroll
      for (int k = 0; k < NV; ++k) p += Ub[s][k] * vzpsi[k];
      psi[s] = p;
      T sn, cs;
      Num<T>::sincos_(p, &sn, &cs);
      cps[s] = cs;
      sps[s] = sn;
    }
  };

  // ---- xi3/xi4 projection of every (circle, obstacle, t), velocity and
  // acceleration, then F^T (F xi - g) into vtr and U^T(psi - psi_hat) into
  // vtpsi.
  auto project_reduce = [&](bool with_psi) {
    T p1x[NV], p2x[NV], p1y[NV], p2y[NV], pps[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) p1x[k] = p2x[k] = p1y[k] = p2y[k] = pps[k] = T(0);
#pragma unroll
    for (int s = 0; s < kSlots; ++s) {
      if (!tv[s]) continue;
      const int t = lane + kWave * s;
      const T ux = slack ? cc[s] : cps[s], uy = slack ? ss[s] : sps[s];
      T Xi[kMaxC], Yi[kMaxC], Sx[kMaxC], Sy[kMaxC];
#pragma unroll
      for (int i = 0; i < kMaxC; ++i) {
        Xi[i] = x[s] + rr[i] * ux;
        Yi[i] = y[s] + rr[i] * uy;
        Sx[i] = T(0);
        Sy[i] = T(0);
      }
      if (!literal_alpha) {
        for (int j = 0; j < n; ++j) {
          const T oxj = ox[j * q + t], oyj = oy[j * q + t];
          const T a2 = op[j * 8 + OP_A2], b2 = op[j * 8 + OP_B2], ab = op[j * 8 + OP_AB];
#pragma unroll
          for (int i = 0; i < kMaxC; ++i) {
            if (i < m) {
              const T xt = Xi[i] - oxj, yt = Yi[i] - oyj;
              const T r2 = b2 * xt * xt + a2 * yt * yt;
              const T f1 = fmax(T(0), ab * Num<T>::rsqrt(r2) - T(1));
              Sx[i] += xt * f1;
              Sy[i] += yt * f1;
            }
          }
        }
      } else {
        for (int j = 0; j < n; ++j) {
          const T oxj = ox[j * q + t], oyj = oy[j * q + t];
          const T a = op[j * 8 + OP_A], b = op[j * 8 + OP_B];
          const T a2 = op[j * 8 + OP_A2], b2 = op[j * 8 + OP_B2];
#pragma unroll
          for (int i = 0; i < kMaxC; ++i) {
            if (i < m) {
              const T xt = Xi[i] - oxj, yt = Yi[i] - oyj;
              const T xx = xt * xt, yy = yt * yt;
              const T kap = fmax(Num<T>::rsqrt(xx + yy), (a * xx + b * yy) / (a2 * xx + b2 * yy));
              Sx[i] += xt * (a * kap - T(1));
              Sy[i] += yt * (b * kap - T(1));
            }
          }
        }
      }
      // Exact zero (or underflowed) offsets make the fast form non-finite;
      // redo those sums element by element (alpha := 0 at the zero vector).
#pragma unroll
      for (int i = 0; i < kMaxC; ++i) {
        if (i < m && !(isfinite(Sx[i]) && isfinite(Sy[i]))) {
          T sx = T(0), sy = T(0);
          for (int j = 0; j < n; ++j) {
            const T xt = Xi[i] - ox[j * q + t], yt = Yi[i] - oy[j * q + t];
            const T a = op[j * 8 + OP_A], b = op[j * 8 + OP_B];
            if (xt == T(0) && yt == T(0)) {
              sx += a;   // alpha = 0, d = 1: target (x_j + a, y_j)
            } else if (!literal_alpha) {
              const T rr_ = Num<T>::hypot_(b * xt, a * yt);
              const T f1 = fmax(T(0), (a * b) / rr_ - T(1));
              sx += xt * f1;
              sy += yt * f1;
            } else {
              const T rho0 = Num<T>::hypot_(xt, yt);
              const T ca = xt / rho0, sa = yt / rho0;
              const T dd = fmax(T(1), (a * xt * ca + b * yt * sa) / (a * a * ca * ca + b * b * sa * sa));
              sx += a * dd * ca - xt;
              sy += b * dd * sa - yt;
            }
          }
          Sx[i] = sx;
          Sy[i] = sy;
        }
      }
      T Dx = 0, Dy = 0, DRx = 0, DRy = 0;
#pragma unroll
      for (int i = 0; i < kMaxC; ++i) {
        Dx += Sx[i]; Dy += Sy[i];
        DRx += rr[i] * Sx[i]; DRy += rr[i] * Sy[i];
      }
      // velocity / acceleration: part of (xdot, ydot) outside the disc
      const T fv = fmax(T(0), T(1) - vmax * Num<T>::rsqrt(xd[s] * xd[s] + yd[s] * yd[s]));
      const T fa = fmax(T(0), T(1) - amax * Num<T>::rsqrt(xdd[s] * xdd[s] + ydd[s] * ydd[s]));
      const T rvx = xd[s] * fv, rvy = yd[s] * fv, rax = xdd[s] * fa, ray = ydd[s] * fa;
      const T dc = cc[s] - cps[s], ds = ss[s] - sps[s];
      const T k1 = slack ? T(0) : s1, k2 = (slack ? T(0) : s2) + T(1);
      const T ro1x = k1 * dc - Dx, ro2x = k2 * dc - DRx;
      const T ro1y = k1 * ds - Dy, ro2y = k2 * ds - DRy;
      const T rp = psi_sign * (psi[s] - psih[s]);
#pragma unroll
      for (int k = 0; k < NV; ++k) {
        p1x[k] += Vb[s][k] * rvx + Wb[s][k] * rax + Ub[s][k] * ro1x;
        p2x[k] += Ub[s][k] * ro2x;
        p1y[k] += Vb[s][k] * rvy + Wb[s][k] * ray + Ub[s][k] * ro1y;
        p2y[k] += Ub[s][k] * ro2y;
        pps[k] += Ub[s][k] * rp;
      }
    }
    const T r0 = wave_sum_rows<T, NV>(p1x, red, lane);
    const T r1 = wave_sum_rows<T, NV>(p2x, red, lane);
    const T r2 = wave_sum_rows<T, NV>(p1y, red, lane);
    const T r3 = wave_sum_rows<T, NV>(p2y, red, lane);
    if (lane < NV) {
      vtr[lane] = r0;
      vtr[NVP + lane] = r1;
      vtr[2 * NVP + lane] = r2;
      vtr[3 * NVP + lane] = r3;
    }
    if (with_psi) {
      const T r4 = wave_sum_rows<T, NV>(pps, red, lane);
      if (lane < NV) vtpsi[lane] = r4;
    }
    wave_sync();
  };

  // lambda + rho (F^T F z - F^T(F xi - g)) for lane k < 4 NV
  auto next_rhs = [&](int k) {
    const int b = k / NV, kk = k % NV, axis = b >> 1;
    const int I = (b & 1) * NV + kk;
    const T *zax = vz + axis * 2 * NVP;
    T gz = T(0);
#pragma unroll
    for (int J = 0; J < 2 * NV; ++J) gz += GF[I * 2 * NV + J] * zax[(J / NV) * NVP + J % NV];
    return vlam[b * NVP + kk] + rho * (gz - vtr[b * NVP + kk]);
  };

  // ---- step 1 of the AM list: initial xi3, xi4 from the given trajectory
  eval_xy();
  eval_psi();
#pragma unroll
  for (int s = 0; s < kSlots; ++s) psih[s] = psi[s];
  project_reduce(false);
  if (lane < 4 * NV) {
    const T v = next_rhs(lane);
    vrhs[(lane / NV) * NVP + lane % NV] = v;
  }
  wave_sync();

  for (int it = 0; it < D.K; ++it) {
    // ---- xi1: [z; mu] = KKT^-1 [lambda + rho F^T g; b]  (eqs. over_3, zeta_1_sepration_3)
    if (lane < 4 * NV) {
      const int b = lane / NV, kk = lane % NV, axis = b >> 1;
      const int I = (b & 1) * NV + kk;
      const T *rax = vrhs + axis * 2 * NVP;
      T acc = vh[b * NVP + kk];
#pragma unroll
      for (int J = 0; J < 2 * NV; ++J) acc += M1[I * 2 * NV + J] * rax[(J / NV) * NVP + J % NV];
      vz[b * NVP + kk] = acc;
    }
    wave_sync();
    eval_xy();

    // ---- xi2: psi_hat = atan2(s, c) on the branch nearest psi^k, then the
    // heading QP (eq. compute_convex_surrogate)
    T pp[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) pp[k] = T(0);
#pragma unroll
    for (int s = 0; s < kSlots; ++s) {
      T ph;
      if (unwrap)
        ph = psi[s] + atan2z(ss[s] * cps[s] - cc[s] * sps[s], cc[s] * cps[s] + ss[s] * sps[s]);
      else
        ph = atan2z(ss[s], cc[s]);
      psih[s] = tv[s] ? ph : T(0);
#pragma unroll
      for (int k = 0; k < NV; ++k) pp[k] += Ub[s][k] * psih[s];
    }
    const T upsi = wave_sum_rows<T, NV>(pp, red, lane);
    if (lane < NV) vtmp[lane] = vlampsi[lane] + rho * upsi;
    wave_sync();
    if (lane < NV) {
      T acc = vh[4 * NVP + lane];
#pragma unroll
      for (int j = 0; j < NV; ++j) acc += M2[lane * NV + j] * vtmp[j];
      vzpsi[lane] = acc;
    }
    wave_sync();
    eval_psi();

    // ---- xi3, xi4 and the multipliers (eqs. update_lambda_1, update_lambda_psi)
    project_reduce(true);
    if (lane < 4 * NV) {
      const int b = lane / NV, kk = lane % NV;
      vlam[b * NVP + kk] -= rho * vtr[b * NVP + kk];
    } else if (lane < 5 * NV) {
      const int kk = lane - 4 * NV;
      vlampsi[kk] -= rhop * vtpsi[kk];
    }
    wave_sync();
    if (lane < 4 * NV) {
      const T v = next_rhs(lane);
      vrhs[(lane / NV) * NVP + lane % NV] = v;
    }
    wave_sync();
  }

  // ---- state back to Bernstein coordinates
  if (lane < 4 * NV) {
    const int b = lane / NV, kk = lane % NV;
    T *dst = static_cast<T *>(b == 0 ? D.cx : (b == 1 ? D.cc : (b == 2 ? D.cy : D.cs)));
    const double coff = (b == 0) ? D.offx : ((b == 2) ? D.offy : 0.0);
    double c = 0.0, lc = 0.0;
    for (int j = kk; j < NV; ++j) c += Rinv[kk * NV + j] * double(vz[b * NVP + j]);
    for (int j = 0; j <= kk; ++j) lc += R[j * NV + kk] * double(vlam[b * NVP + j]);
    dst[size_t(l) * NV + kk] = T(c + coff);
    static_cast<T *>(D.lam)[size_t(l) * 4 * NV + b * NV + kk] = T(lc);
  } else if (lane < 5 * NV) {
    const int kk = lane - 4 * NV;
    double c = 0.0, lc = 0.0;
    for (int j = kk; j < NV; ++j) c += Rinv[kk * NV + j] * double(vzpsi[j]);
    for (int j = 0; j <= kk; ++j) lc += R[j * NV + kk] * double(vlampsi[j]);
    static_cast<T *>(D.cpsi)[size_t(l) * NV + kk] = T(c);
    static_cast<T *>(D.lampsi)[size_t(l) * NV + kk] = T(lc);
  }

  // ---- optional outputs: trajectory and the final (alpha, d) of xi3/xi4
  if (D.traj) {
    T *tr = static_cast<T *>(D.traj) + size_t(l) * 3 * q;
#pragma unroll
    for (int s = 0; s < kSlots; ++s)
      if (tv[s]) {
        const int t = lane + kWave * s;
        tr[t] = x[s] + T(D.offx);
        tr[q + t] = y[s] + T(D.offy);
        tr[2 * q + t] = psi[s];
      }
  }
  if (D.va) {
    T *va = static_cast<T *>(D.va) + size_t(l) * 4 * q;
#pragma unroll
    for (int s = 0; s < kSlots; ++s)
      if (tv[s]) {
        const int t = lane + kWave * s;
        const T av = atan2z(yd[s], xd[s]), aa = atan2z(ydd[s], xdd[s]);
        const T dv = (xd[s] * Num<T>::cos_(av) + yd[s] * Num<T>::sin_(av)) / vmax;
        const T da = (xdd[s] * Num<T>::cos_(aa) + ydd[s] * Num<T>::sin_(aa)) / amax;
        va[t] = av;
        va[q + t] = fmin(T(1), fmax(T(0), dv));
        va[2 * q + t] = aa;
        va[3 * q + t] = fmin(T(1), fmax(T(0), da));
      }
  }
  if (D.alpha || D.d) {
    T *ga = static_cast<T *>(D.alpha), *gd = static_cast<T *>(D.d);
    const size_t base = size_t(l) * m * n * q;
#pragma unroll
    for (int s = 0; s < kSlots; ++s) {
      if (!tv[s]) continue;
      const int t = lane + kWave * s;
      const T ux = slack ? cc[s] : cps[s], uy = slack ? ss[s] : sps[s];
      for (int i = 0; i < m; ++i)
        for (int j = 0; j < n; ++j) {
          const T xt = x[s] + rr[i] * ux - ox[j * q + t];
          const T yt = y[s] + rr[i] * uy - oy[j * q + t];
          const T a = op[j * 8 + OP_A], b = op[j * 8 + OP_B];
          const T al = literal_alpha ? atan2z(yt, xt) : atan2z(a * yt, b * xt);
          const T ca = Num<T>::cos_(al), sa = Num<T>::sin_(al);
          const T dd = fmax(T(1), (a * xt * ca + b * yt * sa) / (a * a * ca * ca + b * b * sa * sa));
          const size_t e = base + size_t(i * n + j) * q + t;
          if (ga) ga[e] = al;
          if (gd) gd[e] = dd;
        }
    }
  }
}

template <typename T, int NV>
__global__ __launch_bounds__(kWave *kWavesPerBlock) void fused_kernel(Desc single, const Desc *table,
                                                                      int nprob) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T *lds = reinterpret_cast<T *>(smem_raw);
  int p = 0;
  if (table) {
    int lo = 0, hi = nprob - 1;
    while (lo < hi) {   // last problem whose first block is <= blockIdx.x
      const int mid = (lo + hi + 1) >> 1;
      if (table[mid].blk0 <= int(blockIdx.x)) lo = mid; else hi = mid - 1;
    }
    p = lo;
  }
  const Desc &D = table ? table[p] : single;
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
  const int q = D.q, n = D.n;
  const FusedLds L = fused_layout(q, n, NV);

  // block-wide: obstacle tables (centred), inflated semi-axes, operators
  const T *gox = static_cast<const T *>(D.ox), *goy = static_cast<const T *>(D.oy);
  const T offx = T(D.offx), offy = T(D.offy);
  for (int i = tid; i < n * q; i += blockDim.x) {
    lds[L.ox + i] = gox[i] - offx;
    lds[L.oy + i] = goy[i] - offy;
  }
  for (int j = tid; j < n; j += blockDim.x) {
    const T a = static_cast<const T *>(D.oa)[j] + T(D.rc);
    const T b = static_cast<const T *>(D.ob)[j] + T(D.rc);
    T *o = lds + L.op + j * 8;
    o[OP_A] = a; o[OP_B] = b; o[OP_A2] = a * a; o[OP_B2] = b * b; o[OP_AB] = a * b;
  }
  const T *gM1 = static_cast<const T *>(D.M1), *gM2 = static_cast<const T *>(D.M2),
          *gGF = static_cast<const T *>(D.GF);
  for (int i = tid; i < 4 * NV * NV; i += blockDim.x) {
    lds[L.m1 + i] = gM1[i];
    lds[L.gf + i] = gGF[i];
  }
  for (int i = tid; i < NV * NV; i += blockDim.x) lds[L.m2 + i] = gM2[i];
  __syncthreads();

  const int l = (int(blockIdx.x) - D.blk0) * kWavesPerBlock + wave;
  if (l >= D.B) return;   // no block-wide barrier follows
  fused_body<T, NV>(D, l, lds, L, lane, wave);
}

template <typename T, int NV>
hipError_t launch_t(const Desc &single, const Desc *table, int nprob, int nblocks, hipStream_t st,
                    size_t lds_bytes) {
  if (lds_bytes > 65536) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&fused_kernel<T, NV>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, int(lds_bytes));
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL((fused_kernel<T, NV>), dim3(nblocks), dim3(kWave * kWavesPerBlock), lds_bytes, st,
                     single, table, nprob);
  return hipGetLastError();
}

}  // namespace

size_t fused_lds_bytes(int q, int n, int nv, bool f64) {
  return size_t(fused_layout(q, n, nv).total) * (f64 ? 8 : 4);
}

hipError_t launch_fused(const Desc &single, const Desc *table, int nprob, int nblocks, bool f64,
                        int nv, hipStream_t st, size_t lds_bytes) {
  if (nblocks <= 0) return hipSuccess;
  if (f64) {
    if (nv == 11) return launch_t<double, 11>(single, table, nprob, nblocks, st, lds_bytes);
    if (nv == 8) return launch_t<double, 8>(single, table, nprob, nblocks, st, lds_bytes);
  } else {
    if (nv == 11) return launch_t<float, 11>(single, table, nprob, nblocks, st, lds_bytes);
    if (nv == 8) return launch_t<float, 8>(single, table, nprob, nblocks, st, lds_bytes);
  }
  return hipErrorInvalidValue;
}

}  // namespace amk
