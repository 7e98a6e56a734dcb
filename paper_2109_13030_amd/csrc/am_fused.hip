// am_fused.hip -- the whole batched AM iteration (Sec. III-D) in one launch.
//
// Two wavefronts own one trajectory for all K iterations: wave h of the pair
// holds the time steps t = h*ceil(q/2) + lane.  A block carries `tile`
// trajectories and shares the LDS copy of the problem's obstacle table and
// KKT operators.  Everything the iteration carries (multipliers,
// coefficients, targets) stays in registers and LDS; global memory is read
// for the initial state and written for the final one only.  Sums over t
// are formed per wave, exchanged through LDS and added in a fixed order, so
// both waves of a pair hold bit-identical copies of the wave-uniform
// vectors (coefficients, multipliers, right-hand sides).
//
// Algebra used (identical to the paper's steps in exact arithmetic):
//  * Coefficients live in the orthonormal basis z = R c (P = U R), so
//    x = U z, xdot = V z, xddot = W z and F^T v is formed with U^T, V^T, W^T.
//  * The xi3/xi4 closed forms are not evaluated through angles inside the
//    loop.  With the elliptic angle alpha = atan2(a y~, b x~) the target of a
//    collision row is g = (x_j, y_j) + (x~, y~) max(1, ab / sqrt(b^2 x~^2 +
//    a^2 y~^2)) (eqs. zeta_2, compute_zeta_3 with d >= 1), and the velocity
//    target is the projection of (xdot, ydot) on the disc of radius vmax
//    (eqs. alpha_v, compute_dv clipped to [0, 1]).  Only the deviation of g
//    from the current point is accumulated, so residuals are formed without
//    cancellation.  That deviation is zero for circle centres outside the
//    ellipse, so obstacles farther from the robot centre than the farthest
//    circle plus the larger semi-axis are skipped (a wave-wide vote per
//    obstacle).
//  * lambda <- lambda - rho F^T (F xi - g) (eq. update_lambda_1) and the
//    next xi1 right-hand side lambda + rho F^T g share the single reduction
//    F^T (F xi - g).
//  * The xi1 step is applied as an update of the current coefficients.  With
//    [M1 H1] the first block row of the KKT inverse (eq. over_3), the identity
//    M1 (Q + rho F^T F) + H1 A = I turns z' = H1 b + M1 (lambda + rho F^T g)
//    into z' = z - H1 (A z - b) + M1 (lambda - rho F^T (F xi - g) - Q z).
//    The update is small once the iteration settles, so the FP32 rounding of
//    the operators and of the large product F^T F z no longer enters z; z,
//    the multipliers, Q z and the update itself are carried in FP64 (Q z' =
//    Q z + Q dz with the product of the small update in T; Q is the
//    block-diagonal smoothness term W^T W), and so are the positions (x' =
//    x + U dz likewise); an offset from an obstacle centre is the FP32
//    difference from the position's FP32 rounding plus the rounding
//    remainder, each rounded once.  A z = b holds after the first update,
//    so the boundary term is applied once.
//  * The heading step (eq. compute_convex_surrogate) is z_psi = h_psi +
//    M2 (lambda_psi + rho U^T psi_hat).  With mu = M2 lambda_psi and the rows
//    of U~ = U M2^T, z_psi = h_psi + mu + rho U~^T psi_hat, and the
//    multiplier update (eq. update_lambda_psi) is mu <- mu - rho_psi U~^T
//    (psi - psi_hat).  Both sums fold into one per iteration: z_psi of
//    iteration k+1 is that of iteration k plus U~^T (rho (psi_hat' -
//    psi_hat) - rho_psi (psi - psi_hat)), so the kernel carries z_psi (FP64)
//    and reduces that per-lane difference only.  lambda_psi itself is
//    linear in the summed residuals, so each lane sums psi - psi_hat over
//    the iterations and lambda_psi is formed once at the end.
//  * Coefficients are shifted by the midpoint of start and goal on entry and
//    back on exit (exact: the basis reproduces constants, P 1 = 1,
//    Pdot 1 = 0).
//  * Each lane holds its rows of U, V, W and U~ in its own order (within
//    groups of 4 rows, slot k holds row k xor (lane mod 4)), so the sums
//    over t combine lanes without selects (wave_sum_perm); the vectors the
//    lanes multiply against those rows are kept in LDS in the four orders.
#include <hip/hip_runtime.h>

#include <limits>
#include <type_traits>

#include "am_device.h"
#include "am_internal.h"

namespace amk {
namespace {

// Circle capacity of a kernel instance: 5 (enough for every robot shape
// here; fewer registers and no dead circle slots) or AM_MAX_CIRCLES.
constexpr int kSmallC = 5;
constexpr int kVoteChunk = 8;   // obstacles whose positions are loaded together in the vote
constexpr double kVoteMargin = 0.25;   // [m] slack of the near-obstacle set, see project_reduce

// Wave-uniform copies of descriptor fields: the compiler then keeps them in
// scalar registers and treats loops over them as uniform.
__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ float uni(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, v)));
}
__device__ __forceinline__ double uni(double v) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_readfirstlane(int(b & 0xffffffffLL));
  const int hi = __builtin_amdgcn_readfirstlane(int(b >> 32));
  return __builtin_bit_cast(double, (static_cast<long long>(hi) << 32) | (static_cast<unsigned int>(lo)));
}

// Value of the neighbouring lane (lane ^ 1) through a DPP quad permutation.
__device__ __forceinline__ float lane_xor1(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), 0xB1, 0xF, 0xF, true));
}
__device__ __forceinline__ double lane_xor1(double v) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_mov_dpp(int(b & 0xffffffffLL), 0xB1, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_mov_dpp(int(b >> 32), 0xB1, 0xF, 0xF, true);
  return __builtin_bit_cast(double, (static_cast<long long>(hi) << 32) | (static_cast<unsigned int>(lo)));
}

// Value of lane ^ 2 (DPP quad permutation [2, 3, 0, 1]).
__device__ __forceinline__ float lane_xor2(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), 0x4E, 0xF, 0xF, true));
}
__device__ __forceinline__ double lane_xor2(double v) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_mov_dpp(int(b & 0xffffffffLL), 0x4E, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_mov_dpp(int(b >> 32), 0x4E, 0xF, 0xF, true);
  return __builtin_bit_cast(double, (static_cast<long long>(hi) << 32) | (static_cast<unsigned int>(lo)));
}

// Total of the 16 quad sums of one reduction row, with four interleaved
// accumulators.
template <typename T>
__device__ __forceinline__ T quad_row_total(const T *row_base) {
#pragma clang fp contract(off)
  const Quad<T> *row = reinterpret_cast<const Quad<T> *>(row_base);
  const Quad<T> v0 = row[0];
  T s0 = v0.a, s1 = v0.b, s2 = v0.c, s3 = v0.d;
#pragma unroll
  for (int c = 1; c < 4; ++c) {
    const Quad<T> v = row[c];
    s0 += v.a; s1 += v.b; s2 += v.c; s3 += v.d;
  }
  return (s0 + s1) + (s2 + s3);
}

// Sums over the 64 lanes of G per-lane partials (G a multiple of 4) that
// come in lane-permuted slots: on lane L, slot 4i + k holds the partial of
// row 4i + (k ^ (L % 4)).  Slot 4i + 1 of the neighbour L ^ 1 holds the row
// of slot 4i here, so one DPP add per row pair gives this row's sum over the
// lane pair; likewise slots 4i + 2 and 4i + 3 give the sum of the row that
// lane L ^ 2 holds, and one more DPP add across the quad leaves lane L with
// row 4i + L % 4 summed over its quad, with no selects.  The 16 quad sums
// of a row go to LDS and lane g adds row g with four interleaved
// accumulators.  Rows go through LDS in passes of ROWS (a multiple of 4).
// On return lane g (g < G) holds the total of row g; the order of the
// additions does not depend on the pass size.  (A plain add takes the
// neighbour through its DPP operand, one instruction; fused into the
// caller's product it would need a separate DPP move and the product twice.)
template <typename T, int G, int ROWS>
__device__ __forceinline__ T wave_sum_perm(const T (&p)[G], T *red, int lane) {
#pragma clang fp contract(off)
  constexpr int NQ = G / 4, RPP = ROWS / 4;   // row groups, per pass
  static_assert(G % 4 == 0 && ROWS <= kRedRows && ROWS % 4 == 0, "row groups");
  T s = T(0);
#pragma unroll
  for (int i0 = 0; i0 < NQ; i0 += RPP) {
#pragma unroll
    for (int i = i0; i < NQ && i < i0 + RPP; ++i) {
      const T a = p[4 * i] + lane_xor1(p[4 * i + 1]);
      const T b = p[4 * i + 2] + lane_xor1(p[4 * i + 3]);
      red[(4 * (i - i0) + (lane & 3)) * kRedRowStride + (lane >> 2)] = a + lane_xor2(b);
    }
    wave_sync();
    const int g0 = 4 * i0;
    if (lane >= g0 && lane < G && lane < g0 + ROWS) s = quad_row_total(red + (lane - g0) * kRedRowStride);
    wave_sync();
  }
  return s;
}

// Row I of a [2nv][2nv] operator stored as Quad [a2/4][2nv] times the
// 2nv-vector v (contiguous, 16-byte aligned, padded to a2).
template <typename T, int NV>
__device__ __forceinline__ T row_dot(const T *op, int I, const T *v) {
  constexpr int N2 = 2 * NV, C = pad4(N2) / 4;
  const Quad<T> *o = reinterpret_cast<const Quad<T> *>(op);
  const Quad<T> *vv = reinterpret_cast<const Quad<T> *>(v);
  T acc0 = T(0), acc1 = T(0);
#pragma unroll
  for (int c = 0; c < C; ++c) {
    const Quad<T> a = o[c * N2 + I], b = vv[c];
    acc0 += a.a * b.a;
    acc1 += a.b * b.b;
    if (4 * c + 2 < N2) acc0 += a.c * b.c;
    if (4 * c + 3 < N2) acc1 += a.d * b.d;
  }
  return acc0 + acc1;
}

template <typename T, int NV, int C, int RED>
__device__ void fused_body(const Desc &Dsrc, int l, bool live, int half, T *lds, const FusedLds &L,
                           int lane, int wave) {
  constexpr int A2 = pad4(2 * NV), N2 = 2 * NV;
  constexpr int NP = pad4(NV);   // basis rows padded to whole 4-row groups
  constexpr int G = 4 * NP;      // rows of the per-iteration reduction (4 blocks of NP)
  constexpr int DW = int(sizeof(double) / sizeof(T));   // elements of T per FP64 value
  // descriptor fields used in the loop, as locals
  const int q = uni(Dsrc.q), m = uni(Dsrc.m), n = uni(Dsrc.n), flags = uni(Dsrc.flags), K = uni(Dsrc.K);
  const T rho = uni(T(Dsrc.rho)), rhop = uni(T(Dsrc.rho_psi)), vmax = uni(T(Dsrc.vmax)),
          amax = uni(T(Dsrc.amax));
  const double rhod = uni(Dsrc.rho);
  const double offx = uni(Dsrc.offx), offy = uni(Dsrc.offy);
  const bool slack = flags & AM_XTILDE_SLACK;
  const bool literal_alpha = flags & AM_ALPHA_LITERAL;
  const bool unwrap = !(flags & AM_PSI_NO_UNWRAP);
  const T psi_sign = (flags & AM_LAMPSI_LITERAL) ? T(-1) : T(1);
  const int hq = (q + 1) / 2;
  const int t = half * hq + lane;
  const bool tv = lane < hq && t < q;
  const int tt = tv ? t : 0;
  // lane roles in the wave-uniform steps: row (axis, I) of the position
  // block for lane < 4 nv, row `lane` of the heading block for lane < nv
  const bool prow = lane < 2 * N2, hrow = lane < NV;
  const int axis = prow ? lane / N2 : 0, I = prow ? lane % N2 : 0;

  const Pair<T> *oxy = reinterpret_cast<const Pair<T> *>(lds + L.oxy);
  const T *op = lds + L.op;
  const Quad<T> *opq = reinterpret_cast<const Quad<T> *>(lds + L.op);
  constexpr int QS = NP;   // row stride of the Q rows and block stride of dz
  static_assert(QS + NV <= A2, "both blocks of dz fit one axis's area");
  // this lane's slot order: slot 4i + k holds row 4i + (k ^ sq)
  const int sq = lane & 3;
  constexpr int DZC = dz_copy_stride(NV), ZPC = zpsi_copy_stride(NV);
  const T *M1 = lds + L.m1, *QL = lds + L.qrows;
  const WaveLds wl = wave_layout(NV, RED, DW);
  T *wb = lds + L.wave0 + wave * L.wave_stride;
  T *vzpsi = wb + wl.zpsi, *vaux = wb + wl.aux;   // vzpsi: copy 0 (natural order)
  T *vw = wb + wl.w, *vdz = wb + wl.dz;            // vdz: copy 0 (natural order)
  const Quad<T> *dzq = reinterpret_cast<const Quad<T> *>(vdz + sq * DZC);      // this lane's copies
  const Quad<T> *zpsiq = reinterpret_cast<const Quad<T> *>(vzpsi + sq * ZPC);
  // element r of a vector held in the four lane-permuted copies
  auto put4 = [](T *v, int stride, int r, T x) {
    const int g = r & ~3, k = r & 3;
#pragma unroll
    for (int c = 0; c < 4; ++c) v[c * stride + g + (k ^ c)] = x;
  };
  double *vzd = reinterpret_cast<double *>(wb + wl.zd), *vwd = reinterpret_cast<double *>(wb + wl.wd);
  T *red = wb + wl.red;
  // exchange area of this trajectory: [half][kXchHalf]
  T *xch = lds + L.xch + (wave >> 1) * 2 * kXchHalf;
  T *xmine = xch + half * kXchHalf;

  T rr[C];
  T s1 = T(0), s2 = T(0), rmax = T(0);
#pragma unroll
  for (int i = 0; i < C; ++i) {
    rr[i] = i < m ? uni(T(Dsrc.r[i])) : T(0);
    s1 += rr[i];
    s2 += rr[i] * rr[i];
    rmax = fmax(rmax, fabs(rr[i]));
  }
  s1 *= T(n);   // n sum r_i
  s2 *= T(n);   // n sum r_i^2

  // ---- per-lane basis rows (constant for the whole solve), U~ = U M2^T
  const T *gU = static_cast<const T *>(Dsrc.U), *gV = static_cast<const T *>(Dsrc.V),
          *gW = static_cast<const T *>(Dsrc.W), *gUt = static_cast<const T *>(Dsrc.Ut),
          *gM2 = static_cast<const T *>(Dsrc.M2);
  // (in this lane's slot order; rows past nv are zero)
  T Ub[NP], Vb[NP], Wb[NP], Ut[NP];
#pragma unroll
  for (int k = 0; k < NP; ++k) {
    const int r = (k & ~3) | ((k & 3) ^ sq);
    const bool use = tv && r < NV;
    const int e = use ? tt * NV + r : 0;
    Ub[k] = use ? gU[e] : T(0);
    Vb[k] = use ? gV[e] : T(0);
    Wb[k] = use ? gW[e] : T(0);
    Ut[k] = use ? gUt[e] : T(0);
  }

  // ---- boundary terms h = H b (centred positions) and the initial state
  const double *R = Dsrc.R, *Rinv = Dsrc.Rinv;
  // lane I of the position block: its coefficient, multiplier and the
  // boundary correction of the first update, in FP64
  double zl = 0.0, lam = 0.0, bcc = 0.0;
  T hpsi = T(0), lampsi0 = T(0);
  // rows of the set-up operators this lane uses after the LDS exchanges
  // below (H1, M2, the FP64 rows of U and Q), loaded first so that their
  // latency overlaps that of the state loads
  double h1r[6], udr[NV], qdr[NV];
  T m2r[NV];
  {
    const int ih = prow ? I : 0, iu = tv ? tt : 0, iq = prow ? I % NV : 0, im = hrow ? lane : 0;
#pragma unroll
    for (int e = 0; e < 6; ++e) h1r[e] = Dsrc.H1d[ih * 6 + e];
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      udr[k] = Dsrc.Ud[iu * NV + k];
      qdr[k] = Dsrc.Qd[iq * NV + k];
      m2r[k] = gM2[im * NV + k];
    }
  }
  if (prow) {
    // z = R (c - off): the basis reproduces constants, so shifting all
    // coefficients of a position shifts its curve
    const int b = axis * 2 + (I >= NV), kk = I % NV;
    const T *src = static_cast<const T *>(b == 0 ? Dsrc.cx : (b == 1 ? Dsrc.cc : (b == 2 ? Dsrc.cy : Dsrc.cs)));
    const double coff = (b == 0) ? offx : ((b == 2) ? offy : 0.0);
    // (the set-up loops run over all NV entries with the unused terms
    // selected away, so that each lane's loads are issued together; the
    // sums keep their order)
    double zz = 0.0;
#pragma unroll
    for (int j = 0; j < NV; ++j) {
      const double t = R[kk * NV + j] * (double(src[size_t(l) * NV + j]) - coff);
      zz += j >= kk ? t : 0.0;
    }
    zl = zz;
    vzd[axis * A2 + I] = zz;
    // (z itself goes through the dz copies for the first evaluation)
    put4(vdz, DZC, axis * A2 + (I / NV) * QS + I % NV, T(zz));
    // lambda_z = R^-T lambda
    const T *glam = static_cast<const T *>(Dsrc.lam);
    double lz = 0.0;
#pragma unroll
    for (int j = 0; j < NV; ++j) {
      const double t = Rinv[j * NV + kk] * double(glam[size_t(l) * 4 * NV + b * NV + j]);
      lz += j <= kk ? t : 0.0;
    }
    lam = lz;
  }
  if (hrow) {
    const int kk = lane;
    const T *H2 = static_cast<const T *>(Dsrc.H2);
    double hsum = 0.0;
#pragma unroll
    for (int e = 0; e < 6; ++e) hsum += double(H2[kk * 6 + e]) * Dsrc.bpsi[e];
    hpsi = T(hsum);
    const T *src = static_cast<const T *>(Dsrc.cpsi);
    double zz = 0.0;
#pragma unroll
    for (int j = 0; j < NV; ++j) {
      const double t = R[kk * NV + j] * double(src[size_t(l) * NV + j]);
      zz += j >= kk ? t : 0.0;
    }
    put4(vzpsi, ZPC, kk, T(zz));
    const T *glp = static_cast<const T *>(Dsrc.lampsi);
    double lz = 0.0;
#pragma unroll
    for (int j = 0; j < NV; ++j) {
      const double t = Rinv[j * NV + kk] * double(glp[size_t(l) * NV + j]);
      lz += j <= kk ? t : 0.0;
    }
    lampsi0 = T(lz);
    vaux[kk] = lampsi0;
  }
  wave_sync();
  // H1 (A z - b) of the given coefficients (centred positions)
  if (prow) {
    const double *bb = axis == 0 ? Dsrc.bx : Dsrc.by;
    const double off = axis == 0 ? offx : offy;
#pragma unroll
    for (int e = 0; e < 6; ++e) {
      double ae = 0.0;
#pragma unroll
      for (int k = 0; k < NV; ++k) ae += Dsrc.Abc[e * NV + k] * vzd[axis * A2 + k];
      const double be = (e == 0 || e == 3) ? bb[e] - off : bb[e];
      bcc += h1r[e] * (ae - be);
    }
  }
  // mu = M2 lambda_psi (heading rows)
  T mu = T(0);
  if (hrow) {
#pragma unroll
    for (int j = 0; j < NV; ++j) mu += m2r[j] * vaux[j];
  }
  wave_sync();

  // ---- per-lane trajectory values at t: positions (absolute, FP64) and
  // the other channels (T).  The positions are formed from the FP64
  // coefficients once and then carried: x' = x + U dz, the product of the
  // small update in T added in FP64.
  double xa = 0.0, ya = 0.0;
  if (tv) {
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      const double u = udr[k];
      xa += u * vzd[k];
      ya += u * vzd[A2 + k];
    }
  }
  xa += offx;
  ya += offy;
  T xd, xdd, cc, yd, ydd, ss, psi, cps, sps, psih;
  T racc = T(0);   // sum over the iterations of psi_sign (psi - psi_hat) at t

  // derivative and slack channels from the initial z (first call: z in the
  // dz copies), then every channel advanced by the product of the update dz
  // (its blocks QS apart in LDS, read in this lane's slot order), the
  // positions in FP64
  auto eval_xy = [&](bool step) {
    T a0 = 0, b0 = 0, a1 = 0, a2 = 0, a3 = 0, b1 = 0, b2 = 0, b3 = 0;
#pragma unroll
    for (int c = 0; c < NP / 4; ++c) {
      const Quad<T> dx = dzq[c], dc = dzq[QS / 4 + c], dy = dzq[A2 / 4 + c], ds = dzq[(A2 + QS) / 4 + c];
      const T *vx = &dx.a, *vc = &dc.a, *vy = &dy.a, *vs = &ds.a;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int k = 4 * c + e;
        a0 += Ub[k] * vx[e]; a1 += Vb[k] * vx[e]; a2 += Wb[k] * vx[e]; a3 += Ub[k] * vc[e];
        b0 += Ub[k] * vy[e]; b1 += Vb[k] * vy[e]; b2 += Wb[k] * vy[e]; b3 += Ub[k] * vs[e];
      }
    }
    if (!step) {
      xd = a1; xdd = a2; cc = a3;
      yd = b1; ydd = b2; ss = b3;
      return;
    }
    xa += double(a0);
    ya += double(b0);
    xd += a1; xdd += a2; cc += a3;
    yd += b1; ydd += b2; ss += b3;
  };
  // offset of this lane's robot centre from an obstacle centre, formed in
  // FP64 and rounded once
  auto off_x = [&](T ox) { return T(xa - double(ox)); };
  auto off_y = [&](T oy) { return T(ya - double(oy)); };
  auto eval_psi = [&]() {
    T p = 0;
#pragma unroll
    for (int c = 0; c < NP / 4; ++c) {
      const Quad<T> z = zpsiq[c];
      p += Ub[4 * c] * z.a;
      p += Ub[4 * c + 1] * z.b;
      p += Ub[4 * c + 2] * z.c;
      p += Ub[4 * c + 3] * z.d;
    }
    psi = p;
    T sn, cs;
    Num<T>::sincos_(p, &sn, &cs);
    cps = cs;
    sps = sn;
  };

  // Both waves' halves of one exchanged sum, added in a fixed order.
  auto exchange_sum = [&](int slot) -> T { return xch[slot] + xch[kXchHalf + slot]; };

  // Projection of one obstacle's rows at this lane's t for every circle
  // (fast form; a non-finite sum, as from a zero or subnormal r2, is redone
  // element by element afterwards).
  // p = (a^2, b^2, ab, max(a, b)) of the inflated ellipse.  The offset of
  // circle i from the obstacle centre is (xh - o.x) + (xl + r_i u): the
  // position split into its FP32 rounding xh and the remainder xl, so the
  // per-obstacle difference is one FP32 subtraction and the remainder joins
  // the circle offsets once per iteration (each part rounded once, as for
  // the FP64 difference).  MC > 0: exactly the first MC circle slots are
  // used (MC = m, a compile-time count), so the circle loop has no
  // per-circle test; MC = 0 tests every slot against m.  FIRST: the first
  // obstacle, whose terms start the sums.
  T Sx[C], Sy[C];
  T xh = T(0), yh = T(0), rxl[C], ryl[C];
  auto project_obstacle = [&](auto count, auto first, const Pair<T> o, const Quad<T> p) {
    constexpr int MC = decltype(count)::value;
    constexpr bool FIRST = decltype(first)::value;
    const T dxj = xh - o.x, dyj = yh - o.y;
#pragma unroll
    for (int i = 0; i < C; ++i) {
      if (MC > 0 ? i < MC : i < m) {
        const T xt = dxj + rxl[i], yt = dyj + ryl[i];
        const T r2 = p.b * xt * xt + p.a * yt * yt;   // b^2 x~^2 + a^2 y~^2
        const T f1 = fmax(T(0), p.c * Num<T>::rsqrt_fast(r2) - T(1));
        if constexpr (FIRST) {
          Sx[i] = xt * f1;
          Sy[i] = yt * f1;
        } else {
          Sx[i] += xt * f1;
          Sy[i] += yt * f1;
        }
      } else if constexpr (FIRST) {
        Sx[i] = T(0);
        Sy[i] = T(0);
      }
    }
  };
  // The near obstacles of the (non-empty) mask, each one's LDS data loaded
  // while the previous one is projected (two register sets in turn).
  auto project_near = [&](auto count, uint64_t mask) {
    int j = __builtin_ctzll(mask);
    mask &= mask - 1;
    Pair<T> o0 = oxy[j * q + tt], o1;
    Quad<T> p0 = opq[j * 2], p1;
    bool more = mask != 0;
    j = more ? __builtin_ctzll(mask) : j;
    mask &= mask - 1;
    o1 = oxy[j * q + tt];
    p1 = opq[j * 2];
    project_obstacle(count, std::true_type(), o0, p0);
    if (!more) return;
    while (true) {
      more = mask != 0;
      j = more ? __builtin_ctzll(mask) : j;
      mask &= mask - 1;
      o0 = oxy[j * q + tt];
      p0 = opq[j * 2];
      project_obstacle(count, std::false_type(), o1, p1);
      if (!more) break;
      more = mask != 0;
      j = more ? __builtin_ctzll(mask) : j;
      mask &= mask - 1;
      o1 = oxy[j * q + tt];
      p1 = opq[j * 2];
      project_obstacle(count, std::false_type(), o0, p0);
      if (!more) break;
    }
  };

  // ---- xi3/xi4 projection of every (circle, obstacle, t), velocity and
  // acceleration, then the per-wave partial sums of F^T (F xi - g) (4
  // blocks of NP rows), exchanged between the two waves; afterwards lane
  // (axis, I) of the position rows holds its row of the total in `tr`.
  // `rp` keeps this lane's heading residual psi_sign (psi - psi_hat) for
  // the next heading step.
  T tr = T(0), rp = T(0);
  // near-obstacle set of the last vote and the positions it was taken at
  T xvote = T(0), yvote = T(0), extvote = T(0);
  uint64_t near_set = 0;
  bool voted = false;
  auto project_reduce = [&](bool with_psi) {
    const T ux = slack ? cc : cps, uy = slack ? ss : sps;
    const T x = T(xa), y = T(ya);   // for the vote and the projection
    if (!literal_alpha) {
      // Wave-wide vote: obstacles within ext + max(a, b) + margin of some
      // lane's robot centre, ext = max|r_i| |u| the reach of its circles.
      // The set stays valid while every lane has moved by less than the
      // margin minus any growth of ext since the vote (an obstacle outside
      // it is then still farther than ext + max(a, b), where every circle
      // is outside the ellipse and contributes exactly zero), so the vote
      // is repeated only when some lane has moved that far.  The positions
      // of a chunk of obstacles are loaded before any is tested.
      // (|u| from the hardware square root, enlarged by 1e-6 so that the
      // rounding of the estimate cannot make ext too small)
      const T ext = rmax * Num<T>::sqrt_fast(ux * ux + uy * uy) * T(1.000001);
      const T margin = T(kVoteMargin);
      const T dxv = x - xvote, dyv = y - yvote, room = margin - (ext - extvote);
      const bool stale = tv & !(room > T(0) && dxv * dxv + dyv * dyv <= room * room);
      if (!voted || __ballot(stale) != 0) {
        voted = true;
        xvote = x;
        yvote = y;
        extvote = ext;
        near_set = 0;
        for (int j0 = 0; j0 < n; j0 += kVoteChunk) {
          Pair<T> o[kVoteChunk];
          T am[kVoteChunk];
#pragma unroll
          for (int k = 0; k < kVoteChunk; ++k) {
            if (j0 + k >= n) break;   // padding of the last chunk
            o[k] = oxy[(j0 + k) * q + tt];
            am[k] = op[(j0 + k) * 8 + OP_AMAX];
          }
#pragma unroll
          for (int k = 0; k < kVoteChunk; ++k) {
            if (j0 + k >= n) break;   // padding of the last chunk
            const T dx = x - o[k].x, dy = y - o[k].y;
            const T reach = ext + am[k] + margin;
            const bool near = tv & (dx * dx + dy * dy < reach * reach);
            if (__ballot(near) != 0) near_set |= uint64_t(1) << (j0 + k);
          }
        }
      }
      // active obstacles
      if (near_set) {
        xh = x;
        yh = y;
        const T xl = T(xa - double(xh)), yl = T(ya - double(yh));
#pragma unroll
        for (int i = 0; i < C; ++i) {
          rxl[i] = xl + rr[i] * ux;
          ryl[i] = yl + rr[i] * uy;
        }
        // exact circle counts for m = C, C - 1 and C - 2 (robots of 3 to 5
        // circles with C = 5), the tested form otherwise
        if (m == C) project_near(std::integral_constant<int, C>(), near_set);
        else if (C > 1 && m == C - 1) project_near(std::integral_constant<int, (C > 1 ? C - 1 : 0)>(), near_set);
        else if (C > 2 && m == C - 2) project_near(std::integral_constant<int, (C > 2 ? C - 2 : 0)>(), near_set);
        else project_near(std::integral_constant<int, 0>(), near_set);
      } else {
#pragma unroll
        for (int i = 0; i < C; ++i) { Sx[i] = T(0); Sy[i] = T(0); }
      }
    } else {
#pragma unroll
      for (int i = 0; i < C; ++i) { Sx[i] = T(0); Sy[i] = T(0); }
      for (int j = 0; j < n; ++j) {
        const Pair<T> o = oxy[j * q + tt];
        const T a = op[j * 8 + OP_A], b = op[j * 8 + OP_B];
        const T a2 = op[j * 8 + OP_A2], b2 = op[j * 8 + OP_B2];
#pragma unroll
        for (int i = 0; i < C; ++i) {
          if (i < m) {
            const T xt = off_x(o.x) + rr[i] * ux, yt = off_y(o.y) + rr[i] * uy;
            const T xx = xt * xt, yy = yt * yt;
            const T kap = fmax(Num<T>::rsqrt(xx + yy), (a * xx + b * yy) / (a2 * xx + b2 * yy));
            Sx[i] += xt * (a * kap - T(1));
            Sy[i] += yt * (b * kap - T(1));
          }
        }
      }
    }
    T Dx = 0, Dy = 0, DRx = 0, DRy = 0;
    auto sum_circles = [&]() {
      Dx = Sx[0]; Dy = Sy[0];
      DRx = rr[0] * Sx[0]; DRy = rr[0] * Sy[0];
#pragma unroll
      for (int i = 1; i < C; ++i) {
        Dx += Sx[i]; Dy += Sy[i];
        DRx += rr[i] * Sx[i]; DRy += rr[i] * Sy[i];
      }
    };
    sum_circles();
    // Exact zero (or underflowed) offsets make the fast form non-finite, and
    // a non-finite term of any circle makes Dx or Dy non-finite: then redo
    // those circles' sums element by element (alpha := 0 at the zero vector).
    if (__ballot(!(isfinite(Dx) && isfinite(Dy))) != 0) {
#pragma unroll
      for (int i = 0; i < C; ++i) {
        if (i < m && !(isfinite(Sx[i]) && isfinite(Sy[i]))) {
          T sx = T(0), sy = T(0);
          for (int j = 0; j < n; ++j) {
            const Pair<T> o = oxy[j * q + tt];
            const T xt = off_x(o.x) + rr[i] * ux, yt = off_y(o.y) + rr[i] * uy;
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
      sum_circles();
    }
    // velocity / acceleration: part of (xdot, ydot) outside the disc
    // (a zero or subnormal speed gives 1/sqrt = +inf and a factor of 0)
    const T fv = fmax(T(0), T(1) - vmax * Num<T>::rsqrt_fast(xd * xd + yd * yd));
    const T fa = fmax(T(0), T(1) - amax * Num<T>::rsqrt_fast(xdd * xdd + ydd * ydd));
    const T rvx = xd * fv, rvy = yd * fv, rax = xdd * fa, ray = ydd * fa;
    const T dc = cc - cps, ds = ss - sps;
    const T k1 = slack ? T(0) : s1, k2 = (slack ? T(0) : s2) + T(1);
    const T ro1x = k1 * dc - Dx, ro2x = k2 * dc - DRx;
    const T ro1y = k1 * ds - Dy, ro2y = k2 * ds - DRy;
    rp = with_psi ? psi_sign * (psi - psih) : T(0);
    racc += rp;
    // partials of F^T (F xi - g) (x: rows 0..2nv-1, y: 2nv..4nv-1, as
    // [V W U] on the position block and U on the slack block)
    // (the velocity and acceleration rows are usually inside their discs on
    // every lane of the wave; their terms are then zero and are left out)
    // (blocks of NP rows, in this lane's slot order)
    T pr[G];
    if (__ballot((fv > T(0)) | (fa > T(0))) != 0) {
#pragma unroll
      for (int k = 0; k < NP; ++k) {
        pr[k] = Vb[k] * rvx + Wb[k] * rax + Ub[k] * ro1x;
        pr[2 * NP + k] = Vb[k] * rvy + Wb[k] * ray + Ub[k] * ro1y;
      }
    } else {
#pragma unroll
      for (int k = 0; k < NP; ++k) {
        pr[k] = Ub[k] * ro1x;
        pr[2 * NP + k] = Ub[k] * ro1y;
      }
    }
#pragma unroll
    for (int k = 0; k < NP; ++k) {
      pr[NP + k] = Ub[k] * ro2x;
      pr[3 * NP + k] = Ub[k] * ro2y;
    }
    // the reduction and exchange are the pair's critical path: while a wave
    // is in them the SIMD issues its instructions first
    __builtin_amdgcn_s_setprio(2);
    const T tot = wave_sum_perm<T, G, RED>(pr, red, lane);
    if (lane < G) xmine[lane] = tot;
    __syncthreads();
    if (prow) tr = exchange_sum((lane / NV) * NP + lane % NV);
    __builtin_amdgcn_s_setprio(0);
  };

  // ---- step 1 of the AM list: initial xi3, xi4 from the given trajectory
  eval_xy(false);
  eval_psi();
  psih = psi;
  // row I of M1 (position block) in registers for the whole solve (WAVES =
  // 2 budget; the three-wavefront build reads it from LDS in every product)
  constexpr int M1Q = pad4(N2) / 4;
  Quad<T> m1r[RED == kRedRows ? M1Q : 1];
  if constexpr (RED == kRedRows) {
    const Quad<T> *o = reinterpret_cast<const Quad<T> *>(M1);
#pragma unroll
    for (int c = 0; c < M1Q; ++c) m1r[c] = o[c * N2 + I];
  }
  auto m1_dot = [&](const T *v) -> T {
    if constexpr (RED == kRedRows) {
      const Quad<T> *vv = reinterpret_cast<const Quad<T> *>(v);
      T acc0 = T(0), acc1 = T(0);
#pragma unroll
      for (int c = 0; c < M1Q; ++c) {
        const Quad<T> x = vv[c];
        acc0 += m1r[c].a * x.a;
        acc1 += m1r[c].b * x.b;
        if (4 * c + 2 < N2) acc0 += m1r[c].c * x.c;
        if (4 * c + 3 < N2) acc1 += m1r[c].d * x.d;
      }
      return acc0 + acc1;
    } else {
      return row_dot<T, NV>(M1, I, v);
    }
  };
  // row I of Q = blockdiag(W^T W, W^T W or 0) times the block of dz it
  // meets (dz is stored with its blocks QS apart; the padding reads zero)
  const int qb = I / NV, qi = I - qb * NV;
  // (in registers under the two-wavefront budget, like the M1 row)
  Quad<T> qr[RED == kRedRows ? QS / 4 : 1];
  if constexpr (RED == kRedRows) {
    const Quad<T> *o = reinterpret_cast<const Quad<T> *>(QL + (qb * NV + qi) * QS);
#pragma unroll
    for (int c = 0; c < QS / 4; ++c) qr[c] = o[c];
  }
  auto q_dot = [&]() {
    const Quad<T> *o = reinterpret_cast<const Quad<T> *>(QL + (qb * NV + qi) * QS);
    const Quad<T> *v = reinterpret_cast<const Quad<T> *>(vdz + axis * A2 + qb * QS);
    T acc0 = T(0), acc1 = T(0);
#pragma unroll
    for (int c = 0; c < QS / 4; ++c) {
      Quad<T> a;
      if constexpr (RED == kRedRows) a = qr[c];
      else a = o[c];
      const Quad<T> b = v[c];
      acc0 += a.a * b.a;
      acc1 += a.b * b.b;
      acc0 += a.c * b.c;
      acc1 += a.d * b.d;
    }
    return acc0 + acc1;
  };
  // Q z, formed once in FP64 and then carried: Q z' = Q z + Q dz
  double qz = 0.0;
  if (prow && (qb == 0 || !(flags & AM_Q_CS_ZERO))) {
#pragma unroll
    for (int k = 0; k < NV; ++k) qz += qdr[k] * vzd[axis * A2 + qb * NV + k];
  }
  project_reduce(false);
  if (prow) vw[axis * A2 + I] = T((lam - rhod * double(tr)) - qz);
  wave_sync();
  // heading coefficients before the first step's sum: h_psi + M2 lambda_psi
  double zpsi_d = double(hpsi) + double(mu);
  T psih_prev = T(0);

  for (int it = 0; it < K; ++it) {
    // ---- xi1 (eqs. over_3, zeta_1_sepration_3) as an update of z:
    // z' = z - H1 (A z - b) + M1 (lambda - rho F^T (F xi - g) - Q z)
    // (every lane computes; lanes past the position rows compute a copy of
    // row 0 and store nothing)
    const double dz = double(m1_dot(vw + axis * A2)) - bcc;
    bcc = 0.0;
    zl += dz;
    if (prow) put4(vdz, DZC, axis * A2 + qb * QS + qi, T(dz));
    wave_sync();
    eval_xy(true);

    // ---- xi2: psi_hat = atan2(s, c) on the branch nearest psi^k, then the
    // heading QP (eq. compute_convex_surrogate) with the multiplier update
    // of the previous iteration folded in:
    // z_psi += U~^T (rho (psi_hat' - psi_hat) - rho_psi psi_sign (psi - psi_hat))
    T dpsi;
    {
      T ph;
      if (unwrap) ph = psi + atan2z(ss * cps - cc * sps, cc * cps + ss * sps);
      else ph = atan2z(ss, cc);
      const T pnew = tv ? ph : T(0);
      dpsi = rho * (pnew - psih_prev) - rhop * rp;
      psih_prev = pnew;
      psih = pnew;
    }
    T pp[NP];
#pragma unroll
    for (int k = 0; k < NP; ++k) pp[k] = Ut[k] * dpsi;
    __builtin_amdgcn_s_setprio(2);
    const T upsi = wave_sum_perm<T, NP, RED>(pp, red, lane);
    if (lane < NV) xmine[kXchBig + lane] = upsi;
    __syncthreads();
    if (hrow) {
      zpsi_d += double(exchange_sum(kXchBig + lane));
      put4(vzpsi, ZPC, lane, T(zpsi_d));
    }
    __builtin_amdgcn_s_setprio(0);
    wave_sync();
    eval_psi();

    // Q z of the new z, for the next update's right-hand side
    qz += double(q_dot());

    // ---- xi3, xi4 and the multipliers (eqs. update_lambda_1, update_lambda_psi)
    project_reduce(true);
    if (prow) {
      lam -= rhod * double(tr);
      vw[axis * A2 + I] = T((lam - rhod * double(tr)) - qz);
    }
    wave_sync();
  }

  // ---- lambda_psi = lambda_psi(0) - rho_psi U^T (sum of psi - psi_hat)
  {
    T pp[NP];
#pragma unroll
    for (int k = 0; k < NP; ++k) pp[k] = Ub[k] * racc;
    const T s = wave_sum_perm<T, NP, RED>(pp, red, lane);
    if (lane < NV) xmine[kXchBig + lane] = s;
    __syncthreads();
    if (hrow) vaux[2 * A2 + lane] = lampsi0 - rhop * exchange_sum(kXchBig + lane);
    if (prow) {
      vzd[axis * A2 + I] = zl;
      vwd[axis * A2 + I] = lam;
    }
    wave_sync();
  }

  // ---- residual statistics of the final state (am_residuals' columns), on
  // request: every (circle, obstacle) at this lane's t, the velocity and
  // acceleration discs, the slack pair, the boundary rows and the cost,
  // reduced over the lanes and the pair (every wave of the block takes part:
  // the exchange has a block barrier)
  if (Dsrc.res) {
    constexpr int NS = 10;
    T fc2 = T(0), fcsq = T(0), lvl2 = T(INFINITY), v2 = T(0), a2 = T(0), slk = T(0), head = T(0), bc = T(0),
      cost = T(0);
    int bad = 0;
    if (tv) {
      for (int j = 0; j < n; ++j) {
        const Pair<T> o = oxy[j * q + t];
        const T a = op[j * 8 + OP_A], b = op[j * 8 + OP_B];
        const T aa = op[j * 8 + OP_A2], bb = op[j * 8 + OP_B2], ab = op[j * 8 + OP_AB];
        const T iaa = op[j * 8 + OP_IA2], ibb = op[j * 8 + OP_IB2];
        const T dxj = off_x(o.x), dyj = off_y(o.y);
#pragma unroll
        for (int i = 0; i < C; ++i) {
          if (i >= m) break;
          const T px = dxj + rr[i] * cps, py = dyj + rr[i] * sps;   // circle centre - obstacle
          const T xt = slack ? dxj + rr[i] * cc : px, yt = slack ? dyj + rr[i] * ss : py;
          T fx, fy;
          if (!literal_alpha) {
            // (a d cos al, b d sin al) = (xt, yt) max(1, ab/r), r = |(b xt, a yt)|;
            // the zero vector (r^2 below the smallest normal) has al = 0, d = 1
            const T r2 = bb * xt * xt + aa * yt * yt;
            const bool zero = !(r2 >= std::numeric_limits<T>::min());
            const T g = zero ? T(1) : fmax(T(1), ab * Num<T>::rsqrt_fast(r2));
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
          fc2 = fmax(fc2, f2);
          fcsq += f2;
          lvl2 = fmin(lvl2, px * px * iaa + py * py * ibb);
        }
      }
      T psd = T(0), psdd = T(0);
#pragma unroll
      for (int c = 0; c < NP / 4; ++c) {
        const Quad<T> z = zpsiq[c];
        const T *zv = &z.a;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          psd += Vb[4 * c + e] * zv[e];
          psdd += Wb[4 * c + e] * zv[e];
        }
      }
      v2 = xd * xd + yd * yd;
      a2 = xdd * xdd + ydd * ydd;
      slk = fmax(fabs(cc - cps), fabs(ss - sps));
      const T pi = T(3.14159265358979323846);
      T dh = atan2z(ss, cc) - psi;
      dh = dh - T(2) * pi * floor((dh + pi) / (T(2) * pi));
      head = fabs(dh);
      cost = xdd * xdd + ydd * ydd + psdd * psdd;
      if (t == 0 || t == q - 1) {
        const int o = t == 0 ? 0 : 3;
        const double vx[3] = {xa, double(xd), double(xdd)}, vy[3] = {ya, double(yd), double(ydd)};
        const double vp[3] = {double(psi), double(psd), double(psdd)};
        for (int e = 0; e < 3; ++e) {
          bc = fmax(bc, T(fabs(vx[e] - Dsrc.bx[o + e])));
          bc = fmax(bc, T(fabs(vy[e] - Dsrc.by[o + e])));
          bc = fmax(bc, T(fabs(vp[e] - Dsrc.bpsi[o + e])));
        }
      }
      bad = !isfinite(xa) || !isfinite(ya) || !isfinite(psi);
    }
    if (prow) bad |= !isfinite(zl) || !isfinite(lam);
    if (hrow) bad |= !isfinite(vzpsi[lane]) || !isfinite(vaux[2 * A2 + lane]);
    auto wmax = [](T v) { return wave_all(v, T(0), [](T a, T b) { return fmax(a, b); }); };   // v >= 0
    auto wmin = [](T v) { return wave_all(v, T(INFINITY), [](T a, T b) { return fmin(a, b); }); };
    auto wadd = [](T v) { return wave_all(v, T(0), [](T a, T b) { return a + b; }); };
    T stv[NS] = {wmax(T(bad ? 1 : 0)), wmax(fc2), wadd(fcsq), wmin(lvl2), wmax(v2), wmax(a2), wmax(slk),
                 wmax(head), wmax(bc), wadd(cost)};
    if (lane == 0) {
#pragma unroll
      for (int k = 0; k < NS; ++k) xmine[k] = stv[k];
    }
    __syncthreads();
    if (live && half == 0 && lane == 0) {
      const T *ot = xch + kXchHalf;   // the partner's statistics
      const T fbad = fmax(stv[0], ot[0]), fcmax = Num<T>::sqrt_(fmax(stv[1], ot[1]));
      const T fcs = stv[2] + ot[2], level = Num<T>::sqrt_(fmin(stv[3], ot[3])) - T(1);
      const T vex = Num<T>::sqrt_(fmax(stv[4], ot[4])) - vmax, aex = Num<T>::sqrt_(fmax(stv[5], ot[5])) - amax;
      T *o = static_cast<T *>(Dsrc.res) + size_t(l) * AM_NRES;
      const int mnq = m * n * q;
      o[AM_RES_FC_MAX] = fcmax;
      o[AM_RES_FC_RMS] = mnq ? Num<T>::sqrt_(fcs / T(mnq)) : T(0);
      o[AM_RES_FV_MAX] = fmax(T(0), vex);
      o[AM_RES_FA_MAX] = fmax(T(0), aex);
      o[AM_RES_SLACK_MAX] = fmax(stv[6], ot[6]);
      o[AM_RES_HEADING_MAX] = fmax(stv[7], ot[7]);
      o[AM_RES_BC_MAX] = fmax(stv[8], ot[8]);
      o[AM_RES_COST] = stv[9] + ot[9];
      o[AM_RES_CLEAR_LEVEL] = mnq ? level : T(INFINITY);
      o[AM_RES_V_EXCESS] = vex;
      o[AM_RES_A_EXCESS] = aex;
      o[AM_RES_NONFINITE] = fbad;
    }
  }

  if (!live) return;   // padding trajectory of a ragged last block

  // ---- state back to Bernstein coordinates (written by the first half)
  if (half == 0) {
    if (prow) {
      const int b = axis * 2 + (I >= NV), kk = I % NV;
      T *dst = static_cast<T *>(b == 0 ? Dsrc.cx : (b == 1 ? Dsrc.cc : (b == 2 ? Dsrc.cy : Dsrc.cs)));
      const double coff = (b == 0) ? offx : ((b == 2) ? offy : 0.0);
      const int base = axis * A2 + (I >= NV ? NV : 0);
      double c = 0.0, lc = 0.0;
#pragma unroll
      for (int j = 0; j < NV; ++j) {
        const double t = Rinv[kk * NV + j] * vzd[base + j], u = R[j * NV + kk] * vwd[base + j];
        c += j >= kk ? t : 0.0;
        lc += j <= kk ? u : 0.0;
      }
      dst[size_t(l) * NV + kk] = T(c + coff);
      static_cast<T *>(Dsrc.lam)[size_t(l) * 4 * NV + b * NV + kk] = T(lc);
    }
    if (hrow) {
      const int kk = lane;
      double c = 0.0, lc = 0.0;
#pragma unroll
      for (int j = 0; j < NV; ++j) {
        const double t = Rinv[kk * NV + j] * double(vzpsi[j]), u = R[j * NV + kk] * double(vaux[2 * A2 + j]);
        c += j >= kk ? t : 0.0;
        lc += j <= kk ? u : 0.0;
      }
      static_cast<T *>(Dsrc.cpsi)[size_t(l) * NV + kk] = T(c);
      static_cast<T *>(Dsrc.lampsi)[size_t(l) * NV + kk] = T(lc);
    }
  }
  if (!tv) return;

  // ---- optional outputs: trajectory and the final (alpha, d) of xi3/xi4
  if (Dsrc.traj) {
    T *trj = static_cast<T *>(Dsrc.traj) + size_t(l) * 3 * q;
    trj[t] = T(xa);
    trj[q + t] = T(ya);
    trj[2 * q + t] = psi;
  }
  if (Dsrc.va) {
    T *va = static_cast<T *>(Dsrc.va) + size_t(l) * 4 * q;
    const T av = atan2z(yd, xd), aa = atan2z(ydd, xdd);
    const T dv = (xd * Num<T>::cos_(av) + yd * Num<T>::sin_(av)) / vmax;
    const T da = (xdd * Num<T>::cos_(aa) + ydd * Num<T>::sin_(aa)) / amax;
    va[t] = av;
    va[q + t] = fmin(T(1), fmax(T(0), dv));
    va[2 * q + t] = aa;
    va[3 * q + t] = fmin(T(1), fmax(T(0), da));
  }
  if (Dsrc.alpha || Dsrc.d) {
    T *ga = static_cast<T *>(Dsrc.alpha), *gd = static_cast<T *>(Dsrc.d);
    const size_t base = size_t(l) * m * n * q;
    const T ux = slack ? cc : cps, uy = slack ? ss : sps;
    for (int i = 0; i < m; ++i)
      for (int j = 0; j < n; ++j) {
        const Pair<T> o = oxy[j * q + t];
        const T xt = off_x(o.x) + rr[i] * ux;
        const T yt = off_y(o.y) + rr[i] * uy;
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

// One block: LDS set-up shared by the block's trajectories, then the loop.
template <typename T, int NV, int C, int TILE, int WAVES>
__device__ __forceinline__ void fused_block(const Desc &D) {
  constexpr int RED = red_rows_for(WAVES);
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T *lds = reinterpret_cast<T *>(smem_raw);
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
  const int q = uni(D.q), n = uni(D.n), B = uni(D.B), blk0 = uni(D.blk0);
  const FusedLds L = fused_layout(q, n, NV, TILE, RED, int(sizeof(double) / sizeof(T)));
  constexpr int N2 = 2 * NV, A2 = pad4(N2);

  // block-wide: obstacle tables ((x, y) pairs), inflated semi-axes,
  // operators as Quad [a2/4][2nv], zeroed per-wave areas (their padding
  // entries are read as zeros)
  const T *gox = static_cast<const T *>(D.ox), *goy = static_cast<const T *>(D.oy);
  const T rc = T(D.rc);
  Pair<T> *oxy = reinterpret_cast<Pair<T> *>(lds + L.oxy);
  for (int i = tid; i < n * q; i += blockDim.x) oxy[i] = Pair<T>{gox[i], goy[i]};
  for (int j = tid; j < n; j += blockDim.x) {
    const T a = static_cast<const T *>(D.oa)[j] + rc;
    const T b = static_cast<const T *>(D.ob)[j] + rc;
    T *o = lds + L.op + j * 8;
    o[OP_A2] = a * a; o[OP_B2] = b * b; o[OP_AB] = a * b; o[OP_AMAX] = fmax(a, b);
    o[OP_A] = a; o[OP_B] = b; o[OP_IA2] = T(1) / (a * a); o[OP_IB2] = T(1) / (b * b);
  }
  const T *gM1 = static_cast<const T *>(D.M1);
  for (int e = tid; e < A2 * N2; e += blockDim.x) {
    // element e of the Quad layout: chunk c, row I, component e % 4
    const int c = e / (4 * N2), rem = e % (4 * N2), I = rem / 4, J = 4 * c + rem % 4;
    lds[L.m1 + e] = J < N2 ? gM1[I * N2 + J] : T(0);
  }
  // Q rows: [block][row][pad4(nv)], the slack block zero under AM_Q_CS_ZERO
  {
    constexpr int QS = pad4(NV);
    const bool qcs = !(uni(D.flags) & AM_Q_CS_ZERO);
    for (int e = tid; e < 2 * NV * QS; e += blockDim.x) {
      const int bq = e / (NV * QS), rem = e % (NV * QS), i = rem / QS, k = rem % QS;
      lds[L.qrows + e] = (k < NV && (bq == 0 || qcs)) ? T(D.Qd[i * NV + k]) : T(0);
    }
  }
  // (the reduction scratch at the end of each wave's area is written before
  // it is read and is left as it is)
  {
    const int zero_len = wave_layout(NV, RED, int(sizeof(double) / sizeof(T))).red;
    for (int i = tid; i < 2 * TILE * zero_len; i += blockDim.x) {
      const int w = i / zero_len;
      lds[L.wave0 + w * L.wave_stride + (i - w * zero_len)] = T(0);
    }
  }
  __syncthreads();

  // Every trajectory slot of the block runs the loop (it has block-wide
  // barriers); a slot past the end of the batch computes a copy of the last
  // trajectory and stores nothing.
  const int lt = (int(blockIdx.x) - blk0) * TILE + (wave >> 1);
  const bool live = lt < B;
  fused_body<T, NV, C, RED>(D, live ? lt : B - 1, live, wave & 1, lds, L, lane, wave);
}

// One problem: the descriptor travels as a kernel argument.  WAVES is the
// register budget: at least that many wavefronts per SIMD (1: up to 512
// VGPRs and AGPRs, 2: up to 256, 3: up to 168).
template <typename T, int NV, int C, int TILE, int WAVES>
__global__ __launch_bounds__(kWave * 2 * TILE) __attribute__((amdgpu_waves_per_eu(WAVES)))
void fused_kernel(Desc single) {
  fused_block<T, NV, C, TILE, WAVES>(single);
}

// Several problems: block b belongs to the last problem whose first block is
// <= b (binary search of the table in global memory).
template <typename T, int NV, int C, int TILE, int WAVES>
__global__ __launch_bounds__(kWave * 2 * TILE) __attribute__((amdgpu_waves_per_eu(WAVES)))
void fused_multi_kernel(const Desc *__restrict__ table, int nprob) {
  int lo = 0, hi = nprob - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (uni(table[mid].blk0) <= int(blockIdx.x)) lo = mid; else hi = mid - 1;
  }
  fused_block<T, NV, C, TILE, WAVES>(table[uni(lo)]);
}

template <typename T, int NV, int C, int TILE, int WAVES>
hipError_t launch_t(const Desc &single, const Desc *table, int nprob, int nblocks, hipStream_t st,
                    size_t lds_bytes) {
  const void *fn = table ? reinterpret_cast<const void *>(&fused_multi_kernel<T, NV, C, TILE, WAVES>)
                         : reinterpret_cast<const void *>(&fused_kernel<T, NV, C, TILE, WAVES>);
  if (lds_bytes > 65536) {
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, int(lds_bytes));
    if (e != hipSuccess) return e;
  }
  if (table)
    hipLaunchKernelGGL((fused_multi_kernel<T, NV, C, TILE, WAVES>), dim3(nblocks), dim3(kWave * 2 * TILE),
                       lds_bytes, st, table, nprob);
  else
    hipLaunchKernelGGL((fused_kernel<T, NV, C, TILE, WAVES>), dim3(nblocks), dim3(kWave * 2 * TILE), lds_bytes,
                       st, single);
  return hipGetLastError();
}

template <typename T, int NV, int C, int WAVES>
hipError_t launch_tile(const Desc &single, const Desc *table, int nprob, int nblocks, hipStream_t st,
                       size_t lds_bytes, int tile) {
  switch (tile) {
    case 1: return launch_t<T, NV, C, 1, WAVES>(single, table, nprob, nblocks, st, lds_bytes);
    case 2: return launch_t<T, NV, C, 2, WAVES>(single, table, nprob, nblocks, st, lds_bytes);
    case 4: return launch_t<T, NV, C, 4, WAVES>(single, table, nprob, nblocks, st, lds_bytes);
    default: return hipErrorInvalidValue;
  }
}

// FP32: the small circle capacity when every problem of the launch fits it.
template <int NV, int WAVES>
hipError_t launch_f32(const Desc &single, const Desc *table, int nprob, int nblocks, hipStream_t st,
                      size_t lds_bytes, int tile, int max_m) {
  if (max_m <= kSmallC)
    return launch_tile<float, NV, kSmallC, WAVES>(single, table, nprob, nblocks, st, lds_bytes, tile);
  return launch_tile<float, NV, AM_MAX_CIRCLES, WAVES>(single, table, nprob, nblocks, st, lds_bytes, tile);
}

}  // namespace

size_t fused_lds_bytes(int q, int n, int nv, bool f64, int tile, int waves) {
  return size_t(fused_layout(q, n, nv, tile, red_rows_for(waves), f64 ? 1 : 2).total) * (f64 ? 8 : 4);
}

// FP64 kernels take the default budget only, built without a wavefront
// target (their registers do not fit 256 without spilling).
hipError_t launch_fused(const Desc &single, const Desc *table, int nprob, int nblocks, bool f64,
                        int nv, int max_m, hipStream_t st, size_t lds_bytes, int tile, int waves) {
  if (nblocks <= 0) return hipSuccess;
  if (max_m < 1 || max_m > AM_MAX_CIRCLES) return hipErrorInvalidValue;
  constexpr int MC = AM_MAX_CIRCLES;
  if (f64) {
    if (waves != 2) return hipErrorInvalidValue;
    if (nv == 11) return launch_tile<double, 11, MC, 1>(single, table, nprob, nblocks, st, lds_bytes, tile);
    if (nv == 8) return launch_tile<double, 8, MC, 1>(single, table, nprob, nblocks, st, lds_bytes, tile);
  } else if (waves == 2) {
    if (nv == 11) return launch_f32<11, 2>(single, table, nprob, nblocks, st, lds_bytes, tile, max_m);
    if (nv == 8) return launch_f32<8, 2>(single, table, nprob, nblocks, st, lds_bytes, tile, max_m);
  } else if (waves == 3) {
    if (nv == 11) return launch_f32<11, 3>(single, table, nprob, nblocks, st, lds_bytes, tile, max_m);
    if (nv == 8) return launch_f32<8, 3>(single, table, nprob, nblocks, st, lds_bytes, tile, max_m);
  }
  return hipErrorInvalidValue;
}

}  // namespace amk
