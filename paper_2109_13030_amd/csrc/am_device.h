// am_device.h -- device helpers shared by the iteration kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "am_internal.h"
#include "am_poly.h"

namespace amk {

template <typename T>
struct Num;

// FP32 atan2 and sincos written for the iteration kernels (fewer
// instructions than the general library routines, which also handle huge
// arguments).  The coefficients (am_poly.h) are near-minimax fits made by
// paper_2109_13030_amd/gen_poly.py (Lawson's iteratively reweighted least
// squares on dense grids, rounded to FP32):
//  * atan(r) = r P(r^2) on [0, 1], P of degree 8, then the octant fix-ups
//    atan2 = pi/2 - atan(1/r), pi - ... and the sign of y; within 3.2e-7 rad
//    with an exact reciprocal, 3.7e-7 rad with the hardware reciprocal's
//    one unit in the last place;
//  * sin r = r + r^3 S(r^2), cos r = 1 - r^2/2 + r^4 C(r^2) on [-pi/4, pi/4],
//    S and C of degree 3, after a two-constant Cody-Waite reduction by
//    pi/2 with fused multiply-adds; within 1e-7 for |a| <= 1e3.
// tests/test_poly.py checks both bounds with an FP32 emulation.
// The zero vector is handled by atan2z, not here.
__device__ __forceinline__ float atan2_f32(float y, float x) {
  const float ax = fabsf(x), ay = fabsf(y);
  const float mx = fmaxf(ax, ay), mn = fminf(ax, ay);
  const float r = mn * __builtin_amdgcn_rcpf(mx), u = r * r;
  float p = kAtanP[0];
#pragma unroll
  for (int i = 1; i < 9; ++i) p = fmaf(p, u, kAtanP[i]);
  float a = r * p;
  a = ay > ax ? kHalfPi - a : a;
  a = x < 0.0f ? kPi - a : a;
  return copysignf(a, y);
}

__device__ __forceinline__ void sincos_f32(float a, float *s, float *c) {
  const float k = rintf(a * kTwoOverPi);                     // nearest multiple of pi/2
  float r = fmaf(-k, kHalfPiHi, a);                          // pi/2 = hi + lo
  r = fmaf(-k, kHalfPiLo, r);
  const float u = r * r;
  float ps = kSinS[0];
#pragma unroll
  for (int i = 1; i < 4; ++i) ps = fmaf(ps, u, kSinS[i]);
  const float sr = fmaf(r * u, ps, r);
  float pc = kCosC[0];
#pragma unroll
  for (int i = 1; i < 4; ++i) pc = fmaf(pc, u, kCosC[i]);
  const float cr = fmaf(u * u, pc, fmaf(-0.5f, u, 1.0f));
  const int qd = int(k) & 3;                                 // quadrant of a
  const float s0 = (qd & 1) ? cr : sr, c0 = (qd & 1) ? sr : cr;
  *s = (qd & 2) ? -s0 : s0;
  *c = ((qd + 1) & 2) ? -c0 : c0;
}

template <>
struct Num<float> {
  static __device__ __forceinline__ float rsqrt(float x) { return rsqrtf(x); }
  // hardware reciprocal square root (about 1 ulp) without the rescaling of
  // subnormal arguments: a zero or subnormal argument may give +inf, which
  // callers must tolerate
  static __device__ __forceinline__ float rsqrt_fast(float x) { return __builtin_amdgcn_rsqf(x); }
  static __device__ __forceinline__ float sqrt_(float x) { return sqrtf(x); }
  // hardware square root (about 1 ulp), for bounds that tolerate it
  static __device__ __forceinline__ float sqrt_fast(float x) { return __builtin_amdgcn_sqrtf(x); }
  static __device__ __forceinline__ float atan2_(float y, float x) { return atan2_f32(y, x); }
  static __device__ __forceinline__ void sincos_(float a, float *s, float *c) { sincos_f32(a, s, c); }
  static __device__ __forceinline__ float hypot_(float a, float b) { return hypotf(a, b); }
  static __device__ __forceinline__ float cos_(float a) { return cosf(a); }
  static __device__ __forceinline__ float sin_(float a) { return sinf(a); }
};

template <>
struct Num<double> {
  static __device__ __forceinline__ double rsqrt(double x) { return 1.0 / ::sqrt(x); }
  static __device__ __forceinline__ double rsqrt_fast(double x) { return 1.0 / ::sqrt(x); }
  static __device__ __forceinline__ double sqrt_(double x) { return ::sqrt(x); }
  static __device__ __forceinline__ double sqrt_fast(double x) { return ::sqrt(x); }
  static __device__ __forceinline__ double atan2_(double y, double x) { return ::atan2(y, x); }
  static __device__ __forceinline__ void sincos_(double a, double *s, double *c) { ::sincos(a, s, c); }
  static __device__ __forceinline__ double hypot_(double a, double b) { return ::hypot(a, b); }
  static __device__ __forceinline__ double cos_(double a) { return ::cos(a); }
  static __device__ __forceinline__ double sin_(double a) { return ::sin(a); }
};

// atan2 with the value 0 for the zero vector (the angle of a zero vector is
// not defined by the paper; this reading is used everywhere).
// (evaluated on every lane and then selected, without a branch)
template <typename T>
__device__ __forceinline__ T atan2z(T y, T x) {
  const T a = Num<T>::atan2_(y, x);
  return (x == T(0) && y == T(0)) ? T(0) : a;
}

// Orders LDS traffic between lanes of one wavefront (the compiler may not
// move memory operations across it; a wavefront's LDS operations complete
// in issue order).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// DPP move with control CTRL on the rows of ROWS; lanes of the other rows
// keep `id`.
template <int CTRL, int ROWS>
__device__ __forceinline__ float dpp_rows(float v, float id) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(__builtin_bit_cast(int, id), __builtin_bit_cast(int, v),
                                                               CTRL, ROWS, 0xF, false));
}
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_rows(double v, double id) {
  const long long b = __builtin_bit_cast(long long, v), i = __builtin_bit_cast(long long, id);
  const int lo = __builtin_amdgcn_update_dpp(int(i & 0xffffffffLL), int(b & 0xffffffffLL), CTRL, ROWS, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(int(i >> 32), int(b >> 32), CTRL, ROWS, 0xF, false);
  return __builtin_bit_cast(double, (static_cast<long long>(hi) << 32) | (static_cast<unsigned int>(lo)));
}
__device__ __forceinline__ float lane63(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), 63));
}
__device__ __forceinline__ double lane63(double v) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_readlane(int(b & 0xffffffffLL), 63);
  const int hi = __builtin_amdgcn_readlane(int(b >> 32), 63);
  return __builtin_bit_cast(double, (static_cast<long long>(hi) << 32) | (static_cast<unsigned int>(lo)));
}

// op over the 64 lanes (id its identity), the same on every lane: quads,
// half rows and rows through lane permutations, then rows 0 + 1 and 2 + 3
// through the row broadcasts of lanes 15 and 31, read from lane 63.
template <typename T, typename Op>
__device__ __forceinline__ T wave_all(T v, T id, Op op) {
  v = op(v, dpp_rows<0xB1, 0xF>(v, id));    // quad_perm [1, 0, 3, 2]
  v = op(v, dpp_rows<0x4E, 0xF>(v, id));    // quad_perm [2, 3, 0, 1]
  v = op(v, dpp_rows<0x141, 0xF>(v, id));   // row_half_mirror
  v = op(v, dpp_rows<0x140, 0xF>(v, id));   // row_mirror
  v = op(v, dpp_rows<0x142, 0xA>(v, id));   // row_bcast:15 into rows 1 and 3
  v = op(v, dpp_rows<0x143, 0xC>(v, id));   // row_bcast:31 into rows 2 and 3
  return lane63(v);
}

__host__ __device__ constexpr int pad4(int v) { return (v + 3) & ~3; }

// Sums exchanged between the two wavefronts of one trajectory: per half, 64
// slots for the per-iteration reduction F^T(F xi - g) and the heading
// multiplier rows, 16 for the heading right-hand side.
constexpr int kXchBig = 64;
constexpr int kXchSmall = 16;
constexpr int kXchHalf = kXchBig + kXchSmall;

// Reduction scratch: up to kRedRows rows of 16 lane-quad sums (a launch
// built for 3 wavefronts per SIMD reduces in passes of kRedRows / 2 rows to
// halve the area).
constexpr int kRedRows = 56;
constexpr int kRedRowStride = 36;
__host__ __device__ constexpr int red_rows_for(int waves) { return waves >= 3 ? kRedRows / 2 : kRedRows; }

// Pairs and quads of T with the alignment of one LDS vector access.
template <typename T>
struct alignas(2 * sizeof(T)) Pair {
  T x, y;
};
template <typename T>
struct alignas(4 * sizeof(T)) Quad {
  T a, b, c, d;
};

// LDS carve-up of the fused kernel, in elements of T.  Offsets are multiples
// of 8 elements, so Pair and Quad reads (and FP64 pairs when T is float)
// are aligned.
struct FusedLds {
  int oxy;                 // obstacle centres, Pair [n][q]
  int op;                  // per-obstacle parameters [n][8] (OP_*)
  int m1;                  // [2nv][2nv] operator M1 as Quad [a2/4][2nv]
  int qrows;               // rows of Q = blockdiag(W^T W, W^T W or 0) as [2][nv][pad4(nv)]
  int xch;                 // [traj][half][kXchHalf] exchange area
  int wave0, wave_stride;  // per-wave areas
  int total;
};

// Per-wave vectors.  Position-block vectors hold one axis in 2nv contiguous
// entries (x block then slack block), padded to a2 = pad4(2nv).  The
// coefficients are kept in FP64 (zd; dw elements of T per double); w and dz
// are the T operands of the coefficient update's two products; wd stages
// the FP64 multipliers for the write-back.  dz (its four blocks pad4(nv)
// apart) and the heading coefficients zpsi are read by every lane against
// its basis rows, which a lane holds in its own order (slot 4i + k holds
// row 4i + (k ^ (lane & 3))); both are stored in four copies, copy s in
// that order for the lanes with lane & 3 = s (copy 0 is the natural
// order).  The copy strides put the four copies' 16-byte groups in
// different LDS banks.
struct WaveLds {
  int w, dz, zd, wd, zpsi, aux, red;
};

__host__ __device__ constexpr int pad8(int v) { return (v + 7) & ~7; }
__host__ __device__ constexpr int dz_copy_stride(int nv) { return 2 * pad4(2 * nv) + 4; }
__host__ __device__ constexpr int zpsi_copy_stride(int nv) { return pad4(nv); }

__host__ __device__ inline WaveLds wave_layout(int nv, int red_rows, int dw) {
  const int p = pad4(nv), a2 = pad4(2 * nv);
  WaveLds w;
  int o = 0;
  w.w = o; o += pad8(2 * a2);                      // lambda - rho F^T (F xi - g)
  w.dz = o; o += pad8(4 * dz_copy_stride(nv));     // the last update of z (4 copies)
  w.zd = o; o += pad8(2 * a2 * dw);                // z in FP64
  w.wd = o; o += pad8(2 * a2 * dw);                // multipliers in FP64 (write-back)
  w.zpsi = o; o += pad8(4 * zpsi_copy_stride(nv)); // heading coefficients (4 copies)
  w.aux = o; o += pad8(2 * a2 + p);                // set-up staging
  w.red = o; o += red_rows * kRedRowStride;
  return w;
}

__host__ __device__ inline FusedLds fused_layout(int q, int n, int nv, int tile, int red_rows, int dw) {
  FusedLds L;
  const int a2 = pad4(2 * nv);
  int o = 0;
  L.oxy = o; o += pad8(2 * n * q);
  L.op = o; o += 8 * n;
  L.m1 = o; o += a2 * 2 * nv;
  L.qrows = o; o += pad8(2 * nv * pad4(nv));
  L.xch = o; o += tile * 2 * kXchHalf;
  const WaveLds w = wave_layout(nv, red_rows, dw);
  L.wave_stride = pad8(w.red + red_rows * kRedRowStride);
  L.wave0 = o; o += 2 * tile * L.wave_stride;
  L.total = o;
  return L;
}

// Per-obstacle parameter slots in the op table (inflated semi-axes a, b):
// the first four are read as one Quad in the projection loop.
enum { OP_A2 = 0, OP_B2 = 1, OP_AB = 2, OP_AMAX = 3, OP_A = 4, OP_B = 5, OP_IA2 = 6, OP_IB2 = 7 };

}  // namespace amk
