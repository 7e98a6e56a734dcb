// am_device.h -- device helpers shared by the iteration kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "am_internal.h"

namespace amk {

template <typename T>
struct Num;

template <>
struct Num<float> {
  static __device__ __forceinline__ float rsqrt(float x) { return rsqrtf(x); }
  static __device__ __forceinline__ float sqrt_(float x) { return sqrtf(x); }
  static __device__ __forceinline__ float atan2_(float y, float x) { return atan2f(y, x); }
  static __device__ __forceinline__ void sincos_(float a, float *s, float *c) { sincosf(a, s, c); }
  static __device__ __forceinline__ float hypot_(float a, float b) { return hypotf(a, b); }
  static __device__ __forceinline__ float cos_(float a) { return cosf(a); }
  static __device__ __forceinline__ float sin_(float a) { return sinf(a); }
};

template <>
struct Num<double> {
  static __device__ __forceinline__ double rsqrt(double x) { return 1.0 / ::sqrt(x); }
  static __device__ __forceinline__ double sqrt_(double x) { return ::sqrt(x); }
  static __device__ __forceinline__ double atan2_(double y, double x) { return ::atan2(y, x); }
  static __device__ __forceinline__ void sincos_(double a, double *s, double *c) { ::sincos(a, s, c); }
  static __device__ __forceinline__ double hypot_(double a, double b) { return ::hypot(a, b); }
  static __device__ __forceinline__ double cos_(double a) { return ::cos(a); }
  static __device__ __forceinline__ double sin_(double a) { return ::sin(a); }
};

// atan2 with the value 0 for the zero vector (the angle of a zero vector is
// not defined by the paper; this reading is used everywhere).
template <typename T>
__device__ __forceinline__ T atan2z(T y, T x) {
  return (x == T(0) && y == T(0)) ? T(0) : Num<T>::atan2_(y, x);
}

// Orders LDS traffic between lanes of one wavefront (the compiler may not
// move memory operations across it; a wavefront's LDS operations complete
// in issue order).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__host__ __device__ constexpr int pad4(int v) { return (v + 3) & ~3; }

// Sums exchanged between the two wavefronts of one trajectory: per half, 64
// slots for the per-iteration reduction F^T(F xi - g) and the heading
// multiplier rows, 16 for the heading right-hand side.
constexpr int kXchBig = 64;
constexpr int kXchSmall = 16;
constexpr int kXchHalf = kXchBig + kXchSmall;

// Reduction scratch: up to kRedRows rows of 32 lane-pair sums.
constexpr int kRedRows = 56;
constexpr int kRedRowStride = 36;

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
// of 4 elements, so Pair and Quad reads are aligned.
struct FusedLds {
  int oxy;                 // centred obstacle centres, Pair [n][q]
  int op;                  // per-obstacle parameters [n][8] (OP_*)
  int m1, gf;              // [2nv][2nv] operators as Quad [a2/4][2nv]
  int xch;                 // [traj][half][kXchHalf] exchange area
  int wave0, wave_stride;  // per-wave areas
  int total;
};

// Per-wave vectors.  Position-block vectors hold one axis in 2nv contiguous
// entries (x block then slack block), padded to a2 = pad4(2nv).
struct WaveLds {
  int z, rhs, zpsi, aux, red;
};

__host__ __device__ inline WaveLds wave_layout(int nv) {
  const int p = pad4(nv), a2 = pad4(2 * nv);
  WaveLds w;
  int o = 0;
  w.z = o; o += 2 * a2;         // z of (x, c) and (y, s)
  w.rhs = o; o += 2 * a2;       // lambda + rho F^T g
  w.zpsi = o; o += p;           // heading coefficients
  w.aux = o; o += 2 * a2 + p;   // set-up and write-back staging
  w.red = o; o += kRedRows * kRedRowStride;
  return w;
}

__host__ __device__ inline FusedLds fused_layout(int q, int n, int nv, int tile) {
  FusedLds L;
  const int a2 = pad4(2 * nv);
  int o = 0;
  L.oxy = o; o += pad4(2 * n * q);
  L.op = o; o += 8 * n;
  L.m1 = o; o += a2 * 2 * nv;
  L.gf = o; o += a2 * 2 * nv;
  L.xch = o; o += tile * 2 * kXchHalf;
  const WaveLds w = wave_layout(nv);
  L.wave_stride = pad4(w.red + kRedRows * kRedRowStride);
  L.wave0 = o; o += 2 * tile * L.wave_stride;
  L.total = o;
  return L;
}

// Per-obstacle parameter slots in the op table (inflated semi-axes a, b):
// the first four are read as one Quad in the projection loop.
enum { OP_A2 = 0, OP_B2 = 1, OP_AB = 2, OP_AMAX = 3, OP_A = 4, OP_B = 5 };

}  // namespace amk
