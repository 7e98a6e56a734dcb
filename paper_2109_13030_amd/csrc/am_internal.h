// am_internal.h -- types shared by the host API and the HIP kernels of the
// batched AM trajectory optimizer (not part of the public C-ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "am.h"

namespace amk {

constexpr int kWave = 64;          // CDNA wavefront width
constexpr int kWavesPerBlock = 4;  // 256-thread blocks (residual kernel)
// Fused kernel: two wavefronts per trajectory, `tile` trajectories per block
// (a launch shape the autotuner chooses among).
constexpr int kTiles[] = {1, 2, 4};
constexpr int kDefaultTile = 2;
constexpr int kWaveBudgets[] = {2, 3};   // register budgets of the fused kernel (wavefronts per SIMD)
constexpr int kDefaultWaves = 2;

// One problem of a launch: handle constants, problem data, state, sizes.
// Pointers to typed data (float or double) are void*; the kernel template
// reinterprets them.
struct Desc {
  // constants built by the setup kernel (orthonormal basis, KKT inverses)
  const void *U, *V, *W;     // [q][nv]: x = U z, xdot = V z, xddot = W z
  const void *M1, *H1;       // xi1: [2nv][2nv] and [2nv][6]
  const void *M2, *H2;       // xi2: [nv][nv] and [nv][6]
  const void *GF;            // [2nv][2nv] F^T F of one axis in the z basis
  const void *N;             // [2nv][2nv] M1 Q (Q: smoothness cost of one axis in the z basis)
  const void *Ut;            // [q][nv] U M2^T (heading rows premultiplied by M2)
  const double *R, *Rinv;    // z = R c (Bernstein c), [nv][nv]
  const double *Ud;          // [q][nv] U in FP64 (positions)
  const double *Abc;         // [6][nv] boundary rows U, V, W at t = 0 and t = q-1 (z basis)
  const double *H1d;         // [2nv][6] H1 in FP64
  const double *Qd;          // [nv][nv] W^T W in the z basis (FP64): the smoothness block of Q
  // problem
  const void *ox, *oy, *oa, *ob;
  // state (Bernstein coordinates at the boundary)
  void *cx, *cc, *cy, *cs, *cpsi, *lam, *lampsi;
  void *alpha, *d, *va, *traj, *res;
  double bx[6], by[6], bpsi[6];
  double offx, offy;         // translation applied inside the kernel
  double rc, vmax, amax, rho, rho_psi;
  double r[AM_MAX_CIRCLES];
  int q, nv, m, n, B, K, flags;
  int blk0, nblk;            // blocks of this problem in a multi-problem grid
};

// Largest descriptor table the multi-problem launch accepts.
constexpr int kMaxProblems = 4096;

// Device buffers of a handle (all inside one FP64 and one typed allocation).
struct Consts {
  double *P, *Pd, *Pdd;          // [q][nv] Bernstein basis and derivatives
  double *U, *V, *W;             // [q][nv]
  double *R, *Rinv;              // [nv][nv]
  double *G;                     // scratch: 3 Gram matrices [3][nv][nv]
  double *K1, *K2;               // z-space KKT [N1][N1], [N2][N2]
  double *A1, *A2;               // Gauss-Jordan work [N][2N]
  double *M1, *H1, *M2, *H2, *GF;
  double *N;                     // [2nv][2nv] M1 Q
  double *Abc;                   // [6][nv] boundary rows in the z basis
  double *K1b_inv, *K2b_inv;     // Bernstein-space inverses (diagnostics)
  double *Ut;                    // [q][nv] U M2^T
  double *status;                // [0]: 0 ok, 1 singular xi1 KKT, 2 singular xi2 KKT
  void *tU, *tV, *tW, *tM1, *tH1, *tM2, *tH2, *tGF;  // typed copies
  void *tP, *tPd, *tPdd, *tUt, *tN;
};

// Launchers (defined in the .hip files).
hipError_t launch_setup(const am_shape &s, const double *r_dev, const Consts &c, bool f64,
                        hipStream_t st);
size_t fused_lds_bytes(int q, int n, int nv, bool f64, int tile, int waves);
// max_m: the largest circle count of the launch's problems (picks the
// kernel's circle capacity)
hipError_t launch_fused(const Desc &single, const Desc *table, int nprob, int nblocks, bool f64,
                        int nv, int max_m, hipStream_t st, size_t lds_bytes, int tile, int waves);
hipError_t launch_select_best(const void *res, int B, double tol, int32_t *idx, void *vals, bool f64,
                              hipStream_t st);
hipError_t launch_residuals(const Desc &d, const void *P, const void *Pd, const void *Pdd, void *out,
                            bool f64, int nv, hipStream_t st);
hipError_t launch_desc_copy(const Desc *host_descs, int count, Desc *dev_dst, hipStream_t st);
// Loads the kernels of the residual/selection/descriptor-copy source file
// (otherwise loaded by the first launch of one of them).
hipError_t preload_kernels();
// Device address of `device`'s copy of the static problem table
// (AM_STATIC_MAX_PROBLEMS descriptors); `device` must be current on the
// first call for it.
hipError_t static_table(int device, Desc **out);
hipError_t launch_plain(const Desc &d, void *ws, size_t ws_bytes, bool f64, int nv, hipStream_t st);
size_t plain_workspace_bytes(int B, int q, int nv, int m, int n, bool f64);

// Records the calling thread's last error message (am_last_error); returns code.
int set_last_error(int code, const char *msg);

// Shape of a handle (for the server).
int handle_q(const am_handle *h);
int handle_nv(const am_handle *h);
int handle_n(const am_handle *h);
int handle_dtype(const am_handle *h);

}  // namespace amk
