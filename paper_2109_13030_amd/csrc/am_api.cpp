// am_api.cpp -- host side of the C-ABI declared in include/am.h: argument
// checks, error reporting, handle lifetime and kernel launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <string>

#include "am.h"
#include "am_internal.h"

using amk::Consts;
using amk::Desc;

struct am_handle {
  am_shape shape;
  double r[AM_MAX_CIRCLES];
  int device;
  bool f64;
  int tile = amk::kDefaultTile;   // trajectories per block of the fused kernel
  int waves = amk::kDefaultWaves; // register budget of the fused kernel (wavefronts per SIMD)
  double *buf64;       // all FP64 constants
  void *bufT;          // typed copies
  Consts c;
};

namespace {

thread_local std::string g_err = "no error";

int fail(int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

int hip_fail(hipError_t e, const char *what) {
  return fail(AM_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

bool is_fin(double v) { return std::isfinite(v); }

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

int check_problem(const am_handle *h, const am_problem *p) {
  if (!p) return fail(AM_ERR_INVALID, "problem is NULL");
  if (h->shape.n_obs > 0 && (!p->obs_x || !p->obs_y || !p->obs_a || !p->obs_b))
    return fail(AM_ERR_INVALID, "obstacle arrays must be non-NULL when n_obs > 0");
  if (!(p->r_circle >= 0.0) || !is_fin(p->r_circle))
    return fail(AM_ERR_INVALID, "r_circle must be finite and >= 0");
  if (!(p->v_max > 0.0) || !(p->a_max > 0.0) || !is_fin(p->v_max) || !is_fin(p->a_max))
    return fail(AM_ERR_INVALID, "v_max and a_max must be finite and > 0");
  for (int e = 0; e < 6; ++e)
    if (!is_fin(p->bc_x[e]) || !is_fin(p->bc_y[e]) || !is_fin(p->bc_psi[e]))
      return fail(AM_ERR_INVALID, "boundary conditions must be finite");
  return AM_OK;
}

int check_state(const am_state *st) {
  if (!st) return fail(AM_ERR_INVALID, "state is NULL");
  if (!st->cx || !st->cc || !st->cy || !st->cs || !st->cpsi || !st->lam || !st->lam_psi)
    return fail(AM_ERR_INVALID, "state coefficient and multiplier arrays must be non-NULL");
  return AM_OK;
}

int check_device(const am_handle *h) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (dev != h->device)
    return fail(AM_ERR_INVALID, "handle was set up on device %d but device %d is current", h->device, dev);
  return AM_OK;
}

Desc make_desc(const am_handle *h, const am_problem *p, int32_t batch, int32_t iters,
               const am_state *st, int tile) {
  Desc d;
  std::memset(&d, 0, sizeof d);
  const Consts &c = h->c;
  d.U = c.tU; d.V = c.tV; d.W = c.tW; d.M1 = c.tM1; d.H1 = c.tH1; d.M2 = c.tM2; d.H2 = c.tH2;
  d.GF = c.tGF; d.N = c.tN; d.Ut = c.tUt; d.R = c.R; d.Rinv = c.Rinv; d.Ud = c.U; d.Abc = c.Abc; d.H1d = c.H1;
  d.Qd = c.G + 2 * size_t(h->shape.nv) * h->shape.nv;   // the third Gram matrix, W^T W
  d.ox = p->obs_x; d.oy = p->obs_y; d.oa = p->obs_a; d.ob = p->obs_b;
  d.cx = st->cx; d.cc = st->cc; d.cy = st->cy; d.cs = st->cs; d.cpsi = st->cpsi;
  d.lam = st->lam; d.lampsi = st->lam_psi;
  d.alpha = st->alpha; d.d = st->d; d.va = st->va; d.traj = st->traj; d.res = st->res;
  for (int e = 0; e < 6; ++e) { d.bx[e] = p->bc_x[e]; d.by[e] = p->bc_y[e]; d.bpsi[e] = p->bc_psi[e]; }
  d.offx = 0.5 * (p->bc_x[0] + p->bc_x[3]);
  d.offy = 0.5 * (p->bc_y[0] + p->bc_y[3]);
  d.rc = p->r_circle; d.vmax = p->v_max; d.amax = p->a_max;
  d.rho = h->shape.rho; d.rho_psi = h->shape.rho_psi;
  for (int i = 0; i < h->shape.m; ++i) d.r[i] = h->r[i];
  d.q = h->shape.q; d.nv = h->shape.nv; d.m = h->shape.m; d.n = h->shape.n_obs;
  d.B = batch; d.K = iters; d.flags = int(h->shape.flags);
  d.blk0 = 0;
  d.nblk = (batch + tile - 1) / tile;
  return d;
}

size_t lds_limit() {
  int dev = 0, v = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 65536;
  if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) return 65536;
  return size_t(v);
}

}  // namespace

namespace {

// Times `reps` launches of fn on the stream with HIP events (after one
// warm-up launch); returns milliseconds per launch or a negative status.
template <class F>
int time_launches(hipStream_t s, int reps, F fn, float *ms) {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int rc = fn();
  if (rc != AM_OK) return rc;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    return fail(AM_ERR_HIP, "hipEventCreate failed");
  }
  (void)hipEventRecord(e0, s);
  for (int r = 0; r < reps && rc == AM_OK; ++r) rc = fn();
  (void)hipEventRecord(e1, s);
  hipError_t e = hipEventSynchronize(e1);
  float t = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc != AM_OK) return rc;
  if (e != hipSuccess) return hip_fail(e, "timing events");
  *ms = t / float(reps);
  return AM_OK;
}


// Times `solve` for every launch configuration (tile x register budget) the
// handle's dtype allows; configs[i] = {tile, waves}.  Leaves the fastest set
// through `apply`.
template <typename Apply, typename Solve>
int tune(bool f64, void *stream, Apply apply, Solve solve, int keep_tile, int keep_waves, int32_t *best_tile,
         int32_t *best_waves, float *times_ms) {
  int bt = keep_tile, bw = keep_waves, idx = 0;
  float best_ms = 0.f;
  bool any = false;
  for (int w : amk::kWaveBudgets)
    for (int t : amk::kTiles) {
      const int i = idx++;
      if (f64 && w != 2) {
        if (times_ms) times_ms[i] = -1.f;
        continue;
      }
      apply(t, w);
      float ms = 0.f;
      const int rc = time_launches(static_cast<hipStream_t>(stream), 3, solve, &ms);
      if (rc != AM_OK) {
        apply(keep_tile, keep_waves);
        return rc;
      }
      if (times_ms) times_ms[i] = ms;
      if (!any || ms < best_ms) { best_ms = ms; bt = t; bw = w; any = true; }
    }
  apply(bt, bw);
  if (best_tile) *best_tile = bt;
  if (best_waves) *best_waves = bw;
  return AM_OK;
}

}  // namespace

namespace amk {
int set_last_error(int code, const char *msg) { return fail(code, "%s", msg); }
int handle_q(const am_handle *h) { return h->shape.q; }
int handle_nv(const am_handle *h) { return h->shape.nv; }
int handle_n(const am_handle *h) { return h->shape.n_obs; }
int handle_dtype(const am_handle *h) { return h->shape.dtype; }
}  // namespace amk

extern "C" {

const char *am_last_error(void) { return g_err.c_str(); }

int am_setup(const am_shape *s, am_handle **out) {
  if (!out) return fail(AM_ERR_INVALID, "out is NULL");
  *out = nullptr;
  if (!s) return fail(AM_ERR_INVALID, "shape is NULL");
  if (s->q <= 2 || s->q > AM_MAX_Q) return fail(AM_ERR_INVALID, "q must be in (2, %d], got %d", AM_MAX_Q, s->q);
  if (s->nv != 8 && s->nv != 11) return fail(AM_ERR_INVALID, "nv must be 8 or 11, got %d", s->nv);
  if (s->q < s->nv) return fail(AM_ERR_INVALID, "q must be >= nv");
  if (!(s->tf > 0.0) || !is_fin(s->tf)) return fail(AM_ERR_INVALID, "tf must be finite and > 0");
  if (s->m < 1 || s->m > AM_MAX_CIRCLES) return fail(AM_ERR_INVALID, "m must be in [1, %d]", AM_MAX_CIRCLES);
  if (!s->r_off) return fail(AM_ERR_INVALID, "r_off is NULL");
  for (int i = 0; i < s->m; ++i)
    if (!is_fin(s->r_off[i])) return fail(AM_ERR_INVALID, "r_off must be finite");
  if (s->n_obs < 0 || s->n_obs > AM_MAX_OBS) return fail(AM_ERR_INVALID, "n_obs must be in [0, %d]", AM_MAX_OBS);
  if (!(s->rho > 0.0) || !is_fin(s->rho)) return fail(AM_ERR_INVALID, "rho must be finite and > 0");
  if (!(s->rho_psi >= 0.0) || !is_fin(s->rho_psi)) return fail(AM_ERR_INVALID, "rho_psi must be finite and >= 0");
  if (s->dtype != AM_F32 && s->dtype != AM_F64) return fail(AM_ERR_INVALID, "dtype must be AM_F32 or AM_F64");
  if (s->flags & ~AM_FLAGS_ALL) return fail(AM_ERR_INVALID, "unknown flag bits 0x%x", s->flags & ~AM_FLAGS_ALL);
  if ((s->flags & AM_PLAIN_BF16X3) && s->dtype != AM_F32)
    return fail(AM_ERR_INVALID, "AM_PLAIN_BF16X3 needs an AM_F32 handle");

  am_handle *h = new am_handle();
  h->shape = *s;
  h->shape.r_off = nullptr;
  for (int i = 0; i < s->m; ++i) h->r[i] = s->r_off[i];
  h->f64 = s->dtype == AM_F64;
  hipError_t e = hipGetDevice(&h->device);
  if (e != hipSuccess) { delete h; return hip_fail(e, "hipGetDevice"); }

  const int q = s->q, nv = s->nv, n2 = 2 * nv, N1 = n2 + 6, N2 = nv + 6;
  // FP64 carve-up (in doubles)
  size_t sizes[] = {size_t(q * nv), size_t(q * nv), size_t(q * nv),      // P Pd Pdd
                    size_t(q * nv), size_t(q * nv), size_t(q * nv),      // U V W
                    size_t(nv * nv), size_t(nv * nv), size_t(3 * nv * nv),
                    size_t(N1 * N1), size_t(N2 * N2), size_t(2 * N1 * N1), size_t(2 * N2 * N2),
                    size_t(n2 * n2), size_t(n2 * 6), size_t(nv * nv), size_t(nv * 6), size_t(n2 * n2),
                    size_t(N1 * N1), size_t(N2 * N2), 8, size_t(AM_MAX_CIRCLES), size_t(q * nv),
                    size_t(n2 * n2), size_t(6 * nv)};
  const int nparts = int(sizeof(sizes) / sizeof(sizes[0]));
  size_t off[32], tot = 0;
  for (int i = 0; i < nparts; ++i) { off[i] = tot; tot += align_up(sizes[i], 32); }
  e = hipMalloc(&h->buf64, tot * sizeof(double));
  if (e != hipSuccess) { delete h; return fail(AM_ERR_NOMEM, "hipMalloc of %zu bytes failed", tot * 8); }
  double *b = h->buf64;
  Consts &c = h->c;
  c.P = b + off[0]; c.Pd = b + off[1]; c.Pdd = b + off[2]; c.U = b + off[3]; c.V = b + off[4];
  c.W = b + off[5]; c.R = b + off[6]; c.Rinv = b + off[7]; c.G = b + off[8]; c.K1 = b + off[9];
  c.K2 = b + off[10]; c.A1 = b + off[11]; c.A2 = b + off[12]; c.M1 = b + off[13]; c.H1 = b + off[14];
  c.M2 = b + off[15]; c.H2 = b + off[16]; c.GF = b + off[17]; c.K1b_inv = b + off[18];
  c.K2b_inv = b + off[19]; c.status = b + off[20];
  double *r_dev = b + off[21];
  c.Ut = b + off[22];
  c.N = b + off[23];
  c.Abc = b + off[24];

  // typed carve-up (in elements)
  const size_t es = h->f64 ? 8 : 4;
  size_t tsz[] = {size_t(q * nv), size_t(q * nv), size_t(q * nv), size_t(n2 * n2), size_t(n2 * 6),
                  size_t(nv * nv), size_t(nv * 6), size_t(n2 * n2), size_t(q * nv), size_t(q * nv),
                  size_t(q * nv), size_t(q * nv), size_t(n2 * n2)};
  constexpr int ntyped = int(sizeof(tsz) / sizeof(tsz[0]));
  size_t toff[16], ttot = 0;
  for (int i = 0; i < ntyped; ++i) { toff[i] = ttot; ttot += align_up(tsz[i], 64); }
  e = hipMalloc(&h->bufT, ttot * es);
  if (e != hipSuccess) {
    (void)hipFree(h->buf64);
    delete h;
    return fail(AM_ERR_NOMEM, "hipMalloc of %zu bytes failed", ttot * es);
  }
  char *tb = static_cast<char *>(h->bufT);
  void **tp[] = {&c.tU, &c.tV, &c.tW, &c.tM1, &c.tH1, &c.tM2, &c.tH2, &c.tGF, &c.tP, &c.tPd, &c.tPdd, &c.tUt, &c.tN};
  static_assert(sizeof(tp) / sizeof(tp[0]) == ntyped, "typed buffers");
  for (int i = 0; i < ntyped; ++i) *tp[i] = tb + toff[i] * es;

  hipStream_t stream = nullptr;
  double status = -1.0;
  int rc = AM_OK;
  if ((e = hipStreamCreateWithFlags(&stream, hipStreamNonBlocking)) != hipSuccess) {
    rc = hip_fail(e, "hipStreamCreateWithFlags");
  } else if ((e = hipMemcpyAsync(r_dev, h->r, sizeof(double) * s->m, hipMemcpyHostToDevice, stream)) != hipSuccess) {
    rc = hip_fail(e, "hipMemcpyAsync");
  } else if ((e = amk::launch_setup(h->shape, r_dev, c, h->f64, stream)) != hipSuccess) {
    rc = hip_fail(e, "setup kernel launch");
  } else if ((e = hipMemcpyAsync(&status, c.status, sizeof(double), hipMemcpyDeviceToHost, stream)) != hipSuccess) {
    rc = hip_fail(e, "hipMemcpyAsync");
  } else if ((e = hipStreamSynchronize(stream)) != hipSuccess) {
    rc = hip_fail(e, "setup kernel");
  } else if (status != 0.0) {
    rc = fail(AM_ERR_SINGULAR, "the %s KKT matrix is numerically singular",
              status == 1.0 ? "xi1" : "xi2");
  }
  if (stream) (void)hipStreamDestroy(stream);
  if (rc == AM_OK) {
    // the static problem table of am_solve_multi_static: its device address
    // on this device, looked up once with the device current
    amk::Desc *tbl = nullptr;
    if ((e = amk::static_table(h->device, &tbl)) != hipSuccess) rc = hip_fail(e, "static problem table");
  }
  if (rc == AM_OK && (e = amk::preload_kernels()) != hipSuccess) rc = hip_fail(e, "kernel load");
  if (rc != AM_OK) {
    am_destroy(h);
    return rc;
  }
  *out = h;
  return AM_OK;
}

void am_destroy(am_handle *h) {
  if (!h) return;
  if (h->buf64) (void)hipFree(h->buf64);
  if (h->bufT) (void)hipFree(h->bufT);
  delete h;
}

int am_solve_batch(am_handle *h, const am_problem *p, int32_t batch, int32_t iters, const am_state *st,
                   void *stream) {
  if (!h) return fail(AM_ERR_INVALID, "handle is NULL");
  if (batch < 0 || iters < 0) return fail(AM_ERR_INVALID, "batch and iters must be >= 0");
  int rc;
  if ((rc = check_problem(h, p)) != AM_OK) return rc;
  if ((rc = check_device(h)) != AM_OK) return rc;
  if (batch == 0) return AM_OK;   // empty arrays may come as NULL
  if ((rc = check_state(st)) != AM_OK) return rc;
  const Desc d = make_desc(h, p, batch, iters, st, h->tile);
  const size_t lds = amk::fused_lds_bytes(h->shape.q, h->shape.n_obs, h->shape.nv, h->f64, h->tile, h->waves);
  if (lds > lds_limit())
    return fail(AM_ERR_INVALID, "problem needs %zu bytes of LDS, device allows %zu", lds, lds_limit());
  hipError_t e = amk::launch_fused(d, nullptr, 1, d.nblk, h->f64, h->shape.nv, h->shape.m,
                                   static_cast<hipStream_t>(stream), lds, h->tile, h->waves);
  if (e != hipSuccess) return hip_fail(e, "fused kernel launch");
  return AM_OK;
}

int am_multi_workspace_size(int32_t nprob, size_t *bytes) {
  if (!bytes) return fail(AM_ERR_INVALID, "bytes is NULL");
  if (nprob < 0 || nprob > amk::kMaxProblems)
    return fail(AM_ERR_INVALID, "nprob must be in [0, %d]", amk::kMaxProblems);
  *bytes = align_up(size_t(nprob) * sizeof(Desc), 256);
  return AM_OK;
}

}  // extern "C"

namespace {

// The multi-problem launch with its problem table at `table` (device memory
// for at least `cap` descriptors).  Two passes over the problems: the first
// checks them and sizes the launch, the second writes the table in chunks
// through kernel arguments; no host or device memory is allocated.
int solve_multi_into(int32_t nprob, am_handle *const *handles, const am_problem *problems, const int32_t *batch,
                     const int32_t *iters, const am_state *states, Desc *table, int cap, void *stream) {
  if (nprob < 0 || nprob > cap) return fail(AM_ERR_INVALID, "nprob must be in [0, %d]", cap);
  if (nprob == 0) return AM_OK;
  if (!handles || !problems || !batch || !iters || !states)
    return fail(AM_ERR_INVALID, "problem arrays must be non-NULL");
  const am_handle *h0 = handles[0];
  if (!h0) return fail(AM_ERR_INVALID, "handle 0 is NULL");
  size_t lds = 0;
  int blocks = 0, max_m = 1;
  for (int k = 0; k < nprob; ++k) {
    const am_handle *h = handles[k];
    if (!h) return fail(AM_ERR_INVALID, "handle %d is NULL", k);
    if (h->f64 != h0->f64 || h->shape.q != h0->shape.q || h->shape.nv != h0->shape.nv)
      return fail(AM_ERR_INVALID, "handle %d differs from handle 0 in dtype, q or nv", k);
    if (batch[k] < 0 || iters[k] < 0) return fail(AM_ERR_INVALID, "problem %d: negative batch or iters", k);
    int rc;
    if ((rc = check_problem(h, &problems[k])) != AM_OK) return rc;
    if (batch[k] > 0 && (rc = check_state(&states[k])) != AM_OK) return rc;
    if ((rc = check_device(h)) != AM_OK) return rc;
    blocks += (batch[k] + h0->tile - 1) / h0->tile;
    lds = std::max(lds, amk::fused_lds_bytes(h->shape.q, h->shape.n_obs, h->shape.nv, h->f64, h0->tile, h0->waves));
    max_m = std::max(max_m, int(h->shape.m));
  }
  if (lds > lds_limit())
    return fail(AM_ERR_INVALID, "a problem needs %zu bytes of LDS, device allows %zu", lds, lds_limit());
  if (blocks == 0) return AM_OK;
  hipStream_t s = static_cast<hipStream_t>(stream);
  constexpr int kChunk = 6;
  Desc chunk[kChunk];
  Desc first{};
  int blk = 0;
  for (int base = 0; base < nprob; base += kChunk) {
    const int cnt = std::min(kChunk, nprob - base);
    for (int k = 0; k < cnt; ++k) {
      const int p = base + k;
      chunk[k] = make_desc(handles[p], &problems[p], batch[p], iters[p], &states[p], h0->tile);
      chunk[k].blk0 = blk;
      blk += chunk[k].nblk;
      if (p == 0) first = chunk[k];
    }
    hipError_t e = amk::launch_desc_copy(chunk, cnt, table + base, s);
    if (e != hipSuccess) return hip_fail(e, "problem table copy");
  }
  hipError_t e = amk::launch_fused(first, table, nprob, blocks, h0->f64, h0->shape.nv, max_m, s, lds, h0->tile,
                                   h0->waves);
  if (e != hipSuccess) return hip_fail(e, "fused kernel launch");
  return AM_OK;
}

}  // namespace

extern "C" {

int am_solve_multi(int32_t nprob, am_handle *const *handles, const am_problem *problems, const int32_t *batch,
                   const int32_t *iters, const am_state *states, void *workspace, size_t workspace_bytes,
                   void *stream) {
  if (nprob < 0 || nprob > amk::kMaxProblems)
    return fail(AM_ERR_INVALID, "nprob must be in [0, %d]", amk::kMaxProblems);
  if (nprob == 0) return AM_OK;
  size_t need = 0;
  am_multi_workspace_size(nprob, &need);
  if (!workspace || workspace_bytes < need)
    return fail(AM_ERR_INVALID, "workspace of %zu bytes needed", need);
  return solve_multi_into(nprob, handles, problems, batch, iters, states, static_cast<Desc *>(workspace),
                          amk::kMaxProblems, stream);
}

int am_solve_multi_static(int32_t nprob, am_handle *const *handles, const am_problem *problems, const int32_t *batch,
                          const int32_t *iters, const am_state *states, void *stream) {
  if (nprob < 0 || nprob > AM_STATIC_MAX_PROBLEMS)
    return fail(AM_ERR_INVALID, "nprob must be in [0, %d] (AM_STATIC_MAX_PROBLEMS)", AM_STATIC_MAX_PROBLEMS);
  if (nprob == 0) return AM_OK;
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  Desc *table = nullptr;
  if ((e = amk::static_table(dev, &table)) != hipSuccess) return hip_fail(e, "static problem table");
  return solve_multi_into(nprob, handles, problems, batch, iters, states, table, AM_STATIC_MAX_PROBLEMS, stream);
}

int am_residuals(am_handle *h, const am_problem *p, int32_t batch, const am_state *st, void *out, void *stream) {
  if (!h) return fail(AM_ERR_INVALID, "handle is NULL");
  if (batch < 0) return fail(AM_ERR_INVALID, "batch must be >= 0");
  if (!out && batch > 0) return fail(AM_ERR_INVALID, "out is NULL");
  int rc;
  if ((rc = check_problem(h, p)) != AM_OK) return rc;
  if ((rc = check_device(h)) != AM_OK) return rc;
  if (batch == 0) return AM_OK;   // empty arrays may come as NULL
  if ((rc = check_state(st)) != AM_OK) return rc;
  const Desc d = make_desc(h, p, batch, 0, st, h->tile);
  hipError_t e = amk::launch_residuals(d, h->c.tP, h->c.tPd, h->c.tPdd, out, h->f64, h->shape.nv,
                                       static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "residual kernel launch");
  return AM_OK;
}

int am_select_best(const am_handle *h, int32_t batch, const void *residuals, double fc_tol, int32_t *best,
                   void *values, void *stream) {
  if (!h) return fail(AM_ERR_INVALID, "handle is NULL");
  if (batch < 0) return fail(AM_ERR_INVALID, "batch must be >= 0");
  if (!best) return fail(AM_ERR_INVALID, "best is NULL");
  if (!residuals && batch > 0) return fail(AM_ERR_INVALID, "residuals is NULL");
  if (!(fc_tol >= 0.0)) return fail(AM_ERR_INVALID, "fc_tol must be >= 0, got %g", fc_tol);
  int rc;
  if ((rc = check_device(h)) != AM_OK) return rc;
  hipError_t e = amk::launch_select_best(residuals, batch, fc_tol, best, values, h->f64,
                                         static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "select kernel launch");
  return AM_OK;
}

int am_setup_matrices(const am_handle *h, double *kkt1_inv, double *kkt2_inv, double *basis) {
  if (!h) return fail(AM_ERR_INVALID, "handle is NULL");
  const int q = h->shape.q, nv = h->shape.nv, N1 = 2 * nv + 6, N2 = nv + 6;
  hipError_t e = hipSuccess;
  if (kkt1_inv && e == hipSuccess)
    e = hipMemcpy(kkt1_inv, h->c.K1b_inv, sizeof(double) * N1 * N1, hipMemcpyDeviceToHost);
  if (kkt2_inv && e == hipSuccess)
    e = hipMemcpy(kkt2_inv, h->c.K2b_inv, sizeof(double) * N2 * N2, hipMemcpyDeviceToHost);
  if (basis && e == hipSuccess) e = hipMemcpy(basis, h->c.P, sizeof(double) * q * nv, hipMemcpyDeviceToHost);
  if (basis && e == hipSuccess)
    e = hipMemcpy(basis + q * nv, h->c.Pd, sizeof(double) * q * nv, hipMemcpyDeviceToHost);
  if (basis && e == hipSuccess)
    e = hipMemcpy(basis + 2 * q * nv, h->c.Pdd, sizeof(double) * q * nv, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(e, "hipMemcpy");
  return AM_OK;
}

int am_set_tile(am_handle *h, int32_t tile) {
  if (!h) return fail(AM_ERR_INVALID, "handle is NULL");
  for (int t : amk::kTiles)
    if (t == tile) {
      h->tile = tile;
      return AM_OK;
    }
  return fail(AM_ERR_INVALID, "tile must be 1, 2 or 4, got %d", tile);
}

int am_get_tile(const am_handle *h, int32_t *tile) {
  if (!h || !tile) return fail(AM_ERR_INVALID, "handle and tile must be non-NULL");
  *tile = h->tile;
  return AM_OK;
}

int am_set_waves(am_handle *h, int32_t waves) {
  if (!h) return fail(AM_ERR_INVALID, "handle is NULL");
  if (h->f64 && waves != 2) return fail(AM_ERR_INVALID, "FP64 handles run with a budget of 2 wavefronts per SIMD");
  for (int w : amk::kWaveBudgets)
    if (w == waves) {
      h->waves = waves;
      return AM_OK;
    }
  return fail(AM_ERR_INVALID, "waves must be 2 or 3, got %d", waves);
}

int am_get_waves(const am_handle *h, int32_t *waves) {
  if (!h || !waves) return fail(AM_ERR_INVALID, "handle and waves must be non-NULL");
  *waves = h->waves;
  return AM_OK;
}


int am_autotune(am_handle *h, const am_problem *p, int32_t batch, int32_t iters, const am_state *scratch,
                void *stream, int32_t *best_tile, int32_t *best_waves, float *times_ms) {
  if (!h) return fail(AM_ERR_INVALID, "handle is NULL");
  return tune(
      h->f64, stream, [&](int t, int w) { h->tile = t; h->waves = w; },
      [&] { return am_solve_batch(h, p, batch, iters, scratch, stream); }, h->tile, h->waves, best_tile, best_waves,
      times_ms);
}

int am_autotune_multi(int32_t nprob, am_handle *const *handles, const am_problem *problems, const int32_t *batch,
                      const int32_t *iters, const am_state *scratch, void *workspace, size_t workspace_bytes,
                      void *stream, int32_t *best_tile, int32_t *best_waves, float *times_ms) {
  if (nprob < 1 || !handles) return fail(AM_ERR_INVALID, "at least one problem is needed");
  for (int k = 0; k < nprob; ++k)
    if (!handles[k]) return fail(AM_ERR_INVALID, "handle %d is NULL", k);
  return tune(
      handles[0]->f64, stream,
      [&](int t, int w) {
        for (int k = 0; k < nprob; ++k) { handles[k]->tile = t; handles[k]->waves = w; }
      },
      [&] {
        return am_solve_multi(nprob, handles, problems, batch, iters, scratch, workspace, workspace_bytes, stream);
      },
      handles[0]->tile, handles[0]->waves, best_tile, best_waves, times_ms);
}

int am_plain_workspace_size(const am_handle *h, int32_t batch, size_t *bytes) {
  if (!h || !bytes) return fail(AM_ERR_INVALID, "handle and bytes must be non-NULL");
  if (batch < 0) return fail(AM_ERR_INVALID, "batch must be >= 0");
  *bytes = amk::plain_workspace_bytes(batch, h->shape.q, h->shape.nv, h->shape.m, h->shape.n_obs, h->f64);
  return AM_OK;
}

int am_solve_batch_plain(am_handle *h, const am_problem *p, int32_t batch, int32_t iters, const am_state *st,
                         void *workspace, size_t workspace_bytes, void *stream) {
  if (!h) return fail(AM_ERR_INVALID, "handle is NULL");
  if (batch < 0 || iters < 0) return fail(AM_ERR_INVALID, "batch and iters must be >= 0");
  int rc;
  if ((rc = check_problem(h, p)) != AM_OK) return rc;
  if ((rc = check_device(h)) != AM_OK) return rc;
  if (batch == 0) return AM_OK;   // empty arrays may come as NULL
  if ((rc = check_state(st)) != AM_OK) return rc;
  const size_t need = amk::plain_workspace_bytes(batch, h->shape.q, h->shape.nv, h->shape.m, h->shape.n_obs, h->f64);
  if (!workspace || workspace_bytes < need)
    return fail(AM_ERR_INVALID, "workspace of %zu bytes needed", need);
  if (reinterpret_cast<uintptr_t>(workspace) % 16 != 0)
    return fail(AM_ERR_INVALID, "workspace must be 16-byte aligned");
  const Desc d = make_desc(h, p, batch, iters, st, h->tile);
  hipError_t e = amk::launch_plain(d, workspace, workspace_bytes, h->f64, h->shape.nv,
                                   static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "plain path launch");
  if (st->res) {
    // the plain path forms the statistics with the residual kernel
    e = amk::launch_residuals(d, h->c.tP, h->c.tPd, h->c.tPdd, st->res, h->f64, h->shape.nv,
                              static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "residual kernel launch");
  }
  return AM_OK;
}

}  // extern "C"
