// am_server.cpp -- continuous-batching replanning server over the batched AM
// solver (C-ABI in include/am.h).
//
// Requests are queued by am_server_submit (any thread).  One scheduler
// thread owns the device side: it retires finished launches (event queries),
// keeps each finished request's state as its client's warm-start block (the
// multipliers seed the client's next request, as the paper's MPC warm-starts
// lambda from the previous control loop), and admits pending requests in
// arrival order into the next free launch slot while the device-memory
// budget allows; when it does not, warm blocks of idle clients are dropped,
// least recently used first (their next request starts from lambda = 0).
// All requests admitted together go out as one multi-problem launch; several
// launches can be in flight on separate streams, so admission does not wait
// for the GPU to drain.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "am.h"
#include "am_internal.h"

namespace {

using Clock = std::chrono::steady_clock;
constexpr int kMaxStreams = 16;
constexpr int kMaxPerLaunch = 256;
constexpr size_t kPinnedArena = size_t(64) << 20;   // pinned host bytes for queued requests' input
constexpr size_t kAlign = 256;

size_t round_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// First-fit allocator over one device allocation (offsets only).
class Arena {
 public:
  void init(size_t bytes) { free_[0] = bytes; cap_ = bytes; }
  bool alloc(size_t bytes, size_t *off) {
    bytes = round_up(bytes);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        *off = it->first;
        const size_t rest = it->second - bytes, start = it->first + bytes;
        free_.erase(it);
        if (rest) free_[start] = rest;
        used_ += bytes;
        peak_ = std::max(peak_, used_);
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    bytes = round_up(bytes);
    used_ -= bytes;
    auto it = free_.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
  size_t capacity() const { return cap_; }
  size_t peak() const { return peak_; }

 private:
  std::map<size_t, size_t> free_;
  size_t cap_ = 0, used_ = 0, peak_ = 0;
};

struct Block {      // one arena allocation
  size_t off = 0, bytes = 0;
  bool live = false;
  int B = 0, nv = 0, q = 0;  // layout of a warm block's state
  uint64_t used = 0;  // last use (warm blocks, LRU)
};

struct Request {
  int64_t ticket;
  am_handle *h;
  int client, B, K, q, nv, n;
  // host input in the solve's precision, laid out as on the device: the
  // obstacle table (x [n][q], y [n][q], a [n], b [n]) then the coefficients
  // [5][B][nv]; written by the submitting thread into the server's pinned
  // arena (copied to the device straight from there), or into in_vec when
  // the arena is full
  char *in = nullptr;
  size_t in_off = 0, in_bytes = 0;
  bool in_pinned = false;
  std::vector<char> in_vec;
  am_problem prob;                 // scalars (device pointers filled at admission)
  Clock::time_point t_submit, t_done;
  bool done = false;
  int status = AM_OK;
  std::string error;               // message of a failed launch
  Block state, table, work;        // state + trajectories, obstacle table, plain workspace
  Block warm_src;                  // the client's warm block used at admission (if any)
  char *best_host = nullptr;       // pinned copy of (cost, max |f_c|, index) of the best trajectory
  int32_t best = -1;               // best trajectory (AM selection rule), -1 if none or not selected
  double best_cost = 0.0, best_fc = 0.0;
};

struct Slot {                      // one launch in flight
  hipStream_t stream = nullptr;
  hipEvent_t event = nullptr;
  void *pinned = nullptr;          // staging for host->device copies
  size_t pinned_bytes = 0;
  Block desc;                      // problem table of multi-problem launches
  std::vector<Request *> reqs;
  bool busy = false;
};

size_t elem_size(int dtype) { return dtype == AM_F64 ? 8 : 4; }

// Device state of one request: cx, cc, cy, cs, cpsi, lam, lam_psi, traj,
// residual rows [B][AM_NRES] and the best-trajectory record (cost, max |f_c|,
// int32 index: 4 elements).
constexpr int kBestElems = 4;
size_t state_elems(int B, int nv, int q) { return size_t(B) * (10 * nv + 3 * q + AM_NRES) + kBestElems; }
size_t table_elems(int n, int q) { return size_t(2 * n * q + 2 * n); }

}  // namespace

struct am_server {
  am_server_config cfg;
  int device = 0;
  char *base = nullptr;
  Arena arena;
  // pinned host arena for the requests' input (its own lock: submitting
  // threads allocate, the scheduler releases at retirement)
  char *pin_base = nullptr;
  Arena pin_arena;
  std::mutex pin_mu;
  std::vector<Slot> slots;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Request *> pending;
  std::unordered_map<int64_t, std::unique_ptr<Request>> all;
  std::unordered_map<int, Block> warm;          // client -> state of its last result
  uint64_t clock = 0;                            // LRU counter of warm blocks
  std::unordered_map<int, int64_t> client_busy;  // client -> ticket in flight
  int64_t next_ticket = 0, completed = 0, launches = 0, memory_waits = 0, evictions = 0;
  bool stop = false;
  Clock::time_point last_activity = Clock::now();   // last launch, retirement or submission
  std::string error;
  std::thread worker;
  // KKT cache: handles built for requests that name a shape instead of a
  // handle, keyed by every field that fixes the KKT and the kernels
  std::mutex cache_mu;
  std::map<std::string, am_handle *> kkt_cache;

  void *ptr(const Block &b) const { return base + b.off; }
  void release_input(Request *r) {
    if (r->in_pinned) {
      std::lock_guard<std::mutex> lk(pin_mu);
      pin_arena.release(r->in_off, r->in_bytes);
      r->in_pinned = false;
    }
    r->in = nullptr;
    std::vector<char>().swap(r->in_vec);
  }
  bool alloc_evicting(size_t bytes, int keep_client, size_t *off);
  void run();
  bool admit(Slot &slot, std::vector<Request *> &batch);
  int launch(Slot &slot);
  void retire(Slot &slot);
};

namespace {

int srv_fail(int code, const std::string &msg) { return amk::set_last_error(code, msg.c_str()); }

}  // namespace

// Request state pointers inside its block.
static am_state state_of(const am_server *s, const Request *r, const Block &b) {
  const size_t es = elem_size(s->cfg.dtype);
  char *p = s->base + b.off;
  const size_t row = size_t(r->B) * r->nv * es;
  am_state st;
  std::memset(&st, 0, sizeof st);
  st.cx = p; st.cc = p + row; st.cy = p + 2 * row; st.cs = p + 3 * row; st.cpsi = p + 4 * row;
  st.lam = p + 5 * row;                 // 4 nv per trajectory
  st.lam_psi = p + 9 * row;
  st.traj = p + 10 * row;               // [B][3][q]
  return st;
}

// Residual rows and best-trajectory record of a request (after traj).
static char *residuals_of(const am_server *s, const Request *r, const Block &b) {
  const size_t es = elem_size(s->cfg.dtype);
  return s->base + b.off + size_t(r->B) * (10 * r->nv + 3 * r->q) * es;
}
static char *best_of(const am_server *s, const Request *r, const Block &b) {
  return residuals_of(s, r, b) + size_t(r->B) * AM_NRES * elem_size(s->cfg.dtype);
}

bool am_server::alloc_evicting(size_t bytes, int keep_client, size_t *off) {
  // mu held
  while (!arena.alloc(bytes, off)) {
    int victim = -1;
    uint64_t oldest = ~uint64_t(0);
    for (auto &kv : warm)
      if (kv.first != keep_client && !client_busy.count(kv.first) && kv.second.used < oldest) {
        oldest = kv.second.used;
        victim = kv.first;
      }
    if (victim < 0) return false;
    arena.release(warm[victim].off, warm[victim].bytes);
    warm.erase(victim);
    ++evictions;
  }
  return true;
}

bool am_server::admit(Slot &slot, std::vector<Request *> &batch) {
  // called with mu held; arrival order, a client's requests one at a time.
  // One launch holds requests of one (q, nv) (the multi-problem launch's
  // condition): the first admissible request fixes them, and requests of
  // another (q, nv) keep their place for a later launch.
  const int cap = cfg.mode == AM_SERVE_CONTINUOUS ? cfg.max_per_launch : 1;
  const size_t es = elem_size(cfg.dtype);
  int q0 = -1, nv0 = -1;
  for (auto it = pending.begin(); it != pending.end() && int(batch.size()) < cap;) {
    Request *r = *it;
    if (client_busy.count(r->client)) { ++it; continue; }
    if (q0 >= 0 && (r->q != q0 || r->nv != nv0)) { ++it; continue; }
    const size_t sb = state_elems(r->B, r->nv, r->q) * es, tb = table_elems(r->n, r->q) * es;
    size_t wb = 0;
    if (cfg.mode == AM_SERVE_PLAIN) am_plain_workspace_size(r->h, r->B, &wb);
    Block st{0, sb, false}, tab{0, tb, false}, wk{0, wb, false};
    bool ok = alloc_evicting(sb, r->client, &st.off);
    if (ok) { st.live = true; ok = alloc_evicting(tb, r->client, &tab.off); if (ok) tab.live = true; }
    if (ok && wb) { ok = alloc_evicting(wb, r->client, &wk.off); if (ok) wk.live = true; }
    if (!ok) {
      if (st.live) arena.release(st.off, st.bytes);
      if (tab.live) arena.release(tab.off, tab.bytes);
      ++memory_waits;
      break;   // keep arrival order: later requests wait behind this one
    }
    r->state = st; r->table = tab; r->work = wk;
    r->warm_src = Block{};
    q0 = r->q;
    nv0 = r->nv;
    // the client's last result seeds the multipliers when its layout matches
    // this request's (same batch, coefficients and time steps)
    auto wit = warm.find(r->client);
    if (wit != warm.end() && wit->second.B == r->B && wit->second.nv == r->nv && wit->second.q == r->q) {
      wit->second.used = ++clock;
      r->warm_src = wit->second;
    }
    client_busy[r->client] = r->ticket;
    batch.push_back(r);
    it = pending.erase(it);
  }
  slot.reqs = batch;
  return !batch.empty();
}

int am_server::launch(Slot &slot) {
  // copies and the solve, all on the slot's stream (mu not held)
  const size_t es = elem_size(cfg.dtype);
  size_t need = 0;
  for (Request *r : slot.reqs) need += (r->in_pinned ? 0 : r->in_bytes) + kBestElems * es;
  if (need > slot.pinned_bytes) {
    if (slot.pinned) (void)hipHostFree(slot.pinned);
    slot.pinned = nullptr;
    slot.pinned_bytes = 0;
    if (hipHostMalloc(&slot.pinned, need * 2) != hipSuccess) return AM_ERR_HIP;
    slot.pinned_bytes = need * 2;
  }
  char *stage = static_cast<char *>(slot.pinned);
  std::vector<am_handle *> hs;
  std::vector<am_problem> ps;
  std::vector<int32_t> bs, ks;
  std::vector<am_state> sts;
  for (Request *r : slot.reqs) {
    const size_t nq = size_t(r->n) * r->q;
    const size_t tab = table_elems(r->n, r->q) * es, coef = size_t(r->B) * r->nv * es;
    // the request's input goes to the device from the pinned arena, or
    // through the slot's staging when it did not fit there
    const char *src = r->in;
    if (!r->in_pinned) {
      std::memcpy(stage, r->in, r->in_bytes);
      src = stage;
      stage += r->in_bytes;
    }
    char *tdev = base + r->table.off;
    if (tab && hipMemcpyAsync(tdev, src, tab, hipMemcpyHostToDevice, slot.stream) != hipSuccess) return AM_ERR_HIP;
    am_problem p = r->prob;
    p.obs_x = tdev; p.obs_y = tdev + nq * es; p.obs_a = tdev + 2 * nq * es; p.obs_b = tdev + (2 * nq + r->n) * es;
    if (r->n == 0) p.obs_x = p.obs_y = p.obs_a = p.obs_b = nullptr;
    // initial coefficients from the request (fresh samples each replan);
    // multipliers from the client's previous result (Sec. IV: lambda is
    // warm-started from the previous control loop), else zero
    const am_state st = state_of(this, r, r->state);
    if (hipMemcpyAsync(st.cx, src + tab, 5 * coef, hipMemcpyHostToDevice, slot.stream) != hipSuccess)
      return AM_ERR_HIP;
    auto wit = r->warm_src;
    // lambda [B][4nv] and lambda_psi [B][nv] are contiguous after the coefficients
    if (wit.live) {
      if (hipMemcpyAsync(st.lam, base + wit.off + 5 * coef, 5 * coef, hipMemcpyDeviceToDevice, slot.stream) !=
          hipSuccess)
        return AM_ERR_HIP;
    } else if (hipMemsetAsync(st.lam, 0, 5 * coef, slot.stream) != hipSuccess) {
      return AM_ERR_HIP;
    }
    am_state sr = st;
    if (cfg.select_best) sr.res = residuals_of(this, r, r->state);   // formed by the solve itself
    hs.push_back(r->h); ps.push_back(p); bs.push_back(r->B); ks.push_back(r->K); sts.push_back(sr);
  }
  int rc = AM_OK;
  if (cfg.mode == AM_SERVE_PLAIN) {
    Request *r = slot.reqs[0];
    rc = am_solve_batch_plain(r->h, &ps[0], r->B, r->K, &sts[0], base + r->work.off, r->work.bytes, slot.stream);
  } else if (hs.size() == 1) {
    // one request: the single-problem launch (descriptor as a kernel
    // argument, no table copy); bit-identical to its multi-problem form
    rc = am_solve_batch(hs[0], &ps[0], bs[0], ks[0], &sts[0], slot.stream);
  } else {
    rc = am_solve_multi(int32_t(hs.size()), hs.data(), ps.data(), bs.data(), ks.data(), sts.data(),
                        base + slot.desc.off, slot.desc.bytes, slot.stream);
  }
  if (rc != AM_OK) return rc;
  if (cfg.select_best) {
    // the best trajectory by the selection rule from the residual rows the
    // solve wrote, and its record to pinned memory (read at retirement)
    for (size_t i = 0; i < slot.reqs.size(); ++i) {
      Request *r = slot.reqs[i];
      char *res = residuals_of(this, r, r->state), *rec = best_of(this, r, r->state);
      if ((rc = am_select_best(r->h, r->B, res, cfg.fc_tol, reinterpret_cast<int32_t *>(rec + 2 * es), rec,
                               slot.stream)) != AM_OK)
        return rc;
      r->best_host = stage;
      if (hipMemcpyAsync(stage, rec, kBestElems * es, hipMemcpyDeviceToHost, slot.stream) != hipSuccess)
        return AM_ERR_HIP;
      stage += kBestElems * es;
    }
  }
  if (hipEventRecord(slot.event, slot.stream) != hipSuccess) return AM_ERR_HIP;
  return AM_OK;
}

void am_server::retire(Slot &slot) {
  // mu held; the slot's event has completed
  const auto now = Clock::now();
  const bool f64 = cfg.dtype == AM_F64;
  for (Request *r : slot.reqs) {
    r->t_done = now;
    r->done = true;
    if (cfg.select_best && r->best_host && r->status == AM_OK) {
      const size_t es = elem_size(cfg.dtype);
      std::memcpy(&r->best, r->best_host + 2 * es, sizeof(int32_t));
      r->best_cost = f64 ? reinterpret_cast<const double *>(r->best_host)[0]
                         : double(reinterpret_cast<const float *>(r->best_host)[0]);
      r->best_fc = f64 ? reinterpret_cast<const double *>(r->best_host)[1]
                       : double(reinterpret_cast<const float *>(r->best_host)[1]);
    }
    r->best_host = nullptr;
    if (r->status == AM_OK) {
      auto wit = warm.find(r->client);
      if (wit != warm.end()) arena.release(wit->second.off, wit->second.bytes);
      Block w = r->state;                  // the result seeds the client's next request
      w.B = r->B;
      w.nv = r->nv;
      w.q = r->q;
      w.used = ++clock;
      warm[r->client] = w;
    } else {
      // a failed launch leaves no result: the client keeps its previous warm block
      arena.release(r->state.off, r->state.bytes);
    }
    arena.release(r->table.off, r->table.bytes);
    if (r->work.live) arena.release(r->work.off, r->work.bytes);
    release_input(r);
    client_busy.erase(r->client);
    ++completed;
  }
  slot.reqs.clear();
  slot.busy = false;
}

void am_server::run() {
  (void)hipSetDevice(device);
  std::unique_lock<std::mutex> lk(mu);
  while (true) {
    bool progressed = false;
    for (Slot &s : slots)
      if (s.busy && hipEventQuery(s.event) == hipSuccess) {
        retire(s);
        progressed = true;
      }
    if (progressed) cv_done.notify_all();
    for (Slot &s : slots) {
      if (s.busy || pending.empty()) continue;
      std::vector<Request *> batch;
      if (!admit(s, batch)) break;
      s.busy = true;
      ++launches;
      lk.unlock();
      const int rc = launch(s);
      lk.lock();
      if (rc != AM_OK) {
        // a failed launch completes its requests with the error (and the
        // message this thread recorded)
        const std::string msg = am_last_error();
        (void)hipStreamSynchronize(s.stream);
        for (Request *r : s.reqs) {
          r->status = rc;
          r->error = msg;
        }
        retire(s);
        cv_done.notify_all();
      }
      progressed = true;
    }
    bool busy = false;
    for (Slot &s : slots) busy |= s.busy;
    if (stop && !busy && pending.empty()) break;
    const auto now = Clock::now();
    if (progressed) last_activity = now;
    if (!progressed) {
      const bool spin = busy || std::chrono::duration_cast<std::chrono::microseconds>(now - last_activity).count() <
                                    cfg.idle_spin_us;
      if (spin) {
        // work in flight (or the idle-spin window): poll without sleeping (a
        // timed wait would add the scheduler's timer slack to every
        // completion, a wake-up the OS wake-up time to every arrival)
        lk.unlock();
        std::this_thread::yield();
        lk.lock();
      } else {
        cv_work.wait_for(lk, std::chrono::milliseconds(5));
      }
    }
  }
}

extern "C" {

int am_server_create(const am_server_config *cfg, am_server **out) {
  if (!out) return srv_fail(AM_ERR_INVALID, "out is NULL");
  *out = nullptr;
  if (!cfg) return srv_fail(AM_ERR_INVALID, "config is NULL");
  if (cfg->hbm_budget == 0) return srv_fail(AM_ERR_INVALID, "hbm_budget must be > 0");
  if (cfg->mode < AM_SERVE_CONTINUOUS || cfg->mode > AM_SERVE_PLAIN) return srv_fail(AM_ERR_INVALID, "bad mode");
  if (cfg->dtype != AM_F32 && cfg->dtype != AM_F64) return srv_fail(AM_ERR_INVALID, "bad dtype");
  if (cfg->streams < 1 || cfg->streams > kMaxStreams) return srv_fail(AM_ERR_INVALID, "streams must be 1..16");
  if (cfg->max_per_launch < 1 || cfg->max_per_launch > kMaxPerLaunch)
    return srv_fail(AM_ERR_INVALID, "max_per_launch must be 1..256");
  if (cfg->select_best && !(cfg->fc_tol >= 0.0)) return srv_fail(AM_ERR_INVALID, "fc_tol must be >= 0");
  if (cfg->idle_spin_us < 0 || cfg->idle_spin_us > 1000000)
    return srv_fail(AM_ERR_INVALID, "idle_spin_us must be 0..1000000");
  auto *s = new am_server();
  s->cfg = *cfg;
  if (cfg->mode != AM_SERVE_CONTINUOUS) { s->cfg.streams = 1; s->cfg.max_per_launch = 1; }
  if (hipGetDevice(&s->device) != hipSuccess) { delete s; return srv_fail(AM_ERR_HIP, "hipGetDevice"); }
  size_t desc_bytes = 0;
  am_multi_workspace_size(s->cfg.max_per_launch, &desc_bytes);
  const size_t total = round_up(cfg->hbm_budget) + size_t(s->cfg.streams) * round_up(desc_bytes);
  if (hipMalloc(reinterpret_cast<void **>(&s->base), total) != hipSuccess) {
    delete s;
    return srv_fail(AM_ERR_NOMEM, "hipMalloc of the server budget failed");
  }
  s->arena.init(round_up(cfg->hbm_budget));
  // (without the pinned arena every request goes through the slots' staging)
  if (hipHostMalloc(reinterpret_cast<void **>(&s->pin_base), kPinnedArena) == hipSuccess)
    s->pin_arena.init(kPinnedArena);
  else
    s->pin_base = nullptr;
  s->slots.resize(s->cfg.streams);
  for (int i = 0; i < s->cfg.streams; ++i) {
    Slot &sl = s->slots[i];
    sl.desc = Block{round_up(cfg->hbm_budget) + size_t(i) * round_up(desc_bytes), desc_bytes, true};
    if (hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&sl.event, hipEventDisableTiming) != hipSuccess) {
      am_server_destroy(s);
      return srv_fail(AM_ERR_HIP, "stream/event creation failed");
    }
    // a first operation on each stream, so that the runtime binds it to a
    // hardware queue now and not during the first request that overlaps
    // another (that first use costs milliseconds)
    if (hipMemsetAsync(s->base, 0, kAlign, sl.stream) != hipSuccess || hipStreamSynchronize(sl.stream) != hipSuccess) {
      am_server_destroy(s);
      return srv_fail(AM_ERR_HIP, "stream warm-up failed");
    }
  }
  s->worker = std::thread([s] { s->run(); });
  *out = s;
  return AM_OK;
}

int am_server_submit(am_server *s, const am_request *r, int64_t *ticket) {
  const auto t_submit = Clock::now();   // latency includes a KKT build on a cache miss
  if (!s || !r || !ticket) return srv_fail(AM_ERR_INVALID, "NULL argument");
  if ((!r->handle && !r->shape) || r->client < 0 || r->batch < 1 || r->iters < 0)
    return srv_fail(AM_ERR_INVALID, "request needs a handle or a shape, client >= 0, batch >= 1, iters >= 0");
  am_handle *handle = r->handle;
  if (!handle) {
    const am_shape &sh = *r->shape;
    if (sh.dtype != s->cfg.dtype) return srv_fail(AM_ERR_INVALID, "shape dtype differs from the server's");
    if (sh.m < 1 || sh.m > AM_MAX_CIRCLES || !sh.r_off) return srv_fail(AM_ERR_INVALID, "bad circle offsets");
    std::string key;
    auto put = [&](const void *p, size_t n) { key.append(static_cast<const char *>(p), n); };
    put(&sh.q, sizeof sh.q); put(&sh.nv, sizeof sh.nv); put(&sh.tf, sizeof sh.tf); put(&sh.m, sizeof sh.m);
    put(sh.r_off, sizeof(double) * size_t(sh.m)); put(&sh.n_obs, sizeof sh.n_obs); put(&sh.rho, sizeof sh.rho);
    put(&sh.rho_psi, sizeof sh.rho_psi); put(&sh.dtype, sizeof sh.dtype); put(&sh.flags, sizeof sh.flags);
    std::lock_guard<std::mutex> lk(s->cache_mu);
    auto it = s->kkt_cache.find(key);
    if (it != s->kkt_cache.end()) {
      handle = it->second;
    } else {
      const int rc = am_setup(&sh, &handle);
      if (rc != AM_OK) return rc;   // am_setup recorded the message
      s->kkt_cache.emplace(key, handle);
    }
  }
  auto req = std::make_unique<Request>();
  req->h = handle;
  req->client = r->client;
  req->B = r->batch;
  req->K = r->iters;
  const int q = amk::handle_q(handle), nv = amk::handle_nv(handle), n = amk::handle_n(handle);
  if (amk::handle_dtype(handle) != s->cfg.dtype) return srv_fail(AM_ERR_INVALID, "handle dtype differs from the server's");
  if (n > 0 && (!r->obs_x || !r->obs_y || !r->obs_a || !r->obs_b))
    return srv_fail(AM_ERR_INVALID, "obstacle arrays are NULL");
  req->q = q; req->nv = nv; req->n = n;
  if (!r->init) return srv_fail(AM_ERR_INVALID, "request needs initial coefficients (init)");
  std::memset(&req->prob, 0, sizeof req->prob);
  req->prob.r_circle = r->r_circle;
  for (int e = 0; e < 6; ++e) { req->prob.bc_x[e] = r->bc_x[e]; req->prob.bc_y[e] = r->bc_y[e]; req->prob.bc_psi[e] = r->bc_psi[e]; }
  req->prob.v_max = r->v_max;
  req->prob.a_max = r->a_max;
  const size_t es = elem_size(s->cfg.dtype);
  size_t wb = 0;
  if (s->cfg.mode == AM_SERVE_PLAIN) am_plain_workspace_size(handle, r->batch, &wb);
  const size_t need = round_up(state_elems(r->batch, nv, q) * es) + round_up(table_elems(n, q) * es) + round_up(wb);
  if (need > s->arena.capacity())
    return srv_fail(AM_ERR_INVALID, "request needs more device memory than the server budget");
  {
    // the input in the solve's precision and the device layout, written once
    const bool f64 = s->cfg.dtype == AM_F64;
    const size_t B = size_t(r->batch);
    req->in_bytes = (table_elems(n, q) + B * 5 * nv) * es;
    {
      std::lock_guard<std::mutex> lk(s->pin_mu);
      if (s->pin_base && s->pin_arena.alloc(req->in_bytes, &req->in_off)) {
        req->in = s->pin_base + req->in_off;
        req->in_pinned = true;
      }
    }
    if (!req->in_pinned) {
      req->in_vec.resize(req->in_bytes);
      req->in = req->in_vec.data();
    }
    char *d = req->in;
    auto put = [&](const double *src, size_t cnt) {
      if (f64) std::memcpy(d, src, cnt * sizeof(double));
      else {
        float *f = reinterpret_cast<float *>(d);
        for (size_t i = 0; i < cnt; ++i) f[i] = float(src[i]);
      }
      d += cnt * es;
    };
    if (n > 0) {
      put(r->obs_x, size_t(n) * q); put(r->obs_y, size_t(n) * q); put(r->obs_a, n); put(r->obs_b, n);
    }
    // [B][5][nv] -> [5][B][nv]
    for (int v = 0; v < 5; ++v)
      for (size_t l = 0; l < B; ++l) put(r->init + (l * 5 + v) * nv, size_t(nv));
  }
  req->t_submit = t_submit;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop) {
      s->release_input(req.get());
      return srv_fail(AM_ERR_INVALID, "server is stopping");
    }
    req->ticket = s->next_ticket++;
    *ticket = req->ticket;
    s->pending.push_back(req.get());
    s->all[req->ticket] = std::move(req);
  }
  s->cv_work.notify_one();
  return AM_OK;
}

int am_server_wait(am_server *s, int64_t ticket, double timeout_s, int32_t *done, double *latency_s, void *traj) {
  if (!s || !done) return srv_fail(AM_ERR_INVALID, "NULL argument");
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->all.find(ticket);
  if (it == s->all.end()) return srv_fail(AM_ERR_INVALID, "unknown ticket");
  Request *r = it->second.get();
  auto pred = [&] { return r->done; };
  if (timeout_s < 0) s->cv_done.wait(lk, pred);
  else s->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), pred);
  *done = r->done ? 1 : 0;
  if (!r->done) return AM_OK;
  if (r->status != AM_OK) return srv_fail(r->status, "request failed on the device: " + r->error);
  if (latency_s) *latency_s = std::chrono::duration<double>(r->t_done - r->t_submit).count();
  if (traj) {
    // the result lives in the client's warm slot until the client's next
    // request is admitted; copy it while holding the lock
    auto wit = s->warm.find(r->client);
    if (wit == s->warm.end() || wit->second.off != r->state.off)
      return srv_fail(AM_ERR_INVALID, "result was replaced by a later request of the same client");
    const am_state st = state_of(s, r, r->state);
    const size_t es = elem_size(s->cfg.dtype);
    if (hipMemcpy(traj, st.traj, size_t(r->B) * 3 * r->q * es, hipMemcpyDeviceToHost) != hipSuccess)
      return srv_fail(AM_ERR_HIP, "result copy failed");
  }
  return AM_OK;
}

int am_server_best(am_server *s, int64_t ticket, int32_t *index, double *cost, double *fc_max) {
  if (!s || !index) return srv_fail(AM_ERR_INVALID, "NULL argument");
  if (!s->cfg.select_best) return srv_fail(AM_ERR_INVALID, "the server was created without select_best");
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->all.find(ticket);
  if (it == s->all.end()) return srv_fail(AM_ERR_INVALID, "unknown ticket");
  const Request *r = it->second.get();
  if (!r->done) return srv_fail(AM_ERR_INVALID, "request " + std::to_string(ticket) + " is not finished");
  if (r->status != AM_OK) return srv_fail(r->status, "request failed on the device: " + r->error);
  *index = r->best;
  if (cost) *cost = r->best_cost;
  if (fc_max) *fc_max = r->best_fc;
  if (r->best < 0) return srv_fail(AM_ERR_NONFINITE, "every trajectory of the request is non-finite");
  return AM_OK;
}

int am_server_stats(am_server *s, int64_t *completed, int64_t *launches, size_t *peak_bytes, int64_t *memory_waits) {
  if (!s) return srv_fail(AM_ERR_INVALID, "server is NULL");
  std::lock_guard<std::mutex> lk(s->mu);
  if (completed) *completed = s->completed;
  if (launches) *launches = s->launches;
  if (peak_bytes) *peak_bytes = s->arena.peak();
  if (memory_waits) *memory_waits = s->memory_waits;
  return AM_OK;
}

void am_server_destroy(am_server *s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv_work.notify_all();
  if (s->worker.joinable()) s->worker.join();
  for (Slot &sl : s->slots) {
    if (sl.stream) { (void)hipStreamSynchronize(sl.stream); (void)hipStreamDestroy(sl.stream); }
    if (sl.event) (void)hipEventDestroy(sl.event);
    if (sl.pinned) (void)hipHostFree(sl.pinned);
  }
  if (s->base) (void)hipFree(s->base);
  if (s->pin_base) (void)hipHostFree(s->pin_base);
  for (auto &kv : s->kkt_cache) am_destroy(kv.second);
  delete s;
}

}  // extern "C"
