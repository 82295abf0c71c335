// Continuous-batching solver service.
//
// Requests (problem, options, host y) queue on the host.  Worker threads, one
// per HIP stream, admit them in arrival order as device memory in the
// caller's pool and request slots free up, and run them as waves:
//  * a persistent wave: every queued OMP problem the one-workgroup-per-problem
//    kernel takes (up to max_wave, same options), solved in one launch;
//  * a lockstep wave: requests the persistent kernel does not take (large N
//    or K, SP, CoSaMP) that share class and N (for SP and CoSaMP also M and
//    K), solved as one lockstep plan.
// With several streams worker 0 runs persistent waves only, so small requests
// never queue behind large ones; the other workers take the oldest large
// request first.  Waves on different streams overlap on the device.  Each request's device state
// (y, tables, kernel vector, h_0, Cholesky factor, x) stays in its wave's
// pool region from admission to completion; results come back to pinned host
// memory and the region is freed.  A request's arithmetic does not depend on
// the requests it shares a wave with.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <unordered_map>

#include "batch.h"
#include "plan.h"

using namespace fcmp;

namespace {

size_t pad256(size_t v) { return (v + 255) & ~(size_t)255; }

struct Req {
  uint64_t ticket = 0;
  fcmp_problem prob{};
  std::vector<int32_t> omega;
  fcmp_options opt{};
  std::vector<unsigned char> y;     // host copy of y
  bool small = false;               // taken by the persistent kernel
  size_t foot = 0;                  // device bytes when admitted alone
  int state = 0;                    // 0 queued, 1 running, 2 done
  int rc = FCMP_OK;
  std::string err;
  std::vector<int32_t> sup;
  std::vector<unsigned char> x;
  fcmp_stats stats{};
  fcmp_times times{};
  size_t wbytes() const { return prob.matrix_class == FCMP_FOURIER ? 16 : 8; }
  size_t ybytes() const { return (size_t)prob.M * wbytes(); }
  size_t io_bytes() const {
    return pad256(ybytes()) + pad256((size_t)prob.K * 4) + pad256((size_t)prob.K * wbytes());
  }
};

// First-fit allocator over the caller's pool (offsets, 256-byte granules).
class Arena {
 public:
  void init(size_t bytes) {
    free_.clear();
    free_[0] = bytes & ~(size_t)255;
    used_ = peak_ = 0;
  }
  size_t largest() const {
    size_t b = 0;
    for (auto& kv : free_) b = std::max(b, kv.second);
    return b;
  }
  bool take(size_t bytes, size_t* off) {
    bytes = pad256(bytes);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < bytes) continue;
      *off = it->first;
      const size_t rest = it->second - bytes;
      const size_t next = it->first + bytes;
      free_.erase(it);
      if (rest) free_[next] = rest;
      used_ += bytes;
      peak_ = std::max(peak_, used_);
      return true;
    }
    return false;
  }
  void give(size_t off, size_t bytes) {
    bytes = pad256(bytes);
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
  size_t peak() const { return peak_; }

 private:
  std::map<size_t, size_t> free_;
  size_t used_ = 0, peak_ = 0;
};

bool same_opts(const fcmp_options& a, const fcmp_options& b) {
  return a.algorithm == b.algorithm && a.corr_method == b.corr_method &&
         a.corr_precision == b.corr_precision && a.max_iter == b.max_iter &&
         a.switch_t == b.switch_t && a.flags == b.flags;
}

// Requests that may share a lockstep wave: OMP plans take per-instance M and
// K, so one (class, N) (an instance whose K selections are made stops taking
// device time; the wave ends with its longest solve); SP and CoSaMP need one
// shape.
bool same_group(const fcmp_problem& a, const fcmp_problem& b, int algorithm) {
  if (a.matrix_class != b.matrix_class || a.N != b.N) return false;
  if (algorithm == FCMP_OMP) return true;
  return a.M == b.M && a.K == b.K;
}

// Device bytes of the solver state of n requests run as one wave.
int wave_state_bytes(const std::vector<Req*>& w, bool small, size_t* bytes) {
  std::vector<fcmp_problem> probs;
  for (Req* r : w) probs.push_back(r->prob);
  int rc;
  if (small) {
    WgBatch B;
    std::vector<int64_t> ids(w.size());
    for (size_t i = 0; i < w.size(); ++i) ids[i] = (int64_t)i;
    if ((rc = wg_plan_init(B, (int64_t)w.size(), probs.data(), ids.data(), &w[0]->opt))) return rc;
    *bytes = pad256(B.total);
  } else {
    fcmp_plan P;
    if ((rc = plan_init(P, (int64_t)w.size(), probs.data(), &w[0]->opt))) return rc;
    *bytes = pad256(P.total);
  }
  return FCMP_OK;
}

double now_ms(std::chrono::steady_clock::time_point t0) {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace

struct fcmp_server {
  int device = 0;
  char* pool = nullptr;
  size_t pool_bytes = 0;
  fcmp_server_config cfg{};
  std::chrono::steady_clock::time_point t0;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Req*> queue;                        // not yet admitted, arrival order
  std::unordered_map<uint64_t, Req*> reqs;       // every request not yet collected
  uint64_t next_ticket = 1;
  int inflight = 0;                              // admitted, not finished
  Arena arena;
  bool stop = false;
  fcmp_server_info info{};
  std::vector<hipStream_t> streams;
  std::vector<std::thread> workers;
};

namespace {

// Pinned staging owned by one worker.
struct Staging {
  unsigned char* p = nullptr;
  size_t bytes = 0;
  int ensure(size_t want) {
    if (want <= bytes) return FCMP_OK;
    if (p) (void)hipHostFree(p);
    p = nullptr;
    bytes = 0;
    size_t b = std::max(want, (size_t)1 << 20);
    if (hipHostMalloc((void**)&p, b, hipHostMallocDefault) != hipSuccess)
      return set_error(FCMP_E_DEVICE, "pinned staging allocation failed");
    bytes = b;
    return FCMP_OK;
  }
  ~Staging() {
    if (p) (void)hipHostFree(p);
  }
};

#define HIP_TRY(expr)                                                              \
  do {                                                                             \
    hipError_t _e = (expr);                                                        \
    if (_e != hipSuccess)                                                          \
      return set_error(FCMP_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(_e)); \
  } while (0)

// Runs one wave in the pool region at base (state bytes, then the requests'
// y / support / x) on stream st and fills the requests' results.
int run_wave(fcmp_server* S, std::vector<Req*>& w, bool small, char* base, size_t state_bytes,
             hipStream_t st, hipEvent_t ev, Staging& stg) {
  const size_t n = w.size();
  std::vector<fcmp_problem> probs;
  for (Req* r : w) probs.push_back(r->prob);
  // io layout: y_0..y_{n-1}, then support_0.., then x_0..
  std::vector<size_t> oy(n), os(n), ox(n);
  size_t o = 0;
  for (size_t i = 0; i < n; ++i) { oy[i] = o; o += pad256(w[i]->ybytes()); }
  const size_t out_begin = o;
  for (size_t i = 0; i < n; ++i) { os[i] = o; o += pad256((size_t)w[i]->prob.K * 4); }
  for (size_t i = 0; i < n; ++i) { ox[i] = o; o += pad256((size_t)w[i]->prob.K * w[i]->wbytes()); }
  const size_t io_total = o;
  const size_t ptr_off = pad256(io_total);
  const size_t st_off = ptr_off + pad256(3 * n * sizeof(void*));
  const size_t stg_total = st_off + n * sizeof(Status);
  int rc = stg.ensure(stg_total);
  if (rc) return rc;
  char* io = base + state_bytes;
  for (size_t i = 0; i < n; ++i) std::memcpy(stg.p + oy[i], w[i]->y.data(), w[i]->ybytes());
  HIP_TRY(hipMemcpyAsync(io, stg.p, out_begin, hipMemcpyHostToDevice, st));
  std::vector<const void*> yd(n);
  std::vector<int32_t*> sd(n);
  std::vector<void*> xd(n);
  for (size_t i = 0; i < n; ++i) {
    yd[i] = io + oy[i];
    sd[i] = (int32_t*)(io + os[i]);
    xd[i] = io + ox[i];
  }
  const Status* dstatus = nullptr;
  std::vector<int64_t> order(n);   // internal position -> wave index
  if (small) {
    WgBatch B;
    std::vector<int64_t> ids(n);
    for (size_t i = 0; i < n; ++i) ids[i] = (int64_t)i;
    if ((rc = wg_plan_init(B, (int64_t)n, probs.data(), ids.data(), &w[0]->opt))) return rc;
    wg_layout(B, probs.data(), base);
    if ((rc = wg_build(B, probs.data(), st))) return rc;
    void** hp = (void**)(stg.p + ptr_off);
    wg_host_ptrs(B, yd.data(), sd.data(), xd.data(), hp);
    HIP_TRY(hipMemcpyAsync(B.ptrs, hp, 3 * n * sizeof(void*), hipMemcpyHostToDevice, st));
    if ((rc = wg_run(B, nullptr, st))) return rc;
    dstatus = B.status;
    for (size_t q = 0; q < n; ++q) order[q] = B.order_ids[q];
  } else {
    fcmp_plan P;
    if ((rc = plan_init(P, (int64_t)n, probs.data(), &w[0]->opt))) return rc;
    plan_layout(P, base);
    if ((rc = plan_build(P, probs.data(), st))) return rc;
    rc = plan_solve(P, nullptr, yd.data(), sd.data(), xd.data(), nullptr, st);
    if (rc && rc != FCMP_E_NUMERIC) return rc;
    dstatus = P.status;
    for (size_t q = 0; q < n; ++q) order[q] = (int64_t)q;
  }
  HIP_TRY(hipMemcpyAsync(stg.p + out_begin, io + out_begin, io_total - out_begin,
                         hipMemcpyDeviceToHost, st));
  HIP_TRY(hipMemcpyAsync(stg.p + st_off, dstatus, n * sizeof(Status), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipEventRecord(ev, st));
  HIP_TRY(hipEventSynchronize(ev));
  const double t = now_ms(S->t0);
  int khz = 100000;
  if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, S->device) != hipSuccess ||
      khz <= 0)
    khz = 100000;
  const Status* hs = (const Status*)(stg.p + st_off);
  for (size_t q = 0; q < n; ++q) {
    Req* r = w[order[q]];
    const size_t i = (size_t)order[q];
    r->sup.assign((const int32_t*)(stg.p + os[i]), (const int32_t*)(stg.p + os[i]) + r->prob.K);
    r->x.assign(stg.p + ox[i], stg.p + ox[i] + (size_t)r->prob.K * r->wbytes());
    r->stats = fcmp_stats{};
    r->stats.iterations = hs[q].iterations;
    r->stats.status_detail = hs[q].numeric ? FCMP_E_NUMERIC : FCMP_OK;
    r->stats.min_gap = hs[q].min_gap;
    const double r2 = hs[q].ynorm2 - hs[q].znorm2;
    r->stats.res_norm = r2 > 0 ? std::sqrt(r2) : 0.0;
    r->stats.ms_total = small ? hs[q].t_done / (double)khz : t - r->times.t_launch;
    r->times.t_done = t;
    r->rc = r->stats.status_detail;
  }
  return FCMP_OK;
}

// Picks the next wave under the lock; returns false when nothing can start.
bool form_wave(fcmp_server* S, int worker, std::vector<Req*>& w, bool& small, size_t& off,
               size_t& state_bytes, size_t& total) {
  w.clear();
  const int slots = S->cfg.max_slots - S->inflight;
  if (slots <= 0 || S->queue.empty()) return false;
  const size_t room = S->arena.largest();
  // large first on the general workers (every worker when there is one stream)
  if (worker > 0 || S->streams.size() == 1) {
    for (size_t k = 0; k < S->queue.size(); ++k) {
      Req* h = S->queue[k];
      if (h->small) continue;
      std::vector<Req*> cand{h};
      for (size_t j = k + 1; j < S->queue.size() && (int)cand.size() < std::min(slots, 64); ++j) {
        Req* r = S->queue[j];
        if (!r->small && same_opts(r->opt, h->opt) &&
            same_group(r->prob, h->prob, h->opt.algorithm))
          cand.push_back(r);
      }
      size_t sb = 0;
      while (!cand.empty()) {
        size_t io = 0;
        for (Req* r : cand) io += r->io_bytes();
        if (wave_state_bytes(cand, false, &sb) == FCMP_OK && sb + io <= room &&
            S->arena.take(sb + io, &off)) {
          w = cand;
          small = false;
          state_bytes = sb;
          total = sb + io;
          return true;
        }
        if (cand.size() == 1) break;
        cand.resize(cand.size() / 2);
      }
      break;   // the oldest large request does not fit yet: keep arrival order among large ones
    }
  }
  // a persistent wave: queued small requests sharing the oldest one's options
  Req* h = nullptr;
  for (Req* r : S->queue)
    if (r->small) { h = r; break; }
  if (!h) return false;
  std::vector<Req*> cand;
  size_t bound = 0;
  const int cap = std::min(slots, S->cfg.max_wave);
  for (Req* r : S->queue) {
    if ((int)cand.size() >= cap) break;
    if (!r->small || !same_opts(r->opt, h->opt)) continue;
    if (bound + r->foot > room) break;
    bound += r->foot;
    cand.push_back(r);
  }
  while (!cand.empty()) {
    size_t io = 0, sb = 0;
    for (Req* r : cand) io += r->io_bytes();
    if (wave_state_bytes(cand, true, &sb) == FCMP_OK && S->arena.take(sb + io, &off)) {
      w = cand;
      small = true;
      state_bytes = sb;
      total = sb + io;
      return true;
    }
    cand.resize(cand.size() / 2);
  }
  return false;
}

void worker_main(fcmp_server* S, int k) {
  // a failure here resurfaces as an error of this worker's first device call
  (void)hipSetDevice(S->device);
  hipStream_t st = S->streams[k];
  hipEvent_t ev = nullptr;
  // without the event every wave of this worker fails with a device error
  if (hipEventCreateWithFlags(&ev, hipEventBlockingSync | hipEventDisableTiming) != hipSuccess)
    ev = nullptr;
  Staging stg;
  std::vector<Req*> w;
  std::unique_lock<std::mutex> lk(S->mu);
  for (;;) {
    bool small = false;
    size_t off = 0, sb = 0, total = 0;
    while (!S->stop && !form_wave(S, k, w, small, off, sb, total)) S->cv_work.wait(lk);
    if (S->stop) break;
    // admit: leave the queue, keep arrival order among the rest
    const double t = now_ms(S->t0);
    for (Req* r : w) {
      r->state = 1;
      r->times.t_launch = t;
      S->queue.erase(std::find(S->queue.begin(), S->queue.end(), r));
    }
    S->inflight += (int)w.size();
    S->info.waves++;
    S->info.pool_peak = std::max<int64_t>(S->info.pool_peak, (int64_t)S->arena.peak());
    lk.unlock();
    int rc = ev ? run_wave(S, w, small, S->pool + off, sb, st, ev, stg)
                : set_error(FCMP_E_DEVICE, "event creation failed");
    std::string msg = rc ? last_error() : std::string();
    if (rc) (void)hipStreamSynchronize(st);   // nothing of the wave may still use the region
    lk.lock();
    for (Req* r : w) {
      if (rc) {
        r->rc = rc;
        r->err = msg;
        r->times.t_done = now_ms(S->t0);
      }
      r->state = 2;
    }
    S->arena.give(off, total);
    S->inflight -= (int)w.size();
    S->info.completed += (int64_t)w.size();
    S->cv_done.notify_all();
    S->cv_work.notify_all();
  }
  lk.unlock();
  if (ev) (void)hipEventDestroy(ev);
}

int request_footprint(const fcmp_problem* prob, const fcmp_options* opt, bool* small,
                      size_t* bytes) {
  int rc = validate_problem(prob, true);
  if (rc) return rc;
  if ((rc = validate_options(prob, opt))) return rc;
  Req r;
  r.prob = *prob;
  r.opt = *opt;
  r.small = !(opt->flags & FCMP_FLAG_NO_PERSISTENT) && wg_eligible(*prob, *opt);
  std::vector<Req*> one{&r};
  size_t sb = 0;
  if ((rc = wave_state_bytes(one, r.small, &sb))) return rc;
  *bytes = sb + r.io_bytes();
  if (small) *small = r.small;
  return FCMP_OK;
}

}  // namespace

extern "C" {

int fcmp_server_footprint(const fcmp_problem* prob, const fcmp_options* opt, size_t* bytes) {
  if (!bytes) return set_error(FCMP_E_INVALID, "bytes is NULL");
  return request_footprint(prob, opt, nullptr, bytes);
}

int fcmp_server_create(fcmp_server** out, void* pool_dev, size_t pool_bytes,
                       const fcmp_server_config* cfg) {
  if (!out) return set_error(FCMP_E_INVALID, "out is NULL");
  *out = nullptr;
  if (!pool_dev || pool_bytes < 4096) return set_error(FCMP_E_INVALID, "pool missing or too small");
  fcmp_server_config c{};
  if (cfg) c = *cfg;
  if (c.max_slots < 0 || c.max_pending < 0 || c.n_streams < 0 || c.n_streams > 8 ||
      c.max_wave < 0)
    return set_error(FCMP_E_INVALID, "bad server configuration");
  if (c.max_slots == 0) c.max_slots = 4096;
  if (c.max_pending == 0) c.max_pending = 1 << 16;
  if (c.n_streams == 0) c.n_streams = 4;
  if (c.max_wave == 0) c.max_wave = 1024;
  fcmp_server* S = new fcmp_server();
  S->cfg = c;
  S->pool = (char*)pool_dev;
  S->pool_bytes = pool_bytes;
  S->arena.init(pool_bytes);
  S->t0 = std::chrono::steady_clock::now();
  if (hipGetDevice(&S->device) != hipSuccess) {
    delete S;
    return set_error(FCMP_E_DEVICE, "hipGetDevice failed");
  }
  for (int k = 0; k < c.n_streams; ++k) {
    hipStream_t st = nullptr;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
      for (hipStream_t s : S->streams) (void)hipStreamDestroy(s);
      delete S;
      return set_error(FCMP_E_DEVICE, "stream creation failed");
    }
    S->streams.push_back(st);
  }
  for (int k = 0; k < c.n_streams; ++k) S->workers.emplace_back(worker_main, S, k);
  *out = S;
  return FCMP_OK;
}

int fcmp_server_submit(fcmp_server* S, const fcmp_problem* prob, const fcmp_options* opt,
                       const void* y_host, uint64_t* ticket) {
  if (!S || !ticket || !y_host) return set_error(FCMP_E_INVALID, "NULL argument");
  bool small = false;
  size_t foot = 0;
  int rc = request_footprint(prob, opt, &small, &foot);
  if (rc) return rc;
  if (pad256(foot) > (S->pool_bytes & ~(size_t)255))
    return set_error(FCMP_E_WORKSPACE, "request needs more device memory than the pool holds");
  Req* r = new Req();
  r->prob = *prob;
  r->omega.assign(prob->omega, prob->omega + prob->M);
  r->prob.omega = r->omega.data();
  r->opt = *opt;
  r->small = small;
  r->foot = foot;
  r->y.assign((const unsigned char*)y_host, (const unsigned char*)y_host + r->ybytes());
  std::lock_guard<std::mutex> lk(S->mu);
  if ((int64_t)S->queue.size() >= S->cfg.max_pending) {
    delete r;
    return set_error(FCMP_E_BUSY, "server queue full");
  }
  r->ticket = S->next_ticket++;
  r->times.t_submit = now_ms(S->t0);
  S->queue.push_back(r);
  S->reqs[r->ticket] = r;
  S->info.submitted++;
  *ticket = r->ticket;
  S->cv_work.notify_all();
  return FCMP_OK;
}

int fcmp_server_poll(fcmp_server* S, uint64_t ticket, int32_t* support_host, void* x_host,
                     fcmp_stats* stats, fcmp_times* times, int32_t* done) {
  if (!S || !done) return set_error(FCMP_E_INVALID, "NULL argument");
  Req* r = nullptr;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->reqs.find(ticket);
    if (it == S->reqs.end()) return set_error(FCMP_E_NOTFOUND, "unknown ticket");
    r = it->second;
    if (r->state != 2) {
      *done = 0;
      return FCMP_OK;
    }
    S->reqs.erase(it);
  }
  *done = 1;
  if (support_host && !r->sup.empty())
    std::memcpy(support_host, r->sup.data(), r->sup.size() * 4);
  if (x_host && !r->x.empty()) std::memcpy(x_host, r->x.data(), r->x.size());
  if (stats) *stats = r->stats;
  if (times) *times = r->times;
  int rc = r->rc;
  if (rc) {
    if (r->err.empty()) set_error(rc, "Cholesky breakdown");
    else set_error(rc, r->err);
  }
  delete r;
  return rc;
}

int fcmp_server_drain(fcmp_server* S, double timeout_ms) {
  if (!S) return set_error(FCMP_E_INVALID, "server is NULL");
  std::unique_lock<std::mutex> lk(S->mu);
  auto idle = [&] { return S->queue.empty() && S->inflight == 0; };
  if (timeout_ms <= 0) {
    S->cv_done.wait(lk, idle);
    return FCMP_OK;
  }
  if (!S->cv_done.wait_for(lk, std::chrono::duration<double, std::milli>(timeout_ms), idle))
    return set_error(FCMP_E_BUSY, "requests still running at the timeout");
  return FCMP_OK;
}

int fcmp_server_get_info(fcmp_server* S, fcmp_server_info* info) {
  if (!S || !info) return set_error(FCMP_E_INVALID, "NULL argument");
  std::lock_guard<std::mutex> lk(S->mu);
  *info = S->info;
  info->queued = (int64_t)S->queue.size();
  info->inflight = S->inflight;
  return FCMP_OK;
}

int fcmp_server_destroy(fcmp_server* S) {
  if (!S) return set_error(FCMP_E_INVALID, "server is NULL");
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stop = true;
    S->cv_work.notify_all();
  }
  for (std::thread& t : S->workers) t.join();
  for (hipStream_t st : S->streams) {
    (void)hipStreamSynchronize(st);
    (void)hipStreamDestroy(st);
  }
  for (auto& kv : S->reqs) delete kv.second;
  delete S;
  return FCMP_OK;
}

}  // extern "C"
