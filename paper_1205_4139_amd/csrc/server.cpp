// Continuous-batching solver service.
//
// Requests (problem, options, host y) queue on the host and are admitted in
// arrival order as request slots and room in the caller's device pool allow.
//  * Slot groups (iteration-granular admission): OMP requests with the
//    conventional correlation fused with the residual join a resident group
//    of slots of their (class, N, options) between two iterations.  Slot s
//    runs iteration step - tofs[s] of its own solve, so a request joins
//    while the others are mid-solve and leaves as soon as its K selections
//    are made.  Each group has a thread and a stream; host threads prepare
//    the Omega tables beforehand, through a cache keyed by (class, N, Omega)
//    (the kernel vector and tables can be stored in advance, Sec. III-A),
//    and a slot whose device tables already hold the request's Omega, or
//    another slot's copy of them, is reused without host work.
//  * Waves, on worker streams: a persistent wave takes every queued OMP
//    problem the one-workgroup-per-problem kernel takes (up to max_wave, same
//    options) in one launch; a lockstep wave takes other requests (SP,
//    CoSaMP, the fast or adaptive methods) that share class and N (for SP and
//    CoSaMP also M and K), solved as one lockstep plan.  With several worker
//    streams worker 0 runs persistent waves only.
// A request's device state (y, tables, kernel vector, h_0, Cholesky factor,
// x) stays in its slot or wave region from admission to completion; results
// come back to pinned host memory.  A request's arithmetic depends neither on
// the requests it runs beside nor on when it joined.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <list>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>

#include "batch.h"
#include "plan.h"

using namespace fcmp;

namespace {

size_t pad256(size_t v) { return (v + 255) & ~(size_t)255; }

// Omega tables of one (class, N, Omega) for the slot-plan geometry, shared by
// every request with that Omega (host table cache).
struct TableEntry {
  int cls = 0;
  int64_t N = 0;
  uint64_t hash = 0;
  std::vector<int32_t> omega;
  HostTables t;
  size_t bytes() const {
    return omega.size() * 4 +
           4 * (t.ent_k.size() + t.perm.size() + t.goff.size() + t.ent2_k.size() +
                t.goff2.size() + t.pos1.size() + t.cst.size() + t.cmask.size() + t.cbase.size()) +
           t.tw64.size() * sizeof(double2) + t.tw32.size() * sizeof(float2);
  }
};

uint64_t omega_hash(int cls, int64_t N, const int32_t* om, int64_t M) {
  uint64_t h = 1469598103934665603ull;   // FNV-1a over (class, N, M, Omega)
  auto mix = [&](uint64_t v) {
    for (int b = 0; b < 8; ++b) {
      h ^= (v >> (8 * b)) & 0xffu;
      h *= 1099511628211ull;
    }
  };
  mix((uint64_t)cls);
  mix((uint64_t)N);
  mix((uint64_t)M);
  for (int64_t i = 0; i < M; ++i) mix((uint64_t)(uint32_t)om[i]);
  return h;
}

// Least-recently-used cache of table entries, bounded in host bytes.
class TableCache {
 public:
  explicit TableCache(size_t cap) : cap_(cap) {}
  std::shared_ptr<const TableEntry> find(int cls, int64_t N, uint64_t hash,
                                         const std::vector<int32_t>& om) {
    std::lock_guard<std::mutex> lk(mu_);
    for (auto it = lru_.begin(); it != lru_.end(); ++it) {
      const TableEntry& e = **it;
      if (e.hash == hash && e.cls == cls && e.N == N && e.omega == om) {
        lru_.splice(lru_.begin(), lru_, it);
        return lru_.front();
      }
    }
    return nullptr;
  }
  void put(std::shared_ptr<const TableEntry> e) {
    std::lock_guard<std::mutex> lk(mu_);
    used_ += e->bytes();
    lru_.push_front(std::move(e));
    while (used_ > cap_ && lru_.size() > 1) {
      used_ -= lru_.back()->bytes();
      lru_.pop_back();
    }
  }

 private:
  std::mutex mu_;
  std::list<std::shared_ptr<const TableEntry>> lru_;
  size_t cap_ = 0, used_ = 0;
};

// Slot capacities of the group a request would create: M up to the smallest
// of N/4, N/2, N that holds it; K up to N/64 (clamped to 256 .. 4096), or the
// next power of two that holds the request's K, so that one group per
// (class, N) usually takes every sparsity of a stream.
void slot_caps(const fcmp_problem& p, int64_t* Mcap, int64_t* Kcap) {
  int64_t m = p.N / 4;
  while (m < p.M) m *= 2;
  int64_t k = std::min<int64_t>(4096, std::max<int64_t>(256, p.N / 64));
  while (k < p.K) k *= 2;
  *Mcap = std::min<int64_t>(m, p.N);
  *Kcap = std::min<int64_t>(k, *Mcap - 1);
}

// Per-slot device io: y, support and x at the capacities.
size_t slot_io_bytes(int cls, int64_t Mcap, int64_t Kcap) {
  const size_t wb = cls == FCMP_FOURIER ? 16 : 8;
  return pad256((size_t)Mcap * wb) + pad256((size_t)Kcap * 4) + pad256((size_t)Kcap * wb);
}

// Device bytes of a slot group of n slots (plan, io, iteration offsets).
int slot_group_bytes(const fcmp_problem& cap, const fcmp_options& opt, int64_t n, size_t* bytes) {
  fcmp_plan P;
  int rc = plan_init_slots(P, n, cap, opt);
  if (rc) return rc;
  *bytes = pad256(P.total) + (size_t)n * slot_io_bytes(cap.matrix_class, cap.M, cap.K) +
           pad256((size_t)n * 4);
  return FCMP_OK;
}

struct Req {
  uint64_t ticket = 0;
  fcmp_problem prob{};
  std::vector<int32_t> omega;
  fcmp_options opt{};
  std::vector<unsigned char> y;     // host copy of y
  bool small = false;               // taken by the persistent kernel
  bool slot = false;                // joins a slot group
  bool prepared = false;            // slot request: tables ready
  std::shared_ptr<const TableEntry> tables;
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

namespace {

// Pinned staging owned by one worker or group index.
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

// A resident group of slots of one (class, N, options) at capacities
// (Mcap, Kcap), run by its own thread on its own stream.
struct SlotGroup {
  int idx = 0;                       // stream and staging index
  int cls = 0;
  int64_t N = 0, Mcap = 0, Kcap = 0;
  fcmp_options opt{};
  int nslot = 0;
  size_t off = 0, bytes = 0;         // pool region
  fcmp_plan P;                       // laid out by the group's thread
  std::vector<Req*> occ;             // occupant of each slot (nullptr: free)
  std::vector<int> joined;           // 1 once the occupant's first iteration is enqueued
  std::vector<std::shared_ptr<const TableEntry>> resident;   // device tables of each slot
  std::vector<int> joins;            // slots assigned, not yet joined
  int64_t idle_since_ms = -1;
  bool exiting = false;
  std::condition_variable cv;
};

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
  // slot groups
  std::vector<SlotGroup*> groups;                // live groups
  std::vector<hipStream_t> gstreams;             // one per group index
  std::vector<char> gidx_used;
  int live_group_threads = 0;
  bool room_wanted = false;                      // a slot request waits for pool room
  std::deque<Req*> prepq;                        // slot requests whose tables are pending
  std::condition_variable cv_prep;
  std::vector<std::thread> preps;
  std::vector<Staging> gstage;                   // pinned staging per group index
  TableCache cache{(size_t)1 << 30};
};

namespace {

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
      if (h->small || h->slot) continue;
      std::vector<Req*> cand{h};
      for (size_t j = k + 1; j < S->queue.size() && (int)cand.size() < std::min(slots, 64); ++j) {
        Req* r = S->queue[j];
        if (!r->small && !r->slot && same_opts(r->opt, h->opt) &&
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

// ------------------------------------------------------------ slot groups

constexpr int SLOT_MAX = 64;             // slots per group
constexpr double GROUP_LINGER_MS = 200;  // an idle group keeps its region this long

void group_main(fcmp_server* S, SlotGroup* G);

// A free slot for r: one whose device tables hold r's Omega, else one with
// no tables, else any.
int pick_slot(const SlotGroup* G, const Req* r) {
  int empty = -1, any = -1;
  for (int s = 0; s < G->nslot; ++s) {
    if (G->occ[s]) continue;
    if (G->resident[s] == r->tables) return s;
    if (!G->resident[s] && empty < 0) empty = s;
    if (any < 0) any = s;
  }
  return empty >= 0 ? empty : any;
}

// A new group for r when a group index and pool room are free (under the
// lock); its thread lays it out and runs it.
SlotGroup* create_group(fcmp_server* S, const Req* r) {
  const int maxg = S->cfg.max_groups;
  if ((int)S->groups.size() >= maxg) return nullptr;
  int idx = -1;
  for (int k = 0; k < maxg; ++k)
    if (!S->gidx_used[k]) { idx = k; break; }
  if (idx < 0) return nullptr;   // a group that left is still winding down
  fcmp_problem cap = r->prob;
  slot_caps(r->prob, &cap.M, &cap.K);
  size_t b1 = 0, b2 = 0;
  if (slot_group_bytes(cap, r->opt, 1, &b1) || slot_group_bytes(cap, r->opt, 2, &b2))
    return nullptr;
  const size_t per = b2 > b1 ? b2 - b1 : b1;
  const size_t base = b1 > per ? b1 - per : 0;
  const size_t room = S->arena.largest();
  if (room < b1) {
    S->room_wanted = true;
    return nullptr;
  }
  // at most a quarter of the pool (at least one slot), at most SLOT_MAX slots
  const size_t budget = std::min(room, std::max(S->pool_bytes / 4, b1));
  int64_t n = (int64_t)((budget - base) / per);
  n = std::max<int64_t>(1, std::min<int64_t>({n, (int64_t)SLOT_MAX, (int64_t)S->cfg.max_slots}));
  size_t bytes = 0;
  for (;;) {
    if (slot_group_bytes(cap, r->opt, n, &bytes)) return nullptr;
    if (bytes <= room || n == 1) break;
    n = std::max<int64_t>(1, n * 3 / 4);
  }
  size_t off = 0;
  if (bytes > room || !S->arena.take(bytes, &off)) {
    S->room_wanted = true;
    return nullptr;
  }
  SlotGroup* G = new SlotGroup();
  G->idx = idx;
  G->cls = r->prob.matrix_class;
  G->N = r->prob.N;
  G->Mcap = cap.M;
  G->Kcap = cap.K;
  G->opt = r->opt;
  G->nslot = (int)n;
  G->off = off;
  G->bytes = bytes;
  if (plan_init_slots(G->P, n, cap, r->opt) != FCMP_OK) {
    S->arena.give(off, bytes);
    delete G;
    return nullptr;
  }
  G->occ.assign((size_t)n, nullptr);
  G->joined.assign((size_t)n, 0);
  G->resident.assign((size_t)n, nullptr);
  S->gidx_used[idx] = 1;
  S->groups.push_back(G);
  S->live_group_threads++;
  S->info.groups++;
  S->info.pool_peak = std::max<int64_t>(S->info.pool_peak, (int64_t)S->arena.peak());
  std::thread(group_main, S, G).detach();
  return G;
}

// Slot requests whose tables are ready join a group with a free slot, in
// arrival order (under the lock).
void place_slot_requests(fcmp_server* S) {
  if (S->stop || S->cfg.max_groups <= 0) return;
  S->room_wanted = false;
  for (size_t k = 0; k < S->queue.size();) {
    Req* r = S->queue[k];
    if (!r->slot || !r->prepared) { ++k; continue; }
    if (S->inflight >= S->cfg.max_slots) return;
    SlotGroup* best = nullptr;
    int bs = -1;
    bool bres = false;
    for (SlotGroup* G : S->groups) {
      if (G->exiting || G->cls != r->prob.matrix_class || G->N != r->prob.N ||
          !same_opts(G->opt, r->opt) || G->Mcap < r->prob.M || G->Kcap < r->prob.K)
        continue;
      const int s = pick_slot(G, r);
      if (s < 0) continue;
      const bool res = G->resident[s] == r->tables;
      // a slot holding the tables first, then the group of smallest capacity
      if (!best || (res && !bres) || (res == bres && G->Kcap < best->Kcap)) {
        best = G;
        bs = s;
        bres = res;
      }
    }
    if (!best) {
      best = create_group(S, r);
      if (best) bs = pick_slot(best, r);
    }
    if (!best || bs < 0) { ++k; continue; }
    best->occ[bs] = r;
    best->joined[bs] = 0;
    best->joins.push_back(bs);
    r->state = 1;
    r->times.t_launch = now_ms(S->t0);
    S->queue.erase(S->queue.begin() + (long)k);
    S->inflight++;
    S->info.slot_joins++;
    best->cv.notify_one();
  }
}

// Host tables of queued slot requests: from the cache, else built here.
void prep_main(fcmp_server* S) {
  std::unique_lock<std::mutex> lk(S->mu);
  for (;;) {
    S->cv_prep.wait(lk, [&] { return S->stop || !S->prepq.empty(); });
    if (S->stop) break;
    Req* r = S->prepq.front();
    S->prepq.pop_front();
    lk.unlock();
    const int cls = r->prob.matrix_class;
    const uint64_t h = omega_hash(cls, r->prob.N, r->omega.data(), r->prob.M);
    std::shared_ptr<const TableEntry> e = S->cache.find(cls, r->prob.N, h, r->omega);
    const bool hit = (bool)e;
    if (!e) {
      auto ne = std::make_shared<TableEntry>();
      ne->cls = cls;
      ne->N = r->prob.N;
      ne->hash = h;
      ne->omega = r->omega;
      const Geo g = make_geo(cls == FCMP_FOURIER, (int)r->prob.N, slot_tile());
      build_tables(g, r->omega.data(), (int)r->prob.M, ne->t);
      S->cache.put(ne);
      e = ne;
    }
    lk.lock();
    if (hit) S->info.tables_cached++;
    else S->info.tables_built++;
    r->tables = e;
    r->prepared = true;
    place_slot_requests(S);
  }
}

void group_main(fcmp_server* S, SlotGroup* G) {
  (void)hipSetDevice(S->device);
  hipStream_t st = S->gstreams[(size_t)G->idx];
  Staging& stg = S->gstage[(size_t)G->idx];
  fcmp_plan& P = G->P;
  const int n = G->nslot;
  const bool F = G->cls == FCMP_FOURIER;
  const size_t wb = F ? 16 : 8;
  char* base = S->pool + G->off;
  plan_layout(P, base);
  char* io = base + pad256(P.total);
  const size_t iob = slot_io_bytes(G->cls, G->Mcap, G->Kcap);
  int32_t* tofs_dev = (int32_t*)(io + (size_t)n * iob);
  auto y_dev = [&](int s) { return io + (size_t)s * iob; };
  auto sup_dev = [&](int s) { return y_dev(s) + pad256((size_t)G->Mcap * wb); };
  auto x_dev = [&](int s) { return sup_dev(s) + pad256((size_t)G->Kcap * 4); };
  // staging sizes: results per slot; uploads per join (y, tables, M, K, tofs)
  const size_t res_b = pad256((size_t)G->Kcap * 4) + pad256((size_t)G->Kcap * wb) +
                       pad256(sizeof(Status));
  const size_t M4 = pad256((size_t)G->Mcap * 4);
  const size_t join_b = pad256((size_t)G->Mcap * wb) + 4 * M4 + pad256((size_t)P.sG * 4) +
                        pad256((size_t)P.sG2 * 4) + 2 * pad256((size_t)P.sC * 4) +
                        pad256((size_t)P.sCs * 4) + 3 * 256;
  const size_t tw_b = pad256((size_t)tw_count(P.g) * sizeof(double2)) +
                      pad256((size_t)tw_count(P.g) * sizeof(float2));
  const size_t ptr_b = pad256((size_t)3 * n * sizeof(void*));
  const size_t seg_b = std::max(ptr_b, tw_b + 4 * join_b);
  int rc = stg.ensure((size_t)n * res_b + 3 * seg_b);
  char* res = (char*)stg.p;
  char* ring = res + (size_t)n * res_b;
  hipEvent_t ev[3] = {nullptr, nullptr, nullptr};
  int64_t ev_cycle[3] = {-1, -1, -1};
  for (int q = 0; q < 3 && !rc; ++q)
    if (hipEventCreateWithFlags(&ev[q], hipEventBlockingSync | hipEventDisableTiming) != hipSuccess)
      rc = set_error(FCMP_E_DEVICE, "event creation failed");
  struct Pend {
    int s;
    Req* r;
    int64_t cycle;
  };
  std::vector<Pend> pend;
  std::vector<int> tofs((size_t)n, 0), Ms((size_t)n, 0), Ks((size_t)n, 0), run((size_t)n, 0);
  int64_t cycle = 0, done_cycle = -1;
  int step = 2;
  bool tw_loaded = false;
  int64_t n_res = 0, n_copy = 0, n_steps = 0;
  std::string msg;
  char* seg = nullptr;
  size_t used = 0;
  auto stage = [&](const void* src, size_t bytes) -> const void* {
    char* d = seg + used;
    std::memcpy(d, src, bytes);
    used += pad256(bytes);
    return d;
  };
  auto wait_cycle = [&](int64_t r) -> int {
    if (r <= done_cycle) return FCMP_OK;
    const int q = (int)(r % 3);
    if (ev_cycle[q] != r) return set_error(FCMP_E_DEVICE, "slot group: cycle event lost");
    HIP_TRY(hipEventSynchronize(ev[q]));
    done_cycle = r;
    return FCMP_OK;
  };
  // results of finished slots whose cycle is complete back to their requests
  auto deliver = [&](bool all) {
    std::vector<Pend> keep;
    std::vector<Req*> fin;
    for (const Pend& d : pend) {
      if (!all && d.cycle > done_cycle) {
        keep.push_back(d);
        continue;
      }
      Req* r = d.r;
      const char* rs = res + (size_t)d.s * res_b;
      const Status* hs = (const Status*)(rs + pad256((size_t)G->Kcap * 4) +
                                         pad256((size_t)G->Kcap * wb));
      r->sup.assign((const int32_t*)rs, (const int32_t*)rs + r->prob.K);
      const unsigned char* xs = (const unsigned char*)rs + pad256((size_t)G->Kcap * 4);
      r->x.assign(xs, xs + (size_t)r->prob.K * wb);
      r->stats = fcmp_stats{};
      r->stats.iterations = hs->iterations;
      r->stats.status_detail = hs->numeric ? FCMP_E_NUMERIC : FCMP_OK;
      r->stats.min_gap = hs->min_gap;
      const double r2 = hs->ynorm2 - hs->znorm2;
      r->stats.res_norm = r2 > 0 ? std::sqrt(r2) : 0.0;
      r->rc = r->stats.status_detail;
      fin.push_back(r);
    }
    pend.swap(keep);
    if (fin.empty() && !n_res && !n_copy && !n_steps) return;
    std::lock_guard<std::mutex> lk(S->mu);
    const double t = now_ms(S->t0);
    for (Req* r : fin) {
      r->times.t_done = t;
      r->stats.ms_total = t - r->times.t_launch;
      r->state = 2;
    }
    S->inflight -= (int)fin.size();
    S->info.completed += (int64_t)fin.size();
    S->info.tables_resident += n_res;
    S->info.tables_copied += n_copy;
    S->info.slot_steps += n_steps;
    n_res = n_copy = n_steps = 0;
    if (!fin.empty()) {
      S->cv_done.notify_all();
      place_slot_requests(S);
    }
  };
  // cycle 0: the slots' device pointers, every slot done, offsets zero
  if (!rc) {
    seg = ring;
    used = 0;
    std::vector<void*> ptrs((size_t)3 * n);
    for (int s = 0; s < n; ++s) {
      ptrs[(size_t)3 * s] = y_dev(s);
      ptrs[(size_t)3 * s + 1] = sup_dev(s);
      ptrs[(size_t)3 * s + 2] = x_dev(s);
    }
    const void* sp = stage(ptrs.data(), ptrs.size() * sizeof(void*));
    if (hipMemcpyAsync(P.dptrs, sp, ptrs.size() * sizeof(void*), hipMemcpyHostToDevice, st) !=
            hipSuccess ||
        launch_status_done(P.status, n, st) != hipSuccess ||
        launch_fill_u32((uint32_t*)tofs_dev, 0u, n, st) != hipSuccess ||
        hipEventRecord(ev[0], st) != hipSuccess)
      rc = set_error(FCMP_E_DEVICE, "slot group set-up failed");
    ev_cycle[0] = 0;
    cycle = 1;
  }
  while (!rc) {
    if (cycle >= 2 && (rc = wait_cycle(cycle - 2))) break;
    deliver(false);
    std::vector<int> js;
    {
      std::unique_lock<std::mutex> lk(S->mu);
      js.swap(G->joins);
      bool busy = !js.empty() || !pend.empty();
      for (int s = 0; s < n && !busy; ++s) busy = run[(size_t)s] != 0;
      if (!busy) {
        // idle: keep the region a while for new requests of this shape,
        // unless the server stops or another request waits for room
        const double t_idle = now_ms(S->t0);
        bool leave = false;
        while (G->joins.empty()) {
          if (S->stop || S->room_wanted || now_ms(S->t0) - t_idle >= GROUP_LINGER_MS) {
            leave = true;
            break;
          }
          G->cv.wait_for(lk, std::chrono::milliseconds(20));
        }
        if (leave) {
          G->exiting = true;
          break;
        }
        continue;
      }
    }
    seg = ring + (size_t)(cycle % 3) * seg_b;
    used = 0;
    std::vector<int> fin_now;   // slots done at their join (K = 1)
    size_t j = 0;
    for (; j < js.size() && !rc; ++j) {
      if (j > 0 && used + join_b > seg_b) break;   // the rest join next cycle
      const int s = js[j];
      Req* r = G->occ[(size_t)s];
      const int32_t M = (int32_t)r->prob.M, K = (int32_t)r->prob.K;
      fcmp_plan V = plan_view(P, s, M, K);
      if (!tw_loaded) {
        if ((rc = plan_upload_twiddles(P, r->tables->t, st, stage))) break;
        tw_loaded = true;
      }
      if (hipMemcpyAsync(y_dev(s), stage(r->y.data(), r->ybytes()), r->ybytes(),
                         hipMemcpyHostToDevice, st) != hipSuccess) {
        rc = set_error(FCMP_E_DEVICE, "slot group: y upload failed");
        break;
      }
      if (G->resident[(size_t)s] == r->tables) {
        n_res++;
      } else {
        int from = -1;
        for (int q = 0; q < n && from < 0; ++q)
          if (q != s && G->resident[(size_t)q] == r->tables) from = q;
        if (from >= 0) {
          fcmp_plan Vf = plan_view(P, from, M, K);
          rc = plan_copy_tables(V, Vf, st);
          n_copy++;
        } else {
          rc = plan_upload_tables(V, r->tables->t, st, stage);
        }
        if (rc) break;
        G->resident[(size_t)s] = r->tables;
      }
      tofs[(size_t)s] = step - 2;   // the next step is its iteration 2
      Ms[(size_t)s] = M;
      Ks[(size_t)s] = K;
      const int32_t mk[3] = {M, K, step - 2};
      const int32_t* smk = (const int32_t*)stage(mk, sizeof(mk));
      if (hipMemcpyAsync(V.Mv, smk, 4, hipMemcpyHostToDevice, st) != hipSuccess ||
          hipMemcpyAsync(V.Kv, smk + 1, 4, hipMemcpyHostToDevice, st) != hipSuccess ||
          hipMemcpyAsync(tofs_dev + s, smk + 2, 4, hipMemcpyHostToDevice, st) != hipSuccess) {
        rc = set_error(FCMP_E_DEVICE, "slot group: slot upload failed");
        break;
      }
      if ((rc = plan_join(V, r->opt, st))) break;
      G->joined[(size_t)s] = 1;
      run[(size_t)s] = 1;
      if (K == 1) fin_now.push_back(s);
    }
    if (rc) break;
    if (j < js.size()) {
      std::lock_guard<std::mutex> lk(S->mu);
      G->joins.insert(G->joins.begin(), js.begin() + (long)j, js.end());
    }
    for (int s : fin_now) run[(size_t)s] = 0;
    // one iteration of every running slot
    int t_lo = 1 << 30, t_hi = 0;
    for (int s = 0; s < n; ++s) {
      if (!run[(size_t)s]) continue;
      const int t = step - tofs[(size_t)s];
      t_lo = std::min(t_lo, t);
      t_hi = std::max(t_hi, t);
    }
    std::vector<int> fin = fin_now;
    if (t_hi >= 2) {
      if ((rc = plan_step_slots(P, step, tofs_dev, t_lo, t_hi, st))) break;
      n_steps++;
      for (int s = 0; s < n; ++s)
        if (run[(size_t)s] && step - tofs[(size_t)s] == Ks[(size_t)s]) fin.push_back(s);
      step++;
    }
    // finished slots: results to their staging, the slot free for a new request
    for (int s : fin) {
      for (const Pend& d : pend)
        if (d.s == s && (rc = wait_cycle(d.cycle))) break;
      if (rc) break;
      deliver(false);
      fcmp_plan V = plan_view(P, s, Ms[(size_t)s], Ks[(size_t)s]);
      if ((rc = plan_finish(V, st))) break;
      char* rs = res + (size_t)s * res_b;
      Req* r = G->occ[(size_t)s];
      if (hipMemcpyAsync(rs, sup_dev(s), (size_t)Ks[(size_t)s] * 4, hipMemcpyDeviceToHost, st) !=
              hipSuccess ||
          hipMemcpyAsync(rs + pad256((size_t)G->Kcap * 4), x_dev(s), (size_t)Ks[(size_t)s] * wb,
                         hipMemcpyDeviceToHost, st) != hipSuccess ||
          hipMemcpyAsync(rs + pad256((size_t)G->Kcap * 4) + pad256((size_t)G->Kcap * wb),
                         V.status, sizeof(Status), hipMemcpyDeviceToHost, st) != hipSuccess) {
        rc = set_error(FCMP_E_DEVICE, "slot group: result copy failed");
        break;
      }
      run[(size_t)s] = 0;
      pend.push_back(Pend{s, r, cycle});
      std::lock_guard<std::mutex> lk(S->mu);
      G->occ[(size_t)s] = nullptr;
      G->joined[(size_t)s] = 0;
      place_slot_requests(S);
    }
    if (rc) break;
    const int q = (int)(cycle % 3);
    if (hipEventRecord(ev[q], st) != hipSuccess) {
      rc = set_error(FCMP_E_DEVICE, "slot group: event record failed");
      break;
    }
    ev_cycle[q] = cycle;
    cycle++;
  }
  // wind down: nothing of the group may still use its region
  if (rc) msg = last_error();
  (void)hipStreamSynchronize(st);
  if (!rc) deliver(true);
  for (int q = 0; q < 3; ++q)
    if (ev[q]) (void)hipEventDestroy(ev[q]);
  std::lock_guard<std::mutex> lk(S->mu);
  G->exiting = true;
  if (rc) {
    // every request of the group fails with the error
    std::vector<Req*> bad;
    for (const Pend& d : pend) bad.push_back(d.r);
    for (Req* r : G->occ)
      if (r) bad.push_back(r);
    const double t = now_ms(S->t0);
    for (Req* r : bad) {
      r->rc = rc;
      r->err = msg;
      r->times.t_done = t;
      r->state = 2;
    }
    S->inflight -= (int)bad.size();
    S->info.completed += (int64_t)bad.size();
  }
  S->groups.erase(std::find(S->groups.begin(), S->groups.end(), G));
  S->arena.give(G->off, G->bytes);
  S->gidx_used[(size_t)G->idx] = 0;
  delete G;
  place_slot_requests(S);
  S->live_group_threads--;
  S->cv_done.notify_all();
  S->cv_work.notify_all();
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
    place_slot_requests(S);
    S->cv_done.notify_all();
    S->cv_work.notify_all();
  }
  lk.unlock();
  if (ev) (void)hipEventDestroy(ev);
}

// Device bytes of one request admitted alone: its wave, or a one-slot group
// at its capacities; slot: whether it runs in a slot group (groups != 0).
int request_footprint(const fcmp_problem* prob, const fcmp_options* opt, bool groups, bool* small,
                      bool* slot, size_t* bytes) {
  int rc = validate_problem(prob, true);
  if (rc) return rc;
  if ((rc = validate_options(prob, opt))) return rc;
  Req r;
  r.prob = *prob;
  r.opt = *opt;
  r.small = !(opt->flags & FCMP_FLAG_NO_PERSISTENT) && wg_eligible(*prob, *opt);
  r.slot = groups && !r.small && prob->K <= 4096 && plan_slots_ok(*prob, *opt);
  size_t sb = 0;
  if (r.slot) {
    fcmp_problem cap = *prob;
    slot_caps(*prob, &cap.M, &cap.K);
    if ((rc = slot_group_bytes(cap, *opt, 1, &sb))) return rc;
    *bytes = sb;
  } else {
    std::vector<Req*> one{&r};
    if ((rc = wave_state_bytes(one, r.small, &sb))) return rc;
    *bytes = sb + r.io_bytes();
  }
  if (small) *small = r.small;
  if (slot) *slot = r.slot;
  return FCMP_OK;
}

}  // namespace

extern "C" {

int fcmp_server_footprint(const fcmp_problem* prob, const fcmp_options* opt, size_t* bytes) {
  if (!bytes) return set_error(FCMP_E_INVALID, "bytes is NULL");
  return request_footprint(prob, opt, true, nullptr, nullptr, bytes);
}

int fcmp_server_create(fcmp_server** out, void* pool_dev, size_t pool_bytes,
                       const fcmp_server_config* cfg) {
  if (!out) return set_error(FCMP_E_INVALID, "out is NULL");
  *out = nullptr;
  if (!pool_dev || pool_bytes < 4096) return set_error(FCMP_E_INVALID, "pool missing or too small");
  fcmp_server_config c{};
  if (cfg) c = *cfg;
  if (c.max_slots < 0 || c.max_pending < 0 || c.n_streams < 0 || c.n_streams > 8 ||
      c.max_wave < 0 || c.max_groups < -1 || c.max_groups > 16)
    return set_error(FCMP_E_INVALID, "bad server configuration");
  if (c.max_slots == 0) c.max_slots = 4096;
  if (c.max_pending == 0) c.max_pending = 1 << 16;
  if (c.n_streams == 0) c.n_streams = 4;
  if (c.max_wave == 0) c.max_wave = 1024;
  if (c.max_groups == 0) c.max_groups = 8;
  if (c.max_groups < 0) c.max_groups = 0;
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
  for (int k = 0; k < c.n_streams + c.max_groups; ++k) {
    hipStream_t st = nullptr;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
      for (hipStream_t s : S->streams) (void)hipStreamDestroy(s);
      for (hipStream_t s : S->gstreams) (void)hipStreamDestroy(s);
      delete S;
      return set_error(FCMP_E_DEVICE, "stream creation failed");
    }
    (k < c.n_streams ? S->streams : S->gstreams).push_back(st);
  }
  S->gidx_used.assign((size_t)c.max_groups, 0);
  S->gstage.resize((size_t)c.max_groups);
  for (int k = 0; k < c.n_streams; ++k) S->workers.emplace_back(worker_main, S, k);
  if (c.max_groups > 0)
    for (int k = 0; k < 2; ++k) S->preps.emplace_back(prep_main, S);
  *out = S;
  return FCMP_OK;
}

int fcmp_server_submit(fcmp_server* S, const fcmp_problem* prob, const fcmp_options* opt,
                       const void* y_host, uint64_t* ticket) {
  if (!S || !ticket || !y_host) return set_error(FCMP_E_INVALID, "NULL argument");
  bool small = false, slot = false;
  size_t foot = 0;
  int rc = request_footprint(prob, opt, S->cfg.max_groups > 0, &small, &slot, &foot);
  if (rc) return rc;
  if (pad256(foot) > (S->pool_bytes & ~(size_t)255))
    return set_error(FCMP_E_WORKSPACE, "request needs more device memory than the pool holds");
  Req* r = new Req();
  r->prob = *prob;
  r->omega.assign(prob->omega, prob->omega + prob->M);
  r->prob.omega = r->omega.data();
  r->opt = *opt;
  r->small = small;
  r->slot = slot;
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
  if (r->slot) {
    S->prepq.push_back(r);
    S->cv_prep.notify_one();
  } else {
    S->cv_work.notify_all();
  }
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
    S->cv_prep.notify_all();
    for (SlotGroup* G : S->groups) G->cv.notify_all();
  }
  for (std::thread& t : S->workers) t.join();
  for (std::thread& t : S->preps) t.join();
  {
    // group threads finish their running requests, then leave
    std::unique_lock<std::mutex> lk(S->mu);
    S->cv_done.wait(lk, [&] { return S->live_group_threads == 0; });
  }
  for (hipStream_t st : S->streams) {
    (void)hipStreamSynchronize(st);
    (void)hipStreamDestroy(st);
  }
  for (hipStream_t st : S->gstreams) (void)hipStreamDestroy(st);
  for (auto& kv : S->reqs) delete kv.second;
  delete S;
  return FCMP_OK;
}

}  // extern "C"
