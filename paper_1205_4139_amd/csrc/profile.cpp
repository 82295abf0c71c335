// Per-phase device timing with hipEvents (fcmp_profile_enable / _read).
#include <mutex>
#include <vector>

#include "engine.h"

namespace fcmp {

namespace {
struct Rec {
  int phase;
  hipEvent_t a, b;
};
std::mutex g_mu;
bool g_on = false;
std::vector<Rec> g_recs;
std::vector<hipEvent_t> g_pool;
double g_ms[FCMP_NPHASE];
int64_t g_n[FCMP_NPHASE];
thread_local int t_suspend = 0;   // > 0 while this thread captures a graph
thread_local SolveTimes* t_solve = nullptr;

hipEvent_t take_event() {
  if (!g_pool.empty()) {
    hipEvent_t e = g_pool.back();
    g_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}
}  // namespace

bool prof_enabled() {
  std::lock_guard<std::mutex> lk(g_mu);
  return g_on;
}

void prof_suspend(bool on) { t_suspend += on ? 1 : -1; }

SolveTimes::~SolveTimes() {
  for (const Rec& r : recs) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
}

SolveTimesScope::SolveTimesScope(SolveTimes* s) : prev_(t_solve) { t_solve = s; }
SolveTimesScope::~SolveTimesScope() { t_solve = prev_; }

int solve_times_read(SolveTimes& s, double* ms) {
  for (int p = 0; p < FCMP_NPHASE; ++p) ms[p] = 0.0;
  for (const SolveTimes::Rec& r : s.recs) {
    float t = 0.f;
    if (hipEventSynchronize(r.b) != hipSuccess || hipEventElapsedTime(&t, r.a, r.b) != hipSuccess)
      return set_error(FCMP_E_DEVICE, "phase event query failed");
    ms[r.phase] += t;
  }
  return FCMP_OK;
}

ProfScope::ProfScope(int phase, hipStream_t st) : phase_(phase), st_(st) {
  if (t_suspend > 0) return;
  if (t_solve) {
    if (hipEventCreate(&sa_) == hipSuccess && hipEventRecord(sa_, st_) == hipSuccess) {
      solve_ = t_solve;
    } else if (sa_) {
      (void)hipEventDestroy(sa_);
      sa_ = nullptr;
    }
  }
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_on) return;
  a_ = take_event();
  if (a_ && hipEventRecord(a_, st_) != hipSuccess) {
    g_pool.push_back(a_);
    a_ = nullptr;
  }
}

ProfScope::~ProfScope() {
  if (solve_) {
    hipEvent_t b = nullptr;
    if (hipEventCreate(&b) == hipSuccess && hipEventRecord(b, st_) == hipSuccess) {
      solve_->recs.push_back(SolveTimes::Rec{phase_, sa_, b});
    } else {
      (void)hipEventDestroy(sa_);
      if (b) (void)hipEventDestroy(b);
    }
  }
  if (!a_) return;
  std::lock_guard<std::mutex> lk(g_mu);
  hipEvent_t b = take_event();
  if (!b || hipEventRecord(b, st_) != hipSuccess) {
    g_pool.push_back(a_);
    if (b) g_pool.push_back(b);
    return;
  }
  g_recs.push_back(Rec{phase_, a_, b});
}

int profile_enable(int enable) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_on = enable != 0;
  return FCMP_OK;
}

int profile_read(fcmp_profile* out, int reset) {
  std::lock_guard<std::mutex> lk(g_mu);
  for (const Rec& r : g_recs) {
    float ms = 0.f;
    if (hipEventSynchronize(r.b) != hipSuccess ||
        hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess)
      return set_error(FCMP_E_DEVICE, "profile event query failed");
    g_ms[r.phase] += ms;
    g_n[r.phase] += 1;
    g_pool.push_back(r.a);
    g_pool.push_back(r.b);
  }
  g_recs.clear();
  if (out) {
    for (int p = 0; p < FCMP_NPHASE; ++p) {
      out->ms[p] = g_ms[p];
      out->launches[p] = g_n[p];
    }
  }
  if (reset) {
    for (int p = 0; p < FCMP_NPHASE; ++p) { g_ms[p] = 0.0; g_n[p] = 0; }
  }
  return FCMP_OK;
}

}  // namespace fcmp
