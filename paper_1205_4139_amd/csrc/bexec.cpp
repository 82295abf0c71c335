// Batches of independent problems: the one-shot fcmp_batch_solve and the
// reusable batch plan whose device work is captured once into a hipGraph.
//
// Problems are split into those the persistent one-workgroup-per-problem
// kernel takes (OMP, transform tile within one workgroup's LDS) and the rest,
// which run as lockstep plans, one per (class, N) for OMP (per-instance M and
// K) and one per (class, N, M, K) for SP and CoSaMP.
#include <algorithm>
#include <cmath>
#include <map>
#include <tuple>

#include "batch.h"
#include "plan.h"

using namespace fcmp;

namespace {

#define HIP_TRY(expr)                                                              \
  do {                                                                             \
    hipError_t _e = (expr);                                                        \
    if (_e != hipSuccess)                                                          \
      return set_error(FCMP_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(_e)); \
  } while (0)

size_t pad256(size_t v) { return (v + 255) & ~(size_t)255; }

struct Split {
  std::vector<int64_t> wg;                  // caller indices of the persistent part
  std::vector<std::vector<int64_t>> rest;   // caller indices per lockstep group
};

int partition(int64_t n, const fcmp_problem* probs, const fcmp_options* opt, Split& S) {
  if (n < 1 || !probs) return set_error(FCMP_E_INVALID, "empty batch");
  if (!opt) return set_error(FCMP_E_INVALID, "options is NULL");
  for (int64_t b = 0; b < n; ++b) {
    int rc = validate_problem(&probs[b], true);
    if (rc) return rc;
    if ((rc = validate_options(&probs[b], opt))) return rc;
  }
  const bool allow = !(opt->flags & FCMP_FLAG_NO_PERSISTENT);
  std::map<std::tuple<int, int64_t, int64_t, int64_t>, size_t> idx;
  for (int64_t b = 0; b < n; ++b) {
    const fcmp_problem& p = probs[b];
    if (allow && wg_eligible(p, *opt)) {
      S.wg.push_back(b);
      continue;
    }
    const bool omp = opt->algorithm == FCMP_OMP;
    const auto key = std::make_tuple(p.matrix_class, p.N, omp ? 0 : p.M, omp ? 0 : p.K);
    auto it = idx.find(key);
    if (it == idx.end()) {
      idx[key] = S.rest.size();
      S.rest.push_back({b});
    } else {
      S.rest[it->second].push_back(b);
    }
  }
  return FCMP_OK;
}

std::vector<fcmp_problem> pick(const fcmp_problem* probs, const std::vector<int64_t>& ids) {
  std::vector<fcmp_problem> g;
  g.reserve(ids.size());
  for (int64_t i : ids) g.push_back(probs[i]);
  return g;
}

// Workspace of the one-shot solve: the persistent part, then the largest
// lockstep plan (the plans run one after another in one region).
int oneshot_sizes(int64_t n, const fcmp_problem* probs, const fcmp_options* opt, Split& S,
                  WgBatch& B, size_t* wg_bytes, size_t* rest_bytes) {
  int rc = partition(n, probs, opt, S);
  if (rc) return rc;
  *wg_bytes = 0;
  *rest_bytes = 0;
  if (!S.wg.empty()) {
    if ((rc = wg_plan_init(B, (int64_t)S.wg.size(), probs, S.wg.data(), opt))) return rc;
    *wg_bytes = pad256(B.total);
  }
  for (const auto& ids : S.rest) {
    const auto g = pick(probs, ids);
    fcmp_plan P;
    if ((rc = plan_init(P, (int64_t)g.size(), g.data(), opt))) return rc;
    *rest_bytes = std::max(*rest_bytes, P.total);
  }
  return FCMP_OK;
}

int check_ptrs(int64_t n, const void* const* y, int32_t* const* sup, void* const* x) {
  if (!y || !sup || !x) return set_error(FCMP_E_INVALID, "NULL pointer array");
  for (int64_t i = 0; i < n; ++i)
    if (!y[i] || !sup[i] || !x[i]) return set_error(FCMP_E_INVALID, "NULL device pointer");
  return FCMP_OK;
}

}  // namespace

// A batch plan: tables, descriptors and kernel vectors built once; the OMP
// device work of a solve is one captured graph replayed per call.
struct fcmp_batch_plan {
  int64_t n = 0;
  fcmp_options opt{};
  Split S;
  WgBatch wg;
  std::vector<fcmp_plan> parts;     // one lockstep plan per rest group
  void** dev_ptrs = nullptr;        // every pointer array, contiguous
  size_t nptrs = 0;
  void** host_ptrs = nullptr;       // pinned staging of dev_ptrs
  hipEvent_t copied = nullptr;      // the staging copy has been consumed
  bool copy_pending = false;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  size_t total = 0;
};

namespace {

int bplan_sizes(fcmp_batch_plan& BP, const fcmp_problem* probs) {
  int rc;
  size_t off = 0;
  if (!BP.S.wg.empty()) {
    if ((rc = wg_plan_init(BP.wg, (int64_t)BP.S.wg.size(), probs, BP.S.wg.data(), &BP.opt)))
      return rc;
    off += pad256(BP.wg.total);
  }
  BP.parts.clear();
  BP.parts.resize(BP.S.rest.size());
  for (size_t k = 0; k < BP.S.rest.size(); ++k) {
    const auto g = pick(probs, BP.S.rest[k]);
    if ((rc = plan_init(BP.parts[k], (int64_t)g.size(), g.data(), &BP.opt))) return rc;
    off += pad256(BP.parts[k].total);
  }
  BP.nptrs = 3 * (size_t)BP.n;
  off += pad256(BP.nptrs * sizeof(void*));
  BP.total = off;
  return FCMP_OK;
}

void bplan_release(fcmp_batch_plan* BP) {
  if (!BP) return;
  if (BP->exec) (void)hipGraphExecDestroy(BP->exec);
  if (BP->graph) (void)hipGraphDestroy(BP->graph);
  if (BP->copied) {
    (void)hipEventSynchronize(BP->copied);
    (void)hipEventDestroy(BP->copied);
  }
  if (BP->host_ptrs) (void)hipHostFree(BP->host_ptrs);
  delete BP;
}

// Device work of one solve on stream st (graph capture or eager).
int bplan_enqueue(fcmp_batch_plan& BP, hipStream_t st) {
  int rc;
  if (!BP.S.wg.empty() && (rc = wg_run(BP.wg, nullptr, st))) return rc;
  for (fcmp_plan& P : BP.parts)
    if ((rc = plan_enqueue(P, BP.opt, st))) return rc;
  return FCMP_OK;
}

}  // namespace

extern "C" {

int fcmp_batch_query_workspace(int64_t n, const fcmp_problem* probs, const fcmp_options* opt,
                               size_t* bytes) {
  if (!bytes) return set_error(FCMP_E_INVALID, "bytes is NULL");
  Split S;
  WgBatch B;
  size_t a = 0, b = 0;
  int rc = oneshot_sizes(n, probs, opt, S, B, &a, &b);
  if (rc) return rc;
  *bytes = a + b;
  return FCMP_OK;
}

int fcmp_batch_solve(int64_t n, const fcmp_problem* probs, const fcmp_options* opt,
                     const void* const* y_dev, void* ws_dev, size_t ws_bytes,
                     int32_t* const* support_dev, void* const* x_dev, fcmp_stats* stats,
                     void* hip_stream) {
  Split S;
  WgBatch B;
  size_t a = 0, b = 0;
  int rc = oneshot_sizes(n, probs, opt, S, B, &a, &b);
  if (rc) return rc;
  if (!ws_dev) return set_error(FCMP_E_INVALID, "workspace is NULL");
  if (ws_bytes < a + b) return set_error(FCMP_E_WORKSPACE, "workspace too small");
  if ((rc = check_ptrs(n, y_dev, support_dev, x_dev))) return rc;
  hipStream_t st = (hipStream_t)hip_stream;
  int worst = FCMP_OK;
  if (!S.wg.empty()) {
    wg_layout(B, probs, (char*)ws_dev);
    rc = wg_solve_batch(B, probs, y_dev, support_dev, x_dev, stats, st);
    if (rc && rc != FCMP_E_NUMERIC) return rc;
    if (rc) worst = rc;
  }
  char* base = (char*)ws_dev + a;
  for (const auto& ids : S.rest) {
    const auto g = pick(probs, ids);
    std::vector<const void*> ys;
    std::vector<int32_t*> ss;
    std::vector<void*> xs;
    for (int64_t i : ids) {
      ys.push_back(y_dev[i]);
      ss.push_back(support_dev[i]);
      xs.push_back(x_dev[i]);
    }
    std::vector<fcmp_stats> sts(ids.size());
    fcmp_plan P;
    if ((rc = plan_init(P, (int64_t)g.size(), g.data(), opt))) return rc;
    plan_layout(P, base);
    if ((rc = plan_build(P, g.data(), st))) return rc;
    rc = plan_solve(P, nullptr, ys.data(), ss.data(), xs.data(), stats ? sts.data() : nullptr,
                    st);
    if (rc && rc != FCMP_E_NUMERIC) return rc;
    if (rc) worst = rc;
    if (stats)
      for (size_t i = 0; i < ids.size(); ++i) stats[ids[i]] = sts[i];
  }
  return worst;
}

int fcmp_batch_plan_query_workspace(int64_t n, const fcmp_problem* probs,
                                    const fcmp_options* opt, size_t* bytes) {
  if (!bytes) return set_error(FCMP_E_INVALID, "bytes is NULL");
  fcmp_batch_plan BP;
  int rc = partition(n, probs, opt, BP.S);
  if (rc) return rc;
  BP.n = n;
  BP.opt = *opt;
  if ((rc = bplan_sizes(BP, probs))) return rc;
  *bytes = BP.total;
  return FCMP_OK;
}

int fcmp_batch_plan_create(fcmp_batch_plan** out, int64_t n, const fcmp_problem* probs,
                           const fcmp_options* opt, void* ws_dev, size_t ws_bytes,
                           void* hip_stream) {
  if (!out) return set_error(FCMP_E_INVALID, "out is NULL");
  *out = nullptr;
  fcmp_batch_plan* BP = new fcmp_batch_plan();
  int rc = partition(n, probs, opt, BP->S);
  if (!rc) {
    BP->n = n;
    BP->opt = *opt;
    rc = bplan_sizes(*BP, probs);
  }
  if (!rc && !ws_dev) rc = set_error(FCMP_E_INVALID, "workspace is NULL");
  if (!rc && ws_bytes < BP->total) rc = set_error(FCMP_E_WORKSPACE, "workspace too small");
  if (rc) {
    delete BP;
    return rc;
  }
  hipStream_t st = (hipStream_t)hip_stream;
  // ---- layout: persistent part, lockstep parts, pointer arrays
  char* base = (char*)ws_dev;
  size_t off = 0;
  if (!BP->S.wg.empty()) {
    wg_layout(BP->wg, probs, base);
    off += pad256(BP->wg.total);
  }
  for (size_t k = 0; k < BP->parts.size(); ++k) {
    plan_layout(BP->parts[k], base + off);
    off += pad256(BP->parts[k].total);
  }
  BP->dev_ptrs = (void**)(base + off);
  {
    size_t o = 0;
    if (!BP->S.wg.empty()) {
      BP->wg.ptrs = BP->dev_ptrs;
      o += 3 * BP->S.wg.size();
    }
    for (fcmp_plan& P : BP->parts) {
      P.dptrs = BP->dev_ptrs + o;
      o += 3 * (size_t)P.n;
    }
  }
  auto fail = [&](int code) {
    bplan_release(BP);
    return code;
  };
  if (hipHostMalloc((void**)&BP->host_ptrs, BP->nptrs * sizeof(void*), hipHostMallocDefault) !=
      hipSuccess)
    return fail(set_error(FCMP_E_DEVICE, "pinned staging allocation failed"));
  if (hipEventCreateWithFlags(&BP->copied, hipEventDisableTiming) != hipSuccess)
    return fail(set_error(FCMP_E_DEVICE, "event creation failed"));
  // ---- tables, descriptors, kernel vectors (synchronising host work)
  if (!BP->S.wg.empty() && (rc = wg_build(BP->wg, probs, st))) return fail(rc);
  for (size_t k = 0; k < BP->parts.size(); ++k) {
    const auto g = pick(probs, BP->S.rest[k]);
    if ((rc = plan_build(BP->parts[k], g.data(), st))) return fail(rc);
  }
  if (BP->opt.algorithm != FCMP_OMP) {
    *out = BP;   // SP / CoSaMP loops read back partial results: run eagerly
    return FCMP_OK;
  }
  if (!BP->S.wg.empty() && BP->wg.per_cu == 0) {
    // fix the persistent grid before capture (an occupancy query per replay
    // would not be recorded anyway)
    WgParams p{};
    p.logT = WG_LOGT;
    p.twS = WG_LOGT / 2;
    p.logNmax = BP->wg.logNmax;
    p.Kmax = BP->wg.Kmax;
    p.tile_bytes = BP->wg.tile_bytes;
    BP->wg.per_cu = omp_wg_per_cu(p, BP->opt.corr_precision);
  }
  // ---- capture the device work on a private stream
  hipStream_t cs = nullptr;
  if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess)
    return fail(set_error(FCMP_E_DEVICE, "stream creation failed"));
  prof_suspend(true);
  hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed);
  if (e == hipSuccess) {
    rc = bplan_enqueue(*BP, cs);
    hipGraph_t g = nullptr;
    hipError_t e2 = hipStreamEndCapture(cs, &g);
    BP->graph = g;
    if (!rc && e2 != hipSuccess)
      rc = set_error(FCMP_E_DEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(e2));
  } else {
    rc = set_error(FCMP_E_DEVICE, std::string("hipStreamBeginCapture: ") + hipGetErrorString(e));
  }
  prof_suspend(false);
  (void)hipStreamDestroy(cs);
  if (rc) return fail(rc);
  e = hipGraphInstantiate(&BP->exec, BP->graph, nullptr, nullptr, 0);
  if (e != hipSuccess)
    return fail(set_error(FCMP_E_DEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e)));
  *out = BP;
  return FCMP_OK;
}

int fcmp_batch_plan_solve(fcmp_batch_plan* BP, const void* const* y_dev,
                          int32_t* const* support_dev, void* const* x_dev, fcmp_stats* stats,
                          void* hip_stream) {
  if (!BP) return set_error(FCMP_E_INVALID, "plan is NULL");
  int rc = check_ptrs(BP->n, y_dev, support_dev, x_dev);
  if (rc) return rc;
  hipStream_t st = (hipStream_t)hip_stream;
  // the previous call's pointer copy must be done before the staging is reused
  if (BP->copy_pending) HIP_TRY(hipEventSynchronize(BP->copied));
  size_t o = 0;
  if (!BP->S.wg.empty()) {
    wg_host_ptrs(BP->wg, y_dev, support_dev, x_dev, BP->host_ptrs);
    o += 3 * BP->S.wg.size();
  }
  for (size_t k = 0; k < BP->parts.size(); ++k) {
    const auto& ids = BP->S.rest[k];
    const size_t m = ids.size();
    for (size_t i = 0; i < m; ++i) {
      BP->host_ptrs[o + i] = const_cast<void*>(y_dev[ids[i]]);
      BP->host_ptrs[o + m + i] = support_dev[ids[i]];
      BP->host_ptrs[o + 2 * m + i] = x_dev[ids[i]];
    }
    o += 3 * m;
  }
  HIP_TRY(hipMemcpyAsync(BP->dev_ptrs, BP->host_ptrs, BP->nptrs * sizeof(void*),
                         hipMemcpyHostToDevice, st));
  HIP_TRY(hipEventRecord(BP->copied, st));
  BP->copy_pending = true;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (stats) {
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    HIP_TRY(hipEventRecord(e0, st));
  }
  if (BP->exec) {
    HIP_TRY(hipGraphLaunch(BP->exec, st));
  } else {
    // SP / CoSaMP: the set loops synchronise internally
    std::vector<fcmp_stats> sts;
    if (!BP->S.wg.empty() && (rc = wg_run(BP->wg, nullptr, st))) return rc;
    for (size_t k = 0; k < BP->parts.size(); ++k) {
      fcmp_plan& P = BP->parts[k];
      const auto& ids = BP->S.rest[k];
      std::vector<const void*> ys;
      std::vector<int32_t*> ss;
      std::vector<void*> xs;
      for (int64_t i : ids) {
        ys.push_back(y_dev[i]);
        ss.push_back(support_dev[i]);
        xs.push_back(x_dev[i]);
      }
      sts.assign(ids.size(), fcmp_stats{});
      rc = plan_solve(P, nullptr, ys.data(), ss.data(), xs.data(), stats ? sts.data() : nullptr,
                      st);
      if (rc && rc != FCMP_E_NUMERIC) return rc;
      if (stats)
        for (size_t i = 0; i < ids.size(); ++i) stats[ids[i]] = sts[i];
    }
  }
  if (!stats) return FCMP_OK;
  HIP_TRY(hipEventRecord(e1, st));
  HIP_TRY(hipStreamSynchronize(st));
  float ms = 0.f;
  if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) ms = 0.f;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  int worst = FCMP_OK;
  if (!BP->S.wg.empty()) {
    rc = wg_stats(BP->wg, stats, st);   // writes through the caller indices
    if (rc && rc != FCMP_E_NUMERIC) return rc;
    if (rc) worst = rc;
  }
  if (BP->exec) {
    for (size_t k = 0; k < BP->parts.size(); ++k) {
      fcmp_plan& P = BP->parts[k];
      const auto& ids = BP->S.rest[k];
      std::vector<Status> hs(ids.size());
      HIP_TRY(hipMemcpy(hs.data(), P.status, hs.size() * sizeof(Status), hipMemcpyDeviceToHost));
      std::vector<fcmp_stats> sts(ids.size());
      rc = plan_stats((int64_t)ids.size(), hs.data(), ms, sts.data());
      if (rc) worst = rc;
      for (size_t i = 0; i < ids.size(); ++i) stats[ids[i]] = sts[i];
    }
  }
  return worst;
}

int fcmp_batch_plan_destroy(fcmp_batch_plan* BP) {
  if (!BP) return set_error(FCMP_E_INVALID, "plan is NULL");
  bplan_release(BP);
  return FCMP_OK;
}

}  // extern "C"
