// Autotuners: the adaptive correlation method's switch iteration, and the
// launch schedule (transform tile and thread counts) of a plan shape.
//
// The paper's adaptive strategy runs the fast method while it is cheaper
// than the conventional one and switches afterwards; Table I's flop counts
// put the crossover at 6(t-1) = 5 log2 N (Fourier) and t-1 = log2 N
// (Hadamard).  On the device the two costs are not flop counts: the fast
// method is a gather stream over the kernel vector and the conventional one
// a residual plus a two-pass transform, so the crossover is measured here,
// per (class, N, precision), by timing both correlation launch sequences of
// a lockstep plan at growing tap counts, and stored in the library's table
// (and optionally a text cache, one "class N precision switch_t" per line).
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <vector>

#include "plan.h"

using namespace fcmp;

namespace {

#define HIP_TRY(expr)                                                              \
  do {                                                                             \
    hipError_t _e = (expr);                                                        \
    if (_e != hipSuccess)                                                          \
      return set_error(FCMP_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(_e)); \
  } while (0)

constexpr int kReps = 4;

int tune_shape(int32_t cls, int64_t N, int64_t M, int32_t batch, int32_t tmax,
               std::vector<int32_t>& omega, std::vector<fcmp_problem>& probs, fcmp_options& opt,
               int32_t precision) {
  if (cls != FCMP_HADAMARD && cls != FCMP_FOURIER) return set_error(FCMP_E_INVALID, "bad class");
  if (M < 2 || M > N) return set_error(FCMP_E_INVALID, "M must be in [2, N]");
  if (batch < 1 || batch > 4096) return set_error(FCMP_E_INVALID, "batch must be in [1, 4096]");
  // rows spread evenly over [0, N): the costs do not depend on which rows
  omega.resize((size_t)M);
  for (int64_t m = 0; m < M; ++m) omega[(size_t)m] = (int32_t)((m * N) / M);
  fcmp_problem p{};
  p.matrix_class = cls;
  p.N = N;
  p.M = M;
  p.K = std::min<int64_t>(tmax, M - 1);
  p.omega = omega.data();
  probs.assign((size_t)batch, p);
  opt = fcmp_options{};
  opt.algorithm = FCMP_OMP;
  opt.corr_method = FCMP_CORR_ADAPTIVE;
  opt.corr_precision = precision;
  return FCMP_OK;
}

}  // namespace

extern "C" {

int fcmp_autotune_query_workspace(int32_t matrix_class, int64_t N, int64_t M,
                                  int32_t corr_precision, int32_t batch, size_t* bytes) {
  if (!bytes) return set_error(FCMP_E_INVALID, "bytes is NULL");
  std::vector<int32_t> om;
  std::vector<fcmp_problem> probs;
  fcmp_options opt;
  int rc = tune_shape(matrix_class, N, M, batch, model_switch_t(matrix_class, N) * 8 + 8, om,
                      probs, opt, corr_precision);
  if (rc) return rc;
  fcmp_plan P;
  if ((rc = plan_init(P, batch, probs.data(), &opt))) return rc;
  *bytes = P.total;
  return FCMP_OK;
}

}  // extern "C"

namespace {

// A lockstep plan of `batch` problems (class, N, M) laid out in the caller's
// workspace with synthetic taps (distinct columns, odd stride; unit
// coefficients) and y = 0, ready for single correlation launch sequences.
struct CurveBench {
  fcmp_plan P;
  std::vector<int32_t> om, lam, hord, hbst;
  std::vector<fcmp_problem> probs;
  hipStream_t st = nullptr;
  hipEvent_t e[3] = {nullptr, nullptr, nullptr};
  ~CurveBench() {
    for (hipEvent_t ev : e)
      if (ev) (void)hipEventDestroy(ev);
  }
};

int curve_setup(CurveBench& C, int32_t cls, int64_t N, int64_t M, int32_t prec, int32_t batch,
                int32_t tmax, void* ws_dev, size_t ws_bytes, hipStream_t st, int tile = 0,
                uint32_t flags = 0) {
  fcmp_options opt;
  int rc = tune_shape(cls, N, M, batch, tmax, C.om, C.probs, opt, prec);
  if (rc) return rc;
  fcmp_plan& P = C.P;
  if ((rc = plan_init(P, batch, C.probs.data(), &opt, tile))) return rc;
  if (!ws_dev) return set_error(FCMP_E_INVALID, "workspace is NULL");
  if (ws_bytes < P.total) return set_error(FCMP_E_WORKSPACE, "workspace too small");
  C.st = st;
  plan_layout(P, (char*)ws_dev);
  if ((rc = plan_build(P, C.probs.data(), st))) return rc;
  const bool F = cls == FCMP_FOURIER;
  const size_t wb = F ? 16 : 8;
  C.lam.assign((size_t)(batch * P.sK), 0);
  std::vector<double> x((size_t)(batch * P.sK) * (wb / 8), 0.0);
  for (int64_t b = 0; b < batch; ++b)
    for (int64_t k = 0; k < P.shape.K; ++k) {
      C.lam[(size_t)(b * P.sK + k)] = (int32_t)((k * 40503 + 17) & (N - 1));
      x[(size_t)(b * P.sK + k) * (wb / 8)] = 1.0;
    }
  HIP_TRY(hipMemcpyAsync(P.lam, C.lam.data(), C.lam.size() * 4, hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(P.x, x.data(), x.size() * 8, hipMemcpyHostToDevice, st));
  HIP_TRY(launch_fill_u32((uint32_t*)P.y_ent, 0u, (int64_t)(batch * P.sM * wb / 4), st));
  HIP_TRY(launch_fill_u32(P.excl, 0u, batch * P.sE, st));
  HIP_TRY(launch_fill_u32((uint32_t*)P.h0, 0u, (int64_t)(batch * P.sN * wb / 4), st));
  HIP_TRY(launch_init_status(P.status, P.y_ent, (int)M, F, P.sM, batch, st));
  for (hipEvent_t& ev : C.e) HIP_TRY(hipEventCreate(&ev));
  P.cur_flags = flags;   // kernel-vector variants of the fast correlation
  // warm up both paths (the host copies of x must land before the vector dies)
  int npart = 0;
  if ((rc = plan_set_tap_order(P, C.lam.data(), 1, st, C.hord, C.hbst)) ||
      (rc = plan_fast_corr(P, 2, &npart, st)) || (rc = plan_conv_corr(P, 2, &npart, st)))
    return rc;
  HIP_TRY(hipStreamSynchronize(st));
  return FCMP_OK;
}

// Mean device time of one fast and one conventional correlation launch
// sequence at iteration t (t - 1 taps), over kReps of each.
int curve_point(CurveBench& C, int t, float* fast_ms, float* conv_ms) {
  fcmp_plan& P = C.P;
  hipStream_t st = C.st;
  int npart = 0, rc;
  if ((rc = plan_set_tap_order(P, C.lam.data(), t - 1, st, C.hord, C.hbst))) return rc;
  HIP_TRY(hipEventRecord(C.e[0], st));
  for (int r = 0; r < kReps; ++r)
    if ((rc = plan_fast_corr(P, t, &npart, st))) return rc;
  HIP_TRY(hipEventRecord(C.e[1], st));
  for (int r = 0; r < kReps; ++r)
    if ((rc = plan_conv_corr(P, t, &npart, st))) return rc;
  HIP_TRY(hipEventRecord(C.e[2], st));
  HIP_TRY(hipEventSynchronize(C.e[2]));
  float a = 0.f, b = 0.f;
  HIP_TRY(hipEventElapsedTime(&a, C.e[0], C.e[1]));
  HIP_TRY(hipEventElapsedTime(&b, C.e[1], C.e[2]));
  *fast_ms = a / kReps;
  *conv_ms = b / kReps;
  return FCMP_OK;
}

// ---- launch schedules

constexpr int kSchedT = 16;   // the conventional correlation is timed at t = 16

// Tiles worth timing for N: each distinct (B1, B2) split once.
std::vector<int> sched_tiles(bool F, int64_t N) {
  std::vector<int> out;
  std::vector<std::pair<int, int>> seen;
  for (int tile = 256; tile <= 8192; tile *= 2) {
    const Geo g = make_geo(F, (int)N, tile);
    const std::pair<int, int> k(g.B1, g.B2);
    if (std::find(seen.begin(), seen.end(), k) != seen.end()) continue;
    seen.push_back(k);
    out.push_back(tile);
    if (!g.grouped) break;   // one workgroup per transform: no tile to choose
  }
  return out;
}

// Device time of one solve's transform work per iteration under the plan's
// schedule: a conventional correlation at t = kSchedT, plus the kernel vector
// and h_0 transforms spread over 255 iterations (both FP64 forward transforms
// of a sparse input; the kernel vector's stands for both).
int sched_cost(CurveBench& C, float* ms) {
  fcmp_plan& P = C.P;
  hipStream_t st = C.st;
  int npart = 0, rc;
  if ((rc = plan_set_tap_order(P, C.lam.data(), kSchedT - 1, st, C.hord, C.hbst))) return rc;
  if ((rc = plan_conv_corr(P, kSchedT, &npart, st)) || (rc = plan_kernel_vector(P, st))) return rc;
  HIP_TRY(hipEventRecord(C.e[0], st));
  for (int r = 0; r < kReps; ++r)
    if ((rc = plan_conv_corr(P, kSchedT, &npart, st))) return rc;
  HIP_TRY(hipEventRecord(C.e[1], st));
  for (int r = 0; r < kReps; ++r)
    if ((rc = plan_kernel_vector(P, st))) return rc;
  HIP_TRY(hipEventRecord(C.e[2], st));
  HIP_TRY(hipEventSynchronize(C.e[2]));
  float a = 0.f, b = 0.f;
  HIP_TRY(hipEventElapsedTime(&a, C.e[0], C.e[1]));
  HIP_TRY(hipEventElapsedTime(&b, C.e[1], C.e[2]));
  *ms = a / kReps + (b / kReps) * 2.0f / 255.0f;
  return FCMP_OK;
}

int sched_args(int32_t cls, int64_t N, int64_t M, int32_t prec, int32_t batch) {
  if (cls != FCMP_HADAMARD && cls != FCMP_FOURIER) return set_error(FCMP_E_INVALID, "bad class");
  if (N < 64 || (N & (N - 1)) != 0 || N > (int64_t(1) << 24))
    return set_error(FCMP_E_INVALID, "N must be a power of two in [64, 2^24]");
  if (M <= kSchedT || M > N) return set_error(FCMP_E_INVALID, "M must be in (16, N]");
  if (prec != FCMP_FP32 && prec != FCMP_FP64) return set_error(FCMP_E_INVALID, "bad precision");
  if (batch < 1 || batch > 4096) return set_error(FCMP_E_INVALID, "batch must be in [1, 4096]");
  return FCMP_OK;
}

std::string g_sched_line(const std::string& arch, int cls, int64_t N, int prec, int bucket,
                         const Sched& s) {
  char buf[256];
  std::snprintf(buf, sizeof buf, "sched %s %d %lld %d %d %d %d %d\n", arch.c_str(), cls,
                (long long)N, prec, bucket, s.tile, s.threads, s.rthreads);
  return buf;
}

}  // namespace

extern "C" {

int fcmp_schedule_query_workspace(int32_t matrix_class, int64_t N, int64_t M,
                                  int32_t corr_precision, int32_t batch, size_t* bytes) {
  if (!bytes) return set_error(FCMP_E_INVALID, "bytes is NULL");
  int rc = sched_args(matrix_class, N, M, corr_precision, batch);
  if (rc) return rc;
  size_t most = 0;
  for (int tile : sched_tiles(matrix_class == FCMP_FOURIER, N)) {
    std::vector<int32_t> om;
    std::vector<fcmp_problem> probs;
    fcmp_options opt;
    if ((rc = tune_shape(matrix_class, N, M, batch, kSchedT + 1, om, probs, opt, corr_precision)))
      return rc;
    fcmp_plan P;
    if ((rc = plan_init(P, batch, probs.data(), &opt, tile))) return rc;
    most = std::max(most, P.total);
  }
  *bytes = most;
  return FCMP_OK;
}

int fcmp_schedule_tune(int32_t matrix_class, int64_t N, int64_t M, int32_t corr_precision,
                       int32_t batch, const char* cache_path, void* ws_dev, size_t ws_bytes,
                       fcmp_schedule* best, float* ms_default, float* ms_best, void* hip_stream) {
  if (!best) return set_error(FCMP_E_INVALID, "best is NULL");
  int rc = sched_args(matrix_class, N, M, corr_precision, batch);
  if (rc) return rc;
  const std::string arch = device_arch();
  const int bucket = batch_bucket(batch);
  if (cache_path && fcmp_autotune_load(cache_path) == FCMP_OK) {
    Sched s;
    if (tuned_sched(matrix_class, N, corr_precision, batch, &s)) {
      *best = fcmp_schedule{s.tile, s.threads, s.rthreads};
      if (ms_default) *ms_default = 0.f;
      if (ms_best) *ms_best = 0.f;
      return FCMP_OK;
    }
  }
  hipStream_t st = (hipStream_t)hip_stream;
  const bool F = matrix_class == FCMP_FOURIER;
  // the default schedule first, then every tile at default threads
  float t_def = 0.f;
  {
    CurveBench C;
    if ((rc = curve_setup(C, matrix_class, N, M, corr_precision, batch, kSchedT + 1, ws_dev,
                          ws_bytes, st, plan_tile(batch))) ||
        (rc = sched_cost(C, &t_def)))
      return rc;
  }
  float t_best = 1e30f;
  int tile_best = plan_tile(batch);
  for (int tile : sched_tiles(F, N)) {
    CurveBench C;
    float t = 0.f;
    if ((rc = curve_setup(C, matrix_class, N, M, corr_precision, batch, kSchedT + 1, ws_dev,
                          ws_bytes, st, tile)) ||
        (rc = sched_cost(C, &t)))
      return rc;
    if (t < t_best) { t_best = t; tile_best = tile; }
  }
  // thread counts at the best tile (neither changes the tables)
  CurveBench C;
  if ((rc = curve_setup(C, matrix_class, N, M, corr_precision, batch, kSchedT + 1, ws_dev,
                        ws_bytes, st, tile_best)))
    return rc;
  Sched sb;
  sb.tile = tile_best;
  for (int th : {64, 128, 256}) {
    float t = 0.f;
    if (plan_set_threads(C.P, th, 0) != FCMP_OK) continue;
    if ((rc = sched_cost(C, &t))) return rc;
    if (t < t_best) { t_best = t; sb.threads = th; }
  }
  if (C.P.fused && !C.P.rreg) {
    for (int rt : {64, 128, 256}) {
      float t = 0.f;
      if (plan_set_threads(C.P, sb.threads, rt) != FCMP_OK) continue;
      if ((rc = sched_cost(C, &t))) return rc;
      if (t < t_best) { t_best = t; sb.rthreads = rt; }
    }
  }
  if (t_def <= t_best) {   // nothing beat the defaults: record them
    sb = Sched{};
    sb.tile = plan_tile(batch);
    t_best = t_def;
  }
  set_tuned_sched(arch, matrix_class, N, corr_precision, bucket, sb);
  *best = fcmp_schedule{sb.tile, sb.threads, sb.rthreads};
  if (ms_default) *ms_default = t_def;
  if (ms_best) *ms_best = t_best;
  if (cache_path) {
    FILE* f = std::fopen(cache_path, "a");
    if (!f) return set_error(FCMP_E_INVALID, "cannot append to the cache file");
    std::fputs(g_sched_line(arch, matrix_class, N, corr_precision, bucket, sb).c_str(), f);
    std::fclose(f);
  }
  return FCMP_OK;
}

int fcmp_schedule_set(int32_t matrix_class, int64_t N, int32_t corr_precision, int32_t batch,
                      const fcmp_schedule* s) {
  if (matrix_class != FCMP_HADAMARD && matrix_class != FCMP_FOURIER)
    return set_error(FCMP_E_INVALID, "bad class");
  if (N < 2 || (N & (N - 1)) != 0) return set_error(FCMP_E_INVALID, "N must be a power of two");
  if (batch < 1) return set_error(FCMP_E_INVALID, "batch must be >= 1");
  const std::string arch = device_arch();
  if (!s) {
    erase_tuned_sched(arch, matrix_class, N, corr_precision, batch_bucket(batch));
    return FCMP_OK;
  }
  if (s->tile < 0 || s->tile > 8192 || (s->tile & (s->tile - 1)) ||
      (s->threads != 0 && s->threads != 64 && s->threads != 128 && s->threads != 256) ||
      (s->rthreads != 0 && s->rthreads != 64 && s->rthreads != 128 && s->rthreads != 256))
    return set_error(FCMP_E_INVALID, "tile must be a power of two <= 8192, threads 64/128/256");
  set_tuned_sched(arch, matrix_class, N, corr_precision, batch_bucket(batch),
                  Sched{s->tile, s->threads, s->rthreads});
  return FCMP_OK;
}

int fcmp_schedule_get(int32_t matrix_class, int64_t N, int32_t corr_precision, int32_t batch,
                      fcmp_schedule* s, int32_t* tuned) {
  if (!s) return set_error(FCMP_E_INVALID, "s is NULL");
  if (batch < 1) return set_error(FCMP_E_INVALID, "batch must be >= 1");
  std::vector<int32_t> om;
  std::vector<fcmp_problem> probs;
  fcmp_options opt;
  int rc = tune_shape(matrix_class, N, std::max<int64_t>(2, N / 4), batch, 2, om, probs, opt,
                      corr_precision);
  if (rc) return rc;
  fcmp_plan P;
  if ((rc = plan_init(P, batch, probs.data(), &opt))) return rc;
  const Sched d = plan_sched(P);
  *s = fcmp_schedule{d.tile, d.threads, d.rthreads};
  if (tuned) *tuned = P.sched_tuned ? 1 : 0;
  return FCMP_OK;
}

int fcmp_autotune(int32_t matrix_class, int64_t N, int64_t M, int32_t corr_precision,
                  int32_t batch, const char* cache_path, void* ws_dev, size_t ws_bytes,
                  int32_t* switch_t, void* hip_stream) {
  if (!switch_t) return set_error(FCMP_E_INVALID, "switch_t is NULL");
  const int tmax = model_switch_t(matrix_class, N) * 8 + 8;
  if (cache_path && fcmp_autotune_load(cache_path) == FCMP_OK) {
    int t = 0;
    if (tuned_switch(matrix_class, N, corr_precision, &t)) {
      *switch_t = t;
      return FCMP_OK;
    }
  }
  CurveBench C;
  int rc = curve_setup(C, matrix_class, N, M, corr_precision, batch, tmax, ws_dev, ws_bytes,
                       (hipStream_t)hip_stream);
  if (rc) return rc;
  int best = 1;
  for (int t = 2; t <= C.P.shape.K; t += std::max(1, (t - 1) / 4)) {
    float fast_ms = 0.f, conv_ms = 0.f;
    if ((rc = curve_point(C, t, &fast_ms, &conv_ms))) return rc;
    if (fast_ms <= conv_ms) best = t;
    else break;   // the fast cost only grows with t
  }
  set_tuned_switch(matrix_class, N, corr_precision, best);
  *switch_t = best;
  if (cache_path) {
    if (FILE* f = std::fopen(cache_path, "a")) {
      std::fprintf(f, "%d %lld %d %d\n", matrix_class, (long long)N, corr_precision, best);
      std::fclose(f);
    } else {
      return set_error(FCMP_E_INVALID, "cannot append to the cache file");
    }
  }
  return FCMP_OK;
}

int fcmp_corr_curve_query_workspace(int32_t matrix_class, int64_t N, int64_t M,
                                    int32_t corr_precision, int32_t batch, int32_t tmax,
                                    size_t* bytes) {
  if (!bytes) return set_error(FCMP_E_INVALID, "bytes is NULL");
  if (tmax < 2) return set_error(FCMP_E_INVALID, "tmax must be >= 2");
  std::vector<int32_t> om;
  std::vector<fcmp_problem> probs;
  fcmp_options opt;
  int rc = tune_shape(matrix_class, N, M, batch, tmax, om, probs, opt, corr_precision);
  if (rc) return rc;
  fcmp_plan P;
  if ((rc = plan_init(P, batch, probs.data(), &opt))) return rc;
  *bytes = P.total;
  return FCMP_OK;
}

int fcmp_corr_curve(int32_t matrix_class, int64_t N, int64_t M, int32_t corr_precision,
                    int32_t batch, uint32_t flags, const int32_t* ts, int32_t nt, void* ws_dev,
                    size_t ws_bytes, float* fast_ms, float* conv_ms, void* hip_stream) {
  if (!ts || !fast_ms || !conv_ms || nt < 1) return set_error(FCMP_E_INVALID, "bad arrays");
  if (flags & ~(FCMP_FLAG_HALF_KERNEL | FCMP_FLAG_CONJ_PAIR | FCMP_FLAG_FLOAT_KERNEL))
    return set_error(FCMP_E_INVALID, "the curve takes only the kernel-vector flags");
  if ((flags & FCMP_FLAG_CONJ_PAIR) && (matrix_class != FCMP_FOURIER || N > 8192))
    return set_error(FCMP_E_INVALID, "FCMP_FLAG_CONJ_PAIR needs the Fourier class and N <= 8192");
  int tmax = 2;
  for (int i = 0; i < nt; ++i) {
    if (ts[i] < 2) return set_error(FCMP_E_INVALID, "every t must be >= 2");
    tmax = std::max(tmax, ts[i]);
  }
  if (tmax > M - 1) return set_error(FCMP_E_INVALID, "t must be <= M - 1");
  CurveBench C;
  int rc = curve_setup(C, matrix_class, N, M, corr_precision, batch, tmax, ws_dev, ws_bytes,
                       (hipStream_t)hip_stream, 0, flags);
  if (rc) return rc;
  for (int i = 0; i < nt; ++i)
    if ((rc = curve_point(C, ts[i], &fast_ms[i], &conv_ms[i]))) return rc;
  return FCMP_OK;
}

int fcmp_autotune_load(const char* cache_path) {
  if (!cache_path) return set_error(FCMP_E_INVALID, "cache_path is NULL");
  FILE* f = std::fopen(cache_path, "r");
  if (!f) return set_error(FCMP_E_NOTFOUND, "no cache file");
  int n = 0;
  char line[512];
  while (std::fgets(line, sizeof line, f)) {
    int cls = 0, prec = 0, t = 0, bucket = 0, tile = 0, th = 0, rth = 0;
    long long N = 0;
    char arch[128] = {0};
    auto shape_ok = [&] {
      return (cls == FCMP_HADAMARD || cls == FCMP_FOURIER) && N >= 2 && (N & (N - 1)) == 0 &&
             (prec == FCMP_FP64 || prec == FCMP_FP32);
    };
    if (std::sscanf(line, "sched %127s %d %lld %d %d %d %d %d", arch, &cls, &N, &prec, &bucket,
                    &tile, &th, &rth) == 8) {
      if (shape_ok() && bucket >= 0 && bucket <= 4 && tile >= 0 && tile <= 8192 &&
          (tile & (tile - 1)) == 0 && th >= 0 && th <= 256 && rth >= 0 && rth <= 256) {
        set_tuned_sched(arch, cls, N, prec, bucket, Sched{tile, th, rth});
        ++n;
      }
    } else if (std::sscanf(line, "%d %lld %d %d", &cls, &N, &prec, &t) == 4) {
      if (shape_ok() && t >= 1) {
        set_tuned_switch(cls, N, prec, t);
        ++n;
      }
    }
  }
  std::fclose(f);
  return n > 0 ? FCMP_OK : set_error(FCMP_E_NOTFOUND, "no valid entries in the cache file");
}

int fcmp_adaptive_switch(int32_t matrix_class, int64_t N, int32_t corr_precision,
                         int32_t* switch_t, int32_t* tuned) {
  if (!switch_t) return set_error(FCMP_E_INVALID, "switch_t is NULL");
  if (matrix_class != FCMP_HADAMARD && matrix_class != FCMP_FOURIER)
    return set_error(FCMP_E_INVALID, "bad class");
  if (N < 2 || (N & (N - 1)) != 0) return set_error(FCMP_E_INVALID, "N must be a power of two");
  int t = 0;
  const bool have = tuned_switch(matrix_class, N, corr_precision, &t);
  *switch_t = have ? t : model_switch_t(matrix_class, N);
  if (tuned) *tuned = have ? 1 : 0;
  return FCMP_OK;
}

}  // extern "C"
