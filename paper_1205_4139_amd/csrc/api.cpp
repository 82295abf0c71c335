// extern "C" entry points of libfcmp.so (declared in include/fcmp.h).
#include <cmath>
#include <cstring>

#include "engine.h"
#include "plan.h"
#include "batch.h"
#include <map>
#include <tuple>

using namespace fcmp;

namespace {

#define HIP_TRY(expr)                                                              \
  do {                                                                             \
    hipError_t _e = (expr);                                                        \
    if (_e != hipSuccess)                                                          \
      return set_error(FCMP_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(_e)); \
  } while (0)

inline int wide_kind(bool fourier) { return fourier ? V_C128 : V_F64; }
inline int prec_kind(bool fourier, int precision) {
  return precision == FCMP_FP32 ? (fourier ? V_C64 : V_F32) : wide_kind(fourier);
}

// Device regions shared by every path that transforms with this geometry.
struct Common {
  int32_t* ent_k = nullptr;
  int32_t* perm = nullptr;
  int32_t* goff = nullptr;
  double2* tw64 = nullptr;
  float2* tw32 = nullptr;
  void* tmp = nullptr;        // N wide values
  Sel* partial = nullptr;
  int npart = 1;
};

void carve_common(Carver& cv, const Geo& g, int M, Common& c) {
  c.ent_k = cv.take<int32_t>(M);
  c.perm = cv.take<int32_t>(M);
  c.goff = cv.take<int32_t>(g.ngroups + 1);
  const size_t ntw = (size_t)tw_count(g);
  c.tw64 = cv.take<double2>(ntw);
  c.tw32 = cv.take<float2>(ntw);
  c.tmp = cv.take_bytes((size_t)g.N * vbytes(wide_kind(g.fourier)));
  c.npart = std::max(transform_partials_max(g), fastcorr_groups(g.N));
  c.partial = cv.take<Sel>(c.npart);
}

int upload_common(const Geo& g, const fcmp_problem* prob, const Common& c, hipStream_t st,
                  HostTables& t) {
  build_tables(g, prob->omega, (int)prob->M, t);
  HIP_TRY(hipMemcpyAsync(c.ent_k, t.ent_k.data(), t.ent_k.size() * 4, hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(c.perm, t.perm.data(), t.perm.size() * 4, hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(c.goff, t.goff.data(), t.goff.size() * 4, hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(c.tw64, t.tw64.data(), t.tw64.size() * sizeof(double2),
                         hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(c.tw32, t.tw32.data(), t.tw32.size() * sizeof(float2),
                         hipMemcpyHostToDevice, st));
  // host tables are stack-owned by the caller; wait for the copies to land
  HIP_TRY(hipStreamSynchronize(st));
  return FCMP_OK;
}

TwDev tw_for(int vk, const Geo& g, const Common& c) {
  const size_t nlo = (size_t)1 << g.twS;
  const size_t nst = nlo + ((size_t)g.N >> g.twS);
  if (vk == V_C64) return TwDev{c.tw32, c.tw32 + nlo, c.tw32 + nst};
  return TwDev{c.tw64, c.tw64 + nlo, c.tw64 + nst};
}

}  // namespace

extern "C" {

int fcmp_abi_version(void) { return FCMP_ABI_VERSION; }

const char* fcmp_status_str(int s) {
  switch (s) {
    case FCMP_OK: return "ok";
    case FCMP_E_INVALID: return "invalid argument";
    case FCMP_E_WORKSPACE: return "workspace too small";
    case FCMP_E_DEVICE: return "device error";
    case FCMP_E_BUSY: return "busy";
    case FCMP_E_NUMERIC: return "numerical breakdown";
    case FCMP_E_NOTFOUND: return "not found";
  }
  return "unknown status";
}

const char* fcmp_last_error(void) { return fcmp::last_error(); }

int fcmp_query_workspace(const fcmp_problem* prob, const fcmp_options* opt, size_t* bytes) {
  if (!bytes) return set_error(FCMP_E_INVALID, "bytes is NULL");
  fcmp_plan P;
  int rc = plan_init(P, 1, prob, opt);
  if (rc) return rc;
  *bytes = P.total;
  return FCMP_OK;
}

int fcmp_solve(const fcmp_problem* prob, const fcmp_options* opt, const void* y_dev,
               void* ws_dev, size_t ws_bytes, int32_t* support_dev, void* x_dev,
               fcmp_stats* stats, void* hip_stream) {
  fcmp_plan P;
  int rc = plan_init(P, 1, prob, opt);
  if (rc) return rc;
  if (!y_dev || !ws_dev || !support_dev || !x_dev)
    return set_error(FCMP_E_INVALID, "NULL device pointer");
  if (ws_bytes < P.total) return set_error(FCMP_E_WORKSPACE, "workspace too small");
  plan_layout(P, (char*)ws_dev);
  hipStream_t st = (hipStream_t)hip_stream;
  if ((rc = plan_build(P, prob, st))) return rc;
  const void* yp[1] = {y_dev};
  int32_t* sp[1] = {support_dev};
  void* xp[1] = {x_dev};
  return plan_solve(P, nullptr, yp, sp, xp, stats, st);
}

int fcmp_plan_query_workspace(int64_t n, const fcmp_problem* probs, const fcmp_options* opt,
                              size_t* bytes) {
  if (!bytes) return set_error(FCMP_E_INVALID, "bytes is NULL");
  fcmp_plan P;
  int rc = plan_init(P, n, probs, opt);
  if (rc) return rc;
  *bytes = P.total;
  return FCMP_OK;
}

int fcmp_plan_create(fcmp_plan** out, int64_t n, const fcmp_problem* probs,
                     const fcmp_options* opt, void* ws_dev, size_t ws_bytes, void* hip_stream) {
  if (!out) return set_error(FCMP_E_INVALID, "out is NULL");
  *out = nullptr;
  fcmp_plan* P = new fcmp_plan();
  int rc = plan_init(*P, n, probs, opt);
  if (rc == FCMP_OK && !ws_dev) rc = set_error(FCMP_E_INVALID, "workspace is NULL");
  if (rc == FCMP_OK && ws_bytes < P->total)
    rc = set_error(FCMP_E_WORKSPACE, "workspace too small");
  if (rc == FCMP_OK) {
    plan_layout(*P, (char*)ws_dev);
    rc = plan_build(*P, probs, (hipStream_t)hip_stream);
  }
  if (rc) {
    delete P;
    return rc;
  }
  *out = P;
  return FCMP_OK;
}

int fcmp_plan_solve(fcmp_plan* plan, const fcmp_options* opt, const void* const* y_dev,
                    int32_t* const* support_dev, void* const* x_dev, fcmp_stats* stats,
                    void* hip_stream) {
  if (!plan) return set_error(FCMP_E_INVALID, "plan is NULL");
  return plan_solve(*plan, opt, y_dev, support_dev, x_dev, stats, (hipStream_t)hip_stream);
}

int fcmp_plan_destroy(fcmp_plan* plan) {
  delete plan;
  return FCMP_OK;
}

int fcmp_profile_enable(int enable) { return profile_enable(enable); }
int fcmp_profile_read(fcmp_profile* out, int reset) { return profile_read(out, reset); }

// ---------------------------------------------------------------- steps
static void carve_kv(Carver& cv, const Geo& g, int M, Common& c) { carve_common(cv, g, M, c); }

int fcmp_kernel_vector_workspace(const fcmp_problem* prob, size_t* bytes) {
  int rc = validate_problem(prob, false);
  if (rc) return rc;
  if (!bytes) return set_error(FCMP_E_INVALID, "bytes is NULL");
  const Geo g = make_geo(prob->matrix_class == FCMP_FOURIER, (int)prob->N, plan_tile(1));
  Carver cv;
  Common c;
  carve_kv(cv, g, (int)prob->M, c);
  *bytes = cv.total();
  return FCMP_OK;
}

int fcmp_kernel_vector(const fcmp_problem* prob, int32_t precision, void* c64_dev, void* cp_dev,
                       void* ws_dev, size_t ws_bytes, void* hip_stream) {
  int rc = validate_problem(prob, false);
  if (rc) return rc;
  if (precision != FCMP_FP64 && precision != FCMP_FP32)
    return set_error(FCMP_E_INVALID, "unknown precision");
  if (!c64_dev || !ws_dev) return set_error(FCMP_E_INVALID, "NULL device pointer");
  size_t need = 0;
  fcmp_kernel_vector_workspace(prob, &need);
  if (ws_bytes < need) return set_error(FCMP_E_WORKSPACE, "workspace too small");
  const bool F = prob->matrix_class == FCMP_FOURIER;
  const Geo g = make_geo(F, (int)prob->N, plan_tile(1));
  Carver cv;
  cv.base = (char*)ws_dev;
  Common c;
  carve_kv(cv, g, (int)prob->M, c);
  hipStream_t st = (hipStream_t)hip_stream;
  HostTables t;
  if ((rc = upload_common(g, prob, c, st, t))) return rc;
  const int wk = wide_kind(F), pk = prec_kind(F, precision);
  XDst d;
  d.out = c64_dev; d.kind = wk;
  if (cp_dev) { d.out2 = cp_dev; d.kind2 = pk; }
  d.scale = 1.0 / (double)prob->N;
  HIP_TRY(run_transform(wk, +1, g, tw_for(wk, g, c), EntDev{c.ent_k, c.goff, (int)prob->M},
                        XSrc{IN_SPARSE_ONES, wk, nullptr}, d, c.tmp, nullptr, st));
  return FCMP_OK;
}

int fcmp_correlate_workspace(const fcmp_problem* prob, int32_t precision, size_t* bytes) {
  int rc = validate_problem(prob, false);
  if (rc) return rc;
  if (precision != FCMP_FP64 && precision != FCMP_FP32)
    return set_error(FCMP_E_INVALID, "unknown precision");
  if (!bytes) return set_error(FCMP_E_INVALID, "bytes is NULL");
  const bool F = prob->matrix_class == FCMP_FOURIER;
  const Geo g = make_geo(F, (int)prob->N, plan_tile(1));
  Carver cv;
  Common c;
  carve_common(cv, g, (int)prob->M, c);
  cv.take_bytes((size_t)prob->M * vbytes(prec_kind(F, precision)));
  *bytes = cv.total();
  return FCMP_OK;
}

int fcmp_correlate(const fcmp_problem* prob, int32_t precision, const void* r_dev, void* h_dev,
                   const uint32_t* excl_dev, void* sel_dev, void* ws_dev, size_t ws_bytes,
                   void* hip_stream) {
  size_t need = 0;
  int rc = fcmp_correlate_workspace(prob, precision, &need);
  if (rc) return rc;
  if (!r_dev || !ws_dev) return set_error(FCMP_E_INVALID, "NULL device pointer");
  if (ws_bytes < need) return set_error(FCMP_E_WORKSPACE, "workspace too small");
  const bool F = prob->matrix_class == FCMP_FOURIER;
  const Geo g = make_geo(F, (int)prob->N, plan_tile(1));
  const int pk = prec_kind(F, precision);
  Carver cv;
  cv.base = (char*)ws_dev;
  Common c;
  carve_common(cv, g, (int)prob->M, c);
  void* r_ent = cv.take_bytes((size_t)prob->M * vbytes(pk));
  hipStream_t st = (hipStream_t)hip_stream;
  HostTables t;
  if ((rc = upload_common(g, prob, c, st, t))) return rc;
  const void* rin = r_dev;
  if (g.grouped) {
    HIP_TRY(launch_gather_wide(pk, r_dev, c.perm, r_ent, prob->M, 0, 0, 0, 1, st));
    rin = r_ent;
  }
  XDst d;
  d.out = h_dev; d.kind = pk;
  d.partial = sel_dev ? c.partial : nullptr;
  d.excl = excl_dev;
  d.scale = 1.0 / std::sqrt((double)prob->N);
  HIP_TRY(run_transform(pk, +1, g, tw_for(pk, g, c), EntDev{c.ent_k, c.goff, (int)prob->M},
                        XSrc{IN_SPARSE, pk, rin}, d, c.tmp, nullptr, st));
  if (sel_dev) HIP_TRY(launch_reduce_sel(c.partial, transform_partials(pk, g, h_dev != nullptr),
                                             (Sel*)sel_dev, st));
  return FCMP_OK;
}

int fcmp_fast_correlate_workspace(const fcmp_problem* prob, size_t* bytes) {
  int rc = validate_problem(prob, false);
  if (rc) return rc;
  if (!bytes) return set_error(FCMP_E_INVALID, "bytes is NULL");
  Carver cv;
  cv.take<Sel>(fastcorr_groups((int)prob->N));
  *bytes = cv.total();
  return FCMP_OK;
}

int fcmp_fast_correlate(const fcmp_problem* prob, int32_t precision, const void* h0_dev,
                        const void* cp_dev, const int32_t* lam_dev, const void* xt_dev,
                        int64_t ntaps, void* h_dev, const uint32_t* excl_dev, void* sel_dev,
                        void* ws_dev, size_t ws_bytes, void* hip_stream) {
  size_t need = 0;
  int rc = fcmp_fast_correlate_workspace(prob, &need);
  if (rc) return rc;
  if (precision != FCMP_FP64 && precision != FCMP_FP32)
    return set_error(FCMP_E_INVALID, "unknown precision");
  if (!h0_dev || !cp_dev || !ws_dev || (ntaps > 0 && (!lam_dev || !xt_dev)))
    return set_error(FCMP_E_INVALID, "NULL device pointer");
  if (ntaps < 0 || ntaps > (int64_t)1 << 24) return set_error(FCMP_E_INVALID, "bad ntaps");
  if (ws_bytes < need) return set_error(FCMP_E_WORKSPACE, "workspace too small");
  const bool F = prob->matrix_class == FCMP_FOURIER;
  Sel* part = (Sel*)ws_dev;
  FParams fp{};
  fp.N = (int)prob->N;
  fp.logN = 0;
  while ((1 << fp.logN) < fp.N) ++fp.logN;
  fp.fourier = F;
  fp.c_kind = prec_kind(F, precision);
  fp.h0 = h0_dev; fp.c = cp_dev; fp.lam = lam_dev; fp.x = xt_dev; fp.ntaps = (int)ntaps;
  fp.h = h_dev; fp.partial = sel_dev ? part : nullptr; fp.excl = excl_dev; fp.status = nullptr;
  hipStream_t st = (hipStream_t)hip_stream;
  int groups = 0;
  HIP_TRY(launch_fastcorr(fp, 1, &groups, st));
  if (sel_dev) HIP_TRY(launch_reduce_sel(part, groups, (Sel*)sel_dev, st));
  return FCMP_OK;
}

int fcmp_topk_workspace(int64_t n, size_t* bytes) {
  if (!bytes) return set_error(FCMP_E_INVALID, "bytes is NULL");
  if (n < 1 || n >= ((int64_t)1 << 31)) return set_error(FCMP_E_INVALID, "n must be in [1, 2^31)");
  *bytes = topk_workspace(n);
  return FCMP_OK;
}

int fcmp_topk(int32_t matrix_class, int32_t precision, const void* v_dev, int64_t n,
              const uint32_t* excl_dev, int64_t K, int32_t* out_dev, void* ws_dev,
              size_t ws_bytes, void* hip_stream) {
  size_t need = 0;
  int rc = fcmp_topk_workspace(n, &need);
  if (rc) return rc;
  if (matrix_class != FCMP_HADAMARD && matrix_class != FCMP_FOURIER)
    return set_error(FCMP_E_INVALID, "matrix_class must be FCMP_HADAMARD or FCMP_FOURIER");
  if (precision != FCMP_FP64 && precision != FCMP_FP32)
    return set_error(FCMP_E_INVALID, "unknown precision");
  if (K < 1 || K > n) return set_error(FCMP_E_INVALID, "K must be in [1, n]");
  if (!v_dev || !out_dev || !ws_dev) return set_error(FCMP_E_INVALID, "NULL device pointer");
  if (ws_bytes < need) return set_error(FCMP_E_WORKSPACE, "workspace too small");
  const int kind = prec_kind(matrix_class == FCMP_FOURIER, precision);
  HIP_TRY(launch_topk(v_dev, kind, n, excl_dev, K, ws_dev, out_dev, (hipStream_t)hip_stream));
  return FCMP_OK;
}

int fcmp_measure_workspace(const fcmp_problem* prob, size_t* bytes) {
  int rc = validate_problem(prob, false);
  if (rc) return rc;
  if (!bytes) return set_error(FCMP_E_INVALID, "bytes is NULL");
  const bool F = prob->matrix_class == FCMP_FOURIER;
  const Geo g = make_geo(F, (int)prob->N, plan_tile(1));
  Carver cv;
  Common c;
  carve_common(cv, g, (int)prob->M, c);
  cv.take<int32_t>(prob->M);
  cv.take_bytes((size_t)prob->N * vbytes(wide_kind(F)));
  cv.take_bytes((size_t)prob->M * vbytes(wide_kind(F)));
  *bytes = cv.total();
  return FCMP_OK;
}

int fcmp_measure(const fcmp_problem* prob, const void* x_dev, const void* noise_dev, double snr_db,
                 void* y_dev, void* ws_dev, size_t ws_bytes, void* hip_stream) {
  size_t need = 0;
  int rc = fcmp_measure_workspace(prob, &need);
  if (rc) return rc;
  if (!x_dev || !y_dev || !ws_dev) return set_error(FCMP_E_INVALID, "NULL device pointer");
  if (ws_bytes < need) return set_error(FCMP_E_WORKSPACE, "workspace too small");
  if (noise_dev && !std::isfinite(snr_db)) return set_error(FCMP_E_INVALID, "snr_db not finite");
  const bool F = prob->matrix_class == FCMP_FOURIER;
  const Geo g = make_geo(F, (int)prob->N, plan_tile(1));
  const int wk = wide_kind(F);
  Carver cv;
  cv.base = (char*)ws_dev;
  Common c;
  carve_common(cv, g, (int)prob->M, c);
  int32_t* om = cv.take<int32_t>(prob->M);
  void* full = cv.take_bytes((size_t)prob->N * vbytes(wk));
  void* clean = cv.take_bytes((size_t)prob->M * vbytes(wk));
  hipStream_t st = (hipStream_t)hip_stream;
  HostTables t;
  if ((rc = upload_common(g, prob, c, st, t))) return rc;
  HIP_TRY(hipMemcpyAsync(om, prob->omega, prob->M * 4, hipMemcpyHostToDevice, st));
  HIP_TRY(hipStreamSynchronize(st));
  XDst d;
  d.out = full; d.kind = wk;
  d.scale = 1.0 / std::sqrt((double)prob->N);
  HIP_TRY(run_transform(wk, -1, g, tw_for(wk, g, c), EntDev{c.ent_k, c.goff, (int)prob->M},
                        XSrc{IN_DENSE, wk, x_dev}, d, c.tmp, nullptr, st));
  void* dst = noise_dev ? clean : y_dev;
  HIP_TRY(launch_gather_wide(wk, full, om, dst, prob->M, 0, 0, 0, 1, st));
  if (noise_dev) HIP_TRY(launch_noise(F, clean, noise_dev, snr_db, y_dev, (int)prob->M, st));
  return FCMP_OK;
}

}  // extern "C"
