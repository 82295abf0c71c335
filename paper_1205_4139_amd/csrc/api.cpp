// extern "C" entry points of libfcmp.so (declared in include/fcmp.h).
#include <cmath>
#include <cstring>

#include "engine.h"

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
  const size_t ntw = ((size_t)1 << g.twS) + ((size_t)g.N >> g.twS);
  c.tw64 = cv.take<double2>(ntw);
  c.tw32 = cv.take<float2>(ntw);
  c.tmp = cv.take_bytes((size_t)g.N * vbytes(wide_kind(g.fourier)));
  c.npart = std::max(std::max(transform_partials(V_F32, g), transform_partials(V_C128, g)),
                     fastcorr_groups(g.N));
  c.npart = std::max(c.npart, transform_partials(V_C64, g));
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
  if (vk == V_C64) return TwDev{c.tw32, c.tw32 + nlo};
  return TwDev{c.tw64, c.tw64 + nlo};
}

// ------------------------------------------------------------------ OMP solve
struct OmpLayout {
  Common com;
  void* y_ent = nullptr;   // wide M (entry order)
  void* r = nullptr;       // prec M
  void* c64 = nullptr;     // wide N
  void* cp = nullptr;      // prec N (aliases c64 for FP64)
  void* h0 = nullptr;      // wide N
  int32_t* lam = nullptr;
  uint32_t* excl = nullptr;
  void* x = nullptr;
  void* z = nullptr;
  void* W = nullptr;
  Status* status = nullptr;
  size_t total = 0;
};

OmpLayout omp_layout(const fcmp_problem* p, const fcmp_options* o, void* base) {
  const bool F = p->matrix_class == FCMP_FOURIER;
  const Geo g = make_geo(F, (int)p->N);
  const int wk = wide_kind(F), pk = prec_kind(F, o->corr_precision);
  const int64_t N = p->N, M = p->M, K = p->K;
  Carver cv;
  cv.base = (char*)base;
  OmpLayout L;
  carve_common(cv, g, (int)M, L.com);
  L.y_ent = cv.take_bytes(M * vbytes(wk));
  L.r = cv.take_bytes(M * vbytes(pk));
  L.c64 = cv.take_bytes(N * vbytes(wk));
  L.cp = pk == wk ? L.c64 : cv.take_bytes(N * vbytes(pk));
  L.h0 = cv.take_bytes(N * vbytes(wk));
  L.lam = cv.take<int32_t>(K);
  L.excl = cv.take<uint32_t>((N + 31) / 32);
  L.x = cv.take_bytes(K * vbytes(wk));
  L.z = cv.take_bytes(K * vbytes(wk));
  L.W = cv.take_bytes((size_t)K * (K + 1) / 2 * vbytes(wk));
  L.status = cv.take<Status>(1);
  L.total = cv.total();
  return L;
}

int omp_enqueue(const fcmp_problem* prob, const fcmp_options* opt, const void* y_dev,
                const OmpLayout& L, int32_t* support_dev, void* x_dev, hipStream_t st) {
  const bool F = prob->matrix_class == FCMP_FOURIER;
  const Geo g = make_geo(F, (int)prob->N);
  const int wk = wide_kind(F), pk = prec_kind(F, opt->corr_precision);
  const int N = (int)prob->N, M = (int)prob->M, K = (int)prob->K;
  HostTables t;
  int rc = upload_common(g, prob, L.com, st, t);
  if (rc) return rc;
  const EntDev en{L.com.ent_k, L.com.goff, M};
  HIP_TRY(launch_fill_u32(L.excl, 0u, (N + 31) / 32, st));
  HIP_TRY(launch_init_status(L.status, y_dev, M, F, 0, 1, st));
  // y in entry order
  const void* yent = y_dev;
  if (g.grouped) {
    HIP_TRY(launch_gather_wide(wk, y_dev, L.com.perm, L.y_ent, M, 0, 0, 0, 1, st));
    yent = L.y_ent;
  }
  // A1: kernel vector c = U^H 1_Omega / N  (definition after eq. (kernelsum))
  {
    XDst d;
    d.out = L.c64; d.kind = wk;
    if (L.cp != L.c64) { d.out2 = L.cp; d.kind2 = pk; }
    d.scale = 1.0 / (double)N;
    HIP_TRY(run_transform(wk, +1, g, tw_for(wk, g, L.com), en, XSrc{IN_SPARSE_ONES, wk, nullptr},
                          d, L.com.tmp, nullptr, st));
  }
  // A2: h_0 = Phi^H y in FP64, with the first identification fused
  {
    XDst d;
    d.out = L.h0; d.kind = wk;
    d.partial = L.com.partial; d.excl = L.excl;
    d.scale = 1.0 / std::sqrt((double)N);
    HIP_TRY(run_transform(wk, +1, g, tw_for(wk, g, L.com), en, XSrc{IN_SPARSE, wk, yent}, d,
                          L.com.tmp, nullptr, st));
  }
  LParams lp{};
  lp.N = N; lp.fourier = F;
  lp.partial = L.com.partial; lp.npart = transform_partials(wk, g);
  lp.c64 = L.c64; lp.h0 = L.h0; lp.W = L.W; lp.z = L.z; lp.x = L.x;
  lp.lam = L.lam; lp.excl = L.excl; lp.status = L.status;
  lp.t = 1;
  HIP_TRY(launch_ls_update(lp, 1, st));
  const int switch_t = opt->switch_t > 0 ? opt->switch_t : (F ? 2 + (5 * g.logN) / 6 : 1 + g.logN);
  for (int t = 2; t <= K; ++t) {
    const bool fast = opt->corr_method == FCMP_CORR_FAST ||
                      (opt->corr_method == FCMP_CORR_ADAPTIVE && t <= switch_t);
    int npart;
    if (fast) {
      FParams fp{};
      fp.N = N; fp.logN = g.logN; fp.fourier = F; fp.c_kind = pk;
      fp.h0 = L.h0; fp.c = L.cp; fp.lam = L.lam; fp.x = L.x; fp.ntaps = t - 1;
      fp.h = nullptr; fp.partial = L.com.partial; fp.excl = L.excl; fp.status = L.status;
      HIP_TRY(launch_fastcorr(fp, 1, &npart, st));
    } else {
      RParams rp{};
      rp.N = N; rp.logN = g.logN; rp.twS = g.twS; rp.fourier = F; rp.M = M;
      rp.ent_k = L.com.ent_k; rp.y = yent; rp.r = L.r; rp.r_kind = pk;
      rp.lam = L.lam; rp.x = L.x; rp.ntaps = t - 1;
      rp.tw_lo = L.com.tw64; rp.tw_hi = L.com.tw64 + ((size_t)1 << g.twS);
      rp.status = L.status;
      HIP_TRY(launch_residual(rp, 1, st));
      XDst d;
      d.partial = L.com.partial; d.excl = L.excl;
      d.scale = 1.0 / std::sqrt((double)N);
      HIP_TRY(run_transform(pk, +1, g, tw_for(pk, g, L.com), en, XSrc{IN_SPARSE, pk, L.r}, d,
                            L.com.tmp, L.status, st));
      npart = transform_partials(pk, g);
    }
    lp.t = t;
    lp.npart = npart;
    HIP_TRY(launch_ls_update(lp, 1, st));
  }
  HIP_TRY(launch_finalize(F, L.status, L.lam, L.x, K, support_dev, x_dev, st));
  return FCMP_OK;
}

int fill_stats(const OmpLayout& L, fcmp_stats* stats, hipEvent_t e0, hipEvent_t e1,
               hipStream_t st) {
  HIP_TRY(hipStreamSynchronize(st));
  Status s;
  HIP_TRY(hipMemcpy(&s, L.status, sizeof(Status), hipMemcpyDeviceToHost));
  float ms = 0.f;
  if (e0 && e1) HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
  stats->iterations = s.iterations;
  stats->status = s.numeric ? FCMP_E_NUMERIC : FCMP_OK;
  const double r2 = s.ynorm2 - s.znorm2;
  stats->res_norm = r2 > 0 ? std::sqrt(r2) : 0.0;
  stats->ms_total = ms;
  return stats->status;
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
  int rc = validate_problem(prob, true);
  if (rc) return rc;
  if ((rc = validate_options(prob, opt))) return rc;
  if (!bytes) return set_error(FCMP_E_INVALID, "bytes is NULL");
  if (opt->algorithm != FCMP_OMP) return set_error(FCMP_E_INVALID, "algorithm not available");
  *bytes = omp_layout(prob, opt, nullptr).total;
  return FCMP_OK;
}

int fcmp_solve(const fcmp_problem* prob, const fcmp_options* opt, const void* y_dev,
               void* ws_dev, size_t ws_bytes, int32_t* support_dev, void* x_dev,
               fcmp_stats* stats, void* hip_stream) {
  int rc = validate_problem(prob, true);
  if (rc) return rc;
  if ((rc = validate_options(prob, opt))) return rc;
  if (!y_dev || !ws_dev || !support_dev || !x_dev)
    return set_error(FCMP_E_INVALID, "NULL device pointer");
  if (opt->algorithm != FCMP_OMP) return set_error(FCMP_E_INVALID, "algorithm not available");
  const OmpLayout need = omp_layout(prob, opt, nullptr);
  if (ws_bytes < need.total) return set_error(FCMP_E_WORKSPACE, "workspace too small");
  hipStream_t st = (hipStream_t)hip_stream;
  const OmpLayout L = omp_layout(prob, opt, ws_dev);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (stats) {
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    HIP_TRY(hipEventRecord(e0, st));
  }
  rc = omp_enqueue(prob, opt, y_dev, L, support_dev, x_dev, st);
  if (stats) {
    if (rc == FCMP_OK) {
      HIP_TRY(hipEventRecord(e1, st));
      rc = fill_stats(L, stats, e0, e1, st);
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
  }
  return rc;
}

// ---------------------------------------------------------------- steps
static void carve_kv(Carver& cv, const Geo& g, int M, Common& c) { carve_common(cv, g, M, c); }

int fcmp_kernel_vector_workspace(const fcmp_problem* prob, size_t* bytes) {
  int rc = validate_problem(prob, false);
  if (rc) return rc;
  if (!bytes) return set_error(FCMP_E_INVALID, "bytes is NULL");
  const Geo g = make_geo(prob->matrix_class == FCMP_FOURIER, (int)prob->N);
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
  const Geo g = make_geo(F, (int)prob->N);
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
  const Geo g = make_geo(F, (int)prob->N);
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
  const Geo g = make_geo(F, (int)prob->N);
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
  if (sel_dev) HIP_TRY(launch_reduce_sel(c.partial, transform_partials(pk, g), (Sel*)sel_dev, st));
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

int fcmp_measure_workspace(const fcmp_problem* prob, size_t* bytes) {
  int rc = validate_problem(prob, false);
  if (rc) return rc;
  if (!bytes) return set_error(FCMP_E_INVALID, "bytes is NULL");
  const bool F = prob->matrix_class == FCMP_FOURIER;
  const Geo g = make_geo(F, (int)prob->N);
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
  const Geo g = make_geo(F, (int)prob->N);
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

int fcmp_batch_query_workspace(int64_t n, const fcmp_problem* probs, const fcmp_options* opt,
                               size_t* bytes) {
  (void)n; (void)probs; (void)opt; (void)bytes;
  return set_error(FCMP_E_INVALID, "batch solve not available");
}

int fcmp_batch_solve(int64_t n, const fcmp_problem* probs, const fcmp_options* opt,
                     const void* const* y_dev, void* ws_dev, size_t ws_bytes,
                     int32_t* const* support_dev, void* const* x_dev, fcmp_stats* stats,
                     void* hip_stream) {
  (void)n; (void)probs; (void)opt; (void)y_dev; (void)ws_dev; (void)ws_bytes;
  (void)support_dev; (void)x_dev; (void)stats; (void)hip_stream;
  return set_error(FCMP_E_INVALID, "batch solve not available");
}

}  // extern "C"
