// Batches of uneven OMP problems: problems whose transform fits one
// workgroup's LDS run whole solves per workgroup in one persistent launch
// (after a lockstep prologue per (class, N, M) group computing the kernel
// vector and h_0); the rest run as lockstep plans per shape.
#include "batch.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <tuple>

namespace fcmp {

#define HIP_TRY(expr)                                                              \
  do {                                                                             \
    hipError_t _e = (expr);                                                        \
    if (_e != hipSuccess)                                                          \
      return set_error(FCMP_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(_e)); \
  } while (0)

static int64_t pad64(int64_t v) { return (v + 63) & ~int64_t(63); }

static int corr_kind(int cls, int precision) {
  const bool F = cls == FCMP_FOURIER;
  if (precision == FCMP_FP32) return F ? V_C64 : V_F32;
  return F ? V_C128 : V_F64;
}

bool wg_eligible(const fcmp_problem& p, const fcmp_options& o) {
  if (o.algorithm != FCMP_OMP || p.K > 1024 || p.N > (1 << 15)) return false;
  const size_t tile = (size_t)(p.N + (p.N >> 5) + 1) * vbytes(corr_kind(p.matrix_class, o.corr_precision));
  return tile <= 140 * 1024;
}

int wg_plan_init(WgBatch& B, int64_t n, const fcmp_problem* probs, const int64_t* ids,
                 const fcmp_options* opt) {
  B.n = n;
  B.opt = *opt;
  B.ids.assign(ids, ids + n);
  // groups by (class, N, M), members contiguous in the internal order
  std::map<std::tuple<int, int64_t, int64_t>, std::vector<int64_t>> gm;
  for (int64_t q = 0; q < n; ++q) {
    const fcmp_problem& p = probs[ids[q]];
    gm[std::make_tuple(p.matrix_class, p.N, p.M)].push_back(ids[q]);
  }
  B.groups.clear();
  B.order_ids.clear();
  for (auto& kv : gm) {
    WgGroup G;
    G.cls = std::get<0>(kv.first);
    G.N = (int)std::get<1>(kv.first);
    G.M = (int)std::get<2>(kv.first);
    G.first = (int64_t)B.order_ids.size();
    G.count = (int64_t)kv.second.size();
    for (int64_t id : kv.second) B.order_ids.push_back(id);
    B.groups.push_back(G);
  }
  B.logNmax = 1;
  B.Kmax = 1;
  B.hmax = 0;
  size_t tile = 64;
  for (int64_t q = 0; q < n; ++q) {
    const fcmp_problem& p = probs[B.order_ids[q]];
    int l = 0;
    while ((int64_t(1) << l) < p.N) ++l;
    B.logNmax = std::max(B.logNmax, l);
    B.Kmax = std::max(B.Kmax, (int)p.K);
    if (p.matrix_class == FCMP_FOURIER && p.N / 16 >= 2) B.hmax = std::max(B.hmax, (int)(p.N / 16));
    const int ck = corr_kind(p.matrix_class, opt->corr_precision);
    tile = std::max(tile, (size_t)(p.N + (p.N >> 5) + 1) * vbytes(ck));
    tile = std::max(tile, (size_t)(2 * p.K + 2) * 16);
  }
  B.tile_bytes = tile;
  wg_layout(B, probs, nullptr);
  return FCMP_OK;
}

void wg_layout(WgBatch& B, const fcmp_problem* probs, char* base) {
  Carver cv;
  cv.base = base;
  const int twS = WG_LOGT / 2;
  const size_t ntw = ((size_t)1 << twS) + (((size_t)1 << WG_LOGT) >> twS) +
                     (size_t)stage_tw_count(B.hmax);
  B.tw64 = cv.take<double2>(ntw);
  B.tw32 = cv.take<float2>(ntw);
  B.desc = cv.take<WgDesc>(B.n);
  B.order = cv.take<int32_t>(B.n);
  B.counter = cv.take<int>(16);
  B.t0 = cv.take<uint64_t>(4);
  B.status = cv.take<Status>(B.n);
  B.ptrs = cv.take<void*>(3 * B.n);
  B.base = base;
  for (WgGroup& G : B.groups) {
    const bool F = G.cls == FCMP_FOURIER;
    const int wk = F ? V_C128 : V_F64;
    const int pk = corr_kind(G.cls, B.opt.corr_precision);
    G.g = make_geo(F, G.N);
    G.sM = pad64(G.M);
    G.sN = pad64(G.N);
    G.sG = pad64(G.g.ngroups + 1);
    const int64_t c = G.count;
    G.tw64 = cv.take<double2>(tw_count(G.g));
    G.tw32 = cv.take<float2>(tw_count(G.g));
    G.ent_k = cv.take<int32_t>(c * G.sM);
    G.perm = cv.take<int32_t>(c * G.sM);
    G.goff = cv.take<int32_t>(c * G.sG);
    G.y_ent = cv.take_bytes(c * G.sM * vbytes(wk));
    G.c64 = cv.take_bytes(c * G.sN * vbytes(wk));
    G.cp = pk == wk ? G.c64 : cv.take_bytes(c * G.sN * vbytes(pk));
    G.h0 = cv.take_bytes(c * G.sN * vbytes(wk));
    G.tmp = cv.take_bytes(c * G.sN * vbytes(wk));
  }
  B.inst_off.assign(B.n, 0);
  for (int64_t q = 0; q < B.n; ++q) {
    const fcmp_problem& p = probs[B.order_ids[q]];
    const size_t wb = p.matrix_class == FCMP_FOURIER ? 16 : 8;
    char* w = (char*)cv.take_bytes((size_t)p.K * (p.K + 1) / 2 * wb + 2 * pad64(p.K) * wb);
    B.inst_off[q] = base ? (int64_t)(w - base) : 0;
  }
  B.total = cv.total();
}

void wg_host_ptrs(const WgBatch& B, const void* const* y, int32_t* const* sup,
                  void* const* xo, void** out) {
  const int64_t n = B.n;
  for (int64_t q = 0; q < n; ++q) {
    const int64_t id = B.order_ids[q];
    out[q] = const_cast<void*>(y[id]);
    out[n + q] = sup[id];
    out[2 * n + q] = xo[id];
  }
}

int wg_solve_batch(WgBatch& B, const fcmp_problem* probs, const void* const* y,
                   int32_t* const* sup, void* const* xo, fcmp_stats* stats, hipStream_t st) {
  int rc = wg_build(B, probs, st);
  if (rc) return rc;
  std::vector<void*> hp(3 * B.n);
  wg_host_ptrs(B, y, sup, xo, hp.data());
  HIP_TRY(hipMemcpyAsync(B.ptrs, hp.data(), hp.size() * sizeof(void*), hipMemcpyHostToDevice, st));
  HIP_TRY(hipStreamSynchronize(st));
  return wg_run(B, stats, st);
}

int wg_build(WgBatch& B, const fcmp_problem* probs, hipStream_t st) {
  const int64_t n = B.n;
  char* base = B.base;
  // ---- host tables and descriptors
  std::vector<WgDesc> desc(n);
  HostTables t;
  for (WgGroup& G : B.groups) {
    const int64_t c = G.count;
    std::vector<int32_t> ent(c * G.sM, 0), perm(c * G.sM, 0), goff(c * G.sG, 0);
    for (int64_t k = 0; k < c; ++k) {
      const fcmp_problem& p = probs[B.order_ids[G.first + k]];
      build_tables(G.g, p.omega, G.M, t);
      std::memcpy(&ent[k * G.sM], t.ent_k.data(), G.M * 4);
      std::memcpy(&perm[k * G.sM], t.perm.data(), G.M * 4);
      std::memcpy(&goff[k * G.sG], t.goff.data(), t.goff.size() * 4);
    }
    HIP_TRY(hipMemcpyAsync(G.tw64, t.tw64.data(), t.tw64.size() * 16, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(G.tw32, t.tw32.data(), t.tw32.size() * 8, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(G.ent_k, ent.data(), ent.size() * 4, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(G.perm, perm.data(), perm.size() * 4, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(G.goff, goff.data(), goff.size() * 4, hipMemcpyHostToDevice, st));
    HIP_TRY(hipStreamSynchronize(st));
  }
  // fixed-size twiddles for the persistent kernel: two-level table of 2^15
  // points, then the stage table up to span B.hmax
  {
    Geo gm = make_geo(true, 1 << WG_LOGT);
    gm.hmax = 0;
    HostTables tf;
    build_tables(gm, nullptr, 0, tf);
    std::vector<double2> s64;
    std::vector<float2> s32;
    build_stage_table(B.hmax, s64, s32);
    tf.tw64.insert(tf.tw64.end(), s64.begin(), s64.end());
    tf.tw32.insert(tf.tw32.end(), s32.begin(), s32.end());
    HIP_TRY(hipMemcpyAsync(B.tw64, tf.tw64.data(), tf.tw64.size() * 16, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(B.tw32, tf.tw32.data(), tf.tw32.size() * 8, hipMemcpyHostToDevice, st));
    HIP_TRY(hipStreamSynchronize(st));   // tf is local
  }
  std::vector<double> cost(n);
  for (WgGroup& G : B.groups) {
    const bool F = G.cls == FCMP_FOURIER;
    const int wk = F ? V_C128 : V_F64;
    const int pk = corr_kind(G.cls, B.opt.corr_precision);
    for (int64_t k = 0; k < G.count; ++k) {
      const int64_t q = G.first + k;
      const fcmp_problem& p = probs[B.order_ids[q]];
      WgDesc& d = desc[q];
      d.cls = p.matrix_class;
      d.N = (int)p.N;
      d.logN = G.g.logN;
      d.M = (int)p.M;
      d.K = (int)p.K;
      d.method = B.opt.corr_method;
      d.switch_t = B.opt.switch_t > 0 ? B.opt.switch_t
                                      : default_switch_t(G.cls, G.N, B.opt.corr_precision);
      d.pad = 0;
      d.off_om = (const char*)(G.ent_k + k * G.sM) - base;
      d.off_y = ((const char*)G.y_ent + k * G.sM * vbytes(wk)) - base;
      d.off_c64 = ((const char*)G.c64 + k * G.sN * vbytes(wk)) - base;
      d.off_cp = ((const char*)G.cp + k * G.sN * (G.cp == G.c64 ? vbytes(wk) : vbytes(pk))) - base;
      d.off_h0 = ((const char*)G.h0 + k * G.sN * vbytes(wk)) - base;
      const size_t wb = vbytes(wk);
      d.off_W = B.inst_off[q];
      d.off_x = d.off_W + (int64_t)((size_t)p.K * (p.K + 1) / 2 * wb);
      d.off_z = d.off_x + pad64(p.K) * (int64_t)wb;
      // largest-first: iteration count times (residual + transform) work
      cost[q] = (double)p.K * ((double)p.M * p.K * 0.5 + (double)p.N * G.g.logN);
    }
  }
  std::vector<int32_t> order(n);
  for (int64_t q = 0; q < n; ++q) order[q] = (int32_t)q;
  std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return cost[a] > cost[b]; });
  HIP_TRY(hipMemcpyAsync(B.desc, desc.data(), n * sizeof(WgDesc), hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(B.order, order.data(), n * 4, hipMemcpyHostToDevice, st));
  HIP_TRY(hipStreamSynchronize(st));
  return FCMP_OK;
}

int wg_run(WgBatch& B, fcmp_stats* stats, hipStream_t st) {
  const int64_t n = B.n;
  HIP_TRY(launch_stamp(B.t0, st));
  {
    // ---- prologue: y in entry order, kernel vector, h_0, per (class, N, M) group
    ProfScope ps(FCMP_PHASE_H0, st);
    for (WgGroup& G : B.groups) {
      const bool F = G.cls == FCMP_FOURIER;
      const int wk = F ? V_C128 : V_F64;
      const int pk = corr_kind(G.cls, B.opt.corr_precision);
      const int c = (int)G.count;
      HIP_TRY(launch_gather_ptr(wk, (const void* const*)(B.ptrs + G.first), G.perm, G.y_ent,
                                G.M, G.sM, G.sM, c, st));
      HIP_TRY(launch_init_status(B.status + G.first, G.y_ent, G.M, F, G.sM, c, st, nullptr,
                                 B.opt.res_tol * B.opt.res_tol));
      const size_t nlo = (size_t)1 << G.g.twS;
      const size_t nhi = (size_t)G.N >> G.g.twS;
      const TwDev tw{G.tw64, G.tw64 + nlo, G.tw64 + nlo + nhi};
      const EntDev en{G.ent_k, G.goff, G.M};
      XDst d;
      d.out = G.c64; d.kind = wk;
      if (G.cp != G.c64) { d.out2 = G.cp; d.kind2 = pk; }
      d.scale = 1.0 / (double)G.N;
      HIP_TRY(run_transform(wk, +1, G.g, tw, en, XSrc{IN_SPARSE_ONES, wk, nullptr}, d, G.tmp,
                            nullptr, st, c, G.sN, G.sM, 0, 0, G.sG));
      XDst h;
      h.out = G.h0; h.kind = wk;
      h.scale = 1.0 / std::sqrt((double)G.N);
      HIP_TRY(run_transform(wk, +1, G.g, tw, en, XSrc{IN_SPARSE, wk, G.y_ent}, h, G.tmp, nullptr,
                            st, c, G.sN, G.sM, 0, 0, G.sG));
    }
  }
  {
    ProfScope ps(FCMP_PHASE_LS, st);
    HIP_TRY(launch_fill_u32((uint32_t*)B.counter, 0u, 1, st));
    WgParams p{};
    p.desc = B.desc;
    p.order = B.order;
    p.n = (int)n;
    p.counter = B.counter;
    p.base = B.base;
    p.status = B.status;
    p.ptrs = B.ptrs;
    p.tw64 = B.tw64;
    p.tw32 = B.tw32;
    {
      const size_t nlo = (size_t)1 << (WG_LOGT / 2), nhi = ((size_t)1 << WG_LOGT) >> (WG_LOGT / 2);
      p.tws64 = B.tw64 + nlo + nhi;
      p.tws32 = B.tw32 + nlo + nhi;
    }
    p.logT = WG_LOGT;
    p.twS = WG_LOGT / 2;
    p.logNmax = B.logNmax;
    p.Kmax = B.Kmax;
    p.tile_bytes = B.tile_bytes;
    p.t0 = B.t0;
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess)
      (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    const int per_cu = B.per_cu > 0 ? B.per_cu : omp_wg_per_cu(p, B.opt.corr_precision);
    const int groups = (int)std::min<int64_t>(n, (int64_t)cus * per_cu);
    HIP_TRY(launch_omp_wg(p, B.opt.corr_precision, groups, st));
  }
  if (stats) return wg_stats(B, stats, st);
  return FCMP_OK;
}

int wg_stats(WgBatch& B, fcmp_stats* stats, hipStream_t st) {
  const int64_t n = B.n;
  {
    std::vector<Status> hs(n);
    HIP_TRY(hipMemcpyAsync(hs.data(), B.status, n * sizeof(Status), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    int dev = 0, khz = 100000;
    if (hipGetDevice(&dev) == hipSuccess)
      (void)hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev);
    if (khz <= 0) khz = 100000;
    int worst = FCMP_OK;
    for (int64_t q = 0; q < n; ++q) {
      fcmp_stats& s = stats[B.order_ids[q]];
      s = fcmp_stats{};
      s.iterations = hs[q].iterations;
      s.status_detail = hs[q].numeric ? FCMP_E_NUMERIC : FCMP_OK;
      s.min_gap = hs[q].min_gap;
      const double r2 = hs[q].ynorm2 - hs[q].znorm2;
      s.res_norm = r2 > 0 ? std::sqrt(r2) : 0.0;
      s.ms_total = hs[q].t_done / (double)khz;   // completion, from the batch start
      if (hs[q].numeric) worst = FCMP_E_NUMERIC;
    }
    if (worst) return set_error(worst, "Cholesky breakdown in at least one instance");
  }
  return FCMP_OK;
}

}  // namespace fcmp
