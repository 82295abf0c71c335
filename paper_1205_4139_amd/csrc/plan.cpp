// Plan construction and the lockstep OMP solve (Algorithm 1.1 with either
// correlation method), n instances of one shape per launch.
#include "plan.h"

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <thread>

namespace fcmp {

#define HIP_TRY(expr)                                                              \
  do {                                                                             \
    hipError_t _e = (expr);                                                        \
    if (_e != hipSuccess)                                                          \
      return set_error(FCMP_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(_e)); \
  } while (0)

static int64_t pad64(int64_t v) { return (v + 63) & ~int64_t(63); }

// Geometry of the fused residual + first-pass launch: the correlation's
// first pass (B1 columns of length N2 per workgroup).
// Columns per workgroup of the fused pass: the most whose tile fits the
// kernel (at most 2048 values, 64 KiB of LDS), a function of (class, N,
// precision) only, so whether a plan fuses the residual never depends on the
// plan's size or launch knobs.
RCParams rcorr_geometry(const fcmp_plan& P) {
  RCParams q{};
  q.N = P.g.N; q.logN = P.g.logN; q.twS = P.g.twS;
  q.L = 1 << P.g.n2; q.logL = P.g.n2; q.logN1 = P.g.n1;
  const int N1 = 1 << P.g.n1;
  int best = 1;
  for (int b = 1; b <= N1 && b * q.L <= 2048; b *= 2) {
    q.B = b;
    if (rcorr_ok(P.pk, P.g.fourier, q, rcorr_threads(q))) best = b;
  }
  q.B = best;
  return q;
}

int rcorr_threads(const RCParams& q) { return std::min(256, std::max(64, q.B * q.L / 8)); }

Sched plan_sched(const fcmp_plan& P) {
  Sched s;
  s.tile = P.g.B1 << P.g.n2;
  s.threads = P.g.threads > 0 ? P.g.threads : tune().threads;
  if (P.fused && !P.rreg) s.rthreads = P.rthreads > 0 ? P.rthreads : rcorr_threads(rcorr_geometry(P));
  return s;
}

int plan_set_threads(fcmp_plan& P, int threads, int rthreads) {
  if (threads != 0 && (threads < 64 || threads > 256 || (threads & (threads - 1))))
    return set_error(FCMP_E_INVALID, "transform threads must be 64, 128 or 256");
  if (rthreads != 0) {
    if (!P.fused || P.rreg) return set_error(FCMP_E_INVALID, "no generic fused first pass");
    const RCParams q = rcorr_geometry(P);
    if (!rcorr_ok(P.pk, P.g.fourier, q, rthreads))
      return set_error(FCMP_E_INVALID, "the fused first pass cannot run with that many threads");
  }
  P.g.threads = threads;
  P.rthreads = rthreads;
  return FCMP_OK;
}

int plan_init(fcmp_plan& P, int64_t n, const fcmp_problem* probs, const fcmp_options* opt,
              int tile) {
  if (n < 1) return set_error(FCMP_E_INVALID, "n must be >= 1");
  if (!probs) return set_error(FCMP_E_INVALID, "problems is NULL");
  if (!opt) return set_error(FCMP_E_INVALID, "options is NULL");
  P.uniform = true;
  P.hM.assign(n, 0);
  P.hK.assign(n, 0);
  fcmp_problem big = probs[0];
  for (int64_t b = 0; b < n; ++b) {
    int rc = validate_problem(&probs[b], true);
    if (rc) return rc;
    if ((rc = validate_options(&probs[b], opt))) return rc;
    if (probs[b].matrix_class != probs[0].matrix_class || probs[b].N != probs[0].N)
      return set_error(FCMP_E_INVALID, "plan problems must share class and N");
    if (probs[b].M != probs[0].M || probs[b].K != probs[0].K) {
      if (opt->algorithm != FCMP_OMP)
        return set_error(FCMP_E_INVALID, "SP/CoSaMP plan problems must share M and K");
      P.uniform = false;
    }
    P.hM[b] = (int32_t)probs[b].M;
    P.hK[b] = (int32_t)probs[b].K;
    big.M = std::max(big.M, probs[b].M);
    big.K = std::max(big.K, probs[b].K);
  }
  if (opt->algorithm != FCMP_OMP && probs[0].K > 2048)
    return set_error(FCMP_E_INVALID, "SP and CoSaMP support K <= 2048");
  P.n = n;
  P.shape = big;
  P.shape.omega = nullptr;
  P.opt = *opt;
  const bool F = P.shape.matrix_class == FCMP_FOURIER;
  Sched sc;
  P.sched_tuned = tile <= 0 && !tune().tile_fixed &&
                  tuned_sched(big.matrix_class, big.N, opt->corr_precision, n, &sc);
  if (P.sched_tuned && sc.tile > 0) tile = sc.tile;
  P.g = make_geo(F, (int)P.shape.N, tile > 0 ? tile : plan_tile(n));
  if (P.sched_tuned) P.g.threads = sc.threads;
  P.wk = F ? V_C128 : V_F64;
  P.pk = opt->corr_precision == FCMP_FP32 ? (F ? V_C64 : V_F32) : P.wk;
  const int64_t N = P.shape.N, M = P.shape.M, K = P.shape.K;
  P.sM = pad64(M);
  P.sN = pad64(N);
  P.sK = pad64(K);
  P.sW = pad64(K * (K + 1) / 2);
  P.sG = pad64(P.g.ngroups + 1);
  P.sG2 = pad64(P.g.ngroups2 + 1);
  const char* rr = std::getenv("FCMP_RESID_RATIO");
  if (rr) P.resid_ratio = std::atof(rr);
  // the residual fused into the correlation's first pass (OMP, two-pass
  // correlation); FCMP_RESID_RATIO selects the separate residual kernels
  if (opt->algorithm == FCMP_OMP && P.g.grouped && !single_ok(P.pk, (int)N) && !rr) {
    RCParams q = rcorr_geometry(P);
    q.cmask = (const uint32_t*)&P;   // presence only: the tables are laid out below
    q.cbase = (const int32_t*)&P;
    P.rreg = rcorr_reg_ok(P.pk, F, q);
    P.fused = P.rreg || rcorr_ok(P.pk, F, q, rcorr_threads(q));
    // a tuned thread count is taken only where the fused pass runs with it
    if (P.sched_tuned && sc.rthreads > 0 && P.fused && !P.rreg &&
        rcorr_ok(P.pk, F, q, sc.rthreads))
      P.rthreads = sc.rthreads;
  }
  P.sC = pad64(N / 32);
  P.sCs = pad64(((int64_t)1 << P.g.n1) + 1);
  P.sB = pad64(((int64_t)1 << P.g.n2) + 1);
  P.npart = std::max(transform_partials_max(P.g), fastcorr_groups((int)N));
  P.sP = pad64(P.npart);
  P.sE = pad64((N + 31) / 32);
  plan_layout(P, nullptr);
  return FCMP_OK;
}

void plan_layout(fcmp_plan& P, char* base) {
  Carver cv;
  cv.base = base;
  const int64_t n = P.n;
  const size_t ntw = (size_t)tw_count(P.g);
  const size_t wb = vbytes(P.wk), pb = vbytes(P.pk);
  P.tw64 = cv.take<double2>(ntw);
  P.tw32 = cv.take<float2>(ntw);
  P.ent_k = cv.take<int32_t>(n * P.sM);
  P.perm = cv.take<int32_t>(n * P.sM);
  P.goff = cv.take<int32_t>(n * P.sG);
  if (!P.g.same_out) {
    P.ent2_k = cv.take<int32_t>(n * P.sM);
    P.goff2 = cv.take<int32_t>(n * P.sG2);
    P.pos1 = cv.take<int32_t>(n * P.sM);
  } else {
    P.ent2_k = P.ent_k;
    P.goff2 = P.goff;
    P.pos1 = nullptr;
  }
  if (P.rreg) {
    P.cmask = cv.take<uint32_t>(n * P.sC);
    P.cbase = cv.take<int32_t>(n * P.sC);
  } else {
    P.cmask = nullptr;
    P.cbase = nullptr;
  }
  P.cst = (P.fused && !P.rreg) ? cv.take<int32_t>(n * P.sCs) : nullptr;
  if (!P.uniform) {
    P.Mv = cv.take<int32_t>(n);
    P.Kv = cv.take<int32_t>(n);
  } else {
    P.Mv = P.Kv = nullptr;
  }
  P.c64 = cv.take_bytes(n * P.sN * wb);
  P.cp = P.pk == P.wk ? P.c64 : cv.take_bytes(n * P.sN * pb);
  // Hadamard: |N c(j)| <= M, so N c fits int16 when M < 2^15 (Sec. III-B:
  // the kernel vector takes few distinct values)
  P.ci16 = (!P.g.fourier && P.shape.M < (1 << 15)) ? cv.take<int16_t>(n * P.sN) : nullptr;
  P.y_ent = cv.take_bytes(n * P.sM * wb);
  P.r = cv.take_bytes(n * P.sM * pb);
  P.h0 = cv.take_bytes(n * P.sN * wb);
  P.tmp = cv.take_bytes(n * P.sN * wb);
  P.partial = cv.take<Sel>(n * P.sP);
  P.lam = cv.take<int32_t>(n * P.sK);
  if (P.fused) {
    P.ord = cv.take<int32_t>(n * 2 * P.sK);
    P.bst = cv.take<int32_t>(n * 2 * P.sB);
  } else {
    P.ord = P.bst = nullptr;
  }
  P.excl = cv.take<uint32_t>(n * P.sE);
  P.x = cv.take_bytes(n * P.sK * wb);
  P.z = cv.take_bytes(n * P.sK * wb);
  P.W = cv.take_bytes(n * P.sW * wb);
  P.wbuf = cv.take_bytes(n * P.sK * wb);
  P.vpart = cv.take_bytes(n * ls_split_groups((int)P.shape.K) * P.sK * wb);
  P.status = cv.take<Status>(n);
  if (P.opt.algorithm != FCMP_OMP) {
    const int64_t K = P.shape.K, N = P.shape.N;
    const int smax = (int)(P.opt.algorithm == FCMP_SP ? 2 * K : 3 * K);
    P.hbuf = cv.take_bytes(N * wb);
    P.Ta = cv.take<int32_t>(3 * K);
    P.Tb = cv.take<int32_t>(3 * K);
    P.Tc = cv.take<int32_t>(3 * K);
    P.Td = cv.take<int32_t>(3 * K);
    P.xa = cv.take_bytes(3 * K * wb);
    P.xb = cv.take_bytes(3 * K * wb);
    P.xc = cv.take_bytes(3 * K * wb);
    P.dws = cv.take_bytes(dense_ls_workspace(smax, P.wk == V_C128));
    P.tkws = cv.take_bytes(topk_workspace(N));
    P.small = cv.take<double>(256);
    P.bad = cv.take<int>(16);
  }
  P.dptrs = cv.take<void*>(3 * n);
  P.total = cv.total();
}

static TwDev tw_for(const fcmp_plan& P, int vk) {
  const size_t nlo = (size_t)1 << P.g.twS;
  const size_t nst = nlo + ((size_t)P.g.N >> P.g.twS);
  if (vk == V_C64) return TwDev{P.tw32, P.tw32 + nlo, P.tw32 + nst};
  return TwDev{P.tw64, P.tw64 + nlo, P.tw64 + nst};
}

int plan_kernel_vector(fcmp_plan& P, hipStream_t st) {
  ProfScope ps(FCMP_PHASE_KERNEL, st);
  XDst d;
  d.out = P.c64; d.kind = P.wk;
  if (P.cp != P.c64) { d.out2 = P.cp; d.kind2 = P.pk; }
  d.scale = 1.0 / (double)P.shape.N;
  HIP_TRY(run_transform(P.wk, +1, P.g, tw_for(P, P.wk),
                        EntDev{P.ent_k, P.goff, (int)P.shape.M}, XSrc{IN_SPARSE_ONES, P.wk, nullptr},
                        d, P.tmp, nullptr, st, (int)P.n, P.sN, P.sM, 0, 0, P.sG));
  if (P.ci16)
    HIP_TRY(launch_to_int16((const double*)P.c64, P.ci16, (double)P.shape.N, P.shape.N, P.sN, P.sN,
                            (int)P.n, st));
  return FCMP_OK;
}

int plan_build(fcmp_plan& P, const fcmp_problem* probs, hipStream_t st) {
  const int64_t n = P.n;
  std::vector<int32_t> ent((size_t)(n * P.sM), 0), perm((size_t)(n * P.sM), 0),
      goff((size_t)(n * P.sG), 0);
  std::vector<int32_t> ent2, goff2, pos1, cbase, cst;
  std::vector<uint32_t> cmask;
  if (P.cst) cst.assign((size_t)(n * P.sCs), 0);
  if (P.rreg) {
    cmask.assign((size_t)(n * P.sC), 0u);
    cbase.assign((size_t)(n * P.sC), 0);
  }
  if (!P.g.same_out) {
    ent2.assign((size_t)(n * P.sM), 0);
    goff2.assign((size_t)(n * P.sG2), 0);
    pos1.assign((size_t)(n * P.sM), 0);
  }
  // the per-instance tables are independent: built by up to eight host
  // threads for large plans, each with its own table set
  int64_t work = 0;
  for (int64_t b = 0; b < n; ++b) work += probs[b].M + P.g.N / 8;
  const int64_t hw = (int64_t)std::max(1u, std::thread::hardware_concurrency());
  const int nth = (int)std::max<int64_t>(1, std::min<int64_t>({n, 8, hw, work / (1 << 18) + 1}));
  std::vector<HostTables> tset((size_t)nth);
  auto fill = [&](int th) {
    HostTables& t = tset[(size_t)th];
    for (int64_t b = th; b < n; b += nth) {
      const int64_t M = probs[b].M;
      build_tables(P.g, probs[b].omega, (int)M, t);
      std::memcpy(&ent[b * P.sM], t.ent_k.data(), M * 4);
      std::memcpy(&perm[b * P.sM], t.perm.data(), M * 4);
      std::memcpy(&goff[b * P.sG], t.goff.data(), t.goff.size() * 4);
      if (P.rreg) {
        std::memcpy(&cmask[b * P.sC], t.cmask.data(), t.cmask.size() * 4);
        std::memcpy(&cbase[b * P.sC], t.cbase.data(), t.cbase.size() * 4);
      }
      if (P.cst) std::memcpy(&cst[b * P.sCs], t.cst.data(), t.cst.size() * 4);
      if (!P.g.same_out) {
        std::memcpy(&ent2[b * P.sM], t.ent2_k.data(), M * 4);
        std::memcpy(&goff2[b * P.sG2], t.goff2.data(), t.goff2.size() * 4);
        std::memcpy(&pos1[b * P.sM], t.pos1.data(), M * 4);
      }
    }
  };
  if (nth == 1) {
    fill(0);
  } else {
    std::vector<std::thread> ths;
    for (int th = 0; th < nth; ++th) ths.emplace_back(fill, th);
    for (std::thread& th : ths) th.join();
  }
  const HostTables& t = tset[0];
  if (!P.g.same_out) {
    HIP_TRY(hipMemcpyAsync(P.ent2_k, ent2.data(), ent2.size() * 4, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(P.goff2, goff2.data(), goff2.size() * 4, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(P.pos1, pos1.data(), pos1.size() * 4, hipMemcpyHostToDevice, st));
  }
  if (P.cst)
    HIP_TRY(hipMemcpyAsync(P.cst, cst.data(), cst.size() * 4, hipMemcpyHostToDevice, st));
  if (P.rreg) {
    HIP_TRY(hipMemcpyAsync(P.cmask, cmask.data(), cmask.size() * 4, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(P.cbase, cbase.data(), cbase.size() * 4, hipMemcpyHostToDevice, st));
  }
  HIP_TRY(hipMemcpyAsync(P.tw64, t.tw64.data(), t.tw64.size() * sizeof(double2),
                         hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(P.tw32, t.tw32.data(), t.tw32.size() * sizeof(float2),
                         hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(P.ent_k, ent.data(), ent.size() * 4, hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(P.perm, perm.data(), perm.size() * 4, hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(P.goff, goff.data(), goff.size() * 4, hipMemcpyHostToDevice, st));
  if (!P.uniform) {
    HIP_TRY(hipMemcpyAsync(P.Mv, P.hM.data(), n * 4, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(P.Kv, P.hK.data(), n * 4, hipMemcpyHostToDevice, st));
  }
  int rc = plan_kernel_vector(P, st);
  if (rc) return rc;
  HIP_TRY(hipStreamSynchronize(st));
  P.last_ptrs.clear();
  return FCMP_OK;
}

static int upload_ptrs(fcmp_plan& P, const void* const* y, int32_t* const* sup, void* const* x,
                       hipStream_t st) {
  std::vector<const void*> want((size_t)(3 * P.n));
  for (int64_t b = 0; b < P.n; ++b) {
    if (!y[b] || !sup[b] || !x[b]) return set_error(FCMP_E_INVALID, "NULL device pointer");
    want[b] = y[b];
    want[P.n + b] = sup[b];
    want[2 * P.n + b] = x[b];
  }
  if (want == P.last_ptrs) return FCMP_OK;
  HIP_TRY(hipMemcpyAsync(P.dptrs, want.data(), want.size() * sizeof(void*),
                         hipMemcpyHostToDevice, st));
  HIP_TRY(hipStreamSynchronize(st));   // the host array is the caller's
  P.last_ptrs = want;
  return FCMP_OK;
}

void stats_phases(fcmp_stats& s, const double* pms) {
  s.ms_corr = (float)(pms[FCMP_PHASE_H0] + pms[FCMP_PHASE_CORR] + pms[FCMP_PHASE_FAST]);
  s.ms_select = (float)pms[FCMP_PHASE_SELECT];
  s.ms_ls = (float)pms[FCMP_PHASE_LS];
  s.ms_resid = (float)pms[FCMP_PHASE_RESID];
}

int plan_stats(int64_t n, const Status* hs, double ms, fcmp_stats* stats, const double* pms) {
  int worst = FCMP_OK;
  for (int64_t b = 0; b < n; ++b) {
    stats[b] = fcmp_stats{};
    stats[b].iterations = hs[b].iterations;
    stats[b].status_detail = hs[b].numeric ? FCMP_E_NUMERIC : FCMP_OK;
    const double r2 = hs[b].ynorm2 - hs[b].znorm2;
    stats[b].res_norm = r2 > 0 ? std::sqrt(r2) : 0.0;
    stats[b].min_gap = hs[b].min_gap;
    if (pms) stats_phases(stats[b], pms);
    stats[b].ms_total = ms;
    if (stats[b].status_detail != FCMP_OK) worst = stats[b].status_detail;
  }
  if (worst != FCMP_OK) return set_error(worst, "Cholesky breakdown in at least one instance");
  return FCMP_OK;
}

// Kernel vector (when asked), exclusion reset, y in entry order, status and
// h_0 with the first identification: device work only.
static int plan_enqueue_prefix(fcmp_plan& P, const fcmp_options& opt, hipStream_t st) {
  int rc = FCMP_OK;
  P.cur_flags = opt.flags;
  const bool F = P.shape.matrix_class == FCMP_FOURIER;
  const int n = (int)P.n;
  const int N = (int)P.shape.N, M = (int)P.shape.M;
  const Geo& g = P.g;
  const EntDev en{P.ent_k, P.goff, M};
  if (opt.flags & FCMP_FLAG_RECOMPUTE_KERNEL) {
    if ((rc = plan_kernel_vector(P, st))) return rc;
  }
  {
    ProfScope ps(FCMP_PHASE_OTHER, st);
    HIP_TRY(launch_fill_u32(P.excl, 0u, P.n * P.sE, st));
    HIP_TRY(launch_gather_ptr(P.wk, (const void* const*)P.dptrs, P.perm, P.y_ent, M, P.sM, P.sM,
                              n, st, P.Mv));
    HIP_TRY(launch_init_status(P.status, P.y_ent, M, F, P.sM, n, st, P.Mv,
                               opt.res_tol * opt.res_tol));
  }
  const double inv_sqrt_n = 1.0 / std::sqrt((double)N);
  {
    // A2: h_0 = Phi^H y in FP64 with the first identification fused
    ProfScope ps(FCMP_PHASE_H0, st);
    XDst d;
    d.out = P.h0; d.kind = P.wk;
    d.partial = P.partial; d.excl = P.excl;
    d.scale = inv_sqrt_n;
    HIP_TRY(run_transform(P.wk, +1, g, tw_for(P, P.wk), en, XSrc{IN_SPARSE, P.wk, P.y_ent}, d,
                          P.tmp, nullptr, st, n, P.sN, P.sM, P.sP, P.sE, P.sG));
  }
  (void)rc;
  return FCMP_OK;
}

int plan_set_tap_order(fcmp_plan& P, const int32_t* lam, int ntaps, hipStream_t st,
                       std::vector<int32_t>& ord, std::vector<int32_t>& bst) {
  if (!P.fused) return FCMP_OK;
  const int NB = 1 << P.g.n2;
  const int shift = P.g.fourier ? 0 : P.g.n1;
  ord.assign((size_t)(P.n * P.sK), 0);
  bst.assign((size_t)(P.n * P.sB), 0);
  for (int64_t b = 0; b < P.n; ++b) {
    const int32_t* l = lam + b * P.sK;
    int32_t* bs = &bst[(size_t)(b * P.sB)];
    for (int k = 0; k < ntaps; ++k) ++bs[((l[k] >> shift) & (NB - 1)) + 1];
    for (int q = 0; q < NB; ++q) bs[q + 1] += bs[q];
    std::vector<int32_t> fill(bs, bs + NB);
    for (int k = 0; k < ntaps; ++k) ord[(size_t)(b * P.sK + fill[(l[k] >> shift) & (NB - 1)]++)] = k;
  }
  const int par = ntaps & 1;
  HIP_TRY(hipMemcpy2DAsync(P.ord + par * P.sK, 2 * P.sK * 4, ord.data(), P.sK * 4, P.sK * 4, P.n,
                           hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpy2DAsync(P.bst + par * P.sB, 2 * P.sB * 4, bst.data(), P.sB * 4, P.sB * 4, P.n,
                           hipMemcpyHostToDevice, st));
  return FCMP_OK;
}

// One fast correlation (eq. (kernelsumOMP)) with t-1 taps and the fused
// identification; returns the number of partials through npart.
int plan_fast_corr(fcmp_plan& P, int t, int* npart, hipStream_t st) {
  ProfScope ps(FCMP_PHASE_FAST, st);
  FParams fp{};
  fp.N = (int)P.shape.N; fp.logN = P.g.logN; fp.fourier = P.g.fourier; fp.c_kind = P.pk;
  fp.h0 = P.h0; fp.c = P.cp; fp.lam = P.lam; fp.x = P.x; fp.ntaps = t - 1;
  fp.c_half = (P.g.fourier && (P.cur_flags & FCMP_FLAG_HALF_KERNEL)) ? 1 : 0;
  if (P.ci16 && !(P.cur_flags & FCMP_FLAG_FLOAT_KERNEL)) {
    fp.c = P.ci16;
    fp.c_int16 = 1;
    fp.cscale = 1.0 / (double)P.shape.N;
  }
  fp.h = nullptr; fp.partial = P.partial; fp.excl = P.excl; fp.status = P.status;
  fp.inst_h0 = P.sN; fp.inst_c = P.sN; fp.inst_lam = P.sK; fp.inst_x = P.sK;
  fp.inst_h = 0; fp.inst_part = P.sP; fp.inst_excl = P.sE;
  if (P.cur_flags & FCMP_FLAG_CONJ_PAIR) {
    fp.c_half = 0;
    HIP_TRY(launch_fastpair(fp, (int)P.n, npart, st));
    return FCMP_OK;
  }
  HIP_TRY(launch_fastcorr(fp, (int)P.n, npart, st));
  return FCMP_OK;
}

// One conventional correlation at iteration t: the FP64 residual of the
// t-1 selected columns (direct while M_i (t-1) <= ratio N log2 N, per
// instance, else through a forward transform of S_Lambda^T x) and the
// transform of the zero-filled residual with the fused identification.
static int conv_corr(fcmp_plan& P, int t, int* npart, hipStream_t st, const int32_t* tofs);

int plan_conv_corr(fcmp_plan& P, int t, int* npart, hipStream_t st) {
  return conv_corr(P, t, npart, st, nullptr);
}

static int conv_corr(fcmp_plan& P, int t, int* npart, hipStream_t st, const int32_t* tofs) {
  const bool F = P.g.fourier;
  const int n = (int)P.n;
  const int N = (int)P.shape.N, M = (int)P.shape.M;
  const Geo& g = P.g;
  const EntDev en{P.ent_k, P.goff, M};
  const double inv_sqrt_n = 1.0 / std::sqrt((double)N);
  if (P.fused) {
    ProfScope ps(FCMP_PHASE_CORR, st);
    const int ntaps = t - 1;
    RCParams q = rcorr_geometry(P);
    q.lam = P.lam; q.x = P.x; q.ntaps = ntaps;
    q.ord = P.ord;
    q.bstart = P.bst;
    q.inst_lam = P.sK; q.inst_x = P.sK; q.inst_ord = 2 * P.sK; q.inst_bstart = 2 * P.sB;
    q.ord_half = P.sK; q.bstart_half = P.sB;
    q.Kv = P.Kv; q.tofs = tofs;
    q.ent_k = P.ent_k; q.goff = P.cst; q.y = P.y_ent;
    q.inst_ent = P.sM; q.inst_goff = P.sCs; q.inst_y = P.sM;
    q.rscale = inv_sqrt_n;
    const TwDev tr = tw_for(P, P.wk), tc = tw_for(P, P.pk);
    q.twr_lo = tr.lo; q.twr_hi = tr.hi; q.twr_st = tr.st;
    q.twc_lo = tc.lo; q.twc_hi = tc.hi; q.twc_st = tc.st;
    q.out = P.tmp; q.inst_out = P.sN;
    q.status = P.status;
    q.cmask = P.cmask; q.cbase = P.cbase; q.inst_cmask = P.sC;
    if (P.rreg) HIP_TRY(launch_rcorr_reg(P.pk, F, q, n, st));
    else HIP_TRY(launch_rcorr(P.pk, F, q, (1 << g.n1) / q.B, n,
                              P.rthreads > 0 ? P.rthreads : rcorr_threads(q), st));
    XDst d;
    d.partial = P.partial; d.excl = P.excl;
    d.scale = inv_sqrt_n;
    XSrc src{IN_SPARSE, P.pk, nullptr};
    src.pass2_only = true;
    HIP_TRY(run_transform(P.pk, +1, g, tw_for(P, P.pk), en, src, d, P.tmp, P.status, st, n,
                          P.sN, P.sM, P.sP, P.sE, P.sG));
    *npart = transform_partials(P.pk, g, false);
    return FCMP_OK;
  }
  if (tofs) return set_error(FCMP_E_INVALID, "slot iterations need the fused residual");
  const double thr = P.resid_ratio * (double)N * (double)g.logN;
  int64_t m_lo = P.hM[0], m_hi = P.hM[0];
  for (int32_t m : P.hM) { m_lo = std::min<int64_t>(m_lo, m); m_hi = std::max<int64_t>(m_hi, m); }
  const double work_lo = (double)m_lo * (double)(t - 1);
  const double work_hi = (double)m_hi * (double)(t - 1);
  if (work_hi > thr) {
    ProfScope ps(FCMP_PHASE_RESID, st);
    XSrc src{IN_TAPS, P.wk, nullptr};
    src.taps_lam = P.lam; src.taps_x = P.x; src.ntaps = t - 1;
    src.inst_lam = P.sK; src.inst_x = P.sK;
    XDst d;
    d.scale = inv_sqrt_n;
    d.resid = true;
    d.ent2_k = P.ent2_k; d.goff2 = P.goff2; d.pos1 = P.pos1; d.nent2 = M;
    d.yres = P.y_ent; d.yres_kind = P.wk; d.rout = P.r; d.r_kind = P.pk;
    d.inst_ent2 = P.sM; d.inst_goff2 = P.g.same_out ? P.sG : P.sG2;
    d.inst_yres = P.sM; d.inst_rout = P.sM;
    if (work_lo <= thr) { d.rsel_M = P.Mv; d.rsel_ntaps = t - 1; d.rsel_thr = thr; }
    HIP_TRY(run_transform(P.wk, -1, g, tw_for(P, P.wk), en, src, d, P.tmp, P.status, st, n,
                          P.sN, P.sM, 0, 0, P.sG));
  }
  if (work_lo <= thr) {
    ProfScope ps(FCMP_PHASE_RESID, st);
    RParams rp{};
    rp.N = N; rp.logN = g.logN; rp.twS = g.twS; rp.fourier = F; rp.M = M;
    rp.ent_k = P.ent_k; rp.y = P.y_ent; rp.r = P.r; rp.r_kind = P.pk;
    rp.lam = P.lam; rp.x = P.x; rp.ntaps = t - 1;
    rp.tw_lo = P.tw64; rp.tw_hi = P.tw64 + ((size_t)1 << g.twS);
    rp.status = P.status;
    rp.inst_ent = P.sM; rp.inst_y = P.sM; rp.inst_r = P.sM; rp.inst_lam = P.sK;
    rp.inst_x = P.sK;
    if (work_hi > thr) { rp.Mv = P.Mv; rp.thr = thr; }
    HIP_TRY(launch_residual(rp, n, st));
  }
  ProfScope ps(FCMP_PHASE_CORR, st);
  XDst d;
  d.partial = P.partial; d.excl = P.excl;
  d.scale = inv_sqrt_n;
  HIP_TRY(run_transform(P.pk, +1, g, tw_for(P, P.pk), en, XSrc{IN_SPARSE, P.pk, P.r}, d, P.tmp,
                        P.status, st, n, P.sN, P.sM, P.sP, P.sE, P.sG));
  *npart = transform_partials(P.pk, g, false);
  return FCMP_OK;
}

// Least-squares launch parameters of the plan (t and npart set by the caller).
static LParams ls_params(const fcmp_plan& P) {
  const bool F = P.shape.matrix_class == FCMP_FOURIER;
  const int N = (int)P.shape.N, K = (int)P.shape.K;
  const Geo& g = P.g;
  LParams lp{};
  lp.N = N; lp.fourier = F;
  lp.partial = P.partial; lp.npart = transform_partials(P.wk, g, true);
  lp.c64 = P.c64; lp.h0 = P.h0; lp.W = P.W; lp.z = P.z; lp.x = P.x;
  lp.lam = P.lam; lp.excl = P.excl; lp.status = P.status;
  lp.inst_part = P.sP; lp.inst_c = P.sN; lp.inst_h0 = P.sN; lp.inst_W = P.sW;
  lp.inst_z = P.sK; lp.inst_x = P.sK; lp.inst_lam = P.sK; lp.inst_excl = P.sE;
  lp.wbuf = P.wbuf; lp.inst_wbuf = P.sK;
  lp.vpart = P.vpart; lp.inst_vpart = ls_split_groups((int)K) * P.sK; lp.vpart_stride = P.sK;
  lp.Kv = P.Kv;
  if (P.fused) {
    lp.ord = P.ord; lp.bstart = P.bst;
    lp.inst_ord = 2 * P.sK; lp.ord_half = P.sK;
    lp.inst_bstart = 2 * P.sB; lp.bstart_half = P.sB;
    lp.nbuck = 1 << g.n2;
    lp.bshift = F ? 0 : g.n1;
  }
  return lp;
}

int plan_enqueue(fcmp_plan& P, const fcmp_options& opt, hipStream_t st) {
  int rc = plan_enqueue_prefix(P, opt, st);
  if (rc) return rc;
  const bool F = P.shape.matrix_class == FCMP_FOURIER;
  const int n = (int)P.n;
  const int N = (int)P.shape.N, K = (int)P.shape.K;
  LParams lp = ls_params(P);
  lp.t = 1;
  {
    ProfScope ps(FCMP_PHASE_LS, st);
    HIP_TRY(launch_ls_update(lp, n, st));
  }
  const int switch_t = opt.switch_t > 0
                           ? opt.switch_t
                           : default_switch_t(P.shape.matrix_class, N, P.opt.corr_precision);
  for (int t = 2; t <= K; ++t) {
    const bool fast = opt.corr_method == FCMP_CORR_FAST ||
                      (opt.corr_method == FCMP_CORR_ADAPTIVE && t <= switch_t);
    int npart = 0;
    if (fast) rc = plan_fast_corr(P, t, &npart, st);
    else rc = plan_conv_corr(P, t, &npart, st);
    if (rc) return rc;
    lp.t = t;
    lp.npart = npart;
    ProfScope ps(FCMP_PHASE_LS, st);
    HIP_TRY(launch_ls_update(lp, n, st));
  }
  {
    ProfScope ps(FCMP_PHASE_OTHER, st);
    HIP_TRY(launch_finalize_ptr(F, P.status, P.lam, P.x, K, P.sK, P.sK,
                                (int32_t* const*)(P.dptrs + P.n), (void* const*)(P.dptrs + 2 * P.n),
                                n, st, P.Kv));
  }
  return FCMP_OK;
}

int plan_solve(fcmp_plan& P, const fcmp_options* o, const void* const* y, int32_t* const* sup,
               void* const* xo, fcmp_stats* stats, hipStream_t st, bool timed) {
  fcmp_options opt = P.opt;
  if (o) {
    int rc = validate_options(&P.shape, o);
    if (rc) return rc;
    if (o->algorithm != P.opt.algorithm || o->corr_precision != P.opt.corr_precision)
      return set_error(FCMP_E_INVALID, "options differ from the plan's algorithm/precision");
    opt = *o;
  }
  if (!y || !sup || !xo) return set_error(FCMP_E_INVALID, "NULL pointer array");
  int rc = upload_ptrs(P, y, sup, xo, st);
  if (rc) return rc;
  const int n = (int)P.n;
  // per-solve phase times: events around every phase of this solve
  SolveTimes stm;
  const bool phase_times = stats && timed && (opt.flags & FCMP_FLAG_PHASE_TIMES);
  SolveTimesScope stm_scope(phase_times ? &stm : nullptr);
  double pms[FCMP_NPHASE] = {0.0};
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (stats && timed) {
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    HIP_TRY(hipEventRecord(e0, st));
  }
  auto drop_events = [&] {
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    e0 = e1 = nullptr;
  };
  if (P.opt.algorithm != FCMP_OMP) {
    rc = plan_enqueue_prefix(P, opt, st);
    if (!rc) rc = plan_solve_set(P, opt, (int32_t* const*)sup, xo, stats, st);
    if (e1 && (!rc || rc == FCMP_E_NUMERIC)) {
      // the loops synchronise the stream themselves; the solve's device time
      float ms = 0.f;
      hipError_t e = hipEventRecord(e1, st);
      if (e == hipSuccess) e = hipEventSynchronize(e1);
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
      if (e == hipSuccess)
        for (int64_t b = 0; b < P.n; ++b) stats[b].ms_total = ms;
    }
    drop_events();
    if (phase_times && (!rc || rc == FCMP_E_NUMERIC)) {
      const int prc = solve_times_read(stm, pms);
      if (prc) return prc;
      for (int64_t b = 0; b < P.n; ++b) stats_phases(stats[b], pms);
    }
    return rc;
  }
  if ((rc = plan_enqueue(P, opt, st))) {
    drop_events();
    return rc;
  }
  if (stats) {
    float ms = 0.f;
    hipError_t e = timed ? hipEventRecord(e1, st) : hipSuccess;
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e == hipSuccess && timed) e = hipEventElapsedTime(&ms, e0, e1);
    drop_events();
    if (e != hipSuccess)
      return set_error(FCMP_E_DEVICE, std::string("plan solve: ") + hipGetErrorString(e));
    std::vector<Status> hs((size_t)n);
    HIP_TRY(hipMemcpy(hs.data(), P.status, n * sizeof(Status), hipMemcpyDeviceToHost));
    if (phase_times) {
      const int prc = solve_times_read(stm, pms);
      if (prc) return prc;
    }
    return plan_stats(n, hs.data(), ms, stats, phase_times ? pms : nullptr);
  }
  return FCMP_OK;
}

// ---------------------------------------------------------------- slot plans

int slot_tile() { return plan_tile(int64_t(1) << 30); }

bool plan_slots_ok(const fcmp_problem& prob, const fcmp_options& opt) {
  if (opt.algorithm != FCMP_OMP || opt.corr_method != FCMP_CORR_CONVENTIONAL ||
      opt.res_tol > 0.0 || (opt.flags & FCMP_FLAG_PHASE_TIMES))
    return false;
  fcmp_plan P;
  std::vector<int32_t> om((size_t)prob.M);
  for (int64_t i = 0; i < prob.M; ++i) om[(size_t)i] = (int32_t)i;
  fcmp_problem q = prob;
  q.omega = om.data();
  if (plan_init(P, 1, &q, &opt, slot_tile()) != FCMP_OK) return false;
  return P.fused;
}

int plan_init_slots(fcmp_plan& P, int64_t n, const fcmp_problem& cap, const fcmp_options& opt) {
  std::vector<int32_t> om((size_t)cap.M);
  for (int64_t i = 0; i < cap.M; ++i) om[(size_t)i] = (int32_t)i;
  fcmp_problem q = cap;
  q.omega = om.data();
  int rc = plan_init(P, 1, &q, &opt, slot_tile());
  if (rc) return rc;
  if (!P.fused) return set_error(FCMP_E_INVALID, "slot plans need the fused residual");
  if (n < 1) return set_error(FCMP_E_INVALID, "n must be >= 1");
  // n slots of the capacity shape, each with its own M and K
  P.n = n;
  P.hM.assign((size_t)n, (int32_t)cap.M);
  P.hK.assign((size_t)n, (int32_t)cap.K);
  P.uniform = false;
  plan_layout(P, nullptr);
  return FCMP_OK;
}

template <class T>
static T* at(T* p, int64_t k) { return p ? p + k : nullptr; }
static void* at_bytes(void* p, int64_t b) { return p ? (void*)((char*)p + b) : nullptr; }

fcmp_plan plan_view(const fcmp_plan& P, int64_t s, int32_t M, int32_t K) {
  fcmp_plan V;
  V.n = 1;
  V.shape = P.shape;
  V.uniform = false;
  V.hM.assign(1, M);
  V.hK.assign(1, K);
  V.opt = P.opt;
  V.g = P.g;
  V.wk = P.wk; V.pk = P.pk;
  V.sM = P.sM; V.sN = P.sN; V.sK = P.sK; V.sW = P.sW; V.sG = P.sG; V.sG2 = P.sG2;
  V.sP = P.sP; V.sE = P.sE; V.sB = P.sB; V.sC = P.sC; V.sCs = P.sCs;
  V.resid_ratio = P.resid_ratio;
  V.fused = P.fused; V.rreg = P.rreg;
  V.npart = P.npart;
  V.tw64 = P.tw64; V.tw32 = P.tw32;
  const int64_t wb = vbytes(P.wk), pb = vbytes(P.pk);
  V.ent_k = at(P.ent_k, s * P.sM);
  V.perm = at(P.perm, s * P.sM);
  V.goff = at(P.goff, s * P.sG);
  if (!P.g.same_out) {
    V.ent2_k = at(P.ent2_k, s * P.sM);
    V.goff2 = at(P.goff2, s * P.sG2);
    V.pos1 = at(P.pos1, s * P.sM);
  } else {
    V.ent2_k = V.ent_k;
    V.goff2 = V.goff;
    V.pos1 = nullptr;
  }
  V.cmask = at(P.cmask, s * P.sC);
  V.cbase = at(P.cbase, s * P.sC);
  V.cst = at(P.cst, s * P.sCs);
  V.Mv = at(P.Mv, s);
  V.Kv = at(P.Kv, s);
  V.c64 = at_bytes(P.c64, s * P.sN * wb);
  V.cp = P.cp == P.c64 ? V.c64 : at_bytes(P.cp, s * P.sN * pb);
  V.ci16 = at(P.ci16, s * P.sN);
  V.y_ent = at_bytes(P.y_ent, s * P.sM * wb);
  V.r = at_bytes(P.r, s * P.sM * pb);
  V.h0 = at_bytes(P.h0, s * P.sN * wb);
  V.tmp = at_bytes(P.tmp, s * P.sN * wb);
  V.partial = at(P.partial, s * P.sP);
  V.lam = at(P.lam, s * P.sK);
  V.ord = at(P.ord, s * 2 * P.sK);
  V.bst = at(P.bst, s * 2 * P.sB);
  V.excl = at(P.excl, s * P.sE);
  V.x = at_bytes(P.x, s * P.sK * wb);
  V.z = at_bytes(P.z, s * P.sK * wb);
  V.W = at_bytes(P.W, s * P.sW * wb);
  V.wbuf = at_bytes(P.wbuf, s * P.sK * wb);
  V.vpart = at_bytes(P.vpart, s * ls_split_groups((int)P.shape.K) * P.sK * wb);
  V.status = at(P.status, s);
  V.dptrs = at(P.dptrs, 3 * s);
  V.total = 0;
  return V;
}

int plan_upload_twiddles(fcmp_plan& P, const HostTables& t, hipStream_t st, const StageFn& stage) {
  if (t.tw64.size() != (size_t)tw_count(P.g)) return set_error(FCMP_E_INVALID, "twiddle geometry");
  const size_t b64 = t.tw64.size() * sizeof(double2), b32 = t.tw32.size() * sizeof(float2);
  HIP_TRY(hipMemcpyAsync(P.tw64, stage ? stage(t.tw64.data(), b64) : t.tw64.data(), b64,
                         hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(P.tw32, stage ? stage(t.tw32.data(), b32) : t.tw32.data(), b32,
                         hipMemcpyHostToDevice, st));
  return FCMP_OK;
}

int plan_upload_tables(fcmp_plan& V, const HostTables& t, hipStream_t st, const StageFn& stage) {
  const size_t M = (size_t)V.hM[0];
  if (t.ent_k.size() < M || t.goff.size() > (size_t)V.sG ||
      (V.rreg && t.cmask.size() > (size_t)V.sC) || (V.cst && t.cst.size() > (size_t)V.sCs) ||
      (!V.g.same_out && t.goff2.size() > (size_t)V.sG2))
    return set_error(FCMP_E_INVALID, "tables do not match the slot");
  auto up = [&](void* dst, const void* src, size_t bytes) {
    if (!bytes) return hipSuccess;
    const void* from = stage ? stage(src, bytes) : src;
    return hipMemcpyAsync(dst, from, bytes, hipMemcpyHostToDevice, st);
  };
  HIP_TRY(up(V.ent_k, t.ent_k.data(), M * 4));
  HIP_TRY(up(V.perm, t.perm.data(), M * 4));
  HIP_TRY(up(V.goff, t.goff.data(), t.goff.size() * 4));
  if (!V.g.same_out) {
    HIP_TRY(up(V.ent2_k, t.ent2_k.data(), M * 4));
    HIP_TRY(up(V.goff2, t.goff2.data(), t.goff2.size() * 4));
    HIP_TRY(up(V.pos1, t.pos1.data(), M * 4));
  }
  if (V.rreg) {
    HIP_TRY(up(V.cmask, t.cmask.data(), t.cmask.size() * 4));
    HIP_TRY(up(V.cbase, t.cbase.data(), t.cbase.size() * 4));
  }
  if (V.cst) HIP_TRY(up(V.cst, t.cst.data(), t.cst.size() * 4));
  return plan_kernel_vector(V, st);
}

int plan_copy_tables(fcmp_plan& V, const fcmp_plan& from, hipStream_t st) {
  auto cp = [&](void* dst, const void* src, size_t bytes) {
    return (dst && src && dst != src)
               ? hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, st)
               : hipSuccess;
  };
  const size_t M = (size_t)V.hM[0];
  const size_t wb = vbytes(V.wk), pb = vbytes(V.pk);
  HIP_TRY(cp(V.ent_k, from.ent_k, M * 4));
  HIP_TRY(cp(V.perm, from.perm, M * 4));
  HIP_TRY(cp(V.goff, from.goff, (size_t)V.sG * 4));
  if (!V.g.same_out) {
    HIP_TRY(cp(V.ent2_k, from.ent2_k, M * 4));
    HIP_TRY(cp(V.goff2, from.goff2, (size_t)V.sG2 * 4));
    HIP_TRY(cp(V.pos1, from.pos1, M * 4));
  }
  HIP_TRY(cp(V.cmask, from.cmask, (size_t)V.sC * 4));
  HIP_TRY(cp(V.cbase, from.cbase, (size_t)V.sC * 4));
  HIP_TRY(cp(V.cst, from.cst, (size_t)V.sCs * 4));
  HIP_TRY(cp(V.c64, from.c64, (size_t)V.shape.N * wb));
  if (V.cp != V.c64) HIP_TRY(cp(V.cp, from.cp, (size_t)V.shape.N * pb));
  HIP_TRY(cp(V.ci16, from.ci16, (size_t)V.shape.N * 2));
  return FCMP_OK;
}

int plan_join(fcmp_plan& V, const fcmp_options& opt, hipStream_t st) {
  int rc = plan_enqueue_prefix(V, opt, st);
  if (rc) return rc;
  LParams lp = ls_params(V);
  lp.t = 1;
  HIP_TRY(launch_ls_update(lp, 1, st));
  return FCMP_OK;
}

int plan_step_slots(fcmp_plan& P, int step, const int32_t* tofs, int t_lo, int t_hi,
                    hipStream_t st) {
  if (!tofs || t_lo < 2 || t_hi < t_lo || t_hi > P.shape.K)
    return set_error(FCMP_E_INVALID, "slot step out of range");
  int npart = 0;
  int rc = conv_corr(P, step, &npart, st, tofs);
  if (rc) return rc;
  LParams lp = ls_params(P);
  lp.t = step;
  lp.tofs = tofs;
  lp.npart = npart;
  HIP_TRY(launch_ls_update_slots(lp, (int)P.n, t_lo, t_hi, st));
  return FCMP_OK;
}

int plan_finish(fcmp_plan& V, hipStream_t st) {
  HIP_TRY(launch_finalize_ptr(V.g.fourier, V.status, V.lam, V.x, (int)V.shape.K, V.sK, V.sK,
                              (int32_t* const*)(V.dptrs + 1), (void* const*)(V.dptrs + 2), 1, st,
                              V.Kv));
  HIP_TRY(launch_status_done(V.status, 1, st));
  return FCMP_OK;
}

}  // namespace fcmp
