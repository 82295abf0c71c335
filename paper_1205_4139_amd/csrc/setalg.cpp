// Set-based pursuits on the GPU, one instance at a time: subspace pursuit and
// CoSaMP, the matching pursuit algorithms the paper cites beside OMP (Sec. I)
// and applies its method to (Sec. IV, CoSaMP).  The paper does not define
// them; the loops follow this library's reading:
//
// SP:     T = top-K |h_0|, x = LS(T).  Repeat: h = Phi^H r; T~ = T + the K
//         largest |h| outside T; x~ = LS(T~); T' = the K largest |x~|;
//         x' = LS(T'); stop when T' = T (keep it) or ||r'|| >= ||r|| (keep T).
// CoSaMP: S = {}, a = 0.  Repeat: u = Phi^H (y - Phi_S a); T = the 2K
//         largest |u| plus S; b = LS(T); S', a' = the K largest |b|; stop when
//         S' = S or ||y - Phi_S' a'|| <= 1e-12 ||y||.  Finally x = LS(S).
//
// The correlation h = Phi^H r uses either method: conventional (FP64 forward
// transform of the current coefficients for the residual, then the transform
// in the correlation precision) or fast (h_0 - sum over the support of
// x P_lambda c, i.e. eq. (kernelsum) with the K-sized support as taps).
// Selection ties go to the lowest index; every support is kept ascending.
#include <algorithm>
#include <cmath>
#include <limits>
#include <vector>

#include "plan.h"

namespace fcmp {

#define HIP_TRY(expr)                                                              \
  do {                                                                             \
    hipError_t _e = (expr);                                                        \
    if (_e != hipSuccess)                                                          \
      return set_error(FCMP_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(_e)); \
  } while (0)

namespace {

struct Inst {
  const int32_t* ent_k; const int32_t* goff;
  const int32_t* ent2_k; const int32_t* goff2; const int32_t* pos1;
  const void* c64; const void* cp; const void* y_ent; void* r; const void* h0; void* tmp;
  Status* status;
};

Inst inst_view(const fcmp_plan& P, int64_t b) {
  const size_t wb = vbytes(P.wk), pb = vbytes(P.pk);
  Inst v;
  v.ent_k = P.ent_k + b * P.sM;
  v.goff = P.goff + b * P.sG;
  v.ent2_k = P.ent2_k + b * P.sM;
  v.goff2 = P.goff2 ? P.goff2 + b * (P.g.same_out ? P.sG : P.sG2) : nullptr;
  v.pos1 = P.pos1 ? P.pos1 + b * P.sM : nullptr;
  v.c64 = (const char*)P.c64 + b * P.sN * wb;
  v.cp = (const char*)P.cp + b * P.sN * (P.cp == P.c64 ? wb : pb);
  v.y_ent = (const char*)P.y_ent + b * P.sM * wb;
  v.r = (char*)P.r + b * P.sM * pb;
  v.h0 = (const char*)P.h0 + b * P.sN * wb;
  v.tmp = (char*)P.tmp + b * P.sN * wb;
  v.status = P.status + b;
  return v;
}

TwDev tw_of(const fcmp_plan& P, int vk) {
  const size_t nlo = (size_t)1 << P.g.twS;
  const size_t nst = nlo + ((size_t)P.g.N >> P.g.twS);
  if (vk == V_C64) return TwDev{P.tw32, P.tw32 + nlo, P.tw32 + nst};
  return TwDev{P.tw64, P.tw64 + nlo, P.tw64 + nst};
}

// h = Phi^H (y - Phi_S a) into P.hbuf; returns the value kind of h.
int correlate_set(const fcmp_plan& P, const Inst& I, bool fast, const int32_t* S, const void* a,
                  int s, hipStream_t st, int* hkind) {
  const int N = (int)P.shape.N, M = (int)P.shape.M;
  const double inv_sqrt_n = 1.0 / std::sqrt((double)N);
  if (fast) {
    ProfScope ps(FCMP_PHASE_FAST, st);
    FParams fp{};
    fp.N = N; fp.logN = P.g.logN; fp.fourier = P.g.fourier; fp.c_kind = P.pk;
    fp.h0 = I.h0; fp.c = I.cp; fp.lam = S; fp.x = a; fp.ntaps = s;
    fp.h = P.hbuf; fp.partial = nullptr; fp.excl = nullptr; fp.status = nullptr;
    int groups = 0;
    if (P.cur_flags & FCMP_FLAG_CONJ_PAIR) HIP_TRY(launch_fastpair(fp, 1, &groups, st));
    else HIP_TRY(launch_fastcorr(fp, 1, &groups, st));
    *hkind = P.wk;
    return FCMP_OK;
  }
  const EntDev en{I.ent_k, I.goff, M};
  {
    ProfScope ps(FCMP_PHASE_RESID, st);
    XSrc src{IN_TAPS, P.wk, nullptr};
    src.taps_lam = S; src.taps_x = a; src.ntaps = s;
    XDst d;
    d.scale = inv_sqrt_n;
    d.resid = true;
    d.ent2_k = I.ent2_k; d.goff2 = I.goff2; d.pos1 = I.pos1; d.nent2 = M;
    d.yres = I.y_ent; d.yres_kind = P.wk; d.rout = I.r; d.r_kind = P.pk;
    HIP_TRY(run_transform(P.wk, -1, P.g, tw_of(P, P.wk), en, src, d, I.tmp, nullptr, st));
  }
  ProfScope ps(FCMP_PHASE_CORR, st);
  XDst d;
  d.out = P.hbuf; d.kind = P.pk;
  d.scale = inv_sqrt_n;
  HIP_TRY(run_transform(P.pk, +1, P.g, tw_of(P, P.pk), en, XSrc{IN_SPARSE, P.pk, I.r}, d, I.tmp,
                        nullptr, st));
  *hkind = P.pk;
  return FCMP_OK;
}

int dense_ls(const fcmp_plan& P, const Inst& I, const int32_t* T, int s, void* x, hipStream_t st) {
  ProfScope ps(FCMP_PHASE_LS, st);
  HIP_TRY(launch_dense_ls(P.g.fourier, I.c64, I.h0, T, s, (int)P.shape.N, P.dws, x, P.bad, st));
  return FCMP_OK;
}

// ||y - Phi_S a||^2 = ||y||^2 - 2 Re(h0(S)^H a) + a^H G_S a
int resid_norm2(const fcmp_plan& P, const Inst& I, const int32_t* S, const void* a, int s,
                double ynorm2, hipStream_t st, double* out) {
  HIP_TRY(launch_set_quad(P.g.fourier, I.c64, I.h0, S, a, s, (int)P.shape.N, P.small, st));
  const int g = set_quad_groups(s);
  std::vector<double> part(2 * g);
  HIP_TRY(hipMemcpyAsync(part.data(), P.small, part.size() * 8, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  double lin = 0.0, quad = 0.0;
  for (int i = 0; i < g; ++i) { lin += part[2 * i]; quad += part[2 * i + 1]; }
  *out = ynorm2 - 2.0 * lin + quad;
  return FCMP_OK;
}

int to_host(std::vector<int32_t>& h, const int32_t* d, int s, hipStream_t st) {
  h.resize(s);
  HIP_TRY(hipMemcpyAsync(h.data(), d, (size_t)s * 4, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  return FCMP_OK;
}

int to_dev(int32_t* d, const std::vector<int32_t>& h, hipStream_t st) {
  HIP_TRY(hipMemcpyAsync(d, h.data(), h.size() * 4, hipMemcpyHostToDevice, st));
  HIP_TRY(hipStreamSynchronize(st));
  return FCMP_OK;
}

std::vector<int32_t> merge_sorted(const std::vector<int32_t>& a, const std::vector<int32_t>& b) {
  std::vector<int32_t> out;
  out.reserve(a.size() + b.size());
  std::set_union(a.begin(), a.end(), b.begin(), b.end(), std::back_inserter(out));
  return out;
}

}  // namespace

int plan_solve_set(fcmp_plan& P, const fcmp_options& opt, int32_t* const* sup, void* const* xo,
                   fcmp_stats* stats, hipStream_t st) {
  const bool F = P.g.fourier;
  const bool fast = opt.corr_method != FCMP_CORR_CONVENTIONAL;
  const int K = (int)P.shape.K;
  const int N = (int)P.shape.N;
  const int max_iter = opt.max_iter > 0 ? opt.max_iter : 50;
  const double rt2 = opt.res_tol * opt.res_tol;   // stop once ||r||^2 <= rt2 ||y||^2
  const size_t wb = vbytes(P.wk);
  // top-K selections, timed as their own phase
  auto topk = [&](const void* v, int kind, int n, const uint32_t* ex, int k, int32_t* out) {
    ProfScope ps(FCMP_PHASE_SELECT, st);
    return launch_topk(v, kind, n, ex, k, P.tkws, out, st);
  };
  int worst = FCMP_OK;
  for (int64_t b = 0; b < P.n; ++b) {
    const Inst I = inst_view(P, b);
    Status hs;
    HIP_TRY(hipMemcpyAsync(&hs, I.status, sizeof(Status), hipMemcpyDeviceToHost, st));
    HIP_TRY(launch_fill_u32((uint32_t*)P.bad, 0u, 1, st));
    HIP_TRY(hipStreamSynchronize(st));
    const double ynorm2 = hs.ynorm2;
    std::vector<int32_t> T, Tn, extra;
    int rc;
    int iters = 0;
    double rn2 = ynorm2;
    int32_t* dT = P.Ta;        // current support
    void* dx = P.xa;           // its coefficients
    // buffers: current / next support and coefficients alternate between
    // (Ta, xa) and (Tc, xb); Tb holds merged supports, Td selected positions,
    // xc the fit on the merged support
    if (opt.algorithm == FCMP_SP) {
      HIP_TRY(topk(I.h0, P.wk, N, nullptr, K, dT));
      if ((rc = dense_ls(P, I, dT, K, dx, st))) return rc;
      if ((rc = resid_norm2(P, I, dT, dx, K, ynorm2, st, &rn2))) return rc;
      if ((rc = to_host(T, dT, K, st))) return rc;
      while (iters < max_iter && !(rt2 > 0.0 && rn2 <= rt2 * ynorm2)) {
        ++iters;
        int hk;
        if ((rc = correlate_set(P, I, fast, dT, dx, K, st, &hk))) return rc;
        HIP_TRY(launch_set_bits(P.excl, P.sE, dT, K, st));
        HIP_TRY(topk(P.hbuf, hk, N, P.excl, K, P.Tb));
        if ((rc = to_host(extra, P.Tb, K, st))) return rc;
        const std::vector<int32_t> Tt = merge_sorted(T, extra);
        const int st_n = (int)Tt.size();
        if ((rc = to_dev(P.Tb, Tt, st))) return rc;
        if ((rc = dense_ls(P, I, P.Tb, st_n, P.xc, st))) return rc;
        HIP_TRY(topk(P.xc, P.wk, st_n, nullptr, K, P.Td));   // positions in Tt
        std::vector<int32_t> keep;
        if ((rc = to_host(keep, P.Td, K, st))) return rc;
        Tn.resize(K);
        for (int i = 0; i < K; ++i) Tn[i] = Tt[keep[i]];
        int32_t* dTn = dT == P.Ta ? P.Tc : P.Ta;
        void* dxn = dx == P.xa ? P.xb : P.xa;
        if ((rc = to_dev(dTn, Tn, st))) return rc;
        if ((rc = dense_ls(P, I, dTn, K, dxn, st))) return rc;
        double rn2n;
        if ((rc = resid_norm2(P, I, dTn, dxn, K, ynorm2, st, &rn2n))) return rc;
        if (Tn == T) {
          dT = dTn; dx = dxn; rn2 = rn2n;
          break;
        }
        if (rn2n >= rn2) break;
        T = Tn; dT = dTn; dx = dxn; rn2 = rn2n;
      }
    } else {
      // CoSaMP
      std::vector<int32_t> S;   // empty
      int32_t* dS = P.Ta;
      void* da = P.xa;
      while (iters < max_iter) {
        ++iters;
        const void* u = I.h0;
        int uk = P.wk;
        if (!S.empty()) {
          if ((rc = correlate_set(P, I, fast, dS, da, (int)S.size(), st, &uk))) return rc;
          u = P.hbuf;
        }
        HIP_TRY(topk(u, uk, N, nullptr, 2 * K, P.Tb));
        if ((rc = to_host(extra, P.Tb, 2 * K, st))) return rc;
        const std::vector<int32_t> Tt = merge_sorted(extra, S);
        const int tn = (int)Tt.size();
        if ((rc = to_dev(P.Tb, Tt, st))) return rc;
        if ((rc = dense_ls(P, I, P.Tb, tn, P.xc, st))) return rc;
        HIP_TRY(topk(P.xc, P.wk, tn, nullptr, K, P.Td));
        std::vector<int32_t> keep;
        if ((rc = to_host(keep, P.Td, K, st))) return rc;
        std::vector<int32_t> Sn(K);
        for (int i = 0; i < K; ++i) Sn[i] = Tt[keep[i]];
        int32_t* dSn = dS == P.Ta ? P.Tc : P.Ta;
        void* dan = da == P.xa ? P.xb : P.xa;
        // a' = b at the kept positions (no refit inside the loop)
        HIP_TRY(launch_gather_wide(P.wk, P.xc, P.Td, dan, K, 0, 0, 0, 1, st));
        if ((rc = to_dev(dSn, Sn, st))) return rc;
        const bool same = Sn == S;
        S = Sn; dS = dSn; da = dan;
        double vn2;
        if ((rc = resid_norm2(P, I, dS, da, K, ynorm2, st, &vn2))) return rc;
        if (same || vn2 <= 1e-24 * ynorm2 || (rt2 > 0.0 && vn2 <= rt2 * ynorm2)) break;
      }
      // final refit on the support
      void* dxf = P.xc;
      if ((rc = dense_ls(P, I, dS, K, dxf, st))) return rc;
      if ((rc = resid_norm2(P, I, dS, dxf, K, ynorm2, st, &rn2))) return rc;
      dT = dS;
      dx = dxf;
    }
    // copy out (support ascending, K entries)
    HIP_TRY(hipMemcpyAsync(sup[b], dT, (size_t)K * 4, hipMemcpyDeviceToDevice, st));
    HIP_TRY(hipMemcpyAsync(xo[b], dx, (size_t)K * wb, hipMemcpyDeviceToDevice, st));
    int bad = 0;
    HIP_TRY(hipMemcpyAsync(&bad, P.bad, sizeof(int), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (bad) worst = FCMP_E_NUMERIC;
    if (stats) {
      stats[b] = fcmp_stats{};
      stats[b].iterations = iters;
      stats[b].status_detail = bad ? FCMP_E_NUMERIC : FCMP_OK;
      stats[b].min_gap = std::numeric_limits<double>::quiet_NaN();
      stats[b].res_norm = rn2 > 0 ? std::sqrt(rn2) : 0.0;
      stats[b].ms_total = 0.0;
    }
    (void)F;
  }
  if (worst) return set_error(worst, "Cholesky breakdown in at least one instance");
  return FCMP_OK;
}

}  // namespace fcmp
