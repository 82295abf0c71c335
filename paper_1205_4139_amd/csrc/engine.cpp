// Host engine: geometry, tables, transform sequencing and validation.
#include "engine.h"

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>

namespace fcmp {

static thread_local std::string g_last_error;

int set_error(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}
const char* last_error() { return g_last_error.c_str(); }

static int ilog2(int64_t n) {
  int l = 0;
  while ((int64_t(1) << l) < n) ++l;
  return l;
}

bool single_ok(int vk, int N) { return (size_t)N * vbytes(vk) <= 131072; }

namespace {
std::mutex g_tune_mu;
std::map<std::tuple<int, int64_t, int>, int> g_switch;
}  // namespace

int model_switch_t(int matrix_class, int64_t N) {
  const int logN = ilog2(N);
  return matrix_class == FCMP_FOURIER ? 2 + (5 * logN) / 6 : 1 + logN;
}

void set_tuned_switch(int matrix_class, int64_t N, int precision, int switch_t) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_switch[std::make_tuple(matrix_class, N, precision)] = switch_t;
}

bool tuned_switch(int matrix_class, int64_t N, int precision, int* switch_t) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  auto it = g_switch.find(std::make_tuple(matrix_class, N, precision));
  if (it == g_switch.end()) return false;
  *switch_t = it->second;
  return true;
}

int default_switch_t(int matrix_class, int64_t N, int precision) {
  int t = 0;
  if (tuned_switch(matrix_class, N, precision, &t)) return t;
  return model_switch_t(matrix_class, N);
}

int plan_tile(int64_t n) {
  if (tune().tile_fixed) return tune().tile;
  if (n <= 1) return 256;
  if (n <= 8) return 512;
  if (n <= 32) return 1024;
  return tune().tile;
}

Geo make_geo(bool fourier, int N, int tile_req) {
  Geo g;
  g.N = N;
  g.fourier = fourier;
  g.logN = ilog2(N);
  g.n2 = g.logN / 2;
  // N = 2^18: columns of 256 rows, so the residual-fused first pass runs
  // register-resident, and rows of 1024 for the second pass
  if (g.logN == 18) g.n2 = 8;
  g.n1 = g.logN - g.n2;
  g.twS = g.n2;
  const int tile = tile_req > 0 ? tile_req : tune().tile;
  g.B1 = std::min(1 << g.n1, std::max(1, tile >> g.n2));
  g.B2 = std::min(1 << g.n2, std::max(1, tile >> g.n1));
  g.grouped = !single_ok(fourier ? V_C128 : V_F64, N);
  g.ngroups = g.grouped ? (1 << g.n1) / g.B1 : 1;
  g.ngroups2 = g.grouped ? (1 << g.n2) / g.B2 : 1;
  g.same_out = !g.grouped || (fourier && g.n1 == g.n2 && g.B1 == g.B2);
  if (fourier) {
    // longest LDS transform of this N: the whole N when complex64 fits one
    // workgroup, else the longer pass
    const int maxL = single_ok(V_C64, N) ? N : (1 << std::max(g.n1, g.n2));
    g.hmax = maxL / 16 >= 2 ? maxL / 16 : 0;
  }
  return g;
}

int64_t tw_count(const Geo& g) {
  return ((int64_t)1 << g.twS) + ((int64_t)g.N >> g.twS) + stage_tw_count(g.hmax);
}

void build_stage_table(int hmax, std::vector<double2>& t64, std::vector<float2>& t32) {
  const int64_t n = stage_tw_count(hmax);
  t64.resize(n);
  t32.resize(n);
  const long double two_pi = 6.283185307179586476925286766559005768L;
  for (int64_t h = 2; h <= hmax; h *= 2) {
    for (int64_t k = 0; k < h; ++k) {
      for (int m = 1; m < 16; ++m) {
        const int r = ((m & 1) << 3) | ((m & 2) << 1) | ((m & 4) >> 1) | ((m & 8) >> 3);
        // exact reduction of the phase r k / (16 h) before the long double angle
        const int64_t q = ((int64_t)r * k) % (16 * h);
        const long double a = two_pi * (long double)q / (long double)(16 * h);
        const long double c = cosl(a), s = sinl(a);
        const int64_t e = stage_tw_offset(h) + 15 * k + m - 1;
        t64[e] = make_double2((double)c, (double)s);
        t32[e] = make_float2((float)c, (float)s);
      }
    }
  }
}

int xrow_rows_per_group(const Geo& g) {
  const int N1 = 1 << g.n1, N2 = 1 << g.n2;
  const int q = N1 == 256 ? 1 : N1 == 512 ? 2 : N1 == 1024 ? 4 : 0;
  return (q && N2 % (16 / q) == 0) ? 16 / q : 0;
}

int transform_partials(int vk, const Geo& g, bool store) {
  if (single_ok(vk, g.N)) return 1;
  if (!store && xrow_rows_per_group(g)) return (1 << g.n2) / xrow_rows_per_group(g);
  return (1 << g.n2) / g.B2;
}

int transform_partials_max(const Geo& g) {
  int n = 1;
  for (int vk : {V_F32, V_F64, V_C64, V_C128})
    n = std::max(n, std::max(transform_partials(vk, g, true), transform_partials(vk, g, false)));
  return n;
}

void build_tables(const Geo& g, const int32_t* omega, int M, HostTables& t) {
  t.ent_k.resize(M);
  t.perm.resize(M);
  if (!g.grouped) {
    for (int m = 0; m < M; ++m) { t.ent_k[m] = omega[m]; t.perm[m] = m; }
    t.goff.assign(2, 0);
    t.goff[1] = M;
  } else {
    // entries sorted by column c = k mod N1, then by row k / N1 (Omega is
    // increasing, so a stable counting sort by column does it); a pass-1
    // workgroup's columns are contiguous in this order for any B1
    const int N1 = 1 << g.n1, N2 = 1 << g.n2;
    const int mask1 = N1 - 1;
    const int logB1 = ilog2(g.B1);
    std::vector<int32_t> cst(N1 + 1, 0);
    for (int m = 0; m < M; ++m) cst[(omega[m] & mask1) + 1]++;
    for (int c = 0; c < N1; ++c) cst[c + 1] += cst[c];
    std::vector<int32_t> fill(cst.begin(), cst.end() - 1);
    const int nw = std::max(1, N2 / 32);
    t.cmask.assign((size_t)N1 * nw, 0u);
    t.cbase.assign((size_t)N1 * nw, 0);
    for (int m = 0; m < M; ++m) {
      const int k = omega[m];
      const int c = k & mask1, row = k >> g.n1;
      const int p = fill[c]++;
      t.perm[p] = m;
      t.ent_k[p] = k;
      t.cmask[(size_t)c * nw + (row >> 5)] |= 1u << (row & 31);
    }
    for (int c = 0; c < N1; ++c) {
      int run = cst[c];
      for (int w = 0; w < nw; ++w) {
        t.cbase[(size_t)c * nw + w] = run;
        run += __builtin_popcount(t.cmask[(size_t)c * nw + w]);
      }
    }
    t.goff.assign(g.ngroups + 1, 0);
    for (int q = 0; q <= g.ngroups; ++q) t.goff[q] = cst[std::min(N1, q << logB1)];
    t.cst = cst;
  }
  // rows grouped by the pass-2 workgroup that produces them (Fourier output
  // j = j2 + N2 j1, Hadamard output j = j1 + N1 j2); pos1 maps back to the
  // pass-1 entry order
  if (!g.same_out) {
    const int logB2 = ilog2(g.B2);
    const int mask2 = (1 << g.n2) - 1;
    std::vector<int32_t> inv(M);
    for (int p = 0; p < M; ++p) inv[t.perm[p]] = p;
    auto grp2 = [&](int k) {
      return g.fourier ? ((k & mask2) >> logB2) : ((k >> g.n1) >> logB2);
    };
    t.goff2.assign(g.ngroups2 + 1, 0);
    for (int m = 0; m < M; ++m) t.goff2[grp2(omega[m]) + 1]++;
    for (int q = 0; q < g.ngroups2; ++q) t.goff2[q + 1] += t.goff2[q];
    std::vector<int32_t> fill(t.goff2.begin(), t.goff2.end() - 1);
    t.ent2_k.resize(M);
    t.pos1.resize(M);
    for (int m = 0; m < M; ++m) {
      const int q = fill[grp2(omega[m])]++;
      t.ent2_k[q] = omega[m];
      t.pos1[q] = inv[m];
    }
  } else {
    t.ent2_k.clear();
    t.goff2.clear();
    t.pos1.clear();
  }
  // twiddles e^{+2 pi i q / N}: lo for q < 2^twS, hi for q * 2^twS, q < N >> twS
  // (kept when this table set already holds them for the same geometry)
  if (t.tw_N == g.N && t.tw_twS == g.twS && t.tw_hmax == g.hmax) return;
  t.tw_N = g.N;
  t.tw_twS = g.twS;
  t.tw_hmax = g.hmax;
  const int nlo = 1 << g.twS, nhi = g.N >> g.twS;
  t.tw64.resize(nlo + nhi);
  t.tw32.resize(nlo + nhi);
  const long double two_pi = 6.283185307179586476925286766559005768L;
  for (int q = 0; q < nlo + nhi; ++q) {
    const long double k = q < nlo ? (long double)q : (long double)(q - nlo) * nlo;
    const long double a = two_pi * k / (long double)g.N;
    const long double c = cosl(a), s = sinl(a);
    t.tw64[q] = make_double2((double)c, (double)s);
    t.tw32[q] = make_float2((float)c, (float)s);
  }
  if (g.hmax >= 2) {
    std::vector<double2> s64;
    std::vector<float2> s32;
    build_stage_table(g.hmax, s64, s32);
    t.tw64.insert(t.tw64.end(), s64.begin(), s64.end());
    t.tw32.insert(t.tw32.end(), s32.begin(), s32.end());
  }
}

const Tune& tune() {
  static const Tune t = [] {
    Tune v;
    if (const char* e = std::getenv("FCMP_TILE")) {
      v.tile = std::max(256, std::min(8192, std::atoi(e)));
      v.tile_fixed = true;
    }
    if (const char* e = std::getenv("FCMP_THREADS")) v.threads = std::max(64, std::min(256, std::atoi(e)));
    return v;
  }();
  return t;
}

int pick_threads(int tile_n, int cap) {
  int t = tile_n / 8;
  if (t < 64) t = 64;
  const int c = cap > 0 ? cap : tune().threads;
  if (t > c) t = c;
  return t;
}

namespace {
std::mutex g_sched_mu;
std::map<std::tuple<std::string, int, int64_t, int, int>, Sched> g_sched;
}  // namespace

int batch_bucket(int64_t n) {
  if (n <= 1) return 0;
  if (n <= 8) return 1;
  if (n <= 32) return 2;
  if (n <= 128) return 3;
  return 4;
}

std::string device_arch() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return std::string();
  static std::mutex mu;
  static std::map<int, std::string> names;
  std::lock_guard<std::mutex> lk(mu);
  auto it = names.find(dev);
  if (it != names.end()) return it->second;
  hipDeviceProp_t prop{};
  std::string a;
  if (hipGetDeviceProperties(&prop, dev) == hipSuccess) {
    a = prop.gcnArchName;
    const size_t c = a.find(':');
    if (c != std::string::npos) a.resize(c);
  }
  names[dev] = a;
  return a;
}

bool tuned_sched(int cls, int64_t N, int prec, int64_t n, Sched* s) {
  {
    std::lock_guard<std::mutex> lk(g_sched_mu);
    if (g_sched.empty()) return false;   // no device query while nothing is tuned
  }
  const std::string arch = device_arch();
  std::lock_guard<std::mutex> lk(g_sched_mu);
  auto it = g_sched.find(std::make_tuple(arch, cls, N, prec, batch_bucket(n)));
  if (it == g_sched.end()) return false;
  *s = it->second;
  return true;
}

void set_tuned_sched(const std::string& arch, int cls, int64_t N, int prec, int bucket,
                     const Sched& s) {
  std::lock_guard<std::mutex> lk(g_sched_mu);
  g_sched[std::make_tuple(arch, cls, N, prec, bucket)] = s;
}

bool erase_tuned_sched(const std::string& arch, int cls, int64_t N, int prec, int bucket) {
  std::lock_guard<std::mutex> lk(g_sched_mu);
  return g_sched.erase(std::make_tuple(arch, cls, N, prec, bucket)) > 0;
}

hipError_t run_transform(int vk, int sign, const Geo& g, const TwDev& tw, const EntDev& en,
                         const XSrc& in, const XDst& out, void* tmp, const Status* status,
                         hipStream_t st, int ninst, int64_t isn, int64_t ism, int64_t isp,
                         int64_t isx, int64_t isg) {
  const bool fft = g.fourier;
  XParams p{};
  p.N = g.N;
  p.logN = g.logN;
  p.twS = g.twS;
  p.sign = sign;
  p.tw_lo = tw.lo;
  p.tw_hi = tw.hi;
  p.tws = tw.st;
  p.status = status;
  p.excl = out.excl;
  p.inst_excl = isx;
  p.inst_goff = isg;
  p.taps_lam = in.taps_lam; p.taps_x = in.taps_x; p.ntaps = in.ntaps;
  p.inst_taps_lam = in.inst_lam; p.inst_taps_x = in.inst_x;
  p.resid = 0;
  p.ent2_k = out.ent2_k; p.goff2 = out.goff2; p.pos1 = out.pos1; p.nent2 = out.nent2;
  p.yres = out.yres; p.yres_kind = out.yres_kind; p.rout = out.rout; p.r_kind = out.r_kind;
  p.inst_ent2 = out.inst_ent2; p.inst_goff2 = out.inst_goff2;
  p.inst_yres = out.inst_yres; p.inst_rout = out.inst_rout;
  p.excl_mode = 0;
  p.rsel_M = out.rsel_M; p.rsel_ntaps = out.rsel_ntaps; p.rsel_thr = out.rsel_thr;
  p.goff_span = 1;
  p.goff2_span = 1;
  if (single_ok(vk, g.N)) {
    p.L = g.N; p.logL = g.logN; p.B = 1;
    p.in_mode = in.mode; p.in_kind = in.kind; p.in = in.ptr;
    p.in_ss = 0; p.in_es = 1;
    p.ent_k = en.ent_k; p.goff = en.goff; p.nent = en.M; p.logN1 = 0;
    // the tables may be grouped for a two-pass transform of the same N in
    // FP64: one workgroup takes every group
    p.goff_span = g.ngroups;
    p.goff2_span = g.same_out ? g.ngroups : g.ngroups2;
    p.inst_in = in.mode == IN_DENSE ? isn : ism;
    p.inst_ent = ism;
    p.out = out.out; p.out_kind = out.out ? out.kind : -1;
    p.out2 = out.out2; p.out2_kind = out.out2 ? out.kind2 : -1;
    p.out_ss = 0; p.out_es = 1;
    p.inst_out = isn; p.inst_out2 = isn;
    p.inter_tw = 0;
    p.scale = out.scale;
    p.partial = out.partial; p.inst_part = isp;
    p.nthreads = pick_threads(g.N, g.threads);
    p.role = 0;
    p.resid = out.resid ? 1 : 0;
    p.log_out_es = 0;
    if (out.partial && out.excl) p.excl_mode = 1;
    return launch_xform(vk, fft, p, 1, ninst, st);
  }
  const int N1 = 1 << g.n1, N2 = 1 << g.n2;
  // pass 1: N1 sequences (columns k1) of length N2 over k2
  XParams a = p;
  a.L = N2; a.logL = g.n2; a.B = g.B1;
  a.in_mode = in.mode; a.in_kind = in.kind; a.in = in.ptr;
  a.in_ss = 1; a.in_es = N1;
  a.ent_k = en.ent_k; a.goff = en.goff; a.nent = en.M; a.logN1 = g.n1;
  a.inst_in = in.mode == IN_DENSE ? isn : ism;
  a.inst_ent = ism;
  a.out = tmp; a.out_kind = vk; a.out2 = nullptr; a.out2_kind = -1;
  a.out_ss = 1; a.out_es = N1; a.inst_out = isn; a.inst_out2 = 0;
  a.inter_tw = fft ? 1 : 0;
  a.scale = 1.0;
  a.partial = nullptr; a.excl = nullptr; a.excl_mode = 0;
  a.resid = 0;
  a.nthreads = pick_threads(a.L * a.B, g.threads);
  a.role = 1;
  if (!in.pass2_only) {
    hipError_t e = (in.mode == IN_TAPS && taps_pass1_ok(a, vk))
                       ? launch_taps_pass1(a, vk, N1 / g.B1, ninst, st)
                       : launch_xform(vk, fft, a, N1 / g.B1, ninst, st);
    if (e != hipSuccess) return e;
  }
  // pass 2: N2 sequences (rows j2) of length N1 over k1
  XParams b = p;
  b.L = N1; b.logL = g.n1; b.B = g.B2;
  b.in_mode = IN_DENSE; b.in_kind = vk; b.in = tmp;
  b.in_ss = N1; b.in_es = 1; b.inst_in = isn;
  b.ent_k = nullptr; b.goff = nullptr; b.nent = 0; b.logN1 = 0; b.inst_ent = 0;
  b.out = out.out; b.out_kind = out.out ? out.kind : -1;
  b.out2 = out.out2; b.out2_kind = out.out2 ? out.kind2 : -1;
  if (fft) { b.out_ss = 1; b.out_es = N2; }
  else { b.out_ss = N1; b.out_es = 1; }
  b.inst_out = isn; b.inst_out2 = isn;
  b.inter_tw = 0;
  b.scale = out.scale;
  b.partial = out.partial; b.inst_part = isp;
  b.nthreads = pick_threads(b.L * b.B, g.threads);
  b.role = 2;
  b.resid = out.resid ? 1 : 0;
  b.log_out_es = fft ? g.n2 : 0;
  if (out.partial && out.excl) {
    if (!fft) b.excl_mode = 1;
    else if ((N2 & 31) == 0 && g.B2 <= 32) b.excl_mode = 2;
  }
  if (xrow_q(b)) return launch_xrow(vk, fft, b, ninst, st);
  return launch_xform(vk, fft, b, N2 / g.B2, ninst, st);
}

int validate_problem(const fcmp_problem* p, bool need_k) {
  if (!p) return set_error(FCMP_E_INVALID, "problem is NULL");
  if (p->matrix_class != FCMP_HADAMARD && p->matrix_class != FCMP_FOURIER)
    return set_error(FCMP_E_INVALID, "matrix_class must be FCMP_HADAMARD or FCMP_FOURIER");
  const int64_t N = p->N, M = p->M, K = p->K;
  if (N < 2 || N > (int64_t(1) << 24) || (N & (N - 1)) != 0)
    return set_error(FCMP_E_INVALID, "N must be a power of two in [2, 2^24]");
  if (p->matrix_class == FCMP_FOURIER && N > (int64_t(1) << 22))
    return set_error(FCMP_E_INVALID, "Fourier N must be <= 2^22");
  if (M < 1 || M > N) return set_error(FCMP_E_INVALID, "M must be in [1, N]");
  if (need_k && (K < 1 || K >= M))
    return set_error(FCMP_E_INVALID, "K must be in [1, M-1]");
  if (!p->omega) return set_error(FCMP_E_INVALID, "omega is NULL");
  int32_t prev = -1;
  for (int64_t m = 0; m < M; ++m) {
    const int32_t k = p->omega[m];
    if (k < 0 || k >= N) return set_error(FCMP_E_INVALID, "omega entry out of [0, N)");
    if (k <= prev) return set_error(FCMP_E_INVALID, "omega must be strictly increasing");
    prev = k;
  }
  return FCMP_OK;
}

int validate_options(const fcmp_problem* p, const fcmp_options* o) {
  if (!o) return set_error(FCMP_E_INVALID, "options is NULL");
  if (o->algorithm < FCMP_OMP || o->algorithm > FCMP_COSAMP)
    return set_error(FCMP_E_INVALID, "unknown algorithm");
  if (o->corr_method < FCMP_CORR_CONVENTIONAL || o->corr_method > FCMP_CORR_ADAPTIVE)
    return set_error(FCMP_E_INVALID, "unknown corr_method");
  if (o->corr_precision != FCMP_FP64 && o->corr_precision != FCMP_FP32)
    return set_error(FCMP_E_INVALID, "unknown corr_precision");
  if (o->max_iter < 0) return set_error(FCMP_E_INVALID, "max_iter must be >= 0");
  if (o->switch_t < 0) return set_error(FCMP_E_INVALID, "switch_t must be >= 0");
  if (!(o->res_tol >= 0.0 && o->res_tol < 1.0))
    return set_error(FCMP_E_INVALID, "res_tol must be in [0, 1)");
  if (o->flags & ~(FCMP_FLAG_RECOMPUTE_KERNEL | FCMP_FLAG_NO_PERSISTENT | FCMP_FLAG_FLOAT_KERNEL |
                   FCMP_FLAG_HALF_KERNEL | FCMP_FLAG_PHASE_TIMES | FCMP_FLAG_CONJ_PAIR))
    return set_error(FCMP_E_INVALID, "unknown flags");
  if ((o->flags & FCMP_FLAG_CONJ_PAIR) && (p->matrix_class != FCMP_FOURIER || p->N > 8192))
    return set_error(FCMP_E_INVALID, "FCMP_FLAG_CONJ_PAIR needs the Fourier class and N <= 8192");
  if (o->algorithm == FCMP_OMP && p->K > 4096)
    return set_error(FCMP_E_INVALID, "OMP supports K <= 4096");
  if (o->algorithm == FCMP_SP && 2 * p->K > p->M)
    return set_error(FCMP_E_INVALID, "SP needs 2K <= M");
  if (o->algorithm == FCMP_COSAMP && 3 * p->K > p->M)
    return set_error(FCMP_E_INVALID, "CoSaMP needs 3K <= M");
  return FCMP_OK;
}

}  // namespace fcmp
