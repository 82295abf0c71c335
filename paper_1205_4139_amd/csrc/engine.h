// Host-side engine: validation, transform geometry, workspace layout and
// launch sequencing behind the C ABI.
#pragma once
#include <string>
#include <vector>

#include "../../include/fcmp.h"
#include "kernels.h"

namespace fcmp {

int set_error(int code, const std::string& msg);
const char* last_error();

// Transform geometry for one N: single workgroup when the values fit in LDS,
// else two passes N = N1 * N2 with B1 (pass 1) / B2 (pass 2) sequences per
// workgroup.  Entries (rows of Phi) are grouped by pass-1 workgroup when any
// FP64 transform of this N needs two passes.
struct Geo {
  int N = 0, logN = 0, twS = 0;
  bool fourier = false;
  int n1 = 0, n2 = 0;        // log2 N1, log2 N2
  int B1 = 1, B2 = 1;
  bool grouped = false;
  int ngroups = 1;           // pass-1 workgroups = N1 / B1
  int ngroups2 = 1;          // pass-2 workgroups = N2 / B2
  bool same_out = true;      // pass-2 output groups coincide with pass-1 input groups
  int hmax = 0;              // largest span of a twiddled radix-16 stage (Fourier)
  int threads = 0;           // most threads per transform workgroup (0: the default)
};
// Twiddle entries per precision: two-level table (lo 2^twS, hi N >> twS) for
// the inter-pass twiddle, then the per-span stage table of the LDS core.
int64_t tw_count(const Geo& g);
// Per-span stage table for spans 2..hmax (see lds_fft), sign +.
void build_stage_table(int hmax, std::vector<double2>& t64, std::vector<float2>& t32);

// Launch-shape knobs (FCMP_TILE: values per workgroup tile in the two-pass
// transforms; FCMP_THREADS: threads per transform workgroup).
struct Tune {
  int tile = 2048;
  int threads = 256;
  bool tile_fixed = false;   // FCMP_TILE given: use it for every plan
};
const Tune& tune();

bool single_ok(int vk, int N);
// Last iteration of the adaptive method that uses the fast correlation: the
// autotuned crossover for (class, N, precision) when one was measured or
// loaded, else the flop model of Table I (fast while 6(t-1) < 5 log2 N for
// Fourier, t-1 < log2 N for Hadamard).
int default_switch_t(int matrix_class, int64_t N, int precision);
int model_switch_t(int matrix_class, int64_t N);
void set_tuned_switch(int matrix_class, int64_t N, int precision, int switch_t);
bool tuned_switch(int matrix_class, int64_t N, int precision, int* switch_t);
// tile: values per workgroup tile of a two-pass transform (0: the tuned
// default).  The tile changes only how work is split over workgroups, never a
// result: every element's arithmetic and the identification's total order are
// the same for any tile.
Geo make_geo(bool fourier, int N, int tile = 0);
// Tile for a lockstep plan of n instances: few instances need small tiles to
// spread one transform over enough workgroups; many fill the chip anyway.
int plan_tile(int64_t n);
// Partials (one identification result per workgroup) written by a
// transform whose outputs are stored (store) or only identified (the
// register-resident second pass); transform_partials_max bounds both.
int transform_partials(int vk, const Geo& g, bool store);
int transform_partials_max(const Geo& g);
int xrow_rows_per_group(const Geo& g);
int pick_threads(int tile_n, int cap = 0);       // threads of a transform workgroup

// Launch schedule of a plan: the transform tile, the most threads of a
// transform workgroup and the threads of the fused residual's first pass
// (0: the defaults).  No field changes a result: each only splits the same
// per-element arithmetic, and the identification's total order, over
// workgroups and threads differently.  Tuned schedules are kept per (device
// architecture, class, N, precision, batch bucket).
struct Sched {
  int tile = 0, threads = 0, rthreads = 0;
};
int batch_bucket(int64_t n);                     // 0: 1, 1: <= 8, 2: <= 32, 3: <= 128, 4: more
std::string device_arch();                       // of the current device ("" without one)
bool tuned_sched(int cls, int64_t N, int prec, int64_t n, Sched* s);
void set_tuned_sched(const std::string& arch, int cls, int64_t N, int prec, int bucket,
                     const Sched& s);
bool erase_tuned_sched(const std::string& arch, int cls, int64_t N, int prec, int bucket);

struct HostTables {
  std::vector<int32_t> ent_k, perm, goff;   // entry order (grouped or Omega order)
  std::vector<int32_t> ent2_k, goff2, pos1; // rows grouped by pass-2 output workgroup
  std::vector<int32_t> cst;                 // grouped: first entry of each column (N1 + 1)
  std::vector<uint32_t> cmask;              // grouped: rows of Omega per column (N / 32 words)
  std::vector<int32_t> cbase;               //   and the entry index of each word's first row
  std::vector<double2> tw64;                // lo (2^twS), hi (N >> twS), stage table; sign +
  std::vector<float2> tw32;
  int tw_N = 0, tw_twS = -1, tw_hmax = -1;  // geometry the twiddles were built for
};
void build_tables(const Geo& g, const int32_t* omega, int M, HostTables& t);

struct TwDev { const void* lo; const void* hi; const void* st; };
struct EntDev { const int32_t* ent_k; const int32_t* goff; int M; };
struct XSrc {
  int mode; int kind; const void* ptr;
  // two-pass transforms only: the first pass's output is already in tmp
  bool pass2_only = false;
  // IN_TAPS
  const int32_t* taps_lam = nullptr; const void* taps_x = nullptr; int ntaps = 0;
  int64_t inst_lam = 0, inst_x = 0;
};
struct XDst {
  // plans with per-instance row counts: the transform residual skips the
  // instances with rsel_M[inst] * rsel_ntaps <= rsel_thr
  const int32_t* rsel_M = nullptr; int rsel_ntaps = 0; double rsel_thr = 0.0;
  void* out = nullptr; int kind = -1;
  void* out2 = nullptr; int kind2 = -1;
  Sel* partial = nullptr; const uint32_t* excl = nullptr;
  double scale = 1.0;
  // residual output (see XParams)
  bool resid = false;
  const int32_t* ent2_k = nullptr; const int32_t* goff2 = nullptr; const int32_t* pos1 = nullptr;
  int nent2 = 0;
  const void* yres = nullptr; int yres_kind = 0; void* rout = nullptr; int r_kind = 0;
  int64_t inst_ent2 = 0, inst_goff2 = 0, inst_yres = 0, inst_rout = 0;
};

// One N-point transform (sign +1: U^H, -1: U) of the zero-filled entries or
// of a dense N-vector.  tmp: N values of kind vk (two-pass only).
hipError_t run_transform(int vk, int sign, const Geo& g, const TwDev& tw, const EntDev& en,
                         const XSrc& in, const XDst& out, void* tmp, const Status* status,
                         hipStream_t st, int ninst = 1, int64_t inst_stride_n = 0,
                         int64_t inst_stride_m = 0, int64_t inst_stride_part = 0,
                         int64_t inst_stride_excl = 0, int64_t inst_stride_goff = 0);

// Workspace carving helper (256-byte aligned regions).
struct Carver {
  size_t off = 0;
  char* base = nullptr;
  template <class T> T* take(size_t count) {
    off = (off + 255) & ~(size_t)255;
    T* p = base ? (T*)(base + off) : nullptr;
    off += count * sizeof(T);
    return p;
  }
  void* take_bytes(size_t bytes) { return take<char>(bytes); }
  size_t total() const { return (off + 255) & ~(size_t)255; }
};

// Per-solve phase times (FCMP_FLAG_PHASE_TIMES): while a SolveTimes is
// installed on the calling thread, every ProfScope also records a pair of
// events for it.
struct SolveTimes {
  struct Rec { int phase; hipEvent_t a, b; };
  std::vector<Rec> recs;
  ~SolveTimes();
};
// RAII installation on the calling thread (nullptr: nothing installed).
class SolveTimesScope {
 public:
  explicit SolveTimesScope(SolveTimes* s);
  ~SolveTimesScope();
  SolveTimesScope(const SolveTimesScope&) = delete;
  SolveTimesScope& operator=(const SolveTimesScope&) = delete;

 private:
  SolveTimes* prev_;
};
// Synchronises the recorded events and sums them per phase (ms[FCMP_NPHASE]).
int solve_times_read(SolveTimes& s, double* ms);

// RAII phase timer: records hipEvents around a launch sequence when profiling
// is enabled (fcmp_profile_enable) or a SolveTimes is installed; no-op
// otherwise.
class ProfScope {
 public:
  ProfScope(int phase, hipStream_t st);
  ~ProfScope();
  ProfScope(const ProfScope&) = delete;
  ProfScope& operator=(const ProfScope&) = delete;

 private:
  int phase_;
  hipStream_t st_;
  hipEvent_t a_ = nullptr;
  hipEvent_t sa_ = nullptr;
  SolveTimes* solve_ = nullptr;
};
bool prof_enabled();
// Phase events are not recorded by this thread while suspended (graph capture).
void prof_suspend(bool on);
int profile_enable(int enable);
int profile_read(fcmp_profile* out, int reset);

int validate_problem(const fcmp_problem* p, bool need_k);
int validate_options(const fcmp_problem* p, const fcmp_options* o);

}  // namespace fcmp
