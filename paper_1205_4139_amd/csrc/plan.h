// Plans: Omega-derived tables, the kernel vector and per-solve buffers for n
// problems of one shape, solved in lockstep.
#pragma once
#include <functional>
#include <vector>

#include "engine.h"

struct fcmp_plan {
  int64_t n = 0;
  fcmp_problem shape{};        // class, N, largest M and K (omega not kept)
  bool uniform = true;         // every instance has the same M and K
  std::vector<int32_t> hM, hK; // per-instance M and K
  int32_t* Mv = nullptr;       // device copies (only when not uniform)
  int32_t* Kv = nullptr;
  fcmp_options opt{};          // algorithm and precision fixed at creation
  fcmp::Geo g;
  int wk = 0, pk = 0;          // wide and correlation-precision value kinds
  // per-instance strides in elements
  int64_t sM = 0, sN = 0, sK = 0, sW = 0, sG = 0, sG2 = 0, sP = 0, sE = 0;
  double resid_ratio = 1.0;    // transform residual when M (t-1) > ratio * N log2 N
  bool fused = false;          // residual fused into the correlation's first pass
  bool rreg = false;           //   by the register-resident kernel (N2 = 256)
  int rthreads = 0;            //   threads of the generic fused first pass (0: default)
  bool sched_tuned = false;    // the launch schedule came from the tuned table
  int64_t sB = 0;              // bucket starts per buffer (N2 + 1, padded)
  int npart = 1;
  // shared
  double2* tw64 = nullptr;
  float2* tw32 = nullptr;
  // per instance (n * stride)
  int32_t* ent_k = nullptr;
  int32_t* perm = nullptr;
  int32_t* goff = nullptr;
  int32_t* ent2_k = nullptr;   // rows grouped by pass-2 output (absent when identical)
  int32_t* goff2 = nullptr;
  int32_t* pos1 = nullptr;
  uint32_t* cmask = nullptr;   // register-resident fused residual: rows of Omega
  int32_t* cbase = nullptr;    //   per column and their positions in y
  int64_t sC = 0;              //   words per instance (N / 32, padded)
  int32_t* cst = nullptr;      // fused residual (other N): first entry of each column
  int64_t sCs = 0;             //   N1 + 1 values per instance, padded
  void* c64 = nullptr;
  void* cp = nullptr;
  int16_t* ci16 = nullptr;     // Hadamard, M < 2^15: the integers N c (fast gathers)
  uint32_t cur_flags = 0;      // flags of the solve being enqueued
  void* y_ent = nullptr;
  void* r = nullptr;
  void* h0 = nullptr;
  void* tmp = nullptr;
  fcmp::Sel* partial = nullptr;
  int32_t* lam = nullptr;
  int32_t* ord = nullptr;      // fused residual: taps in bucket order, two buffers
  int32_t* bst = nullptr;      //   and the bucket starts, two buffers
  uint32_t* excl = nullptr;
  void* x = nullptr;
  void* z = nullptr;
  void* W = nullptr;
  void* wbuf = nullptr;        // split least squares: w and the partial rows
  void* vpart = nullptr;
  fcmp::Status* status = nullptr;
  // set-based pursuits (SP, CoSaMP), one instance at a time
  void* hbuf = nullptr;        // N correlation values (FP64-sized)
  int32_t* Ta = nullptr;       // index lists of up to 3K entries
  int32_t* Tb = nullptr;
  int32_t* Tc = nullptr;
  int32_t* Td = nullptr;
  void* xa = nullptr;          // coefficient lists of up to 3K FP64 values
  void* xb = nullptr;
  void* xc = nullptr;
  void* dws = nullptr;         // dense least-squares workspace
  void* tkws = nullptr;        // top-K workspace
  double* small = nullptr;     // partial sums read back by the host
  int* bad = nullptr;          // Cholesky breakdown flag
  void** dptrs = nullptr;      // 3n device pointers: y, support, x
  std::vector<const void*> last_ptrs;
  size_t total = 0;
};

namespace fcmp {

// Lays out the plan's buffers from base (nullptr: sizes only).
void plan_layout(fcmp_plan& P, char* base);
// tile: transform tile (0: plan_tile(n)); it never changes a result.
int plan_init(fcmp_plan& P, int64_t n, const fcmp_problem* probs, const fcmp_options* opt,
              int tile = 0);
int plan_build(fcmp_plan& P, const fcmp_problem* probs, hipStream_t st);
// timed = false: stats (when given) carry no device time (ms_total = 0) and
// no hipEvent is created.
int plan_solve(fcmp_plan& P, const fcmp_options* opt, const void* const* y,
               int32_t* const* sup, void* const* x, fcmp_stats* stats, hipStream_t st,
               bool timed = true);
int plan_kernel_vector(fcmp_plan& P, hipStream_t st);
// OMP device work of one solve (no host synchronisation, so it can be
// captured in a graph); the pointer array dptrs must already be uploaded.
int plan_enqueue(fcmp_plan& P, const fcmp_options& opt, hipStream_t st);
// One correlation of iteration t (t-1 selected columns) with the fused
// identification, by the fast method or the conventional one (residual and
// transform); npart receives the number of identification partials.
int plan_fast_corr(fcmp_plan& P, int t, int* npart, hipStream_t st);
int plan_conv_corr(fcmp_plan& P, int t, int* npart, hipStream_t st);
// Fused-residual plans: uploads the bucket order of taps 0..ntaps-1 given on
// the host (lam: n * sK values), for conventional correlations run outside a
// solve; ord and bst are host staging kept alive by the caller.
int plan_set_tap_order(fcmp_plan& P, const int32_t* lam, int ntaps, hipStream_t st,
                       std::vector<int32_t>& ord, std::vector<int32_t>& bst);
RCParams rcorr_geometry(const fcmp_plan& P);
int rcorr_threads(const RCParams& q);
// The launch schedule the plan uses (tile, transform threads, first-pass threads).
Sched plan_sched(const fcmp_plan& P);
// Sets the plan's thread counts (0: defaults); FCMP_E_INVALID when the fused
// first pass cannot run with rthreads.
int plan_set_threads(fcmp_plan& P, int threads, int rthreads);
// Fills stats from host copies of the status records; FCMP_E_NUMERIC when any
// instance broke down.
int plan_stats(int64_t n, const Status* hs, double ms, fcmp_stats* stats,
               const double* phase_ms = nullptr);
// Per-solve phase times (ms per FCMP_PHASE_*) into the stats fields.
void stats_phases(fcmp_stats& s, const double* phase_ms);
// ---- slot plans (continuous batching)
// n slots of one (class, N) and options, sized for M <= cap.M and K <= cap.K;
// requests join a free slot and leave it between iterations, and slot s runs
// iteration step - tofs[s] of its own solve (tofs on the device).  Every
// slot starts done.  Only OMP with the conventional correlation fused with
// the residual (plan_slots_ok) runs this way.
bool plan_slots_ok(const fcmp_problem& prob, const fcmp_options& opt);
int plan_init_slots(fcmp_plan& P, int64_t n, const fcmp_problem& cap, const fcmp_options& opt);
// The transform tile of every slot plan (tables are built for its geometry).
int slot_tile();
// One-instance view of slot s: every per-instance buffer offset to the slot;
// dptrs points at the slot's three device pointers (y, support, x).
fcmp_plan plan_view(const fcmp_plan& P, int64_t s, int32_t M, int32_t K);
// stage (nullable) returns a pinned copy of host bytes to copy from, which
// must stay unchanged until the stream has run the copy.
using StageFn = std::function<const void*(const void*, size_t)>;
int plan_upload_twiddles(fcmp_plan& P, const HostTables& t, hipStream_t st,
                         const StageFn& stage = nullptr);
// The view's Omega tables from host tables built for its problem (slot_tile
// geometry), then its kernel vector; or the tables and kernel vector of
// another slot's view.
int plan_upload_tables(fcmp_plan& V, const HostTables& t, hipStream_t st,
                       const StageFn& stage = nullptr);
int plan_copy_tables(fcmp_plan& V, const fcmp_plan& from, hipStream_t st);
// The view's first iteration: exclusions, y in entry order, status, h_0 with
// the first identification and the t = 1 update (its y at dptrs[0]).
int plan_join(fcmp_plan& V, const fcmp_options& opt, hipStream_t st);
// One iteration of every slot that is not done: the fused conventional
// correlation and the update, t_lo .. t_hi spanning the slots' iterations.
int plan_step_slots(fcmp_plan& P, int step, const int32_t* tofs, int t_lo, int t_hi,
                    hipStream_t st);
// The view's support and x to its output pointers; then the slot is done.
int plan_finish(fcmp_plan& V, hipStream_t st);

// SP / CoSaMP for every instance of the plan (after h_0 is in place)
int plan_solve_set(fcmp_plan& P, const fcmp_options& opt, int32_t* const* sup, void* const* xo,
                   fcmp_stats* stats, hipStream_t st);

}  // namespace fcmp
