// Persistent per-instance OMP batches (host side).
#pragma once
#include <vector>

#include "engine.h"

namespace fcmp {

// Twiddle table size of the persistent kernel: fixed (not the batch's
// largest N) so an instance's arithmetic never depends on its batch mates.
constexpr int WG_LOGT = 15;
// The persistent kernel's LDS transforms read the per-span stage table up to
// span (largest Fourier N of the batch) / 16; an entry's value depends only
// on its span, so the table's extent never changes an instance's arithmetic.

struct WgGroup {
  int cls = 0, N = 0, M = 0;
  int64_t first = 0, count = 0;   // members: internal positions [first, first + count)
  Geo g;
  int64_t sM = 0, sN = 0, sG = 0;
  double2* tw64 = nullptr;
  float2* tw32 = nullptr;
  int32_t* ent_k = nullptr;
  int32_t* perm = nullptr;
  int32_t* goff = nullptr;
  void* y_ent = nullptr;
  void* c64 = nullptr;
  void* cp = nullptr;
  void* h0 = nullptr;
  void* tmp = nullptr;
};

struct WgBatch {
  int64_t n = 0;
  fcmp_options opt{};
  std::vector<int64_t> ids;        // caller indices of the batch members
  std::vector<int64_t> order_ids;  // caller index of each internal position
  std::vector<WgGroup> groups;
  std::vector<int64_t> inst_off;   // per internal position: W, x, z region offset
  int logNmax = 1, Kmax = 1;
  int hmax = 0;                    // stage-table extent (Fourier instances)
  int per_cu = 0;                  // resident workgroups per CU (0: occupancy query)
  size_t tile_bytes = 0;
  char* base = nullptr;
  double2* tw64 = nullptr;
  float2* tw32 = nullptr;
  WgDesc* desc = nullptr;
  int32_t* order = nullptr;
  int* counter = nullptr;
  uint64_t* t0 = nullptr;          // device clock at the batch start
  Status* status = nullptr;
  void** ptrs = nullptr;           // 3n: y, support, x (internal order)
  size_t total = 0;
};

bool wg_eligible(const fcmp_problem& p, const fcmp_options& o);
int wg_plan_init(WgBatch& B, int64_t n, const fcmp_problem* probs, const int64_t* ids,
                 const fcmp_options* opt);
void wg_layout(WgBatch& B, const fcmp_problem* probs, char* base);
// Builds the tables and descriptors and uploads them (host work; synchronises).
int wg_build(WgBatch& B, const fcmp_problem* probs, hipStream_t st);
// Host array of 3n pointers (y, support, x) in the internal order.
void wg_host_ptrs(const WgBatch& B, const void* const* y, int32_t* const* sup,
                  void* const* xo, void** out);
// wg_build + pointer upload + wg_run.
int wg_solve_batch(WgBatch& B, const fcmp_problem* probs, const void* const* y,
                   int32_t* const* sup, void* const* xo, fcmp_stats* stats, hipStream_t st);
// Device work only: prologue + persistent launch (stats synchronise).
int wg_run(WgBatch& B, fcmp_stats* stats, hipStream_t st);
// Reads the per-instance status (synchronises): iterations, residual norm,
// completion time from the batch start in ms_total.
int wg_stats(WgBatch& B, fcmp_stats* stats, hipStream_t st);

}  // namespace fcmp
