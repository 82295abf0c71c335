// Persistent per-instance OMP batches (host side).
#pragma once
#include <vector>

#include "engine.h"

namespace fcmp {

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
  size_t tile_bytes = 0;
  char* base = nullptr;
  double2* tw64 = nullptr;
  float2* tw32 = nullptr;
  WgDesc* desc = nullptr;
  int32_t* order = nullptr;
  int* counter = nullptr;
  Status* status = nullptr;
  void** yptrs = nullptr;
  size_t total = 0;
};

bool wg_eligible(const fcmp_problem& p, const fcmp_options& o);
int wg_plan_init(WgBatch& B, int64_t n, const fcmp_problem* probs, const int64_t* ids,
                 const fcmp_options* opt);
void wg_layout(WgBatch& B, const fcmp_problem* probs, char* base);
// Builds the tables and descriptors (host work, synchronises) then runs.
int wg_solve_batch(WgBatch& B, const fcmp_problem* probs, const void* const* y,
                   int32_t* const* sup, void* const* xo, fcmp_stats* stats, hipStream_t st);
// Device work only: prologue + persistent launch (stats synchronise).
int wg_run(WgBatch& B, fcmp_stats* stats, hipStream_t st);

}  // namespace fcmp
