// fcmp_solve_noalloc: fcmp_solve for callers that cannot allocate device
// memory.  The solve's workspace (the plan tables, the kernel vector, h_0,
// the transform intermediate, the inverse Cholesky factor, ...) is carved
// from a file-scope device array instead of a caller buffer; the kernels are
// the ones fcmp_solve launches, with the same arguments apart from where the
// workspace lives, so results are bit-identical.
#include <mutex>
#include <vector>

#include "engine.h"
#include "plan.h"

using namespace fcmp;

namespace {

// Each device the library runs on holds its own copy of this array for the
// life of the process.  Host code never uses the array's name as an address:
// the device address comes from hipGetSymbolAddress, once per device.
static __device__ __align__(256) unsigned char scratch[FCMP_NOALLOC_SCRATCH_BYTES];

std::mutex g_scratch_mu;
std::vector<void*> g_scratch_ptr;   // indexed by device ordinal

// Device address of this device's scratch (looked up on the first call made
// with that device current).
int scratch_for_current_device(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess || dev < 0)
    return set_error(FCMP_E_DEVICE, std::string("hipGetDevice: ") + hipGetErrorString(e));
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if ((size_t)dev >= g_scratch_ptr.size()) g_scratch_ptr.resize((size_t)dev + 1, nullptr);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return set_error(FCMP_E_DEVICE, std::string("hipGetSymbolAddress(scratch): ") +
                                          hipGetErrorString(e));
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return FCMP_OK;
}

}  // namespace

extern "C" int fcmp_solve_noalloc(const fcmp_problem* prob, const fcmp_options* opt,
                                  const void* y_dev, int32_t* support_dev, void* x_dev,
                                  fcmp_stats* stats, void* hip_stream) {
  fcmp_plan P;
  int rc = plan_init(P, 1, prob, opt);
  if (rc) return rc;
  if (!y_dev || !support_dev || !x_dev) return set_error(FCMP_E_INVALID, "NULL device pointer");
  if (P.total > (size_t)FCMP_NOALLOC_SCRATCH_BYTES)
    return set_error(FCMP_E_WORKSPACE,
                     "problem needs " + std::to_string(P.total) +
                         " bytes of workspace, more than the static scratch of " +
                         std::to_string((size_t)FCMP_NOALLOC_SCRATCH_BYTES));
  void* ws = nullptr;
  if ((rc = scratch_for_current_device(&ws))) return rc;
  plan_layout(P, (char*)ws);
  hipStream_t st = (hipStream_t)hip_stream;
  if ((rc = plan_build(P, prob, st))) return rc;
  const void* yp[1] = {y_dev};
  int32_t* sp[1] = {support_dev};
  void* xp[1] = {x_dev};
  return plan_solve(P, nullptr, yp, sp, xp, stats, st, /*timed=*/false);
}
