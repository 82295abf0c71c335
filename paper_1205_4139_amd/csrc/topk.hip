// Deterministic top-K selection for the set-based pursuits (SP, CoSaMP):
// the K entries of largest |v|^2 (ties to the lowest index), optionally
// skipping excluded indices, returned as an ascending index list.
//
// The key of entry j is the IEEE bit pattern of |v(j)|^2 (a non-negative
// double, so the bit pattern orders like the value).  Eight radix rounds of 8
// bits find the exact K-th key kappa; a counting pass and an ordered write
// then emit every key > kappa and the lowest-index keys == kappa.
#include "kernels.h"

namespace fcmp {

constexpr int TK_THREADS = 256;
constexpr int TK_CHUNK = 4096;     // elements per workgroup in the counting passes

__device__ __forceinline__ double key_of(const void* v, int kind, int64_t j) {
  switch (kind) {
    case V_F32: { const float a = ((const float*)v)[j]; return (double)(a * a); }
    case V_F64: { const double a = ((const double*)v)[j]; return a * a; }
    case V_C64: { const float2 a = ((const float2*)v)[j]; return (double)(a.x * a.x + a.y * a.y); }
    default: { const double2 a = ((const double2*)v)[j]; return a.x * a.x + a.y * a.y; }
  }
}

__device__ __forceinline__ bool tk_excluded(const uint32_t* excl, int64_t j) {
  return excl && ((excl[j >> 5] >> (j & 31)) & 1u);
}

// st: [0] prefix, [1] prefix mask, [2] still needed, [3] count strictly above,
// [4] 1 when fewer eligible entries than requested, [5] total count of keys
// above the K-th (from the counting pass).  Digits of 8 bits.
__global__ void tk_hist_kernel(const void* v, int kind, int64_t n, const uint32_t* excl,
                               const uint64_t* st, int shift, uint32_t* hist) {
  __shared__ uint32_t lh[256];
  for (int b = threadIdx.x; b < 256; b += blockDim.x) lh[b] = 0;
  __syncthreads();
  const uint64_t prefix = st[0], pmask = st[1];
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n;
       j += (int64_t)gridDim.x * blockDim.x) {
    if (tk_excluded(excl, j)) continue;
    const uint64_t k = (uint64_t)__double_as_longlong(key_of(v, kind, j));
    if ((k & pmask) != prefix) continue;
    atomicAdd(&lh[(k >> shift) & 0xFFu], 1u);
  }
  __syncthreads();
  for (int b = threadIdx.x; b < 256; b += blockDim.x)
    if (lh[b]) atomicAdd(&hist[b], lh[b]);
}

// One workgroup of 256: thread t looks at bucket 255 - t (largest first), finds
// the digit that holds the still-needed K-th key, updates the state and
// clears the histogram for the next digit.
__global__ void tk_pick_kernel(uint32_t* hist, uint64_t* st, int shift) {
  __shared__ uint32_t part[256];
  const int t = threadIdx.x;
  const uint32_t c = hist[255 - t];
  part[t] = c;
  __syncthreads();
  for (int off = 1; off < 256; off <<= 1) {
    const uint32_t a = t >= off ? part[t - off] : 0u;
    __syncthreads();
    part[t] += a;
    __syncthreads();
  }
  const uint64_t need = st[2];
  const uint32_t before = part[t] - c;
  __syncthreads();
  if (need > 0 && before < need && part[t] >= need) {
    st[3] += before;
    st[2] = need - before;
    st[0] |= (uint64_t)(255 - t) << shift;
    st[1] |= (uint64_t)0xFFu << shift;
  }
  if (t == 255 && need > 0 && part[255] < need) st[4] = 1;
  hist[255 - t] = 0;
}

// counts[wg] = (#keys > kappa, #keys == kappa) over this workgroup's chunk
__global__ void tk_count_kernel(const void* v, int kind, int64_t n, const uint32_t* excl,
                                const uint64_t* st, uint32_t* counts) {
  __shared__ uint32_t sg[TK_THREADS], se[TK_THREADS];
  const uint64_t kappa = st[0];
  const int64_t base = (int64_t)blockIdx.x * TK_CHUNK;
  uint32_t g = 0, e = 0;
  for (int i = threadIdx.x; i < TK_CHUNK; i += TK_THREADS) {
    const int64_t j = base + i;
    if (j >= n || tk_excluded(excl, j)) continue;
    const uint64_t k = (uint64_t)__double_as_longlong(key_of(v, kind, j));
    g += k > kappa;
    e += k == kappa;
  }
  sg[threadIdx.x] = g;
  se[threadIdx.x] = e;
  __syncthreads();
  for (int off = TK_THREADS / 2; off; off >>= 1) {
    if (threadIdx.x < off) {
      sg[threadIdx.x] += sg[threadIdx.x + off];
      se[threadIdx.x] += se[threadIdx.x + off];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    counts[2 * blockIdx.x] = sg[0];
    counts[2 * blockIdx.x + 1] = se[0];
  }
}

// exclusive scan of the per-workgroup counts (one workgroup, sequential per
// thread block of 1024); st[5] receives the total count of keys > kappa
__global__ void tk_scan_kernel(uint32_t* counts, int nwg, uint32_t* offs, uint64_t* st) {
  __shared__ uint32_t pg[1024], pe[1024];
  const int t = threadIdx.x;
  const int per = (nwg + 1023) / 1024;
  uint32_t g = 0, e = 0;
  for (int i = 0; i < per; ++i) {
    const int w = t * per + i;
    if (w < nwg) { g += counts[2 * w]; e += counts[2 * w + 1]; }
  }
  pg[t] = g;
  pe[t] = e;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    const uint32_t a = t >= off ? pg[t - off] : 0u, b = t >= off ? pe[t - off] : 0u;
    __syncthreads();
    pg[t] += a;
    pe[t] += b;
    __syncthreads();
  }
  uint32_t rg = t ? pg[t - 1] : 0u, re = t ? pe[t - 1] : 0u;
  if (t == 1023) st[5] = pg[1023];
  for (int i = 0; i < per; ++i) {
    const int w = t * per + i;
    if (w < nwg) {
      offs[2 * w] = rg;
      offs[2 * w + 1] = re;
      rg += counts[2 * w];
      re += counts[2 * w + 1];
    }
  }
}

// Ordered write: keys > kappa to out[0 .. above), the first K - above keys
// == kappa to out[above .. K), both in index order.  When fewer than K
// entries are eligible (st[4]), kappa stays 0 and every eligible entry is
// written; the remaining slots keep the -1 they were filled with.
__global__ void tk_write_kernel(const void* v, int kind, int64_t n, const uint32_t* excl,
                                const uint64_t* st, const uint32_t* offs, int32_t* out,
                                int64_t K) {
  __shared__ uint32_t sg[TK_THREADS], se[TK_THREADS];
  const uint64_t kappa = st[0];
  const uint64_t above = st[5];
  const uint64_t need = above < (uint64_t)K ? (uint64_t)K - above : 0;
  const int64_t base = (int64_t)blockIdx.x * TK_CHUNK;
  constexpr int PER = TK_CHUNK / TK_THREADS;
  // each thread owns PER consecutive elements
  uint32_t g = 0, e = 0;
  uint8_t fl[PER];
  for (int i = 0; i < PER; ++i) {
    const int64_t j = base + (int64_t)threadIdx.x * PER + i;
    uint8_t f = 0;
    if (j < n && !tk_excluded(excl, j)) {
      const uint64_t k = (uint64_t)__double_as_longlong(key_of(v, kind, j));
      f = k > kappa ? 1 : (k == kappa ? 2 : 0);
    }
    fl[i] = f;
    g += f == 1;
    e += f == 2;
  }
  sg[threadIdx.x] = g;
  se[threadIdx.x] = e;
  __syncthreads();
  for (int off = 1; off < TK_THREADS; off <<= 1) {
    const uint32_t a = threadIdx.x >= off ? sg[threadIdx.x - off] : 0u;
    const uint32_t b = threadIdx.x >= off ? se[threadIdx.x - off] : 0u;
    __syncthreads();
    sg[threadIdx.x] += a;
    se[threadIdx.x] += b;
    __syncthreads();
  }
  uint32_t rg = offs[2 * blockIdx.x] + sg[threadIdx.x] - g;
  uint32_t re = offs[2 * blockIdx.x + 1] + se[threadIdx.x] - e;
  for (int i = 0; i < PER; ++i) {
    const int64_t j = base + (int64_t)threadIdx.x * PER + i;
    if (fl[i] == 1) {
      out[rg++] = (int32_t)j;
    } else if (fl[i] == 2) {
      if (re < need) out[above + re] = (int32_t)j;
      ++re;
    }
  }
}

// Merge the two index-ordered runs out[0..a) and out[a..K) into ascending
// order (one workgroup, bitonic sort over the next power of two); unused
// slots (-1) sort last and stay -1.
__global__ void tk_sort_kernel(int32_t* out, int K) {
  extern __shared__ int32_t sk[];
  int P = 1;
  while (P < K) P <<= 1;
  for (int i = threadIdx.x; i < P; i += blockDim.x)
    sk[i] = (i < K && out[i] >= 0) ? out[i] : 0x7fffffff;
  __syncthreads();
  for (int size = 2; size <= P; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int i = threadIdx.x; i < P; i += blockDim.x) {
        const int pr = i ^ stride;
        if (pr > i) {
          const bool up = (i & size) == 0;
          const int32_t a = sk[i], b = sk[pr];
          if ((a > b) == up) { sk[i] = b; sk[pr] = a; }
        }
      }
      __syncthreads();
    }
  }
  for (int i = threadIdx.x; i < K; i += blockDim.x) out[i] = sk[i] == 0x7fffffff ? -1 : sk[i];
}

__global__ void tk_init_kernel(uint64_t* st, int64_t K) {
  if (threadIdx.x == 0) {
    st[0] = 0; st[1] = 0; st[2] = (uint64_t)K; st[3] = 0; st[4] = 0; st[5] = 0;
  }
}

size_t topk_workspace(int64_t n) {
  const int64_t nwg = (n + TK_CHUNK - 1) / TK_CHUNK;
  return 1024 + 64 + (size_t)nwg * 16 + 256;
}

hipError_t launch_topk(const void* v, int kind, int64_t n, const uint32_t* excl, int64_t K,
                       void* ws, int32_t* out, hipStream_t st) {
  if (K <= 0) return hipSuccess;
  char* w = (char*)ws;
  uint32_t* hist = (uint32_t*)w;
  uint64_t* state = (uint64_t*)(w + 1024);
  const int64_t nwg = (n + TK_CHUNK - 1) / TK_CHUNK;
  uint32_t* counts = (uint32_t*)(w + 1024 + 64);
  uint32_t* offs = counts + 2 * nwg;
  hipError_t e = launch_fill_u32(hist, 0u, 256, st);
  if (e != hipSuccess) return e;
  e = launch_fill_u32((uint32_t*)out, 0xFFFFFFFFu, K, st);   // -1: unused slot
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(tk_init_kernel, dim3(1), dim3(64), 0, st, state, K);
  int hgroups = (int)std::min<int64_t>(2048, (n + 1023) / 1024);
  if (hgroups < 1) hgroups = 1;
  for (int round = 0; round < 8; ++round) {
    const int shift = 56 - 8 * round;
    hipLaunchKernelGGL(tk_hist_kernel, dim3(hgroups), dim3(TK_THREADS), 0, st, v, kind, n, excl,
                       state, shift, hist);
    hipLaunchKernelGGL(tk_pick_kernel, dim3(1), dim3(256), 0, st, hist, state, shift);
  }
  hipLaunchKernelGGL(tk_count_kernel, dim3((unsigned)nwg), dim3(TK_THREADS), 0, st, v, kind, n,
                     excl, state, counts);
  hipLaunchKernelGGL(tk_scan_kernel, dim3(1), dim3(1024), 0, st, counts, (int)nwg, offs, state);
  hipLaunchKernelGGL(tk_write_kernel, dim3((unsigned)nwg), dim3(TK_THREADS), 0, st, v, kind, n,
                     excl, state, offs, out, K);
  int P = 1;
  while (P < K) P <<= 1;
  hipLaunchKernelGGL(tk_sort_kernel, dim3(1), dim3(1024), (size_t)P * 4, st, out, (int)K);
  return hipGetLastError();
}

}  // namespace fcmp
