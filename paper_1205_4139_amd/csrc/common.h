// Shared device/host definitions for libfcmp (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fcmp {

// ---------------------------------------------------------------- values
// Value types: float / double (Hadamard, real) and float2 / double2
// (Fourier, complex, interleaved re/im).  Wide<V> is the FP64 type of the
// same kind, used for h_0, the kernel-vector Gram entries and least squares.
template <class V> struct VT;
template <> struct VT<float>   { using S = float;  using Wide = double;  static constexpr bool cplx = false; };
template <> struct VT<double>  { using S = double; using Wide = double;  static constexpr bool cplx = false; };
template <> struct VT<float2>  { using S = float;  using Wide = double2; static constexpr bool cplx = true; };
template <> struct VT<double2> { using S = double; using Wide = double2; static constexpr bool cplx = true; };
// Hadamard kernel vector stored as the integers N c (F3 variant)
template <> struct VT<int16_t> { using S = int16_t; using Wide = double; static constexpr bool cplx = false; };

__host__ __device__ inline float  vzero(float)   { return 0.f; }
__host__ __device__ inline double vzero(double)  { return 0.0; }
__host__ __device__ inline float2 vzero(float2)  { return make_float2(0.f, 0.f); }
__host__ __device__ inline double2 vzero(double2){ return make_double2(0.0, 0.0); }

__device__ inline float  vadd(float a, float b)   { return a + b; }
__device__ inline double vadd(double a, double b) { return a + b; }
__device__ inline float2 vadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ inline double2 vadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ inline float  vsub(float a, float b)   { return a - b; }
__device__ inline double vsub(double a, double b) { return a - b; }
__device__ inline float2 vsub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ inline double2 vsub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }

template <class S> __device__ inline float  vscale(float a, S s)  { return a * (float)s; }
template <class S> __device__ inline double vscale(double a, S s) { return a * (double)s; }
template <class S> __device__ inline float2 vscale(float2 a, S s) { return make_float2(a.x * (float)s, a.y * (float)s); }
template <class S> __device__ inline double2 vscale(double2 a, S s) { return make_double2(a.x * (double)s, a.y * (double)s); }

// complex products
__device__ inline float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ inline double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ inline double2 cconj(double2 a) { return make_double2(a.x, -a.y); }
// conj(a) * b
__device__ inline double2 cmulc(double2 a, double2 b) {
  return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}

// |v|^2 in the value's own precision, returned as double (exact widening)
__device__ inline double vmag2(float a)   { return (double)(a * a); }
__device__ inline double vmag2(double a)  { return a * a; }
__device__ inline double vmag2(float2 a)  { return (double)(a.x * a.x + a.y * a.y); }
__device__ inline double vmag2(double2 a) { return a.x * a.x + a.y * a.y; }

// conversions between precisions (round to nearest)
__device__ inline float  vnarrow(double a, float)    { return (float)a; }
__device__ inline double vnarrow(double a, double)   { return a; }
__device__ inline float2 vnarrow(double2 a, float2)  { return make_float2((float)a.x, (float)a.y); }
__device__ inline double2 vnarrow(double2 a, double2){ return a; }
__device__ inline double  vwiden(float a)   { return (double)a; }
__device__ inline double  vwiden(double a)  { return a; }
__device__ inline double2 vwiden(float2 a)  { return make_double2((double)a.x, (double)a.y); }
__device__ inline double2 vwiden(double2 a) { return a; }

// ---------------------------------------------------------------- selection
// Identification key: larger |h|^2 wins, ties go to the lower index.  key2
// carries the runner-up's key (the largest key among the other candidates),
// from which a solve reports its identification gap.
struct Sel {
  double key;   // |h|^2, or -1 when nothing was eligible
  int64_t idx;  // column index, -1 when nothing was eligible
  double key2;  // runner-up |h|^2, or -1 when there was no other candidate
};

__device__ inline bool sel_better(double k1, int64_t i1, double k2, int64_t i2) {
  return (k1 > k2) || (k1 == k2 && (uint64_t)i1 < (uint64_t)i2);
}

// Adds one candidate (k, i) to a running (best, runner-up): the loser of the
// comparison becomes a runner-up candidate.
template <class K>
__device__ inline void sel_add(K k, int64_t i, K& key, int64_t& idx, K& key2) {
  if (sel_better((double)k, i, (double)key, idx)) {
    key2 = key > key2 ? key : key2;
    key = k;
    idx = i;
  } else if (k > key2) {
    key2 = k;
  }
}

// Merges another (best, runner-up) into a running one.
__device__ inline void sel_merge(double ok, int64_t oi, double ok2, double& key, int64_t& idx,
                                 double& key2) {
  if (sel_better(ok, oi, key, idx)) {
    key2 = key > ok2 ? key : ok2;
    key = ok;
    idx = oi;
  } else {
    key2 = ok > key2 ? ok : key2;
  }
}

// Wave64 reduction of (key, idx, key2) by xor shuffles.
__device__ inline void wave_sel_reduce(double& key, int64_t& idx, double& key2) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    const double ok = __shfl_xor(key, off, 64);
    const int64_t oi = __shfl_xor(idx, off, 64);
    const double ok2 = __shfl_xor(key2, off, 64);
    sel_merge(ok, oi, ok2, key, idx, key2);
  }
}

// Block reduction; every thread must call it.  scratch: >= 2*(nwaves) slots.
__device__ inline Sel block_sel_reduce(double key, int64_t idx, double key2, Sel* scratch) {
  wave_sel_reduce(key, idx, key2);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nwaves = (blockDim.x + 63) >> 6;
  if (lane == 0) scratch[wave] = Sel{key, idx, key2};
  __syncthreads();
  if (wave == 0) {
    Sel s = lane < nwaves ? scratch[lane] : Sel{-1.0, -1, -1.0};
    double k = s.key, k2 = s.key2;
    int64_t i = s.idx;
    wave_sel_reduce(k, i, k2);
    if (lane == 0) scratch[0] = Sel{k, i, k2};
  }
  __syncthreads();
  Sel r = scratch[0];
  __syncthreads();
  return r;
}

// Relative identification gap (|h|_(1) - |h|_(2)) / |h|_(1) from the keys
// |h|^2 of a winner and its runner-up (1 when there is no runner-up).
__device__ inline double sel_gap(const Sel& s) {
  if (!(s.key > 0.0)) return 0.0;
  const double a = sqrt(s.key);
  return s.key2 > 0.0 ? (a - sqrt(s.key2)) / a : 1.0;
}

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Block sum of a double; every thread must call it; scratch >= nwaves doubles.
__device__ inline double block_sum(double v, double* scratch) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nwaves = (blockDim.x + 63) >> 6;
  if (lane == 0) scratch[wave] = v;
  __syncthreads();
  double r = 0.0;
  for (int w = 0; w < nwaves; ++w) r += scratch[w];
  __syncthreads();
  return r;
}

__device__ inline bool bit_is_set(const uint32_t* bm, int64_t j) {
  return (bm[j >> 5] >> (j & 31)) & 1u;
}

// ---------------------------------------------------------------- index maps
// P_lambda of Thm 2-1 as index arithmetic: cyclic shift (Fourier) or XOR
// (Hadamard); c is gathered at j (-) lambda.
__device__ inline uint32_t perm_index(bool fourier, uint32_t j, uint32_t lam, uint32_t mask) {
  return (fourier ? (j - lam) : (j ^ lam)) & mask;
}

// ---------------------------------------------------------------- device status
// Per-solve control block in device memory.
struct Status {
  int32_t done;        // 1: stop (all later iteration kernels return at once)
  int32_t numeric;     // 1: Cholesky breakdown
  int32_t iterations;  // selections made (OMP) / outer iterations (SP, CoSaMP)
  int32_t cur_j;       // column picked by the current iteration
  double  znorm2;      // ||z||^2 = ||y||^2 - ||r||^2
  double  ynorm2;      // ||y||^2
  double  last_key;    // |h|^2 of the last pick
  double  t_done;      // persistent batches: device wall-clock ticks at completion
  double  min_gap;     // smallest identification gap so far (+inf before any)
  double  res_tol2;    // stop once ||r||^2 <= res_tol2 ||y||^2 (0: never)
};

}  // namespace fcmp
