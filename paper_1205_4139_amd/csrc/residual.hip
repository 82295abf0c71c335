// Residual update r_t = y - Phi_t x_t (Algorithm 1.1, step 7) in FP64, for
// the conventional correlation path.  Each entry e holds a row k = Omega_m of
// Phi; its residual sums the current support directly:
//   Fourier : U(k, lam) = exp(-2 pi i (k lam mod N) / N) / sqrt(N)
//   Hadamard: U(k, lam) = (-1)^popcount(k & lam) / sqrt(N)
// The phase index k*lam mod N is exact in 32-bit unsigned arithmetic because N
// is a power of two; the phase itself comes from a two-level FP64 table in LDS.
#include "kernels.h"

namespace fcmp {

constexpr int R_THREADS = 256;
constexpr int R_EPT = 4;       // entries per thread
constexpr int R_TCH = 512;     // taps staged in LDS per chunk

__device__ __forceinline__ void store_r(void* b, int64_t i, int kind, double v) {
  if (kind == V_F32) ((float*)b)[i] = (float)v; else ((double*)b)[i] = v;
}
__device__ __forceinline__ void store_r(void* b, int64_t i, int kind, double2 v) {
  if (kind == V_C64) ((float2*)b)[i] = make_float2((float)v.x, (float)v.y);
  else ((double2*)b)[i] = v;
}

template <bool FOURIER>
__global__ void __launch_bounds__(R_THREADS) residual_kernel(RParams p) {
  using Wd = typename std::conditional<FOURIER, double2, double>::type;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int inst = blockIdx.y;
  if (p.status && p.status[inst].done) return;
  const int64_t Mi = p.Mv ? (int64_t)p.Mv[inst] : (int64_t)p.M;
  if (p.Mv && (double)Mi * (double)p.ntaps > p.thr) return;   // transform residual's
  if ((int64_t)blockIdx.x * (R_THREADS * R_EPT) >= Mi) return;
  const int tid = threadIdx.x;
  const int nlo = FOURIER ? (1 << p.twS) : 0;
  const int nhi = FOURIER ? (p.N >> p.twS) : 0;
  double2* tlo = (double2*)smem_raw;
  double2* thi = tlo + nlo;
  Wd* sx = (Wd*)(thi + nhi);
  int32_t* sl = (int32_t*)(sx + R_TCH);
  if (FOURIER) {
    const double2* glo = (const double2*)p.tw_lo;
    const double2* ghi = (const double2*)p.tw_hi;
    for (int e = tid; e < nlo; e += R_THREADS) tlo[e] = glo[e];
    for (int e = tid; e < nhi; e += R_THREADS) thi[e] = ghi[e];
  }
  const int32_t* ek = p.ent_k + (int64_t)inst * p.inst_ent;
  const Wd* y = (const Wd*)p.y + (int64_t)inst * p.inst_y;
  const int32_t* lam = p.lam + (int64_t)inst * p.inst_lam;
  const Wd* xg = (const Wd*)p.x + (int64_t)inst * p.inst_x;
  const int64_t e0 = (int64_t)blockIdx.x * (R_THREADS * R_EPT) + tid;
  uint32_t kk[R_EPT];
  Wd acc[R_EPT];
#pragma unroll
  for (int u = 0; u < R_EPT; ++u) {
    const int64_t e = e0 + (int64_t)u * R_THREADS;
    kk[u] = e < Mi ? (uint32_t)ek[e] : 0u;
    acc[u] = vzero(Wd());
  }
  const uint32_t mask = (uint32_t)p.N - 1u;
  const uint32_t lomask = (1u << p.twS) - 1u;
  for (int base = 0; base < p.ntaps; base += R_TCH) {
    const int n = min(R_TCH, p.ntaps - base);
    __syncthreads();
    for (int e = tid; e < n; e += R_THREADS) {
      sl[e] = lam[base + e];
      sx[e] = xg[base + e];
    }
    __syncthreads();
    for (int tau = 0; tau < n; ++tau) {
      const uint32_t l = (uint32_t)sl[tau];
      const Wd xv = sx[tau];
#pragma unroll
      for (int u = 0; u < R_EPT; ++u) {
        if constexpr (FOURIER) {
          const uint32_t ph = (kk[u] * l) & mask;
          const double2 w = cmul(thi[ph >> p.twS], tlo[ph & lomask]);   // e^{+2 pi i ph/N}
          const double2 t = cmulc(w, xv);                                // conj(w) x
          acc[u].x += t.x;
          acc[u].y += t.y;
        } else {
          const bool neg = __popc(kk[u] & l) & 1;
          acc[u] += neg ? -xv : xv;
        }
      }
    }
  }
  const double sc = 1.0 / sqrt((double)p.N);
#pragma unroll
  for (int u = 0; u < R_EPT; ++u) {
    const int64_t e = e0 + (int64_t)u * R_THREADS;
    if (e < Mi) {
      Wd r = y[e];
      if constexpr (FOURIER) { r.x -= acc[u].x * sc; r.y -= acc[u].y * sc; }
      else r -= acc[u] * sc;
      store_r(p.r, (int64_t)inst * p.inst_r + e, p.r_kind, r);
    }
  }
}

hipError_t launch_residual(const RParams& p, int ninst, hipStream_t st) {
  const int groups = (p.M + R_THREADS * R_EPT - 1) / (R_THREADS * R_EPT);
  const size_t tw = p.fourier ? (((size_t)1 << p.twS) + ((size_t)p.N >> p.twS)) * 16 : 0;
  const size_t lds = tw + (size_t)R_TCH * (p.fourier ? 16 : 8) + (size_t)R_TCH * 4;
  if (p.fourier) {
    hipError_t e = raise_lds_limit((const void*)residual_kernel<true>, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(residual_kernel<true>, dim3(groups, ninst), dim3(R_THREADS), lds, st, p);
  } else {
    hipLaunchKernelGGL(residual_kernel<false>, dim3(groups, ninst), dim3(R_THREADS), lds, st, p);
  }
  return hipGetLastError();
}

}  // namespace fcmp
