// The paper's fast correlation, eq. (kernelsum) / (kernelsumOMP):
//   h(j) = h_0(j) - sum_tau x(tau) (P_{lam_tau} c)(j),
// where P_lambda (Thm 2-1) is the cyclic shift c((j - lambda) mod N) for the
// Fourier class and the dyadic shift c(j XOR lambda) for the Hadamard class
// (Sec. III-B).  h_0 and the taps are FP64, the kernel vector c is stored in
// the correlation precision and every product is accumulated in FP64.  Lanes
// of a wave take consecutive j, so each tap's gather of c is one contiguous
// (shift) or in-block-permuted (XOR) 64-element run.  The identification
// argmax over the columns not yet selected is fused into the epilogue.
#include "kernels.h"

namespace fcmp {

constexpr int F_THREADS = 256;
constexpr int F_TCH = 1024;   // taps staged in LDS per chunk

template <class VC> __device__ __forceinline__ double cwiden(VC v);
template <> __device__ __forceinline__ double cwiden<float>(float v) { return (double)v; }
template <> __device__ __forceinline__ double cwiden<double>(double v) { return v; }
template <> __device__ __forceinline__ double cwiden<int16_t>(int16_t v) { return (double)v; }
template <class VC> __device__ __forceinline__ double2 cwiden2(VC v);
template <> __device__ __forceinline__ double2 cwiden2<float2>(float2 v) {
  return make_double2((double)v.x, (double)v.y);
}
template <> __device__ __forceinline__ double2 cwiden2<double2>(double2 v) { return v; }

template <class VC, int JPT>
__global__ void __launch_bounds__(F_THREADS) fastcorr_kernel(FParams p) {
  constexpr bool FOURIER = VT<VC>::cplx;
  using Wd = typename VT<VC>::Wide;
  __shared__ int32_t sl[F_TCH];
  __shared__ Wd sx[F_TCH];
  __shared__ Sel red[16];
  // Workgroups are dispatched to the eight XCDs round-robin by linear id.
  // With xcd_map, the one-dimensional grid is read so that XCD x runs the
  // instances x, x + 8, ... one after another: an instance's kernel vector
  // then stays in one XCD's L2 while its workgroups gather from it.
  int inst, grp;
  if (p.xcd_map) {
    const int L = blockIdx.x, k = L >> 3;
    inst = (L & 7) + 8 * (k / p.groups);
    grp = k % p.groups;
  } else {
    inst = blockIdx.y;
    grp = blockIdx.x;
  }
  if (p.status && p.status[inst].done) return;
  const int tid = threadIdx.x;
  const uint32_t mask = (uint32_t)p.N - 1u;
  const bool half = p.c_half != 0;
  const uint32_t half_n = (uint32_t)p.N >> 1;
  const int64_t jb = (int64_t)grp * (F_THREADS * JPT) + tid;
  const Wd* h0 = (const Wd*)p.h0 + (int64_t)inst * p.inst_h0;
  const VC* c = (const VC*)p.c + (int64_t)inst * p.inst_c;
  const int32_t* lam = p.lam + (int64_t)inst * p.inst_lam;
  const Wd* xg = (const Wd*)p.x + (int64_t)inst * p.inst_x;
  Wd acc[JPT];
#pragma unroll
  for (int u = 0; u < JPT; ++u) {
    const int64_t j = jb + (int64_t)u * F_THREADS;
    acc[u] = j < p.N ? h0[j] : vzero(Wd());
  }
  for (int base = 0; base < p.ntaps; base += F_TCH) {
    const int n = min(F_TCH, p.ntaps - base);
    __syncthreads();
    for (int e = tid; e < n; e += F_THREADS) {
      sl[e] = lam[base + e];
      sx[e] = xg[base + e];
    }
    __syncthreads();
    // FTU taps per step: their gathers are all in flight before the first
    // product (the products are still accumulated in tap order)
    constexpr int FTU = JPT == 1 ? 8 : (JPT == 2 ? 4 : 2);
    for (int tau0 = 0; tau0 < n; tau0 += FTU) {
      VC cv[FTU][JPT];
#pragma unroll
      for (int q = 0; q < FTU; ++q) {
        const uint32_t l = (uint32_t)sl[min(tau0 + q, n - 1)];
#pragma unroll
        for (int u = 0; u < JPT; ++u) {
          const uint32_t j = (uint32_t)(jb + u * F_THREADS) & mask;
          const uint32_t m = perm_index(FOURIER, j, l, mask);
          if constexpr (FOURIER) {
            // conjugate symmetry: c(m) = conj(c(N - m)); a wave crosses N/2 at
            // most once per tap, so the two halves are read as contiguous runs
            const bool up = half && m > half_n;
            cv[q][u] = c[up ? p.N - m : m];
            if (up) cv[q][u].y = -cv[q][u].y;
          } else {
            cv[q][u] = c[m];
          }
        }
      }
#pragma unroll
      for (int q = 0; q < FTU; ++q) {
        if (tau0 + q < n) {   // uniform
          const Wd xv = sx[tau0 + q];
#pragma unroll
          for (int u = 0; u < JPT; ++u) {
            if constexpr (FOURIER) {
              const double2 cw = cwiden2<VC>(cv[q][u]);
              acc[u].x -= xv.x * cw.x - xv.y * cw.y;
              acc[u].y -= xv.x * cw.y + xv.y * cw.x;
            } else if constexpr (std::is_same<VC, int16_t>::value) {
              // (N c) / N is exact, so this equals the floating-point kernel path
              acc[u] -= xv * (cwiden<VC>(cv[q][u]) * p.cscale);
            } else {
              acc[u] -= xv * cwiden<VC>(cv[q][u]);
            }
          }
        }
      }
    }
  }
  double bkey = -1.0, bkey2 = -1.0;
  int64_t bidx = -1;
  const uint32_t* excl = p.excl ? p.excl + (int64_t)inst * p.inst_excl : nullptr;
  Wd* hout = p.h ? (Wd*)p.h + (int64_t)inst * p.inst_h : nullptr;
#pragma unroll
  for (int u = 0; u < JPT; ++u) {
    const int64_t j = jb + (int64_t)u * F_THREADS;
    if (j < p.N) {
      if (hout) hout[j] = acc[u];
      if (p.partial && (!excl || !bit_is_set(excl, j))) sel_add(vmag2(acc[u]), j, bkey, bidx, bkey2);
    }
  }
  if (p.partial) {
    const Sel r = block_sel_reduce(bkey, bidx, bkey2, red);
    if (tid == 0) p.partial[(int64_t)inst * p.inst_part + grp] = r;
  }
}

// ---------------------------------------------------------------------------
// The conjugate-symmetric pairing of Sec. III-B (complexity, partial Fourier):
// c(N - m) = conj(c(m)), so for a tap (lam, x) the four real products of
// x c(m) give both x c(m), added at h(lam + m), and x conj(c(m)) = x c(N - m),
// added at h(lam - m): (N/2) complex multiplications per tap instead of N.
// The two outputs of a product are mirrors about the tap's own lam, so one
// workgroup holds the whole h of its instance in LDS (N <= 8192 complex FP64)
// and takes the taps in order: within a tap the outputs lam + m (m <= N/2)
// and lam - m (0 < m < N/2) are all distinct, so each is updated by exactly
// one thread, and a barrier separates taps.  Each thread keeps the kernel
// vector values of its m in registers for the whole correlation.
constexpr int FP_THREADS = 512;
constexpr int FP_TCH = 256;     // taps staged per chunk
constexpr int FP_NMAX = 8192;
constexpr int FP_MPT = (FP_NMAX / 2 + FP_THREADS) / FP_THREADS;   // m values per thread

template <class VC>
__global__ void __launch_bounds__(FP_THREADS) fastpair_kernel(FParams p) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ Sel red[16];
  const int inst = blockIdx.x;
  if (p.status && p.status[inst].done) return;
  const int tid = threadIdx.x;
  const int N = p.N, half = p.N >> 1;
  const uint32_t mask = (uint32_t)p.N - 1u;
  double2* hs = (double2*)smem_raw;
  int32_t* sl = (int32_t*)(hs + N);
  double2* sx = (double2*)(sl + FP_TCH);
  const double2* h0 = (const double2*)p.h0 + (int64_t)inst * p.inst_h0;
  const VC* c = (const VC*)p.c + (int64_t)inst * p.inst_c;
  const int32_t* lam = p.lam + (int64_t)inst * p.inst_lam;
  const double2* xg = (const double2*)p.x + (int64_t)inst * p.inst_x;
  for (int j = tid; j < N; j += FP_THREADS) hs[j] = h0[j];
  double2 cm[FP_MPT];
#pragma unroll
  for (int q = 0; q < FP_MPT; ++q) {
    const int m = tid + q * FP_THREADS;
    cm[q] = m <= half ? cwiden2<VC>(c[m]) : make_double2(0.0, 0.0);
  }
  for (int base = 0; base < p.ntaps; base += FP_TCH) {
    const int n = min(FP_TCH, p.ntaps - base);
    __syncthreads();   // h loaded / the previous chunk's last tap is done
    for (int e = tid; e < n; e += FP_THREADS) {
      sl[e] = lam[base + e];
      sx[e] = xg[base + e];
    }
    __syncthreads();
    for (int tau = 0; tau < n; ++tau) {
      const uint32_t l = (uint32_t)sl[tau];
      const double2 xv = sx[tau];
#pragma unroll
      for (int q = 0; q < FP_MPT; ++q) {
        const int m = tid + q * FP_THREADS;
        if (m <= half) {
          const double a = xv.x * cm[q].x, b = xv.y * cm[q].y;
          const double e = xv.x * cm[q].y, f = xv.y * cm[q].x;
          const uint32_t j1 = (l + (uint32_t)m) & mask;
          hs[j1].x -= a - b;   // x c(m)
          hs[j1].y -= e + f;
          if (m != 0 && m != half) {
            const uint32_t j2 = (l - (uint32_t)m) & mask;
            hs[j2].x -= a + b;   // x conj(c(m))
            hs[j2].y -= f - e;
          }
        }
      }
      __syncthreads();   // the next tap updates the same outputs
    }
  }
  __syncthreads();
  double bkey = -1.0, bkey2 = -1.0;
  int64_t bidx = -1;
  const uint32_t* excl = p.excl ? p.excl + (int64_t)inst * p.inst_excl : nullptr;
  double2* hout = p.h ? (double2*)p.h + (int64_t)inst * p.inst_h : nullptr;
  for (int j = tid; j < N; j += FP_THREADS) {
    const double2 v = hs[j];
    if (hout) hout[j] = v;
    if (p.partial && (!excl || !bit_is_set(excl, j))) sel_add(vmag2(v), (int64_t)j, bkey, bidx, bkey2);
  }
  if (p.partial) {
    const Sel r = block_sel_reduce(bkey, bidx, bkey2, red);
    if (tid == 0) p.partial[(int64_t)inst * p.inst_part] = r;
  }
}

bool fastpair_ok(const FParams& p) {
  return p.fourier && p.N >= 2 && p.N <= FP_NMAX && (p.c_kind == V_C64 || p.c_kind == V_C128);
}

hipError_t launch_fastpair(const FParams& p, int ninst, int* groups_out, hipStream_t st) {
  if (!fastpair_ok(p)) return hipErrorInvalidValue;
  if (groups_out) *groups_out = 1;
  const size_t lds = (size_t)p.N * 16 + (size_t)FP_TCH * 20;
  if (p.c_kind == V_C64) {
    hipError_t e = raise_lds_limit((const void*)fastpair_kernel<float2>, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(fastpair_kernel<float2>, dim3(ninst), dim3(FP_THREADS), lds, st, p);
  } else {
    hipError_t e = raise_lds_limit((const void*)fastpair_kernel<double2>, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(fastpair_kernel<double2>, dim3(ninst), dim3(FP_THREADS), lds, st, p);
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Outputs per thread: enough workgroups to cover the chip (about 16 per CU)
// for the whole launch, wider tiles (fewer workgroups, less per-workgroup
// staging) beyond.  Each output's sum runs over the taps in order whatever
// the width, so the width never changes a result.
static int jpt_for(int N, int ninst) {
  int jpt = N <= (1 << 17) ? 1 : (N <= (1 << 19) ? 2 : 4);
  while (jpt < 8 && (int64_t)ninst * (N / (F_THREADS * jpt * 2)) >= 4096) jpt *= 2;
  return jpt;
}

int fastcorr_groups(int N) {
  const int jpt = jpt_for(N, 1);
  return (N + F_THREADS * jpt - 1) / (F_THREADS * jpt);
}

template <class VC>
static hipError_t launch_v(FParams p, int ninst, int jpt, hipStream_t st) {
  p.groups = (p.N + F_THREADS * jpt - 1) / (F_THREADS * jpt);
  p.xcd_map = ninst >= 8 && ninst % 8 == 0 && (int64_t)p.groups * ninst < (int64_t(1) << 31);
  const dim3 grid = p.xcd_map ? dim3(p.groups * ninst) : dim3(p.groups, ninst);
  switch (jpt) {
    case 1: hipLaunchKernelGGL((fastcorr_kernel<VC, 1>), grid, dim3(F_THREADS), 0, st, p); break;
    case 2: hipLaunchKernelGGL((fastcorr_kernel<VC, 2>), grid, dim3(F_THREADS), 0, st, p); break;
    case 4: hipLaunchKernelGGL((fastcorr_kernel<VC, 4>), grid, dim3(F_THREADS), 0, st, p); break;
    default: hipLaunchKernelGGL((fastcorr_kernel<VC, 8>), grid, dim3(F_THREADS), 0, st, p); break;
  }
  return hipGetLastError();
}

hipError_t launch_fastcorr(const FParams& p, int ninst, int* groups_out, hipStream_t st) {
  const int jpt = jpt_for(p.N, ninst);
  if (groups_out) *groups_out = (p.N + F_THREADS * jpt - 1) / (F_THREADS * jpt);
  if (p.c_int16) return launch_v<int16_t>(p, ninst, jpt, st);
  switch (p.c_kind) {
    case V_F32: return launch_v<float>(p, ninst, jpt, st);
    case V_F64: return launch_v<double>(p, ninst, jpt, st);
    case V_C64: return launch_v<float2>(p, ninst, jpt, st);
    case V_C128: return launch_v<double2>(p, ninst, jpt, st);
  }
  return hipErrorInvalidValue;
}

}  // namespace fcmp
