// First pass of the residual's forward transform evaluated directly from
// the taps.  The residual r = y - Phi_Lambda x (Algorithm 1.1, step 7) needs
// S_Omega U applied to S_Lambda^T x, a vector with only t-1 nonzeros.  In the
// two-pass transform N = N1 N2 the first pass takes column k1 (entries
// k1 + N1 k2) through an N2-point transform and multiplies by W_N^{k1 j2};
// for the Fourier class the two factors combine to
//   out(k1, j2) = sum over taps lam = k1 + N1 k2 of x_lam W_N^{-lam j2},
// and for the Hadamard class the column WHT gives
//   out(k1, j2) = sum over the same taps of x_lam (-1)^popcount(k2 & j2).
// With about one tap per column this is a few products per output instead
// of log2 N2 butterfly levels.  A workgroup owns B columns: it compacts
// their taps, in tap order, into LDS and each thread accumulates its outputs
// over that list in FP64 (one thread keeps one column), then writes the
// intermediate for the second pass exactly where the transform would.
#include "kernels.h"

namespace fcmp {

constexpr int T_THREADS = 256;
constexpr int T_EPT = 8;       // outputs per thread: tile B * N2 <= 2048
constexpr int T_CH = T_THREADS;

template <bool FOURIER>
__global__ void __launch_bounds__(T_THREADS) taps_pass1_kernel(XParams p) {
  using Wd = typename std::conditional<FOURIER, double2, double>::type;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ int32_t tl_s[T_CH];
  __shared__ Wd tx_s[T_CH];
  __shared__ int32_t wsum[T_THREADS / 64 + 1];
  const int inst = blockIdx.y;
  if (p.status && p.status[inst].done) return;
  if (p.rsel_M && (double)p.rsel_M[inst] * (double)p.rsel_ntaps <= p.rsel_thr) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int B = p.B, L = p.L;
  const int logB = __ffs(B) - 1;
  const int s0 = blockIdx.x * B;
  const int mask1 = (1 << p.logN1) - 1;
  const uint32_t maskN = (uint32_t)p.N - 1u;
  // two-level twiddle table (sign +) in LDS
  double2* tlo = (double2*)smem_raw;
  const int nlo = FOURIER ? (1 << p.twS) : 0;
  const int nhi = FOURIER ? (p.N >> p.twS) : 0;
  double2* thi = tlo + nlo;
  if constexpr (FOURIER) {
    const double2* glo = (const double2*)p.tw_lo;
    const double2* ghi = (const double2*)p.tw_hi;
    for (int e = tid; e < nlo + nhi; e += T_THREADS) tlo[e] = e < nlo ? glo[e] : ghi[e - nlo];
  }
  // this thread's column and output rows j = j0 + u * (T_THREADS / B)
  const int c = tid & (B - 1);
  const int j0 = tid >> logB;
  const int jstep = T_THREADS >> logB;
  Wd acc[T_EPT];
#pragma unroll
  for (int u = 0; u < T_EPT; ++u) acc[u] = vzero(Wd());
  const int32_t* lam = p.taps_lam + (int64_t)inst * p.inst_taps_lam;
  const Wd* xg = (const Wd*)p.taps_x + (int64_t)inst * p.inst_taps_x;
  for (int base = 0; base < p.ntaps; base += T_CH) {
    const int e = base + tid;
    int32_t l = 0;
    Wd xv = vzero(Wd());
    bool mine = false;
    if (e < p.ntaps) {
      l = lam[e];
      const int cc = (l & mask1) - s0;
      mine = cc >= 0 && cc < B;
      if (mine) xv = xg[e];
    }
    // compaction in tap order: wave ballots, then wave offsets
    const uint64_t bal = __ballot(mine);
    const int before = __popcll(bal & ((1ull << lane) - 1ull));
    __syncthreads();   // the previous chunk's list is no longer read
    if (lane == 0) wsum[wave] = __popcll(bal);
    __syncthreads();
    int off = 0, count = 0;
    for (int w = 0; w < T_THREADS / 64; ++w) {
      if (w < wave) off += wsum[w];
      count += wsum[w];
    }
    if (mine) {
      tl_s[off + before] = l;
      tx_s[off + before] = xv;
    }
    __syncthreads();
    for (int q = 0; q < count; ++q) {
      const int32_t lq = tl_s[q];
      if ((lq & mask1) - s0 != c) continue;
      const Wd xq = tx_s[q];
#pragma unroll
      for (int u = 0; u < T_EPT; ++u) {
        const int j = j0 + u * jstep;
        if (j < L) {
          if constexpr (FOURIER) {
            const uint32_t ph = ((uint32_t)lq * (uint32_t)j) & maskN;
            double2 w = cmul(thi[ph >> p.twS], tlo[ph & ((1u << p.twS) - 1u)]);
            if (p.sign < 0) w.y = -w.y;
            const double2 t = cmul(xq, w);
            acc[u].x += t.x;
            acc[u].y += t.y;
          } else {
            const int k2 = lq >> p.logN1;
            acc[u] += (__popc(k2 & j) & 1) ? -xq : xq;
          }
        }
      }
    }
  }
  Wd* out = (Wd*)p.out + (int64_t)inst * p.inst_out;
#pragma unroll
  for (int u = 0; u < T_EPT; ++u) {
    const int j = j0 + u * jstep;
    if (j < L) out[(int64_t)(s0 + c) * p.out_ss + (int64_t)j * p.out_es] = acc[u];
  }
}

bool taps_pass1_ok(const XParams& a, int vk) {
  return (vk == V_C128 || vk == V_F64) && a.B * a.L <= T_THREADS * T_EPT &&
         (T_THREADS % a.B) == 0 && a.ntaps <= 2 * (1 << a.logN1);
}

hipError_t launch_taps_pass1(const XParams& a, int vk, int groups, int ninst, hipStream_t st) {
  const size_t lds = vk == V_C128 ? (((size_t)1 << a.twS) + ((size_t)a.N >> a.twS)) * 16 : 16;
  if (vk == V_C128) {
    hipError_t e = raise_lds_limit((const void*)taps_pass1_kernel<true>, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(taps_pass1_kernel<true>, dim3(groups, ninst), dim3(T_THREADS), lds, st, a);
  } else {
    hipLaunchKernelGGL(taps_pass1_kernel<false>, dim3(groups, ninst), dim3(T_THREADS), lds, st, a);
  }
  return hipGetLastError();
}

}  // namespace fcmp
