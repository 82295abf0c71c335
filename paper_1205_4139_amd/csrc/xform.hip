// N-point transforms for the correlation h = U^H S_Omega^T r (Algorithm 1.1
// step 2 computed as in Sec. III-B: one FFT for the Fourier class, one FHT
// for the Hadamard class), staged through LDS, with the identification
// argmax of step 3 fused into the output loop.
//
// A transform of length N runs either in one workgroup (N values fit in
// LDS) or as two passes N = N1 * N2 (k = k1 + N1 k2):
//   pass 1: N1 length-N2 transforms over k2 (stride N1 in memory), then the
//           Fourier twiddle W_N^{k1 j2};
//   pass 2: N2 length-N1 transforms over k1 (contiguous rows).
// Fourier output lands at j = j2 + N2 j1; Hadamard output at j = j1 + N1 j2.
#include "kernels.h"

namespace fcmp {

__device__ __forceinline__ int lds_addr(int e) { return e + (e >> 5); }

__device__ __forceinline__ int bitrev(int i, int logL) {
  return logL == 0 ? 0 : (int)(__brev((unsigned)i) >> (32 - logL));
}

// value conversions to the transform type
template <class V> __device__ __forceinline__ V load_as(const void* b, int64_t i, int kind);
template <> __device__ __forceinline__ float load_as<float>(const void* b, int64_t i, int kind) {
  return kind == V_F32 ? ((const float*)b)[i] : (float)((const double*)b)[i];
}
template <> __device__ __forceinline__ double load_as<double>(const void* b, int64_t i, int kind) {
  return kind == V_F32 ? (double)((const float*)b)[i] : ((const double*)b)[i];
}
template <> __device__ __forceinline__ float2 load_as<float2>(const void* b, int64_t i, int kind) {
  if (kind == V_C64) return ((const float2*)b)[i];
  double2 v = ((const double2*)b)[i];
  return make_float2((float)v.x, (float)v.y);
}
template <> __device__ __forceinline__ double2 load_as<double2>(const void* b, int64_t i, int kind) {
  if (kind == V_C128) return ((const double2*)b)[i];
  float2 v = ((const float2*)b)[i];
  return make_double2((double)v.x, (double)v.y);
}

__device__ __forceinline__ void store_as(void* b, int64_t i, int kind, float v) {
  if (kind == V_F32) ((float*)b)[i] = v; else ((double*)b)[i] = (double)v;
}
__device__ __forceinline__ void store_as(void* b, int64_t i, int kind, double v) {
  if (kind == V_F32) ((float*)b)[i] = (float)v; else ((double*)b)[i] = v;
}
__device__ __forceinline__ void store_as(void* b, int64_t i, int kind, float2 v) {
  if (kind == V_C64) ((float2*)b)[i] = v;
  else ((double2*)b)[i] = make_double2((double)v.x, (double)v.y);
}
__device__ __forceinline__ void store_as(void* b, int64_t i, int kind, double2 v) {
  if (kind == V_C128) ((double2*)b)[i] = v;
  else ((float2*)b)[i] = make_float2((float)v.x, (float)v.y);
}

template <class V> __device__ __forceinline__ V vone();
template <> __device__ __forceinline__ float vone<float>() { return 1.f; }
template <> __device__ __forceinline__ double vone<double>() { return 1.0; }
template <> __device__ __forceinline__ float2 vone<float2>() { return make_float2(1.f, 0.f); }
template <> __device__ __forceinline__ double2 vone<double2>() { return make_double2(1.0, 0.0); }

// W_N^p = e^{sign 2 pi i p / N} from the two-level table (p already mod N).
template <class V>
__device__ __forceinline__ V tw_lookup(const V* lo, const V* hi, uint32_t p, int twS, int sign) {
  V w = cmul(hi[p >> twS], lo[p & ((1u << twS) - 1u)]);
  if (sign < 0) w.y = -w.y;
  return w;
}

// multiply by (sign * i)
template <class V> __device__ __forceinline__ V mul_i(V a, int sign) {
  V r;
  if (sign > 0) { r.x = -a.y; r.y = a.x; } else { r.x = a.y; r.y = -a.x; }
  return r;
}

// e^{sign 2 pi i j / 2^(s+1)} for s < 4, j < 2^s: the constant twiddles inside
// a radix-16 block (cos and sin of multiples of pi/8).
template <int S, int J> struct CTw;
#define FCMP_CTW(S_, J_, C_, SN_) \
  template <> struct CTw<S_, J_> { static constexpr double c = C_; static constexpr double s = SN_; };
FCMP_CTW(0, 0, 1.0, 0.0)
FCMP_CTW(1, 0, 1.0, 0.0)
FCMP_CTW(1, 1, 0.0, 1.0)
FCMP_CTW(2, 0, 1.0, 0.0)
FCMP_CTW(2, 1, 0.70710678118654752440, 0.70710678118654752440)
FCMP_CTW(2, 2, 0.0, 1.0)
FCMP_CTW(2, 3, -0.70710678118654752440, 0.70710678118654752440)
FCMP_CTW(3, 0, 1.0, 0.0)
FCMP_CTW(3, 1, 0.92387953251128675613, 0.38268343236508977173)
FCMP_CTW(3, 2, 0.70710678118654752440, 0.70710678118654752440)
FCMP_CTW(3, 3, 0.38268343236508977173, 0.92387953251128675613)
FCMP_CTW(3, 4, 0.0, 1.0)
FCMP_CTW(3, 5, -0.38268343236508977173, 0.92387953251128675613)
FCMP_CTW(3, 6, -0.70710678118654752440, 0.70710678118654752440)
FCMP_CTW(3, 7, -0.92387953251128675613, 0.38268343236508977173)
#undef FCMP_CTW

// b * e^{sign 2 pi i J / 2^(S+1)}
template <int S, int J, class V>
__device__ __forceinline__ V twc(V b, int sign) {
  using T = decltype(b.x);
  if constexpr (J == 0) {
    return b;
  } else if constexpr (CTw<S, J>::c == 0.0) {   // +-i
    return mul_i(b, sign);
  } else {
    V w;
    w.x = (T)CTw<S, J>::c;
    w.y = sign > 0 ? (T)CTw<S, J>::s : -(T)CTw<S, J>::s;
    return cmul(b, w);
  }
}

// Radix-2 DIT sub-stage s over the R = 2^S registers of one block: pairs
// (m, m + 2^s) with twiddle b[s] * w_{2^(s+1)}^(m mod 2^s).
template <int S, int s, int M, class V>
__device__ __forceinline__ void dit_pairs(V* x, const V* b, int sign) {
  if constexpr (M < (1 << S)) {
    constexpr int half = 1 << s;
    if constexpr ((M & half) == 0) {
      const V w = twc<s, (M & (half - 1))>(b[s], sign);
      const V t = cmul(w, x[M + half]);
      x[M + half] = vsub(x[M], t);
      x[M] = vadd(x[M], t);
    }
    dit_pairs<S, s, M + 1>(x, b, sign);
  }
}

template <int S, int s, class V>
__device__ __forceinline__ void dit_block(V* x, const V* b, int sign) {
  if constexpr (s < S) {
    dit_pairs<S, s, 0>(x, b, sign);
    dit_block<S, s + 1>(x, b, sign);
  }
}

template <int S, int s, int M, class V>
__device__ __forceinline__ void wht_pairs(V* x) {
  if constexpr (M < (1 << S)) {
    constexpr int half = 1 << s;
    if constexpr ((M & half) == 0) {
      const V a = x[M], c = x[M + half];
      x[M] = vadd(a, c);
      x[M + half] = vsub(a, c);
    }
    wht_pairs<S, s, M + 1>(x);
  }
}

template <int S, int s, class V>
__device__ __forceinline__ void wht_block(V* x) {
  if constexpr (s < S) {
    wht_pairs<S, s, 0>(x);
    wht_block<S, s + 1>(x);
  }
}

// One radix-2^S stage over the LDS tile: each group holds the 2^S elements
// base + k + m h (m < 2^S) of one sequence in registers and applies S
// consecutive radix-2 levels (spans h .. 2^(S-1) h) to them.  The Fourier
// form is the in-place decimation-in-time DFT on bit-reversed input, the
// Hadamard form the in-place natural-order WHT.  Element (i, c) of the tile
// lives at lds_addr(i*B + c).
template <int S, bool FFT, class V>
__device__ __forceinline__ void lds_stage(V* t, int L, int B, int logB, int logh, const V* lo,
                                          const V* hi, int twS, int logN, int sign) {
  constexpr int R = 1 << S;
  const int h = 1 << logh;
  const int ngrp = (B * L) >> S;
  for (int grp = threadIdx.x; grp < ngrp; grp += blockDim.x) {
    const int c = grp & (B - 1);
    const int q = grp >> logB;
    const int k = q & (h - 1);
    const int base = ((q >> logh) << (logh + S)) + k;
    V x[R];
#pragma unroll
    for (int m = 0; m < R; ++m) x[m] = t[lds_addr((base + m * h) * B + c)];
    if constexpr (FFT) {
      V b[S];
#pragma unroll
      for (int s = 0; s < S; ++s)
        b[s] = tw_lookup(lo, hi, (uint32_t)k << (logN - logh - s - 1), twS, sign);  // w_{2^(s+1) h}^k
      dit_block<S, 0>(x, b, sign);
    } else {
      wht_block<S, 0>(x);
    }
#pragma unroll
    for (int m = 0; m < R; ++m) t[lds_addr((base + m * h) * B + c)] = x[m];
  }
  __syncthreads();
}

// B interleaved length-L transforms in LDS: radix-8 stages from the
// smallest span up, then one radix-2/4 stage for the remaining levels (radix
// 8 keeps the block in about 60 VGPRs, so four waves per SIMD stay resident).
template <bool FFT, class V>
__device__ void lds_transform(V* t, int L, int logL, int B, int logB, const V* lo, const V* hi,
                              int twS, int logN, int sign) {
  int logh = 0;
  for (; logh + 3 <= logL; logh += 3)
    lds_stage<3, FFT>(t, L, B, logB, logh, lo, hi, twS, logN, sign);
  switch (logL - logh) {
    case 2: lds_stage<2, FFT>(t, L, B, logB, logh, lo, hi, twS, logN, sign); break;
    case 1: lds_stage<1, FFT>(t, L, B, logB, logh, lo, hi, twS, logN, sign); break;
    default: break;
  }
}

// ROLE only names the launch for profilers: 0 one workgroup per transform,
// 1 first pass (columns), 2 second pass (rows).
template <class V, bool FFT, int ROLE>
__global__ void __launch_bounds__(256) xform_kernel(XParams p) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int inst = blockIdx.y;
  if (p.status && p.status[inst].done) return;
  const int tid = threadIdx.x, nt = blockDim.x;
  const int g = blockIdx.x;
  const int B = p.B, L = p.L, logL = p.logL;
  const int logB = __ffs(B) - 1;
  const int s0 = g * B;
  const int tile_n = B * L;
  const int tile_alloc = tile_n + (tile_n >> 5) + 1;
  V* tile = (V*)smem_raw;
  V* twlo = tile + tile_alloc;
  const int nlo = FFT ? (1 << p.twS) : 0;
  const int nhi = FFT ? (p.N >> p.twS) : 0;
  V* twhi = twlo + nlo;
  Sel* red = (Sel*)(((uintptr_t)(twhi + nhi) + 15) & ~(uintptr_t)15);

  if constexpr (FFT) {
    const V* glo = (const V*)p.tw_lo;
    const V* ghi = (const V*)p.tw_hi;
    for (int e = tid; e < nlo; e += nt) twlo[e] = glo[e];
    for (int e = tid; e < nhi; e += nt) twhi[e] = ghi[e];
  }

  // ---- load
  if (p.in_mode == IN_DENSE) {
    const int64_t ib = (int64_t)inst * p.inst_in;
    for (int e = tid; e < tile_n; e += nt) {
      int c, i;
      if (p.in_es == 1) { c = e >> logL; i = e & (L - 1); }
      else { c = e & (B - 1); i = e >> logB; }
      const V v = load_as<V>(p.in, ib + (int64_t)(s0 + c) * p.in_ss + (int64_t)i * p.in_es,
                             p.in_kind);
      const int pos = FFT ? bitrev(i, logL) : i;
      tile[lds_addr(pos * B + c)] = v;
    }
  } else if (p.in_mode == IN_TAPS) {
    // zero-filled sparse vector S_Lambda^T x: this workgroup keeps the taps
    // whose column falls in its sequences
    const V z = vzero(V());
    for (int e = tid; e < tile_alloc; e += nt) tile[e] = z;
    __syncthreads();
    const int32_t* tl = p.taps_lam + (int64_t)inst * p.inst_taps_lam;
    const int mask1 = (1 << p.logN1) - 1;
    for (int e = tid; e < p.ntaps; e += nt) {
      const int k = tl[e];
      const int i = k >> p.logN1;
      const int c = (k & mask1) - s0;
      if (c >= 0 && c < B) {
        const V v = load_as<V>(p.taps_x, (int64_t)inst * p.inst_taps_x + e, p.in_kind);
        const int pos = FFT ? bitrev(i, logL) : i;
        tile[lds_addr(pos * B + c)] = v;
      }
    }
  } else {
    const V z = vzero(V());
    for (int e = tid; e < tile_alloc; e += nt) tile[e] = z;
    __syncthreads();
    int lo = 0, hi = p.nent;
    if (p.goff) {
      const int32_t* go = p.goff + (int64_t)inst * p.inst_goff;
      lo = go[g];
      hi = go[g + 1];
    }
    const int32_t* ek = p.ent_k + (int64_t)inst * p.inst_ent;
    const int mask1 = (1 << p.logN1) - 1;
    const int64_t ib = (int64_t)inst * p.inst_in;
    for (int e = lo + tid; e < hi; e += nt) {
      const int k = ek[e];
      const int i = k >> p.logN1;
      const int c = (k & mask1) - s0;
      const V v = (p.in_mode == IN_SPARSE_ONES) ? vone<V>() : load_as<V>(p.in, ib + e, p.in_kind);
      const int pos = FFT ? bitrev(i, logL) : i;
      tile[lds_addr(pos * B + c)] = v;
    }
  }
  __syncthreads();

  // ---- transform
  lds_transform<FFT>(tile, L, logL, B, logB, twlo, twhi, p.twS, p.logN, p.sign);

  // ---- residual output: r = y - (S_Omega U s) at the rows of Phi this
  // workgroup produced (forward transform of the support, Algorithm 1.1 step 7)
  if (p.resid) {
    int lo = 0, hi = p.nent2;
    if (p.goff2) {
      const int32_t* go = p.goff2 + (int64_t)inst * p.inst_goff2;
      lo = go[g];
      hi = go[g + 1];
    }
    const int32_t* ek = p.ent2_k + (int64_t)inst * p.inst_ent2;
    const int32_t* pos1 = p.pos1 ? p.pos1 + (int64_t)inst * p.inst_ent2 : nullptr;
    const int esmask = (1 << p.log_out_es) - 1;
    for (int e = lo + tid; e < hi; e += nt) {
      const int k = ek[e];
      int c, j;
      if (p.out_es == 1) { j = k & (L - 1); c = (k >> logL) - s0; }
      else { c = (k & esmask) - s0; j = k >> p.log_out_es; }
      const V v = vscale(tile[lds_addr(j * B + c)], p.scale);
      const int64_t q = pos1 ? (int64_t)pos1[e] : (int64_t)e;
      const V yv = load_as<V>(p.yres, (int64_t)inst * p.inst_yres + q, p.yres_kind);
      store_as(p.rout, (int64_t)inst * p.inst_rout + q, p.r_kind, vsub(yv, v));
    }
    return;
  }

  // ---- store / identify
  double bkey = -1.0;
  int64_t bidx = -1;
  const uint32_t* excl = p.excl ? p.excl + (int64_t)inst * p.inst_excl : nullptr;
  // stage the exclusion bits this workgroup needs
  uint32_t* xw = (uint32_t*)(red + 16);
  int64_t xbase = 0;
  if (p.partial && excl && p.excl_mode) {
    if (p.excl_mode == 1) {
      const int64_t o0 = (int64_t)s0 * p.out_ss;
      xbase = o0 >> 5;
      const int nw = (int)(((o0 + tile_n - 1) >> 5) - xbase + 1);
      for (int e = tid; e < nw; e += nt) xw[e] = excl[xbase + e];
    } else {
      const int64_t wstride = p.out_es >> 5;
      for (int e = tid; e < L; e += nt) xw[e] = excl[(s0 >> 5) + e * wstride];
    }
    __syncthreads();
  }
  for (int e = tid; e < tile_n; e += nt) {
    int c, j;
    if (p.out_es == 1) { c = e >> logL; j = e & (L - 1); }
    else { c = e & (B - 1); j = e >> logB; }
    V v = tile[lds_addr(j * B + c)];
    if constexpr (FFT) {
      if (p.inter_tw) {
        const uint32_t q = ((uint32_t)(s0 + c) * (uint32_t)j) & (uint32_t)(p.N - 1);
        v = cmul(v, tw_lookup(twlo, twhi, q, p.twS, p.sign));
      }
    }
    v = vscale(v, p.scale);
    const int64_t o = (int64_t)(s0 + c) * p.out_ss + (int64_t)j * p.out_es;
    if (p.out_kind >= 0) store_as(p.out, (int64_t)inst * p.inst_out + o, p.out_kind, v);
    if (p.out2_kind >= 0) store_as(p.out2, (int64_t)inst * p.inst_out2 + o, p.out2_kind, v);
    if (p.partial) {
      bool ex = false;
      if (excl) {
        if (p.excl_mode == 1) ex = (xw[(o >> 5) - xbase] >> (o & 31)) & 1u;
        else if (p.excl_mode == 2) ex = (xw[j] >> ((s0 + c) & 31)) & 1u;
        else ex = bit_is_set(excl, o);
      }
      if (!ex) {
        const double kk = vmag2(v);
        if (sel_better(kk, o, bkey, bidx)) { bkey = kk; bidx = o; }
      }
    }
  }
  if (p.partial) {
    const Sel r = block_sel_reduce(bkey, bidx, red);
    if (tid == 0) p.partial[(int64_t)inst * p.inst_part + g] = r;
  }
}

size_t xform_lds_bytes(int vk, bool fft, const XParams& p) {
  const size_t vb = vbytes(vk);
  const size_t tile_n = (size_t)p.B * p.L;
  const size_t tile_alloc = tile_n + (tile_n >> 5) + 1;
  const size_t ntw = fft ? ((size_t)1 << p.twS) + ((size_t)p.N >> p.twS) : 0;
  size_t bytes = (tile_alloc + ntw) * vb;
  bytes = (bytes + 15) & ~(size_t)15;
  bytes += 16 * sizeof(Sel);
  if (p.excl_mode == 1) bytes += (tile_n / 32 + 2) * 4;
  else if (p.excl_mode == 2) bytes += (size_t)p.L * 4;
  return bytes;
}

template <class V, bool FFT, int ROLE>
static hipError_t launch_r(const XParams& p, int groups, int ninst, size_t lds, hipStream_t st) {
  auto kfn = xform_kernel<V, FFT, ROLE>;
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute((const void*)kfn,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(kfn, dim3(groups, ninst), dim3(p.nthreads), lds, st, p);
  return hipGetLastError();
}

template <class V, bool FFT>
static hipError_t launch_t(const XParams& p, int groups, int ninst, size_t lds, hipStream_t st) {
  if (p.role == 1) return launch_r<V, FFT, 1>(p, groups, ninst, lds, st);
  if (p.role == 2) return launch_r<V, FFT, 2>(p, groups, ninst, lds, st);
  return launch_r<V, FFT, 0>(p, groups, ninst, lds, st);
}

hipError_t launch_xform(int vk, bool fft, const XParams& p, int groups, int ninst,
                        hipStream_t st) {
  const size_t lds = xform_lds_bytes(vk, fft, p);
  if (fft) {
    if (vk == V_C64) return launch_t<float2, true>(p, groups, ninst, lds, st);
    if (vk == V_C128) return launch_t<double2, true>(p, groups, ninst, lds, st);
  } else {
    if (vk == V_F32) return launch_t<float, false>(p, groups, ninst, lds, st);
    if (vk == V_F64) return launch_t<double, false>(p, groups, ninst, lds, st);
  }
  return hipErrorInvalidValue;
}

}  // namespace fcmp
