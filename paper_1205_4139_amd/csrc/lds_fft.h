// LDS-resident transforms shared by the transform kernels and the
// persistent per-instance OMP kernel: two-level twiddle lookup, value
// conversions and the in-place radix-8 FFT / WHT over B interleaved sequences.
#pragma once
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


}  // namespace fcmp
