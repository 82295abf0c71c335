// LDS-resident transforms shared by the transform kernels and the
// persistent per-instance OMP kernel: two-level twiddle lookup, value
// conversions and the in-place radix-16 FFT / WHT over B interleaved sequences.
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

// b * e^{+2 pi i J / 2^(s+1)} with the constant folded: the transform core
// always runs with the + sign (callers conjugate input and output for the -
// sign, since conj(F(conj x)) is the transform with the opposite sign).
template <int s, int J, class V>
__device__ __forceinline__ V twp(V b) {
  using T = decltype(b.x);
  constexpr double c = CTw<s, J>::c, sn = CTw<s, J>::s;
  V r;
  if constexpr (J == 0) {
    r = b;
  } else if constexpr (c == 0.0) {          // i b
    r.x = -b.y; r.y = b.x;
  } else if constexpr (c == sn) {           // (1 + i) b / sqrt(2)
    r.x = (T)c * (b.x - b.y); r.y = (T)c * (b.x + b.y);
  } else if constexpr (c == -sn) {          // (-1 + i) b / sqrt(2)
    r.x = -(T)sn * (b.x + b.y); r.y = (T)sn * (b.x - b.y);
  } else {
    r.x = (T)c * b.x - (T)sn * b.y;
    r.y = (T)c * b.y + (T)sn * b.x;
  }
  return r;
}

// Radix-2 DIT level s over the R = 2^S registers of one block (held in
// bit-reversed sub-block order): pairs (m, m + 2^s) with the constant twiddle
// e^{2 pi i (m mod 2^s) / 2^(s+1)}.
template <int S, int s, int M, class V>
__device__ __forceinline__ void dit_cpairs(V* x) {
  if constexpr (M < (1 << S)) {
    constexpr int half = 1 << s;
    if constexpr ((M & half) == 0) {
      const V t = twp<s, (M & (half - 1))>(x[M + half]);
      x[M + half] = vsub(x[M], t);
      x[M] = vadd(x[M], t);
    }
    dit_cpairs<S, s, M + 1>(x);
  }
}

template <int S, int s, class V>
__device__ __forceinline__ void dit_const(V* x) {
  if constexpr (s < S) {
    dit_cpairs<S, s, 0>(x);
    dit_const<S, s + 1>(x);
  }
}

// The transposed network (decimation in frequency): levels from the largest
// span down, pairs (m, m + 2^s) -> (a + b, w (a - b)); natural-order input,
// bit-reversed output within the block.
template <int S, int s, int M, class V>
__device__ __forceinline__ void dif_cpairs(V* x) {
  if constexpr (M < (1 << S)) {
    constexpr int half = 1 << s;
    if constexpr ((M & half) == 0) {
      const V a = x[M], b = x[M + half];
      x[M] = vadd(a, b);
      x[M + half] = twp<s, (M & (half - 1))>(vsub(a, b));
    }
    dif_cpairs<S, s, M + 1>(x);
  }
}

template <int S, int s, class V>
__device__ __forceinline__ void dif_const(V* x) {
  if constexpr (s >= 0) {
    dif_cpairs<S, s, 0>(x);
    dif_const<S, s - 1>(x);
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

__device__ __forceinline__ float vconj(float v) { return v; }
__device__ __forceinline__ double vconj(double v) { return v; }
__device__ __forceinline__ float2 vconj(float2 v) { return make_float2(v.x, -v.y); }
__device__ __forceinline__ double2 vconj(double2 v) { return make_double2(v.x, -v.y); }

// One in-place stage over the LDS tile: each group holds the 2^S elements
// base + k + m h (m < 2^S) of one sequence.  Fourier: the sub-blocks hold
// decimated sub-transforms in bit-reversed order; register m is multiplied
// by W_{2^S h}^{rev(m) k} (table, radix-16 stages only; the radix-2^r stage
// runs first at span 1 where every twiddle is 1) and then combined by a
// constant-twiddle DIT network (in-place decimation-in-time DFT on
// bit-reversed input).  Hadamard: the natural-order WHT butterflies.
// Element (i, c) of the tile lives at lds_addr(i*B + c).
template <int S, bool FFT, bool DIF, class V>
__device__ __forceinline__ void fft_stage(V* t, int L, int B, int logB, int logh, const V* tws) {
  constexpr int R = 1 << S;
  const int h = 1 << logh;
  const int ngrp = (B * L) >> S;
  const int hb = h * B;
  const bool affine = (hb & 31) == 0;   // padded addresses step by hb + hb/32
  const int hs = hb + (hb >> 5);
  for (int grp = threadIdx.x; grp < ngrp; grp += blockDim.x) {
    const int c = grp & (B - 1);
    const int q = grp >> logB;
    const int k = q & (h - 1);
    const int base = ((q >> logh) << (logh + S)) + k;
    const int e0 = base * B + c;
    int a[R];
    if (affine) {
      const int a0 = lds_addr(e0);
#pragma unroll
      for (int m = 0; m < R; ++m) a[m] = a0 + m * hs;
    } else {
#pragma unroll
      for (int m = 0; m < R; ++m) a[m] = lds_addr(e0 + m * hb);
    }
    V x[R];
#pragma unroll
    for (int m = 0; m < R; ++m) x[m] = t[a[m]];
    if constexpr (FFT && !DIF) {
      if constexpr (S == 4) {
        if (logh > 0) {
          const V* tk = tws + stage_tw_offset(h) + 15 * k - 1;
#pragma unroll
          for (int m = 1; m < R; ++m) x[m] = cmul(x[m], tk[m]);
        }
      }
      dit_const<S, 0>(x);
    } else if constexpr (FFT) {
      // transposed stage: network first, then the same per-register twiddles
      dif_const<S, S - 1>(x);
      if constexpr (S == 4) {
        if (logh > 0) {
          const V* tk = tws + stage_tw_offset(h) + 15 * k - 1;
#pragma unroll
          for (int m = 1; m < R; ++m) x[m] = cmul(x[m], tk[m]);
        }
      }
    } else {
      wht_block<S, 0>(x);
    }
#pragma unroll
    for (int m = 0; m < R; ++m) t[a[m]] = x[m];
  }
  __syncthreads();
}

// B interleaved length-L transforms in LDS with the + sign.  Fourier,
// DIF = false: input placed in bit-reversed order (position bitrev(i) of each
// sequence), output in natural order -- a radix-2^(logL mod 4) stage at span
// 1, then radix-16 stages.  DIF = true (the transposed algorithm): natural
// input, output at position bitrev(j) -- the same stages in reverse order,
// each transposed.  Hadamard: natural in and out either way.  tws is the
// per-span twiddle table (spans up to L/16; unused for Hadamard).  Ends with
// a barrier.
template <bool FFT, bool DIF, class V>
__device__ __forceinline__ void lds_fft(V* t, int L, int logL, int B, int logB, const V* tws) {
  const int r = logL & 3;
  if constexpr (!DIF || !FFT) {
    switch (r) {
      case 1: fft_stage<1, FFT, false>(t, L, B, logB, 0, tws); break;
      case 2: fft_stage<2, FFT, false>(t, L, B, logB, 0, tws); break;
      case 3: fft_stage<3, FFT, false>(t, L, B, logB, 0, tws); break;
      default: break;
    }
    for (int logh = r; logh < logL; logh += 4) fft_stage<4, FFT, false>(t, L, B, logB, logh, tws);
  } else {
    for (int logh = logL - 4; logh >= r; logh -= 4) fft_stage<4, true, true>(t, L, B, logB, logh, tws);
    switch (r) {
      case 1: fft_stage<1, true, true>(t, L, B, logB, 0, tws); break;
      case 2: fft_stage<2, true, true>(t, L, B, logB, 0, tws); break;
      case 3: fft_stage<3, true, true>(t, L, B, logB, 0, tws); break;
      default: break;
    }
  }
}

}  // namespace fcmp
