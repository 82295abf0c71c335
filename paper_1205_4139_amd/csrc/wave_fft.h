// Register-resident transform pieces shared by the second-pass kernel and
// the fused residual + first-pass kernel: a row of 16 P values is held by P
// lanes of one wavefront (16 per lane); 16-point transforms run in registers,
// the lanes exchange values through a wavefront-private LDS region, and
// butterflies between lanes use wavefront shuffles.
#pragma once
#include "lds_fft.h"

namespace fcmp {

__device__ __forceinline__ float kmag2r(float v) { return v * v; }
__device__ __forceinline__ float kmag2r(float2 v) { return v.x * v.x + v.y * v.y; }
__device__ __forceinline__ double kmag2r(double v) { return v * v; }
__device__ __forceinline__ double kmag2r(double2 v) { return v.x * v.x + v.y * v.y; }

constexpr int rev4(int m) { return ((m & 1) << 3) | ((m & 2) << 1) | ((m & 4) >> 1) | ((m & 8) >> 3); }

template <class S> __device__ __forceinline__ S shx(S v, int m) { return __shfl_xor(v, m, 64); }
__device__ __forceinline__ float2 shx(float2 v, int m) {
  return make_float2(__shfl_xor(v.x, m, 64), __shfl_xor(v.y, m, 64));
}
__device__ __forceinline__ double2 shx(double2 v, int m) {
  return make_double2(__shfl_xor(v.x, m, 64), __shfl_xor(v.y, m, 64));
}

template <class S> __device__ __forceinline__ S& cre(S& v) { return v; }
__device__ __forceinline__ float& cre(float2& v) { return v.x; }
__device__ __forceinline__ double& cre(double2& v) { return v.x; }
template <class S> __device__ __forceinline__ S& cim(S& v) { return v; }
__device__ __forceinline__ float& cim(float2& v) { return v.y; }
__device__ __forceinline__ double& cim(double2& v) { return v.y; }

// Lane pl writes its 16 values (register a) to buf[a (P + 1) + pl]; lane
// (a2 = pl mod 16, p1 = pl / 16) reads buf[a2 (P + 1) + p1 + Q p2] into
// register dst(p2).  One scalar component at a time.  LDS operations of a
// wavefront complete in issue order, so the wave barrier only keeps the
// compiler from moving them.
template <int P, int Q, bool REV, class S>
__device__ __forceinline__ void wave_xchg(S* buf, const S (&src)[16], S (&dst)[16], int pl) {
#pragma unroll
  for (int a = 0; a < 16; ++a) buf[a * (P + 1) + pl] = src[a];
  __builtin_amdgcn_wave_barrier();
  const int a2 = pl & 15, p1 = pl >> 4;
  const S* rb = buf + a2 * (P + 1) + p1;
#pragma unroll
  for (int p2 = 0; p2 < 16; ++p2) dst[REV ? rev4(p2) : p2] = rb[Q * p2];
  __builtin_amdgcn_wave_barrier();
}

template <int P, int Q, bool REV, class V, class S>
__device__ __forceinline__ void wave_xchg_v(S* buf, V (&v)[16], int pl) {
  S a[16], b[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) a[i] = cre(v[i]);
  wave_xchg<P, Q, REV>(buf, a, b, pl);
  if constexpr (VT<V>::cplx) {
    S c[16], d[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) c[i] = cim(v[i]);
    wave_xchg<P, Q, REV>(buf, c, d, pl);
#pragma unroll
    for (int i = 0; i < 16; ++i) { cre(v[i]) = b[i]; cim(v[i]) = d[i]; }
  } else {
#pragma unroll
    for (int i = 0; i < 16; ++i) v[i] = b[i];
  }
}


// dit_const<4, 0> with the scheduler kept from interleaving its four levels
// (in FP64 the interleaving makes the compiler hold far more temporaries than
// the 16 values)
template <class V>
__device__ __forceinline__ void dit16_levels(V* x) {
  dit_cpairs<4, 0, 0>(x);
  __builtin_amdgcn_sched_barrier(0);
  dit_cpairs<4, 1, 0>(x);
  __builtin_amdgcn_sched_barrier(0);
  dit_cpairs<4, 2, 0>(x);
  __builtin_amdgcn_sched_barrier(0);
  dit_cpairs<4, 3, 0>(x);
}

// 256-point transforms held by 16 lanes (lane pl, registers v[0..15]) with
// the + sign; xbuf: the group's exchange region (16 x 17 scalars).
// Fourier: lane pl holds x[pl + 16 m] in v[m] on entry and X[pl + 16 r] in
// v[r] on exit; tw(q) returns W_256^q = e^{2 pi i q / 256}.  RECUR: the
// twiddles W_256^{pl a} of register a are the powers of tw(pl) by repeated
// multiplication (FP64 only: an error of a few tens of ulps, two values live
// instead of fifteen) rather than fifteen lookups.
template <bool RECUR = false, class V, class TW>
__device__ __forceinline__ void reg_fft256(V (&v)[16], typename VT<V>::S* xbuf, int pl, TW tw) {
  V r[16];
#pragma unroll
  for (int m = 0; m < 16; ++m) r[rev4(m)] = v[m];
  if constexpr (RECUR) dit16_levels(r);
  else dit_const<4, 0>(r);
  if constexpr (RECUR) {
    const V w1 = tw(pl);
    V w = w1;
#pragma unroll
    for (int a = 1; a < 16; ++a) {
      r[a] = cmul(r[a], w);
      if (a < 15) w = cmul(w, w1);
    }
  } else {
#pragma unroll
    for (int a = 1; a < 16; ++a) r[a] = cmul(r[a], tw(pl * a));
  }
  wave_xchg_v<16, 1, true>(xbuf, r, pl);
  if constexpr (RECUR) dit16_levels(r);
  else dit_const<4, 0>(r);
#pragma unroll
  for (int i = 0; i < 16; ++i) v[i] = r[i];
}

// Hadamard: with the index split into a lane nibble and a register nibble,
// X(j) = sum_k x(k) (-1)^popcount(k & j) leaves the lane and register nibbles
// swapped: an entry index A pl + B m (A, B = 1, 16 or 16, 1) becomes the
// output index A r + B pl.
template <class V>
__device__ __forceinline__ void reg_wht256(V (&v)[16], typename VT<V>::S* xbuf, int pl) {
  wht_block<4, 0>(v);
  wave_xchg_v<16, 1, false>(xbuf, v, pl);
  wht_block<4, 0>(v);
}

}  // namespace fcmp
