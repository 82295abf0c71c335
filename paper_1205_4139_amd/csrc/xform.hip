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

// In-place natural-order WHT of B interleaved sequences of length L
// (element (i, c) at lds_addr(i*B + c)): radix-4 stages, one radix-2 stage
// when log2 L is odd.
template <class V>
__device__ void lds_wht(V* t, int L, int logL, int B, int logB) {
  const int tid = threadIdx.x, nt = blockDim.x;
  int logh = 0;
  for (; logh + 2 <= logL; logh += 2) {
    const int h = 1 << logh;
    const int ngrp = (B * L) >> 2;
    for (int grp = tid; grp < ngrp; grp += nt) {
      const int c = grp & (B - 1);
      const int q = grp >> logB;
      const int k = q & (h - 1);
      const int base = ((q >> logh) << (logh + 2)) + k;
      const int a0 = lds_addr(base * B + c), a1 = lds_addr((base + h) * B + c);
      const int a2 = lds_addr((base + 2 * h) * B + c), a3 = lds_addr((base + 3 * h) * B + c);
      const V e0 = t[a0], e1 = t[a1], e2 = t[a2], e3 = t[a3];
      const V s01 = vadd(e0, e1), d01 = vsub(e0, e1), s23 = vadd(e2, e3), d23 = vsub(e2, e3);
      t[a0] = vadd(s01, s23);
      t[a1] = vadd(d01, d23);
      t[a2] = vsub(s01, s23);
      t[a3] = vsub(d01, d23);
    }
    __syncthreads();
  }
  if (logh < logL) {
    const int h = 1 << logh;
    const int ngrp = (B * L) >> 1;
    for (int grp = tid; grp < ngrp; grp += nt) {
      const int c = grp & (B - 1);
      const int q = grp >> logB;
      const int k = q & (h - 1);
      const int base = ((q >> logh) << (logh + 1)) + k;
      const int a0 = lds_addr(base * B + c), a1 = lds_addr((base + h) * B + c);
      const V e0 = t[a0], e1 = t[a1];
      t[a0] = vadd(e0, e1);
      t[a1] = vsub(e0, e1);
    }
    __syncthreads();
  }
}

// In-place decimation-in-time DFT with kernel e^{sign 2 pi i j k / L} of B
// interleaved sequences whose elements were placed in bit-reversed order;
// the result is in natural order.  Stage twiddles w_{m}^k = W_N^{k N/m}.
template <class V>
__device__ void lds_fft(V* t, int L, int logL, int B, int logB, const V* lo, const V* hi,
                        int twS, int logN, int sign) {
  const int tid = threadIdx.x, nt = blockDim.x;
  int logh = 0;
  for (; logh + 2 <= logL; logh += 2) {
    const int h = 1 << logh;
    const int sh = logN - logh - 2;
    const int ngrp = (B * L) >> 2;
    for (int grp = tid; grp < ngrp; grp += nt) {
      const int c = grp & (B - 1);
      const int q = grp >> logB;
      const int k = q & (h - 1);
      const int base = ((q >> logh) << (logh + 2)) + k;
      const int a0 = lds_addr(base * B + c), a1 = lds_addr((base + h) * B + c);
      const int a2 = lds_addr((base + 2 * h) * B + c), a3 = lds_addr((base + 3 * h) * B + c);
      const V e0 = t[a0], e1 = t[a1], e2 = t[a2], e3 = t[a3];
      const uint32_t pk = (uint32_t)k << sh;
      const V w2 = tw_lookup(lo, hi, pk, twS, sign);        // w_{4h}^k
      const V w1 = tw_lookup(lo, hi, pk << 1, twS, sign);   // w_{2h}^k
      const V w3 = mul_i(w2, sign);                         // w_{4h}^{k+h}
      const V t1 = cmul(w1, e1), t3 = cmul(w1, e3);
      const V e0p = vadd(e0, t1), e1p = vsub(e0, t1), e2p = vadd(e2, t3), e3p = vsub(e2, t3);
      const V u2 = cmul(w2, e2p), u3 = cmul(w3, e3p);
      t[a0] = vadd(e0p, u2);
      t[a2] = vsub(e0p, u2);
      t[a1] = vadd(e1p, u3);
      t[a3] = vsub(e1p, u3);
    }
    __syncthreads();
  }
  if (logh < logL) {
    const int h = 1 << logh;
    const int sh = logN - logh - 1;
    const int ngrp = (B * L) >> 1;
    for (int grp = tid; grp < ngrp; grp += nt) {
      const int c = grp & (B - 1);
      const int q = grp >> logB;
      const int k = q & (h - 1);
      const int base = ((q >> logh) << (logh + 1)) + k;
      const int a0 = lds_addr(base * B + c), a1 = lds_addr((base + h) * B + c);
      const V e0 = t[a0], e1 = t[a1];
      const V w = tw_lookup(lo, hi, (uint32_t)k << sh, twS, sign);
      const V t1 = cmul(w, e1);
      t[a0] = vadd(e0, t1);
      t[a1] = vsub(e0, t1);
    }
    __syncthreads();
  }
}

// ROLE only names the launch for profilers: 0 one workgroup per transform,
// 1 first pass (columns), 2 second pass (rows).
template <class V, bool FFT, int ROLE>
__global__ void __launch_bounds__(1024) xform_kernel(XParams p) {
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
  if constexpr (FFT) lds_fft<V>(tile, L, logL, B, logB, twlo, twhi, p.twS, p.logN, p.sign);
  else lds_wht<V>(tile, L, logL, B, logB);

  // ---- store / identify
  double bkey = -1.0;
  int64_t bidx = -1;
  const uint32_t* excl = p.excl ? p.excl + (int64_t)inst * p.inst_excl : nullptr;
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
      if (!excl || !bit_is_set(excl, o)) {
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

size_t xform_lds_bytes(int vk, bool fft, int L, int B, int N, int twS) {
  const size_t vb = vbytes(vk);
  const size_t tile_n = (size_t)B * L;
  const size_t tile_alloc = tile_n + (tile_n >> 5) + 1;
  const size_t ntw = fft ? ((size_t)1 << twS) + ((size_t)N >> twS) : 0;
  size_t bytes = (tile_alloc + ntw) * vb;
  bytes = (bytes + 15) & ~(size_t)15;
  bytes += 16 * sizeof(Sel);
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
  const size_t lds = xform_lds_bytes(vk, fft, p.L, p.B, p.N, p.twS);
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
