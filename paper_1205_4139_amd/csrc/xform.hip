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
#include "lds_fft.h"

namespace fcmp {

// Identification key type: |h|^2 in the correlation precision.
template <class V> struct KeyOf { using T = double; };
template <> struct KeyOf<float> { using T = float; };
template <> struct KeyOf<float2> { using T = float; };
__device__ __forceinline__ float kmag2(float v) { return v * v; }
__device__ __forceinline__ float kmag2(float2 v) { return v.x * v.x + v.y * v.y; }
__device__ __forceinline__ double kmag2(double v) { return v * v; }
__device__ __forceinline__ double kmag2(double2 v) { return v.x * v.x + v.y * v.y; }

// ROLE: 0 one workgroup per transform, 1 first pass (columns), 2 second pass
// (rows; dense input, so the Fourier core runs transposed: natural input,
// bit-reversed output positions).
template <class V, bool FFT, int ROLE>
__global__ void __launch_bounds__(256) xform_kernel(XParams p) {
  constexpr bool DIF = FFT && ROLE == 2;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int inst = blockIdx.y;
  if (p.status && p.status[inst].done) return;
  if (p.rsel_M && (double)p.rsel_M[inst] * (double)p.rsel_ntaps <= p.rsel_thr) return;
  const int tid = threadIdx.x, nt = blockDim.x;
  const int g = blockIdx.x;
  const int B = p.B, L = p.L, logL = p.logL;
  const int logB = __ffs(B) - 1;
  const int s0 = g * B;
  const int tile_n = B * L;
  const int tile_alloc = tile_n + (tile_n >> 5) + 1;
  V* tile = (V*)smem_raw;
  V* twlo = tile + tile_alloc;
  const bool itw = FFT && p.inter_tw;
  const int nlo = itw ? (1 << p.twS) : 0;
  const int nhi = itw ? (p.N >> p.twS) : 0;
  V* twhi = twlo + nlo;
  Sel* red = (Sel*)(((uintptr_t)(twhi + nhi) + 15) & ~(uintptr_t)15);
  const bool neg = p.sign < 0;   // conj(F(conj x)): the core runs with the + sign

  // Global loads are issued XU at a time (from clamped, always valid
  // addresses) before their LDS writes, so each thread waits for memory once
  // per batch rather than once per element.
  constexpr int XU = sizeof(V) >= 16 ? 4 : 8;
  // inter-pass twiddles: the first two per thread are loaded now (clamped
  // indices, so the loads are unconditional) and stored with the inputs
  const V* glo = (const V*)p.tw_lo;
  const V* ghi = (const V*)p.tw_hi;
  const int ntw = nlo + nhi;
  V tw0 = vzero(V()), tw1 = vzero(V());
  if (itw) {
    const int e0 = min(tid, ntw - 1), e1 = min(tid + nt, ntw - 1);
    tw0 = e0 < nlo ? glo[e0] : ghi[e0 - nlo];
    tw1 = e1 < nlo ? glo[e1] : ghi[e1 - nlo];
  }

  // the exclusion words the identification needs: the first one per thread
  // is loaded now, in flight with the input loads, and written to LDS with
  // them (the transform's barriers order it before its use)
  const uint32_t* excl = p.excl ? p.excl + (int64_t)inst * p.inst_excl : nullptr;
  uint32_t* xw = (uint32_t*)(red + 16);
  int64_t xbase = 0, xstride = 1;
  int nxw = 0;
  if (p.partial && excl && p.excl_mode == 1) {
    const int64_t o0 = (int64_t)s0 * p.out_ss;
    xbase = o0 >> 5;
    nxw = (int)(((o0 + tile_n - 1) >> 5) - xbase + 1);
  } else if (p.partial && excl && p.excl_mode == 2) {
    xbase = s0 >> 5;
    xstride = p.out_es >> 5;
    nxw = L;
  }
  uint32_t xw0 = 0;
  if (tid < nxw) xw0 = excl[xbase + (int64_t)tid * xstride];

  // ---- load
  if (p.in_mode == IN_DENSE) {
    const int64_t ib = (int64_t)inst * p.inst_in;
    for (int e0 = tid; e0 < tile_n; e0 += nt * XU) {
      V v[XU];
      int a[XU];
#pragma unroll
      for (int u = 0; u < XU; ++u) {
        const int e = min(e0 + u * nt, tile_n - 1);
        int c, i;
        if (p.in_es == 1) { c = e >> logL; i = e & (L - 1); }
        else { c = e & (B - 1); i = e >> logB; }
        v[u] = load_as<V>(p.in, ib + (int64_t)(s0 + c) * p.in_ss + (int64_t)i * p.in_es,
                          p.in_kind);
        const int pos = (FFT && !DIF) ? bitrev(i, logL) : i;
        a[u] = lds_addr(pos * B + c);
      }
#pragma unroll
      for (int u = 0; u < XU; ++u) {
        if (e0 + u * nt < tile_n) tile[a[u]] = neg ? vconj(v[u]) : v[u];
      }
    }
  } else if (p.in_mode == IN_TAPS) {
    // zero-filled sparse vector S_Lambda^T x: this workgroup keeps the taps
    // whose column falls in its sequences
    const V z = vzero(V());
    for (int e = tid; e < tile_alloc; e += nt) tile[e] = z;
    __syncthreads();
    const int32_t* tl = p.taps_lam + (int64_t)inst * p.inst_taps_lam;
    const int mask1 = (1 << p.logN1) - 1;
    for (int e0 = tid; e0 < p.ntaps; e0 += nt * XU) {
      int kk[XU];
#pragma unroll
      for (int u = 0; u < XU; ++u) {
        const int e = e0 + u * nt;
        kk[u] = tl[min(e, p.ntaps - 1)];
        if (e >= p.ntaps) kk[u] = -1;
      }
      V v[XU];
#pragma unroll
      for (int u = 0; u < XU; ++u)
        v[u] = load_as<V>(p.taps_x, (int64_t)inst * p.inst_taps_x + min(e0 + u * nt, p.ntaps - 1),
                          p.in_kind);
#pragma unroll
      for (int u = 0; u < XU; ++u) {
        const int c = (kk[u] & mask1) - s0;
        if (kk[u] >= 0 && c >= 0 && c < B) {
          const int i = kk[u] >> p.logN1;
          const int pos = FFT ? bitrev(i, logL) : i;
          tile[lds_addr(pos * B + c)] = neg ? vconj(v[u]) : v[u];
        }
      }
    }
  } else {
    const V z = vzero(V());
    for (int e = tid; e < tile_alloc; e += nt) tile[e] = z;
    __syncthreads();
    int lo = 0, hi = p.nent;
    if (p.goff) {
      const int32_t* go = p.goff + (int64_t)inst * p.inst_goff;
      lo = go[g * p.goff_span];
      hi = go[(g + 1) * p.goff_span];
    }
    const int32_t* ek = p.ent_k + (int64_t)inst * p.inst_ent;
    const int mask1 = (1 << p.logN1) - 1;
    const int64_t ib = (int64_t)inst * p.inst_in;
    const bool ones = p.in_mode == IN_SPARSE_ONES;
    for (int e0 = lo + tid; e0 < hi; e0 += nt * XU) {
      int kk[XU];
      V v[XU];
#pragma unroll
      for (int u = 0; u < XU; ++u) {
        const int e = min(e0 + u * nt, hi - 1);
        kk[u] = ek[e];
        v[u] = ones ? vone<V>() : load_as<V>(p.in, ib + e, p.in_kind);
      }
#pragma unroll
      for (int u = 0; u < XU; ++u) {
        if (e0 + u * nt < hi) {
          const int i = kk[u] >> p.logN1;
          const int c = (kk[u] & mask1) - s0;
          const int pos = FFT ? bitrev(i, logL) : i;
          tile[lds_addr(pos * B + c)] = neg ? vconj(v[u]) : v[u];
        }
      }
    }
  }
  if (itw) {
    twlo[min(tid, ntw - 1)] = tw0;   // twhi follows twlo contiguously
    twlo[min(tid + nt, ntw - 1)] = tw1;
    for (int e = tid + 2 * nt; e < ntw; e += nt) twlo[e] = e < nlo ? glo[e] : ghi[e - nlo];
  }
  if (tid < nxw) xw[tid] = xw0;
  for (int e = tid + nt; e < nxw; e += nt) xw[e] = excl[xbase + (int64_t)e * xstride];
  __syncthreads();

  // ---- transform
  lds_fft<FFT, DIF>(tile, L, logL, B, logB, (const V*)p.tws);

  // ---- residual output: r = y - (S_Omega U s) at the rows of Phi this
  // workgroup produced (forward transform of the support, Algorithm 1.1 step 7)
  if (p.resid) {
    int lo = 0, hi = p.nent2;
    if (p.goff2) {
      const int32_t* go = p.goff2 + (int64_t)inst * p.inst_goff2;
      lo = go[g * p.goff2_span];
      hi = go[(g + 1) * p.goff2_span];
    }
    const int32_t* ek = p.ent2_k + (int64_t)inst * p.inst_ent2;
    const int32_t* pos1 = p.pos1 ? p.pos1 + (int64_t)inst * p.inst_ent2 : nullptr;
    const int esmask = (1 << p.log_out_es) - 1;
    constexpr int RU = sizeof(V) >= 16 ? 2 : 4;
    for (int e0 = lo + tid; e0 < hi; e0 += nt * RU) {
      int kk[RU], qq[RU];
#pragma unroll
      for (int u = 0; u < RU; ++u) {
        const int e = min(e0 + u * nt, hi - 1);
        kk[u] = ek[e];
        qq[u] = pos1 ? pos1[e] : e;
      }
      V yv[RU];
#pragma unroll
      for (int u = 0; u < RU; ++u)
        yv[u] = load_as<V>(p.yres, (int64_t)inst * p.inst_yres + qq[u], p.yres_kind);
#pragma unroll
      for (int u = 0; u < RU; ++u) {
        if (e0 + u * nt < hi) {
          const int k = kk[u];
          int c, j;
          if (p.out_es == 1) { j = k & (L - 1); c = (k >> logL) - s0; }
          else { c = (k & esmask) - s0; j = k >> p.log_out_es; }
          V v = tile[lds_addr((DIF ? bitrev(j, logL) : j) * B + c)];
          if (neg) v = vconj(v);
          v = vscale(v, p.scale);
          store_as(p.rout, (int64_t)inst * p.inst_rout + qq[u], p.r_kind, vsub(yv[u], v));
        }
      }
    }
    return;
  }

  // ---- store / identify (keys |v|^2 unscaled in the transform precision;
  // the winner's key is scaled once at the end)
  using KT = typename KeyOf<V>::T;
  KT bkey = (KT)-1, bkey2 = (KT)-1;
  int64_t bidx = -1;
  const bool store = p.out_kind >= 0 || p.out2_kind >= 0;
  const int out_ss = (int)p.out_ss, out_es = (int)p.out_es;
  for (int e = tid; e < tile_n; e += nt) {
    int c, j, pos;
    if (out_es == 1) {
      c = e >> logL; j = e & (L - 1);
      pos = DIF ? bitrev(j, logL) : j;
    } else {
      c = e & (B - 1);
      const int q = e >> logB;
      // transposed core: walk the LDS positions (conflict-free) unless the
      // values are stored, then walk the outputs (coalesced)
      if (DIF && !store) { pos = q; j = bitrev(q, logL); }
      else { j = q; pos = DIF ? bitrev(q, logL) : q; }
    }
    V v = tile[lds_addr(pos * B + c)];
    if (neg) v = vconj(v);
    if constexpr (FFT) {
      if (p.inter_tw) {
        const uint32_t q = ((uint32_t)(s0 + c) * (uint32_t)j) & (uint32_t)(p.N - 1);
        v = cmul(v, tw_lookup(twlo, twhi, q, p.twS, p.sign));
      }
    }
    const int o = (s0 + c) * out_ss + j * out_es;   // < N <= 2^24
    if (store) {
      const V vs = vscale(v, p.scale);
      if (p.out_kind >= 0) store_as(p.out, (int64_t)inst * p.inst_out + o, p.out_kind, vs);
      if (p.out2_kind >= 0) store_as(p.out2, (int64_t)inst * p.inst_out2 + o, p.out2_kind, vs);
    }
    if (p.partial) {
      bool ex = false;
      if (excl) {
        if (p.excl_mode == 1) ex = (xw[(o >> 5) - xbase] >> (o & 31)) & 1u;
        else if (p.excl_mode == 2) ex = (xw[j] >> ((s0 + c) & 31)) & 1u;
        else ex = bit_is_set(excl, o);
      }
      if (!ex) sel_add(kmag2(v), (int64_t)o, bkey, bidx, bkey2);
    }
  }
  if (p.partial) {
    const double s2 = p.scale * p.scale;
    const double key = bidx >= 0 ? (double)bkey * s2 : -1.0;
    const double key2 = bkey2 >= (KT)0 ? (double)bkey2 * s2 : -1.0;
    const Sel r = block_sel_reduce(key, bidx, key2, red);
    if (tid == 0) p.partial[(int64_t)inst * p.inst_part + g] = r;
  }
}

size_t xform_lds_bytes(int vk, bool fft, const XParams& p) {
  const size_t vb = vbytes(vk);
  const size_t tile_n = (size_t)p.B * p.L;
  const size_t tile_alloc = tile_n + (tile_n >> 5) + 1;
  const size_t ntw = (fft && p.inter_tw) ? ((size_t)1 << p.twS) + ((size_t)p.N >> p.twS) : 0;
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
  hipError_t e = raise_lds_limit((const void*)kfn, lds);
  if (e != hipSuccess) return e;
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
