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

// ROLE only names the launch for profilers: 0 one workgroup per transform,
// 1 first pass (columns), 2 second pass (rows).
template <class V, bool FFT, int ROLE>
__global__ void __launch_bounds__(256) xform_kernel(XParams p) {
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

  if (itw) {
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
      V v = load_as<V>(p.in, ib + (int64_t)(s0 + c) * p.in_ss + (int64_t)i * p.in_es,
                       p.in_kind);
      if (neg) v = vconj(v);
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
        V v = load_as<V>(p.taps_x, (int64_t)inst * p.inst_taps_x + e, p.in_kind);
        if (neg) v = vconj(v);
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
      lo = go[g * p.goff_span];
      hi = go[(g + 1) * p.goff_span];
    }
    const int32_t* ek = p.ent_k + (int64_t)inst * p.inst_ent;
    const int mask1 = (1 << p.logN1) - 1;
    const int64_t ib = (int64_t)inst * p.inst_in;
    for (int e = lo + tid; e < hi; e += nt) {
      const int k = ek[e];
      const int i = k >> p.logN1;
      const int c = (k & mask1) - s0;
      V v = (p.in_mode == IN_SPARSE_ONES) ? vone<V>() : load_as<V>(p.in, ib + e, p.in_kind);
      if (neg) v = vconj(v);
      const int pos = FFT ? bitrev(i, logL) : i;
      tile[lds_addr(pos * B + c)] = v;
    }
  }
  __syncthreads();

  // ---- transform
  lds_fft<FFT>(tile, L, logL, B, logB, (const V*)p.tws);

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
    for (int e = lo + tid; e < hi; e += nt) {
      const int k = ek[e];
      int c, j;
      if (p.out_es == 1) { j = k & (L - 1); c = (k >> logL) - s0; }
      else { c = (k & esmask) - s0; j = k >> p.log_out_es; }
      V v = tile[lds_addr(j * B + c)];
      if (neg) v = vconj(v);
      v = vscale(v, p.scale);
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
    if (neg) v = vconj(v);
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
