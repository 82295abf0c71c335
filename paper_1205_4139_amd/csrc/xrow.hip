// Second pass of a two-pass correlation transform (rows of length
// L = N1 = 256 Q, Q = 1, 2, 4) with the identification argmax of Algorithm
// 1.1 step 3 fused: the outputs h(j) are never stored, each workgroup writes
// its best (|h|^2, index) over the columns not yet selected.
//
// A row is held by P = 16 Q lanes of one wavefront, 16 values per lane, and
// transformed in registers.  With the row index k = p + P m (lane p,
// register m), p = p1 + Q p2 and the output j = a + 16 b, b = b1 + 16 b2:
//   Fourier (W_n = e^{+2 pi i / n}):
//     Y_p[a]  = sum_m x[p + P m] W_16^{m a}            16 points in registers
//     Y_p[a] *= W_L^{p a}
//     Z[b1]   = sum_p2 Y_{p1 + Q p2}[a] W_16^{p2 b1}    after a wave-private LDS
//                                                       exchange, in registers
//     Z[b1]  *= W_L^{16 p1 b1}
//     X[a + 16 b1 + 256 b2] = sum_p1 Z_p1[b1] W_Q^{p1 b2}   across the Q lanes
//                                                       by wavefront shuffles
//   Hadamard: the same split with (-1)^popcount in place of every W and no
//   twiddles (popcount(k & j) is the sum of the popcounts of the bit groups).
// The transposition needs no workgroup barrier: each wavefront exchanges
// through its own LDS region.  Row lengths that need more than one
// wavefront per row, and passes that store their outputs, use xform_kernel.
#include "wave_fft.h"

namespace fcmp {


template <class V, bool FFT, int Q>
__global__ void __launch_bounds__(256) xrow_kernel(XParams p) {
  using S = typename VT<V>::S;
  constexpr int P = 16 * Q;           // lanes per row
  constexpr int GPW = 4 / Q;          // rows per wavefront
  constexpr int RPB = 4 * GPW;        // rows per workgroup (four wavefronts)
  constexpr int BUFW = GPW * 16 * (P + 1);
  constexpr int L = 256 * Q;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int inst = blockIdx.y;
  if (p.status && p.status[inst].done) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int grp = lane / P, pl = lane % P;
  const int row = blockIdx.x * RPB + wave * GPW + grp;
  S* xbuf = (S*)smem_raw + wave * BUFW + grp * 16 * (P + 1);
  V* twl = (V*)((S*)smem_raw + 4 * BUFW);
  uint32_t* xws = (uint32_t*)(twl + (FFT ? L : 0));
  Sel* red = (Sel*)(((uintptr_t)(xws + (FFT ? L : RPB * (L / 32))) + 15) & ~(uintptr_t)15);

  // ---- loads: lane pl takes x[pl + P m], m < 16 (P consecutive values of
  // the row per load), and the exclusion words of its 16 outputs
  const V* in = (const V*)p.in + (int64_t)inst * p.inst_in + (int64_t)row * p.in_ss;
  V x[16];
#pragma unroll
  for (int m = 0; m < 16; ++m) x[m] = in[pl + P * m];
  const int a2 = pl & 15, p1 = pl >> 4;
  // output j1 of register r (see the header): Fourier a2 + 16 r + 256 b2(p1),
  // Hadamard a1(p1) + Q r + P a2
  int j1base, j1step;
  if constexpr (FFT) {
    const int b2 = Q == 4 ? ((p1 >> 1) + 2 * (p1 & 1)) : p1;
    j1base = a2 + 256 * b2;
    j1step = 16;
  } else {
    j1base = p1 + P * a2;
    j1step = Q;
  }
  // exclusion words of the workgroup's outputs, staged in LDS (the rows of a
  // workgroup lie in one block of 32): Fourier o = row + N2 j1, one word per
  // j1; Hadamard o = row L + j1, L / 32 words per row
  const uint32_t* ex = p.excl ? p.excl + (int64_t)inst * p.inst_excl : nullptr;
  const int row0 = blockIdx.x * RPB;
  const int n2 = p.N / L;
  constexpr int NXW = FFT ? L : RPB * (L / 32);
  for (int e = tid; e < NXW; e += 256) {
    const int64_t w = FFT ? (int64_t)(row0 >> 5) + (int64_t)(n2 >> 5) * e
                          : (int64_t)row0 * (L / 32) + e;
    xws[e] = ex ? ex[w] : 0u;
  }
  if constexpr (FFT) {
    const V* hi = (const V*)p.tw_hi;   // W_N^{q N2} = W_L^q for q < L
    for (int e = tid; e < L; e += 256) twl[e] = hi[e];
  }
  __syncthreads();
  if (p.sign < 0) {
#pragma unroll
    for (int m = 0; m < 16; ++m) x[m] = vconj(x[m]);
  }

  V s[16];
  if constexpr (FFT) {
    V r[16];
#pragma unroll
    for (int m = 0; m < 16; ++m) r[rev4(m)] = x[m];
    dit_const<4, 0>(r);
#pragma unroll
    for (int a = 1; a < 16; ++a) r[a] = cmul(r[a], twl[pl * a]);
    wave_xchg_v<P, Q, true>(xbuf, r, pl);
#pragma unroll
    for (int i = 0; i < 16; ++i) s[i] = r[i];
    dit_const<4, 0>(s);
    if constexpr (Q > 1) {
#pragma unroll
      for (int b1 = 1; b1 < 16; ++b1) s[b1] = cmul(s[b1], twl[16 * p1 * b1]);
    }
    if constexpr (Q == 2) {
#pragma unroll
      for (int b1 = 0; b1 < 16; ++b1) {
        const V o = shx(s[b1], 16);
        s[b1] = p1 == 0 ? vadd(s[b1], o) : vsub(o, s[b1]);
      }
    } else if constexpr (Q == 4) {
      const int plo = p1 & 1, phi = p1 >> 1;
#pragma unroll
      for (int b1 = 0; b1 < 16; ++b1) {
        V o = shx(s[b1], 32);
        const V e = phi == 0 ? vadd(s[b1], o) : vsub(o, s[b1]);
        o = shx(e, 16);
        const V e1 = plo ? e : o, e0 = plo ? o : e;
        const V t = phi ? mul_i(e1, +1) : e1;
        s[b1] = plo ? vsub(e0, t) : vadd(e0, t);
      }
    }
  } else {
#pragma unroll
    for (int m = 0; m < 16; ++m) s[m] = x[m];
    wht_block<4, 0>(s);
    wave_xchg_v<P, Q, false>(xbuf, s, pl);
    wht_block<4, 0>(s);
    if constexpr (Q >= 2) {
      if constexpr (Q == 4) {
        const int phi = p1 >> 1;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const V o = shx(s[r], 32);
          s[r] = phi == 0 ? vadd(s[r], o) : vsub(o, s[r]);
        }
      }
      const int plo = p1 & 1;
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const V o = shx(s[r], 16);
        s[r] = plo == 0 ? vadd(s[r], o) : vsub(o, s[r]);
      }
    }
  }

  // ---- identification over the lane's 16 outputs (keys |v|^2 unscaled in
  // the transform precision; the winner's key is scaled once)
  using KT = decltype(kmag2r(V()));
  KT bkey = (KT)-1, bkey2 = (KT)-1;
  int64_t bidx = -1;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int j1 = j1base + j1step * r;
    const int o = FFT ? row + n2 * j1 : row * L + j1;
    const uint32_t xw = FFT ? xws[j1] : xws[(row - row0) * (L / 32) + (j1 >> 5)];
    if (!((xw >> (o & 31)) & 1u)) sel_add(kmag2r(s[r]), (int64_t)o, bkey, bidx, bkey2);
  }
  const double s2 = p.scale * p.scale;
  const double key = bidx >= 0 ? (double)bkey * s2 : -1.0;
  const double key2 = bkey2 >= (KT)0 ? (double)bkey2 * s2 : -1.0;
  const Sel sel = block_sel_reduce(key, bidx, key2, red);
  if (tid == 0) p.partial[(int64_t)inst * p.inst_part + blockIdx.x] = sel;
}

int xrow_q(const XParams& b) {
  if (!b.partial || b.out_kind >= 0 || b.out2_kind >= 0 || b.resid || b.in_mode != IN_DENSE ||
      b.in_es != 1 || b.in_ss != b.L)
    return 0;
  const int q = b.L == 256 ? 1 : b.L == 512 ? 2 : b.L == 1024 ? 4 : 0;
  if (!q) return 0;
  const int n2 = b.N / b.L;
  return (n2 % (16 / q) == 0) ? q : 0;
}

int xrow_groups(const XParams& b) {
  const int q = xrow_q(b);
  return q ? (b.N / b.L) / (16 / q) : 0;
}

static size_t xrow_lds_bytes(int vk, bool fft, int q) {
  const size_t sb = (vk == V_F32 || vk == V_C64) ? 4 : 8;
  const size_t P = 16 * q;
  size_t bytes = 4 * (4 / q) * 16 * (P + 1) * sb;
  if (fft) bytes += (size_t)256 * q * vbytes(vk) + (size_t)256 * q * 4;
  else bytes += (size_t)(16 / q) * (256 * q / 32) * 4;
  bytes = (bytes + 15) & ~(size_t)15;
  return bytes + 16 * sizeof(Sel);
}

template <class V, bool FFT, int Q>
static hipError_t launch_xr(const XParams& b, int ninst, size_t lds, hipStream_t st) {
  auto kfn = xrow_kernel<V, FFT, Q>;
  hipError_t e = raise_lds_limit((const void*)kfn, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(kfn, dim3(xrow_groups(b), ninst), dim3(256), lds, st, b);
  return hipGetLastError();
}

template <class V, bool FFT>
static hipError_t launch_xq(const XParams& b, int q, int ninst, size_t lds, hipStream_t st) {
  if (q == 1) return launch_xr<V, FFT, 1>(b, ninst, lds, st);
  if (q == 2) return launch_xr<V, FFT, 2>(b, ninst, lds, st);
  return launch_xr<V, FFT, 4>(b, ninst, lds, st);
}

hipError_t launch_xrow(int vk, bool fft, const XParams& b, int ninst, hipStream_t st) {
  const int q = xrow_q(b);
  if (!q) return hipErrorInvalidValue;
  const size_t lds = xrow_lds_bytes(vk, fft, q);
  if (fft) {
    if (vk == V_C64) return launch_xq<float2, true>(b, q, ninst, lds, st);
    if (vk == V_C128) return launch_xq<double2, true>(b, q, ninst, lds, st);
  } else {
    if (vk == V_F32) return launch_xq<float, false>(b, q, ninst, lds, st);
    if (vk == V_F64) return launch_xq<double, false>(b, q, ninst, lds, st);
  }
  return hipErrorInvalidValue;
}

}  // namespace fcmp
