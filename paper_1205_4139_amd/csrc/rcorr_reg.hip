// Residual (Algorithm 1.1, step 7) fused with the first pass of the next
// correlation (step 2), register-resident, for columns of N2 = 256 rows
// (N = 2^16, 2^17 and 2^18).
//
// The algebra is that of rcorr_kernel: with bucket l of a tap lam (lam mod N2
// for Fourier, lam >> log2 N1 for Hadamard),
//   A(c, l) = sum_{taps in bucket l} x_lam W(lam, c),
//   (U s)[c + N1 m] = N^{-1/2} sum_l A(c, l) e^{-2 pi i l m / N2}   (Fourier)
// (Hadamard: W = (-1)^popcount(lam & c) on the low bits and a WHT over l).
// Here each column is held by 16 lanes of one wavefront, 16 values per lane:
// lane p accumulates A(c, p + 16 a) for a < 16 in registers, the FP64 N2-point
// transform over l runs in registers with one wavefront-private LDS exchange,
// the residual r = y - U s is formed in registers at the rows of Omega the
// lane holds (column masks and rank bases give each row's position in y),
// and the correlation's first pass (the N2-point transform over the rows,
// correlation precision) runs the same way.  A workgroup holds 16 columns
// (four per wavefront); the first-pass outputs are transposed through LDS so
// each output row segment of 16 columns is written as one 128-byte run.
#include "wave_fft.h"

namespace fcmp {

namespace {
constexpr int RR_COLS = 16;    // columns per workgroup
constexpr int RR_TAPS = 256;   // taps staged in LDS per chunk
constexpr int RR_L = 256;      // rows per column (N2)
constexpr int RR_XW = 4 * 16 * 17;   // exchange scalars per wavefront (4 columns)
// region A: the FP64 exchange buffers of four wavefronts, or the output
// tile (256 rows x 17 slots), whichever is larger
constexpr size_t rr_region_a(size_t vc_bytes) {
  return (size_t)4 * RR_XW * 8 > (size_t)RR_L * 17 * vc_bytes ? (size_t)4 * RR_XW * 8
                                                                : (size_t)RR_L * 17 * vc_bytes;
}
}  // namespace

// Four workgroups per CU (four waves per SIMD) when the LDS footprint allows:
// the kernel is latency-bound, so residency matters more than the few
// registers the bound costs.
template <bool FFT, class VC>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4)))
rcorr_reg_kernel(RCParams p) {
  using VR = typename std::conditional<FFT, double2, double>::type;
  using SC = typename VT<VC>::S;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int inst = blockIdx.y;
  if (p.status && p.status[inst].done) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int col = tid >> 4;           // column within the workgroup
  const int pl = tid & 15;            // lane within the column's group
  const int grp = lane >> 4;          // column within the wavefront
  const int s0 = blockIdx.x * RR_COLS;
  const uint32_t cg = (uint32_t)(s0 + col);
  const uint32_t maskN = (uint32_t)p.N - 1u;
  const uint32_t mask1 = (1u << p.logN1) - 1u;
  const int dsh = p.logN1 - 8;        // W_256^q = W_N1^(q << dsh)
  const int ntaps = p.tofs ? p.ntaps - p.tofs[inst] : p.ntaps;
  if (p.Kv && ntaps >= p.Kv[inst]) return;   // its K selections are made

  // LDS: region A (staged taps; then the exchange buffers; then the output
  // tile), then W_N1^q in FP64 (the tap sums' factors, and, rounded to the
  // correlation precision, the twiddles of the first-pass transform)
  constexpr size_t bytesA = rr_region_a(sizeof(VC));
  int32_t* tl = (int32_t*)smem_raw;
  VR* tx = (VR*)(smem_raw + RR_TAPS * 4);
  int32_t* bsl = (int32_t*)(smem_raw + RR_TAPS * (4 + sizeof(VR)));
  double* xr = (double*)smem_raw + wave * RR_XW + grp * (16 * 17);
  SC* xc = (SC*)((double*)smem_raw + wave * RR_XW) + grp * (16 * 17);
  VC* tile = (VC*)smem_raw;
  const int nhi = p.N >> p.twS;       // N1
  double2* t1 = (double2*)(smem_raw + bytesA);

  // Global loads with no dependence on this workgroup's LDS are issued first,
  // so their latencies overlap: the first chunk of taps and the tables.  The
  // column masks and the per-register twiddle factors are loaded after the
  // tap sums (fewer registers live during them).
  const int32_t* bs = p.bstart + (int64_t)inst * p.inst_bstart + (ntaps & 1) * p.bstart_half;
  const int32_t* od = p.ord + (int64_t)inst * p.inst_ord + (ntaps & 1) * p.ord_half;
  const int32_t* lm = p.lam + (int64_t)inst * p.inst_lam;
  const VR* xs = (const VR*)p.x + (int64_t)inst * p.inst_x;
  int tlv0 = 0;
  VR txv0 = vzero(VR());
  if (ntaps > 0) {
    const int tau = od[min(tid, ntaps - 1)];
    tlv0 = lm[tau];
    txv0 = xs[tau];
  }
  for (int b = tid; b <= RR_L; b += 256) bsl[b] = ntaps > 0 ? bs[b] : 0;
  if constexpr (FFT) {
    const double2* g1 = (const double2*)p.twr_hi;   // W_N^{q N2} = W_N1^q
    for (int e = tid; e < nhi; e += 256) t1[e] = g1[e];
  }

  // ---- A(c, l) for l = pl + 16 a, a < 16, summed over the bucket's taps in
  // bucket order (FP64; stored conjugated for the Fourier class, whose
  // transform core runs with the + sign).  Fourier: with lam = l + N2 lam2,
  //   conj(A(c, l)) = W_N^{l c} sum_taps conj(x) W_N1^{lam2 c}   (W_n = e^{+2 pi i / n}),
  // so a tap costs one lookup in the N1-entry table and one multiply-add; the
  // factor W_N^{l c} is applied once per register afterwards.
  VR acc[16];
#pragma unroll
  for (int a = 0; a < 16; ++a) acc[a] = vzero(VR());
  const uint32_t mask1n = (uint32_t)nhi - 1u;   // N1 - 1
  for (int i0 = 0; i0 < ntaps; i0 += RR_TAPS) {
    const int nc = min(RR_TAPS, ntaps - i0);
    __syncthreads();   // tables staged; the previous chunk is consumed
    if (tid < nc) {
      int lv;
      VR xv;
      if (i0 == 0) {
        lv = tlv0;
        xv = txv0;
      } else {
        const int tau = od[i0 + tid];
        lv = lm[tau];
        xv = xs[tau];
      }
      tl[tid] = FFT ? (lv >> p.twS) : lv;   // Fourier: lam2 = lam / N2
      tx[tid] = xv;
    }
    __syncthreads();
    // the first tap of every bucket for the 16 registers at once (independent
    // lookups in flight; an empty bucket adds a zero), then the rest of each
    // bucket in order
    auto add_tap = [&](VR& ac, int li, bool on) {
      const uint32_t lv = (uint32_t)tl[li];
      VR xv = tx[li];
      if (!on) xv = vzero(VR());
      if constexpr (FFT) {
        const double2 w = t1[(lv * cg) & mask1n];
        ac.x += xv.x * w.x + xv.y * w.y;   // conj(x) w
        ac.y += xv.x * w.y - xv.y * w.x;
      } else {
        ac += (__popc(lv & mask1 & cg) & 1) ? -xv : xv;
      }
    };
#pragma unroll
    for (int a0 = 0; a0 < 16; a0 += 4) {
      int ib[4], ie[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int l = pl + 16 * (a0 + u);
        ib[u] = max(bsl[l], i0) - i0;
        ie[u] = min(bsl[l + 1], i0 + nc) - i0;
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) add_tap(acc[a0 + u], min(ib[u], nc - 1), ib[u] < ie[u]);
#pragma unroll
      for (int u = 0; u < 4; ++u)
        for (int i = ib[u] + 1; i < ie[u]; ++i) add_tap(acc[a0 + u], i, true);
      __builtin_amdgcn_sched_barrier(0);
    }
  }
  const uint32_t* cm = p.cmask + (int64_t)inst * p.inst_cmask + (int64_t)cg * 8;
  const int32_t* cb = p.cbase + (int64_t)inst * p.inst_cmask + (int64_t)cg * 8;
  uint32_t mwv[FFT ? 8 : 1];
  int32_t bwv[FFT ? 8 : 1];
#pragma unroll
  for (int w = 0; w < (FFT ? 8 : 1); ++w) {
    mwv[w] = cm[FFT ? w : (pl >> 1)];
    bwv[w] = cb[FFT ? w : (pl >> 1)];
  }
  // W_N^{pl c} and W_N^{16 c} (FP64): the powers W_N^{(pl + 16 a) c} are
  // both the factor of register a of the tap sums and the inter-pass
  // twiddle of output j2 = pl + 16 a (loaded twice rather than held)
  auto lane_twiddles = [&](double2& w0, double2& w16) {
    const double2* rlo = (const double2*)p.twr_lo;
    const double2* rhi = (const double2*)p.twr_hi;
    const uint32_t lomask = (1u << p.twS) - 1u;
    const uint32_t q0 = ((uint32_t)pl * cg) & maskN, q1 = (16u * cg) & maskN;
    w0 = cmul(rhi[q0 >> p.twS], rlo[q0 & lomask]);
    w16 = cmul(rhi[q1 >> p.twS], rlo[q1 & lomask]);
  };
  if constexpr (FFT) {
    // the factor W_N^{l c}, powers by repeated multiplication (FP64)
    double2 wl0, wl16;
    lane_twiddles(wl0, wl16);
    double2 w = wl0;
#pragma unroll
    for (int a = 0; a < 16; ++a) {
      acc[a] = cmul(acc[a], w);
      if (a < 15) w = cmul(w, wl16);
    }
  }
  __syncthreads();   // taps consumed: region A becomes the exchange buffers

  // ---- FP64 transform over l: Fourier, lane pl ends with the rows
  // m = pl + 16 r; Hadamard (l = pl + 16 a in, nibbles swap) m = r + 16 pl
  if constexpr (FFT) {
    reg_fft256<true>(acc, xr, pl, [&](int q) { return t1[q << dsh]; });
  } else {
    reg_wht256(acc, xr, pl);
  }

  // ---- r = y - N^{-1/2} U s at the rows of Omega among the lane's 16 rows.
  // Column masks: bit m of word m / 32 of column c says whether row c + N1 m
  // is in Omega; the rank base of that word is the position in y of the
  // first such row at or after 32 (m / 32).
  const VR* yv = (const VR*)p.y + (int64_t)inst * p.inst_y;
  const int ylast = (int)p.inst_y - 1;   // y holds inst_y >= M slots per instance
  VC rc[16];
  // four rows at a time, the loads of each group not hoisted above the
  // previous one (fewer registers live beside the 16 FP64 values)
#pragma unroll
  for (int h = 0; h < 4; ++h) {
    __builtin_amdgcn_sched_barrier(0);
    VR yy[4];
    bool pres[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int r = 4 * h + u;
      const int m = FFT ? pl + 16 * r : r + 16 * pl;
      const int w = FFT ? (m >> 5) : 0;
      const uint32_t mw = mwv[w];
      const uint32_t bit = (uint32_t)(m & 31);
      pres[u] = (mw >> bit) & 1u;
      // unconditional load (rows not in Omega read a valid neighbour, and
      // their value is discarded), so no branch splits the groups
      const int rank = bwv[w] + __popc(mw & ((1u << bit) - 1u));
      yy[u] = yv[min(rank, ylast)];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int r = 4 * h + u;
      VR X = acc[r];
      if constexpr (FFT) X = vconj(X);
      const VR rr = vsub(yy[u], vscale(X, p.rscale));
      rc[r] = pres[u] ? vnarrow(rr, VC()) : vzero(VC());
    }
  }

  // ---- the correlation's first pass over the rows, + sign.  Fourier: rows
  // m = pl + 16 r in, outputs j2 = pl + 16 r; Hadamard: rows m = r + 16 pl
  // in, outputs j2 = pl + 16 r
  double2 wj = make_double2(1.0, 0.0), wj16 = wj;
  if constexpr (FFT) {
    lane_twiddles(wj, wj16);
    // W_256^q rounded from FP64 (the same values as a table built in the
    // correlation precision: every entry rounds once to the same float)
    reg_fft256(rc, xc, pl, [&](int q) { return vnarrow(t1[q << dsh], VC()); });
  } else {
    reg_wht256(rc, xc, pl);
  }
  __syncthreads();   // every exchange is done: region A becomes the output tile
  // wj: W_N^{c j2}, powers in FP64, rounded once per output
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int j2 = pl + 16 * r;
    VC v = rc[r];
    if constexpr (FFT) {
      v = cmul(v, vnarrow(wj, VC()));
      if (r < 15) wj = cmul(wj, wj16);
    }
    tile[j2 * 17 + col] = v;
  }
  __syncthreads();
  VC* out = (VC*)p.out + (int64_t)inst * p.inst_out;
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    const int e = tid + 256 * k;
    const int j2 = e >> 4, c = e & 15;
    out[(int64_t)(s0 + c) + ((int64_t)j2 << p.logN1)] = tile[j2 * 17 + c];
  }
}

bool rcorr_reg_ok(int pk, bool fft, const RCParams& p) {
  return p.L == RR_L && p.logN1 >= 8 && p.logN1 <= 10 && p.cmask && p.cbase &&
         (fft ? (pk == V_C64 || pk == V_C128) : (pk == V_F32 || pk == V_F64));
}

static size_t rcorr_reg_lds(int pk, bool fft, const RCParams& p) {
  const size_t bytesA = rr_region_a(vbytes(pk));
  const size_t t1b = fft ? ((size_t)p.N >> p.twS) * 16 : 0;
  return bytesA + t1b;
}

template <bool FFT, class VC>
static hipError_t launch_rr(const RCParams& p, int ninst, size_t lds, hipStream_t st) {
  auto kfn = rcorr_reg_kernel<FFT, VC>;
  hipError_t e = raise_lds_limit((const void*)kfn, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(kfn, dim3((1 << p.logN1) / RR_COLS, ninst), dim3(256), lds, st, p);
  return hipGetLastError();
}

hipError_t launch_rcorr_reg(int pk, bool fft, const RCParams& p, int ninst, hipStream_t st) {
  if (!rcorr_reg_ok(pk, fft, p)) return hipErrorInvalidValue;
  const size_t lds = rcorr_reg_lds(pk, fft, p);
  if (fft) {
    if (pk == V_C64) return launch_rr<true, float2>(p, ninst, lds, st);
    return launch_rr<true, double2>(p, ninst, lds, st);
  }
  if (pk == V_F32) return launch_rr<false, float>(p, ninst, lds, st);
  return launch_rr<false, double>(p, ninst, lds, st);
}

}  // namespace fcmp
