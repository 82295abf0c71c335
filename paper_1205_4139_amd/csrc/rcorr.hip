// Residual (Algorithm 1.1, step 7) fused with the first pass of the next
// correlation (step 2), for transforms too long for one workgroup.
//
// The correlation's first pass owns the rows k = c + N1 m of Phi^H's input
// with c in a block of B classes mod N1 (m < N2).  The residual at exactly
// those rows needs only the taps:
//   Fourier:  (U s)[c + N1 m] = N^{-1/2} sum_{l < N2} A(c, l) e^{-2 pi i l m / N2},
//             A(c, l) = sum over taps lam = l (mod N2) of x_lam e^{-2 pi i lam c / N};
//   Hadamard: (U s)[c + N1 m] = N^{-1/2} sum_{l < N2} A(c, l) (-1)^popcount(l & m),
//             A(c, l) = sum over taps with lam >> log2 N1 = l of x_lam (-1)^popcount(lam & c),
// where s = S_Lambda^T x.  So one workgroup builds A from the taps (kept in
// bucket order by the least-squares update, bucket l as above), runs B
// length-N2 transforms in FP64 in LDS, forms r = y - U s at its rows of Omega,
// and runs the correlation's first pass on the same LDS tile in the
// correlation precision: r never goes to memory, and no intermediate of the
// residual's own two-pass transform is written.
#include "lds_fft.h"

namespace fcmp {

constexpr int RC_RMAX = 8;   // tile values per thread (tile <= RC_RMAX * threads)

__device__ __forceinline__ float2 narrow_to(float2, double2 v) {
  return make_float2((float)v.x, (float)v.y);
}
__device__ __forceinline__ double2 narrow_to(double2, double2 v) { return v; }
__device__ __forceinline__ float narrow_to(float, double v) { return (float)v; }
__device__ __forceinline__ double narrow_to(double, double v) { return v; }

template <bool FFT, class VC>
__global__ void __launch_bounds__(256) rcorr_kernel(RCParams p) {
  using VR = typename std::conditional<FFT, double2, double>::type;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int inst = blockIdx.y;
  if (p.status && p.status[inst].done) return;
  const int tid = threadIdx.x, nt = blockDim.x, g = blockIdx.x;
  const int B = p.B, L = p.L, logL = p.logL;
  const int logB = __ffs(B) - 1;
  const int s0 = g * B;
  const int tile_n = B * L;
  const int tile_alloc = tile_n + (tile_n >> 5) + 1;
  VR* tr = (VR*)smem_raw;
  VC* tc = (VC*)smem_raw;   // the correlation tile reuses the residual tile
  // after the tile: the staged taps (one per thread), later the inter-pass twiddles
  unsigned char* reg2 = smem_raw + (size_t)tile_alloc * sizeof(VR);
  VR* tx = (VR*)reg2;
  int32_t* tl = (int32_t*)(tx + nt);
  VC* twlo = (VC*)reg2;
  const int nlo = FFT ? (1 << p.twS) : 0;
  const int nhi = FFT ? (p.N >> p.twS) : 0;
  const int ntw = nlo + nhi;
  VC* twhi = twlo + nlo;
  const uint32_t maskN = (uint32_t)p.N - 1u;
  const uint32_t mask1 = (1u << p.logN1) - 1u;
  const int ntaps = p.tofs ? p.ntaps - p.tofs[inst] : p.ntaps;
  if (p.Kv && ntaps >= p.Kv[inst]) return;   // its K selections are made

  // The loads of the taps (first chunk, in bucket order) and of the bucket
  // starts are issued together, before any of them is waited for.  (The rows
  // of Omega are loaded after the FP64 transform: values held in registers
  // across it would cost occupancy.)
  const int32_t* bs = p.bstart + (int64_t)inst * p.inst_bstart + (ntaps & 1) * p.bstart_half;
  const int32_t* od = p.ord + (int64_t)inst * p.inst_ord + (ntaps & 1) * p.ord_half;
  const int32_t* lm = p.lam + (int64_t)inst * p.inst_lam;
  const VR* xs = (const VR*)p.x + (int64_t)inst * p.inst_x;
  int32_t* bsl = tl + nt;   // bucket starts in LDS (L + 1)
  int32_t tlv = 0;
  VR txv = vzero(VR());
  if (ntaps > 0) {
    const int tau = od[min(tid, ntaps - 1)];
    tlv = lm[tau];
    txv = xs[tau];
  }
  const int b0 = ntaps > 0 ? bs[min(tid, L)] : 0;
  const int b1 = ntaps > 0 ? bs[min(tid + nt, L)] : 0;
  // entries are sorted by column: this workgroup's rows of Omega are those
  // of columns s0 .. s0 + B - 1
  const int32_t* go = p.goff + (int64_t)inst * p.inst_goff;
  const int lo = go[s0], hi = go[s0 + B];
  const int32_t* ek = p.ent_k + (int64_t)inst * p.inst_ent;
  const VR* yv = (const VR*)p.y + (int64_t)inst * p.inst_y;
  bsl[min(tid, L)] = b0;
  bsl[min(tid + nt, L)] = b1;
  for (int b = tid + 2 * nt; b <= L; b += nt) bsl[b] = ntaps > 0 ? bs[b] : 0;

  // ---- A(c, l) from the taps of bucket l, summed in bucket order (a
  // running sum in the tile entry, whatever the chunking); stored conjugated
  // for the Fourier class (the LDS core runs with the + sign).  A thread
  // takes bucket l for a run of up to 8 consecutive columns.  The twiddle
  // e^{2 pi i lam c / N} is the two-level table product hi[p >> s] lo[p & (2^s - 1)]
  // of p = lam c mod N, the same operations whatever the tile; the loads of
  // four columns are issued together.
  {
    const double2* rlo = (const double2*)p.twr_lo;
    const double2* rhi = (const double2*)p.twr_hi;
    const uint32_t lomask = (1u << p.twS) - 1u;
    const int logR = min(logB, 3);
    const int R = 1 << logR;          // columns per run
    const int logRuns = logB - logR;  // runs per bucket: B / R
    const int npair = L << logRuns;
    for (int i0 = 0; i0 == 0 || i0 < ntaps; i0 += nt) {
      const int nc = max(0, min(nt, ntaps - i0));
      if (i0 > 0) {
        __syncthreads();   // the previous chunk is consumed
        const int tau = od[i0 + min(tid, nc - 1)];
        tlv = lm[tau];
        txv = xs[tau];
      }
      if (tid < nc) {
        tl[tid] = tlv;
        tx[tid] = txv;
      }
      __syncthreads();
      const int ie = i0 + nc;
      for (int pr = tid; pr < npair; pr += nt) {
        const int l = pr >> logRuns;
        const int u0 = (pr & ((1 << logRuns) - 1)) << logR;
        const uint32_t c0 = (uint32_t)(s0 + u0);
        VR acc[8];
#pragma unroll
        for (int j = 0; j < 8; ++j)
          acc[j] = (j < R && i0 > 0) ? tr[lds_addr(l * B + u0 + j)] : vzero(VR());
        const int i1 = min(bsl[l + 1], ie);
        for (int i = max(bsl[l], i0); i < i1; ++i) {
          const int li = i - i0;
          const uint32_t lv = (uint32_t)tl[li];
          if constexpr (FFT) {
            const double2 xv = tx[li];
#pragma unroll
            for (int h = 0; h < 8; h += 4) {
              if (h < R) {
                double2 wh[4], wl[4];
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                  const uint32_t ph = (lv * (c0 + (uint32_t)(h + j))) & maskN;
                  wh[j] = rhi[ph >> p.twS];
                  wl[j] = rlo[ph & lomask];
                }
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                  if (h + j < R) {
                    const double2 w = cmul(wh[j], wl[j]);
                    acc[h + j].x += xv.x * w.x + xv.y * w.y;   // conj(x) w
                    acc[h + j].y += xv.x * w.y - xv.y * w.x;
                  }
                }
              }
            }
          } else {
            const double xv = tx[li];
#pragma unroll
            for (int j = 0; j < 8; ++j)
              if (j < R) acc[j] += (__popc(lv & mask1 & (c0 + j)) & 1) ? -xv : xv;
          }
        }
#pragma unroll
        for (int j = 0; j < 8; ++j)
          if (j < R) tr[lds_addr(l * B + u0 + j)] = acc[j];
      }
    }
  }
  __syncthreads();
  if constexpr (FFT) {
    // the staged taps are consumed: the inter-pass twiddles take their place
    const VC* glo = (const VC*)p.twc_lo;
    const VC* ghi = (const VC*)p.twc_hi;
    for (int e = tid; e < ntw; e += nt) twlo[e] = e < nlo ? glo[e] : ghi[e - nlo];
  }
  // natural input; Fourier output at position bitrev(m), Hadamard at m
  lds_fft<FFT, FFT>(tr, L, logL, B, logB, (const VR*)p.twr_st);

  // ---- r = y - U s at this workgroup's rows of Omega, kept in registers
  // at their tile positions (the correlation's first pass places row
  // c + N1 m at the same position: bitrev(m) for its decimation-in-time core)
  VC rv[RC_RMAX];
  int rp[RC_RMAX];
#pragma unroll
  for (int q = 0; q < RC_RMAX; ++q) { rp[q] = -1; rv[q] = vzero(VC()); }
  if (hi > lo) {
    const int qn = (hi - lo + nt - 1) / nt;   // row slots in use (same for the workgroup)
    int kk[RC_RMAX];
    VR yy[RC_RMAX];
#pragma unroll
    for (int q = 0; q < RC_RMAX; ++q) {
      if (q < qn) {
        const int e = min(lo + tid + q * nt, hi - 1);
        kk[q] = ek[e];
        yy[q] = yv[e];
      }
    }
#pragma unroll
    for (int q = 0; q < RC_RMAX; ++q) {
      if (lo + tid + q * nt < hi) {
        const int k = kk[q];
        const int cc = (int)((uint32_t)k & mask1) - s0;
        const int m = k >> p.logN1;
        const int pos = lds_addr((FFT ? bitrev(m, logL) : m) * B + cc);
        VR X = tr[pos];
        if constexpr (FFT) X = vconj(X);
        const VR r = vsub(yy[q], vscale(X, p.rscale));
        rv[q] = narrow_to(VC(), r);
        rp[q] = pos;
      }
    }
  }
  __syncthreads();   // every residual-tile read is done
  for (int e = tid; e < tile_alloc; e += nt) tc[e] = vzero(VC());
  __syncthreads();
#pragma unroll
  for (int q = 0; q < RC_RMAX; ++q)
    if (rp[q] >= 0) tc[rp[q]] = rv[q];
  __syncthreads();

  // ---- the correlation's first pass: B length-N2 transforms with the + sign,
  // then the inter-pass twiddle W_N^{(s0 + c) j}; out(s0 + c, j) at
  // out[(s0 + c) + N1 j]
  lds_fft<FFT, false>(tc, L, logL, B, logB, (const VC*)p.twc_st);
  VC* out = (VC*)p.out + (int64_t)inst * p.inst_out;
  for (int e = tid; e < tile_n; e += nt) {
    const int cc = e & (B - 1);
    const int j = e >> logB;
    VC v = tc[lds_addr(j * B + cc)];
    if constexpr (FFT) {
      const uint32_t q = ((uint32_t)(s0 + cc) * (uint32_t)j) & maskN;
      v = cmul(v, tw_lookup(twlo, twhi, q, p.twS, +1));
    }
    out[(int64_t)(s0 + cc) + ((int64_t)j << p.logN1)] = v;
  }
}

size_t rcorr_lds_bytes(int pk, bool fft, const RCParams& p) {
  const size_t tile_n = (size_t)p.B * p.L;
  const size_t tile_alloc = tile_n + (tile_n >> 5) + 1;
  const size_t rb = fft ? 16 : 8;
  const size_t ntw = fft ? ((size_t)1 << p.twS) + ((size_t)p.N >> p.twS) : 0;
  // one tap per thread, and the bucket starts
  const size_t staged = (size_t)256 * (rb + 4) + ((size_t)p.L + 1) * 4;
  return tile_alloc * rb + std::max(ntw * vbytes(pk), staged);
}

bool rcorr_ok(int pk, bool fft, const RCParams& p, int nthreads) {
  const int tile_n = p.B * p.L;
  return nthreads >= 64 && nthreads <= 256 && tile_n >= nthreads && tile_n <= RC_RMAX * nthreads &&
         (fft ? (pk == V_C64 || pk == V_C128) : (pk == V_F32 || pk == V_F64)) &&
         rcorr_lds_bytes(pk, fft, p) <= 65536;
}

template <bool FFT, class VC>
static hipError_t launch_rc(const RCParams& p, int groups, int ninst, int nthreads, size_t lds,
                            hipStream_t st) {
  auto kfn = rcorr_kernel<FFT, VC>;
  hipError_t e = raise_lds_limit((const void*)kfn, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(kfn, dim3(groups, ninst), dim3(nthreads), lds, st, p);
  return hipGetLastError();
}

hipError_t launch_rcorr(int pk, bool fft, const RCParams& p, int groups, int ninst, int nthreads,
                        hipStream_t st) {
  if (!rcorr_ok(pk, fft, p, nthreads)) return hipErrorInvalidValue;
  const size_t lds = rcorr_lds_bytes(pk, fft, p);
  if (fft) {
    if (pk == V_C64) return launch_rc<true, float2>(p, groups, ninst, nthreads, lds, st);
    return launch_rc<true, double2>(p, groups, ninst, nthreads, lds, st);
  }
  if (pk == V_F32) return launch_rc<false, float>(p, groups, ninst, nthreads, lds, st);
  return launch_rc<false, double>(p, groups, ninst, nthreads, lds, st);
}

}  // namespace fcmp
