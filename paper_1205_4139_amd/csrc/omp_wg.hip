// Persistent OMP, one workgroup per instance (Algorithm 1.1 end to end):
// for problems whose N-point transform fits in one workgroup's LDS, a
// workgroup pulls an instance from an atomic queue and runs every iteration
// itself -- correlation (conventional: FP64 residual, zero-fill and the LDS
// transform; fast: eq. (kernelsumOMP) against the kernel vector), the
// identification, and the FP64 inverse-Cholesky least-squares update -- then
// takes the next instance.  Every workgroup leaves the loop once the queue is
// exhausted.  The kernel vector and h_0 come from a lockstep prologue.
#include "../../include/fcmp.h"
#include "lds_fft.h"

namespace fcmp {

constexpr int WG_THREADS = 512;

struct WgLds {
  unsigned char* tile;   // transform tile (also g, w of the least squares)
  double2* tw64lo; double2* tw64hi;   // two-level FP64 table (residual phases)
  uint32_t* excl;        // N bits
  int32_t* lam;          // support in selection order
  Sel* red;
  double* dred;
};

template <class T> __device__ __forceinline__ T wsh(T v, int src);
template <> __device__ __forceinline__ double wsh<double>(double v, int src) { return __shfl(v, src, 64); }

// per-span stage twiddles (global) for the corr type
template <class V> __device__ __forceinline__ const V* stage_tw(const WgParams& p);
template <> __device__ __forceinline__ const float2* stage_tw<float2>(const WgParams& p) { return p.tws32; }
template <> __device__ __forceinline__ const double2* stage_tw<double2>(const WgParams& p) { return p.tws64; }
template <> __device__ __forceinline__ const float* stage_tw<float>(const WgParams&) { return nullptr; }
template <> __device__ __forceinline__ const double* stage_tw<double>(const WgParams&) { return nullptr; }

// Identification + least-squares update for selection number t (1-based);
// returns false on a Cholesky breakdown.  g and w live in the tile region.
template <bool FOURIER>
__device__ bool wg_ls(const WgDesc& d, char* base, const WgLds& s, int t, uint32_t j,
                      double& znorm2) {
  using Wd = typename std::conditional<FOURIER, double2, double>::type;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int nwaves = WG_THREADS / 64;
  const int n = t - 1;
  const uint32_t mask = (uint32_t)d.N - 1u;
  const Wd* c64 = (const Wd*)(base + d.off_c64);
  const Wd* h0 = (const Wd*)(base + d.off_h0);
  Wd* W = (Wd*)(base + d.off_W);
  Wd* x = (Wd*)(base + d.off_x);
  Wd* z = (Wd*)(base + d.off_z);
  Wd* g = (Wd*)s.tile;
  Wd* w = g + (n > 0 ? n : 1);
  for (int i = tid; i < n; i += WG_THREADS) g[i] = c64[perm_index(FOURIER, (uint32_t)s.lam[i], j, mask)];
  __syncthreads();
  for (int i = wave; i < n; i += nwaves) {
    const Wd* Wi = W + (int64_t)i * (i + 1) / 2;
    Wd a = vzero(Wd());
    for (int k = lane; k <= i; k += 64) {
      if constexpr (FOURIER) { const double2 q = cmul(Wi[k], g[k]); a.x += q.x; a.y += q.y; }
      else a += Wi[k] * g[k];
    }
    if constexpr (FOURIER) { a.x = wave_sum(a.x); a.y = wave_sum(a.y); }
    else a = wave_sum(a);
    if (lane == 0) w[i] = a;
  }
  __syncthreads();
  double nw = 0.0, wzr = 0.0, wzi = 0.0;
  for (int i = tid; i < n; i += WG_THREADS) {
    nw += vmag2(w[i]);
    if constexpr (FOURIER) { const double2 q = cmulc(w[i], z[i]); wzr += q.x; wzi += q.y; }
    else wzr += w[i] * z[i];
  }
  nw = block_sum(nw, s.dred);
  wzr = block_sum(wzr, s.dred);
  if (FOURIER) wzi = block_sum(wzi, s.dred);
  double gamma;
  if constexpr (FOURIER) gamma = c64[0].x; else gamma = c64[0];
  const double d2 = gamma - nw;
  if (!(d2 > 1e-13 * gamma)) return false;
  const double invd = 1.0 / sqrt(d2);
  const Wd bj = h0[j];
  Wd zt;
  if constexpr (FOURIER) zt = make_double2((bj.x - wzr) * invd, (bj.y - wzi) * invd);
  else zt = (bj - wzr) * invd;
  Wd* Wn = W + (int64_t)n * (n + 1) / 2;
  // new row of W: v_k = -(sum_{i >= k} conj(w_i) W(i,k)) / d, one column per
  // thread and chunk; rows are read whole across the workgroup
  for (int k0 = 0; k0 < n; k0 += WG_THREADS) {
    const int k = k0 + tid;
    Wd acc = vzero(Wd());
    for (int i = k0; i < n; ++i) {
      if (k <= i) {
        const Wd Wik = W[(int64_t)i * (i + 1) / 2 + k];
        if constexpr (FOURIER) { const double2 q = cmulc(w[i], Wik); acc.x += q.x; acc.y += q.y; }
        else acc += w[i] * Wik;
      }
    }
    if (k < n) {
      Wd v;
      if constexpr (FOURIER) {
        v = make_double2(-acc.x * invd, -acc.y * invd);
        const double2 q = cmulc(v, zt);
        x[k].x += q.x;
        x[k].y += q.y;
      } else {
        v = -acc * invd;
        x[k] += v * zt;
      }
      Wn[k] = v;
    }
  }
  if (tid == 0) {
    if constexpr (FOURIER) {
      Wn[n] = make_double2(invd, 0.0);
      x[n] = make_double2(zt.x * invd, zt.y * invd);
    } else {
      Wn[n] = invd;
      x[n] = zt * invd;
    }
    z[n] = zt;
    s.lam[n] = (int32_t)j;
    s.excl[j >> 5] |= 1u << (j & 31);
  }
  znorm2 += vmag2(zt);
  __syncthreads();
  return true;
}

// One OMP solve; V is the correlation type (float/double for Hadamard,
// float2/double2 for Fourier).
template <class V>
__device__ void wg_solve(const WgParams& p, const WgDesc& d, const WgLds& s, Status* stat,
                         int32_t* sup_out, void* x_out) {
  constexpr bool F = VT<V>::cplx;
  using Wd = typename VT<V>::Wide;
  const int tid = threadIdx.x;
  const int N = d.N, logN = d.logN, M = d.M, K = d.K;
  char* base = p.base;
  const Wd* h0 = (const Wd*)(base + d.off_h0);
  const V* cp = (const V*)(base + d.off_cp);
  const int32_t* om = (const int32_t*)(base + d.off_om);
  const Wd* y = (const Wd*)(base + d.off_y);
  const Wd* x = (const Wd*)(base + d.off_x);
  const uint32_t mask = (uint32_t)N - 1u;
  const int upshift = p.logT - logN;   // twiddle index scaling to the fixed tables
  const double inv_sqrt_n = 1.0 / sqrt((double)N);
  for (int e = tid; e < (N + 31) / 32; e += WG_THREADS) s.excl[e] = 0u;
  __syncthreads();
  double znorm2 = 0.0, min_gap = __builtin_inf();
  const double ynorm2 = stat->ynorm2, res_tol2 = stat->res_tol2;
  int iters = 0;
  bool numeric = false;
  V* tile = (V*)s.tile;
  // fast iterations gather the kernel vector from LDS: the transform tile
  // (at least N values) holds it until the first conventional iteration;
  // the least-squares update borrows the tile's first 2(t - 1) wide values
  // for g and w, so later fast iterations restore only that prefix
  bool c_in_tile = false;
  for (int t = 1; t <= K; ++t) {
    double bk = -1.0, bk2 = -1.0;
    int64_t bi = -1;
    const bool fast = d.method == FCMP_CORR_FAST ||
                      (d.method == FCMP_CORR_ADAPTIVE && t <= d.switch_t);
    if (t == 1) {
      for (int j = tid; j < N; j += WG_THREADS) sel_add(vmag2(h0[j]), (int64_t)j, bk, bi, bk2);
    } else if (fast) {
      const int cl = c_in_tile
                         ? min(N, (int)((2 * (size_t)t * sizeof(Wd) + sizeof(V) - 1) / sizeof(V)))
                         : N;
      for (int jj = tid; jj < cl; jj += WG_THREADS) tile[jj] = cp[jj];
      __syncthreads();
      c_in_tile = true;
      // eq. (kernelsumOMP): h = h_0 - sum_tau x_tau P_{lam_tau} c, FP64 accumulation
      for (int j0 = tid; j0 < N; j0 += WG_THREADS * 4) {
        Wd acc[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int j = j0 + u * WG_THREADS;
          acc[u] = j < N ? h0[j] : vzero(Wd());
        }
        for (int tau = 0; tau < t - 1; ++tau) {
          const uint32_t l = (uint32_t)s.lam[tau];
          const Wd xv = x[tau];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const uint32_t j = (uint32_t)(j0 + u * WG_THREADS) & mask;
            const Wd cw = vwiden(tile[perm_index(F, j, l, mask)]);
            if constexpr (F) {
              acc[u].x -= xv.x * cw.x - xv.y * cw.y;
              acc[u].y -= xv.x * cw.y + xv.y * cw.x;
            } else {
              acc[u] -= xv * cw;
            }
          }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int j = j0 + u * WG_THREADS;
          if (j < N && !((s.excl[j >> 5] >> (j & 31)) & 1u))
            sel_add(vmag2(acc[u]), (int64_t)j, bk, bi, bk2);
        }
      }
    } else {
      // conventional: FP64 residual r = y - Phi_t x_t, zero-filled into the tile
      c_in_tile = false;
      for (int e = tid; e < N + (N >> 5) + 1; e += WG_THREADS) tile[e] = vzero(V());
      __syncthreads();
      for (int m0 = tid; m0 < M; m0 += WG_THREADS * 4) {
        Wd acc[4];
        uint32_t kk[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int m = m0 + u * WG_THREADS;
          kk[u] = m < M ? (uint32_t)om[m] : 0u;
          acc[u] = vzero(Wd());
        }
        for (int tau = 0; tau < t - 1; ++tau) {
          const uint32_t l = (uint32_t)s.lam[tau];
          const Wd xv = x[tau];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            if constexpr (F) {
              const uint32_t ph = ((kk[u] * l) & mask) << upshift;
              const double2 wv = cmul(s.tw64hi[ph >> p.twS], s.tw64lo[ph & ((1u << p.twS) - 1u)]);
              const double2 q = cmulc(wv, xv);   // conj(e^{+i..}) x = e^{-2 pi i k lam / N} x
              acc[u].x += q.x;
              acc[u].y += q.y;
            } else {
              acc[u] += (__popc(kk[u] & l) & 1) ? -xv : xv;
            }
          }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int m = m0 + u * WG_THREADS;
          if (m < M) {
            Wd r = y[m];
            if constexpr (F) { r.x -= acc[u].x * inv_sqrt_n; r.y -= acc[u].y * inv_sqrt_n; }
            else r -= acc[u] * inv_sqrt_n;
            const int pos = F ? bitrev((int)kk[u], logN) : (int)kk[u];
            tile[lds_addr(pos)] = vnarrow(r, V());
          }
        }
      }
      __syncthreads();
      lds_fft<F, false>(tile, N, logN, 1, 0, stage_tw<V>(p));
      for (int j = tid; j < N; j += WG_THREADS) {
        if ((s.excl[j >> 5] >> (j & 31)) & 1u) continue;
        sel_add(vmag2(vscale(tile[lds_addr(j)], inv_sqrt_n)), (int64_t)j, bk, bi, bk2);
      }
    }
    const Sel best = block_sel_reduce(bk, bi, bk2, s.red);
    if (best.idx < 0 || !(best.key > 0.0)) break;
    min_gap = fmin(min_gap, sel_gap(best));
    if (!wg_ls<F>(d, base, s, t, (uint32_t)best.idx, znorm2)) {
      numeric = true;
      break;
    }
    iters = t;
    // optional early stop on the residual norm, ||r||^2 = ||y||^2 - ||z||^2
    if (res_tol2 > 0.0 && ynorm2 - znorm2 <= res_tol2 * ynorm2) break;
  }
  // results
  const Wd* xr = (const Wd*)(base + d.off_x);
  Wd* xo = (Wd*)x_out;
  for (int i = tid; i < K; i += WG_THREADS) {
    const bool ok = i < iters;
    sup_out[i] = ok ? s.lam[i] : -1;
    xo[i] = ok ? xr[i] : vzero(Wd());
  }
  if (tid == 0) {
    stat->iterations = iters;
    stat->numeric = numeric ? 1 : 0;
    stat->znorm2 = znorm2;
    stat->min_gap = min_gap;
    stat->t_done = (double)(wall_clock64() - *p.t0);
    stat->done = 1;
  }
  __syncthreads();
}

template <int PREC>
__global__ void __launch_bounds__(WG_THREADS) omp_wg_kernel(WgParams p) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ int cur;
  WgLds s;
  s.tile = smem_raw;
  const int nlo = 1 << p.twS, nhi = (1 << p.logT) >> p.twS;
  unsigned char* q = smem_raw + ((p.tile_bytes + 15) & ~(size_t)15);
  s.tw64lo = (double2*)q; q += nlo * 16;
  s.tw64hi = (double2*)q; q += nhi * 16;
  s.excl = (uint32_t*)q; q += (((1 << p.logNmax) + 31) / 32) * 4;
  s.lam = (int32_t*)q; q += ((p.Kmax + 3) & ~3) * 4;
  q = (unsigned char*)(((uintptr_t)q + 15) & ~(uintptr_t)15);
  s.red = (Sel*)q; q += 16 * sizeof(Sel);
  s.dred = (double*)q;
  for (int e = threadIdx.x; e < nlo + nhi; e += WG_THREADS) {
    const double2 a = p.tw64[e];
    if (e < nlo) s.tw64lo[e] = a;
    else s.tw64hi[e - nlo] = a;
  }
  __syncthreads();
  for (;;) {
    if (threadIdx.x == 0) cur = atomicAdd(p.counter, 1);
    __syncthreads();
    const int i = cur;
    __syncthreads();
    if (i >= p.n) break;   // uniform: every wave reads the same slot
    const int di = p.order[i];
    const WgDesc d = p.desc[di];
    int32_t* so = (int32_t*)p.ptrs[p.n + di];
    void* xo = p.ptrs[2 * p.n + di];
    if (d.cls == FCMP_FOURIER) {
      if (PREC == FCMP_FP32) wg_solve<float2>(p, d, s, p.status + di, so, xo);
      else wg_solve<double2>(p, d, s, p.status + di, so, xo);
    } else {
      if (PREC == FCMP_FP32) wg_solve<float>(p, d, s, p.status + di, so, xo);
      else wg_solve<double>(p, d, s, p.status + di, so, xo);
    }
  }
}

size_t omp_wg_lds_bytes(const WgParams& p) {
  const size_t nlo = (size_t)1 << p.twS, nhi = ((size_t)1 << p.logT) >> p.twS;
  size_t b = (p.tile_bytes + 15) & ~(size_t)15;
  b += (nlo + nhi) * 16;
  b += (((size_t)1 << p.logNmax) + 31) / 32 * 4;
  b += (size_t)((p.Kmax + 3) & ~3) * 4;
  b = (b + 15) & ~(size_t)15;
  b += 16 * sizeof(Sel) + 16 * sizeof(double);
  return b;
}

__global__ void stamp_kernel(uint64_t* dst) {
  if (threadIdx.x == 0) *dst = wall_clock64();
}

hipError_t launch_stamp(uint64_t* dst, hipStream_t st) {
  hipLaunchKernelGGL(stamp_kernel, dim3(1), dim3(64), 0, st, dst);
  return hipGetLastError();
}

int omp_wg_per_cu(const WgParams& p, int precision) {
  const size_t lds = omp_wg_lds_bytes(p);
  const void* f = precision == FCMP_FP32 ? (const void*)omp_wg_kernel<FCMP_FP32>
                                         : (const void*)omp_wg_kernel<FCMP_FP64>;
  if (raise_lds_limit(f, lds) != hipSuccess) return 1;
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, f, WG_THREADS, lds) != hipSuccess || nb < 1)
    return 1;
  return nb;
}

hipError_t launch_omp_wg(const WgParams& p, int precision, int groups, hipStream_t st) {
  const size_t lds = omp_wg_lds_bytes(p);
  if (precision == FCMP_FP32) {
    hipError_t e = raise_lds_limit((const void*)omp_wg_kernel<FCMP_FP32>, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(omp_wg_kernel<FCMP_FP32>, dim3(groups), dim3(WG_THREADS), lds, st, p);
  } else {
    hipError_t e = raise_lds_limit((const void*)omp_wg_kernel<FCMP_FP64>, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(omp_wg_kernel<FCMP_FP64>, dim3(groups), dim3(WG_THREADS), lds, st, p);
  }
  return hipGetLastError();
}

}  // namespace fcmp
