// Identification + least squares for one OMP iteration (Algorithm 1.1,
// steps 3-6), one workgroup per instance, all in FP64.
//
// With Lambda_{t-1} selected and lambda_t new, the Gram column is
//   g_i = phi_{lam_i}^H phi_{lam_t} = c(lam_i (-) lam_t),
// because column lambda of Phi^H Phi is P_lambda c (the chain of eqs.
// (corr_com)-(kernelsum) with x = e_lambda); (-) is subtraction mod N
// (Fourier) or XOR (Hadamard).  The library keeps W = L^{-1}, the inverse of
// the Gram's Cholesky factor, as packed rows.  Appending a column:
//   w = W g,  d = sqrt(c(0) - ||w||^2),  new row of W = [-(w^H W)/d, 1/d],
//   z_t = (b_t - w^H z)/d with b_t = h_0(lam_t) = phi_{lam_t}^H y,
//   x  += z_t * conj(new row of W)^T,
// which keeps x = (Phi_t^H Phi_t)^{-1} Phi_t^H y (step 6) with two
// parallel matrix-vector products per iteration and no triangular solve.
#include "kernels.h"

namespace fcmp {

constexpr int L_THREADS = 256;
constexpr int L_KPT = 16;     // most columns per thread in the w^H W product: K <= 4096
constexpr int L_RB = 4;       // rows per wave in w = W g (independent loads in flight)
constexpr int L_KU = 2;       // lane-strided column chunks per step in w = W g
constexpr int L_VB = 8;       // rows per step in w^H W (independent loads in flight)

// w_i = sum_{k <= i} W(i,k) g_k for the rows i = i0 .. i0+L_RB-1 (< n) of one
// wave: lane-strided partial sums over k, then a butterfly sum per row.  The
// order of additions within a row does not depend on how rows are grouped.
template <bool FOURIER, class Wd>
__device__ __forceinline__ void ls_rows_wg(const Wd* W, const Wd* g, int i0, int n, int lane,
                                           Wd* wout) {
  Wd s[L_RB];
#pragma unroll
  for (int u = 0; u < L_RB; ++u) s[u] = vzero(Wd());
  const int imax = min(i0 + L_RB, n) - 1;
  // L_KU lane-strided chunks of k per step, their loads (clamped to valid
  // entries) issued together; each lane still adds its k in increasing order
  for (int k0 = lane; k0 <= imax; k0 += 64 * L_KU) {
    Wd a[L_KU][L_RB], gk[L_KU];
#pragma unroll
    for (int v = 0; v < L_KU; ++v) {
      const int kc = min(k0 + 64 * v, imax);
      gk[v] = g[kc];
#pragma unroll
      for (int u = 0; u < L_RB; ++u) {
        const int i = min(i0 + u, imax);
        a[v][u] = W[(int64_t)i * (i + 1) / 2 + min(kc, i)];
      }
    }
#pragma unroll
    for (int v = 0; v < L_KU; ++v) {
      const int k = k0 + 64 * v;
#pragma unroll
      for (int u = 0; u < L_RB; ++u) {
        const int i = i0 + u;
        if (k <= imax && i <= imax && k <= i) {
          if constexpr (FOURIER) {
            const double2 t = cmul(a[v][u], gk[v]);
            s[u].x += t.x;
            s[u].y += t.y;
          } else {
            s[u] += a[v][u] * gk[v];
          }
        }
      }
    }
  }
#pragma unroll
  for (int u = 0; u < L_RB; ++u) {
    if constexpr (FOURIER) { s[u].x = wave_sum(s[u].x); s[u].y = wave_sum(s[u].y); }
    else s[u] = wave_sum(s[u]);
    if (lane == 0 && i0 + u < n) wout[i0 + u] = s[u];
  }
}

// acc[q] += sum over rows i = i_first, i_first + step, ... (< n) of
// conj(w_i) W(i, k) for k = tid + q L_THREADS <= i, rows in increasing order,
// VB rows per step with their loads issued together.  KPT (columns per
// thread, a compile-time bound on nq) sizes the accumulators, so short
// supports keep few registers; neither KPT nor VB changes the order of the
// additions.
template <bool FOURIER, int KPT, int VB, class Wd>
__device__ __forceinline__ void ls_rows_wh(const Wd* W, const Wd* w, int i_first, int step, int n,
                                           int nq, int tid, Wd* acc) {
  int i = i_first;
  for (; i + (VB - 1) * step < n; i += VB * step) {
    Wd wv[VB];
#pragma unroll
    for (int u = 0; u < VB; ++u) wv[u] = w[i + u * step];
#pragma unroll
    for (int q = 0; q < KPT; ++q) {
      const int k = tid + q * L_THREADS;
      if (q < nq) {
        Wd a[VB];
#pragma unroll
        for (int u = 0; u < VB; ++u) {
          const int r = i + u * step;
          a[u] = k <= r ? W[(int64_t)r * (r + 1) / 2 + k] : vzero(Wd());
        }
#pragma unroll
        for (int u = 0; u < VB; ++u) {
          const int r = i + u * step;
          if (k <= r) {
            if constexpr (FOURIER) { const double2 t = cmulc(wv[u], a[u]); acc[q].x += t.x; acc[q].y += t.y; }
            else acc[q] += wv[u] * a[u];
          }
        }
      }
    }
  }
  for (; i < n; i += step) {
    const Wd* Wi = W + (int64_t)i * (i + 1) / 2;
    const Wd wi = w[i];
#pragma unroll
    for (int q = 0; q < KPT; ++q) {
      const int k = tid + q * L_THREADS;
      if (q < nq && k <= i) {
        if constexpr (FOURIER) { const double2 t = cmulc(wi, Wi[k]); acc[q].x += t.x; acc[q].y += t.y; }
        else acc[q] += wi * Wi[k];
      }
    }
  }
}

// Bucket order of the taps for the fused residual: with taps 0..n-1 in
// buffer n & 1 (tap indices sorted by (bucket, index) and the bucket starts),
// writes taps 0..n, the new one being tap n of column j, to buffer (n+1) & 1.
// The new tap has the largest index, so it goes to the end of its bucket.
__device__ __forceinline__ void tap_order_insert(const LParams& p, int inst, int n, uint32_t j) {
  const int NB = p.nbuck;
  int32_t* ob = p.ord + (int64_t)inst * p.inst_ord;
  int32_t* bb = p.bstart + (int64_t)inst * p.inst_bstart;
  const int32_t* oold = ob + (n & 1) * p.ord_half;
  int32_t* onew = ob + ((n + 1) & 1) * p.ord_half;
  const int32_t* bold = bb + (n & 1) * p.bstart_half;
  int32_t* bnew = bb + ((n + 1) & 1) * p.bstart_half;
  const int key = (int)((j >> p.bshift) & (uint32_t)(NB - 1));
  const int pos = n > 0 ? bold[key + 1] : 0;
  for (int i = threadIdx.x; i <= n; i += blockDim.x)
    onew[i] = i < pos ? oold[i] : (i == pos ? n : oold[i - 1]);
  for (int b = threadIdx.x; b <= NB; b += blockDim.x)
    bnew[b] = (n > 0 ? bold[b] : 0) + (b > key ? 1 : 0);
}

template <bool FOURIER, int KPT>
__global__ void __launch_bounds__(L_THREADS) ls_kernel(LParams p) {
  using Wd = typename std::conditional<FOURIER, double2, double>::type;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ Sel red[16];
  __shared__ double dred[16];
  const int inst = blockIdx.x;
  Status* st = p.status + inst;
  if (st->done) return;
  const int t = p.tofs ? p.t - p.tofs[inst] : p.t;
  if (p.tofs && ls_split_groups(t) > 1) return;   // the split update takes it
  if (p.Kv && t > p.Kv[inst]) {   // its K selections are made
    __syncthreads();
    if (threadIdx.x == 0) st->done = 1;
    return;
  }
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int nwaves = L_THREADS / 64;
  const int n = t - 1;       // previous selections
  Wd* g = (Wd*)smem_raw;     // g, then the new row of W
  Wd* w = g + (n > 0 ? n : 1);
  int32_t* sl = (int32_t*)(w + (n > 0 ? n : 1));

  // ---- step 3: reduce the per-workgroup partials
  const Sel* part = p.partial + (int64_t)inst * p.inst_part;
  double bk = -1.0, bk2 = -1.0;
  int64_t bi = -1;
  for (int e = tid; e < p.npart; e += L_THREADS) {
    const Sel s = part[e];
    if (s.idx >= 0) sel_merge(s.key, s.idx, s.key2, bk, bi, bk2);
  }
  const Sel best = block_sel_reduce(bk, bi, bk2, red);
  if (best.idx < 0 || !(best.key > 0.0)) {
    if (tid == 0) st->done = 1;
    return;
  }
  const uint32_t j = (uint32_t)best.idx;
  const uint32_t mask = (uint32_t)p.N - 1u;
  int32_t* lam = p.lam + (int64_t)inst * p.inst_lam;
  const Wd* c64 = (const Wd*)p.c64 + (int64_t)inst * p.inst_c;
  Wd* W = (Wd*)p.W + (int64_t)inst * p.inst_W;
  Wd* z = (Wd*)p.z + (int64_t)inst * p.inst_z;
  Wd* x = (Wd*)p.x + (int64_t)inst * p.inst_x;

  // ---- Gram column from the kernel vector
  for (int i = tid; i < n; i += L_THREADS) {
    const uint32_t li = (uint32_t)lam[i];
    sl[i] = (int32_t)li;
    g[i] = c64[perm_index(FOURIER, li, j, mask)];
  }
  __syncthreads();

  // ---- w = W g (row i of W has i+1 entries starting at i(i+1)/2)
  for (int i0 = wave * L_RB; i0 < n; i0 += nwaves * L_RB) ls_rows_wg<FOURIER>(W, g, i0, n, lane, w);
  __syncthreads();

  // ---- d^2 = c(0) - ||w||^2, and w^H z
  double nw = 0.0, wzr = 0.0, wzi = 0.0;
  for (int i = tid; i < n; i += L_THREADS) {
    nw += vmag2(w[i]);
    if constexpr (FOURIER) { const double2 t = cmulc(w[i], z[i]); wzr += t.x; wzi += t.y; }
    else wzr += w[i] * z[i];
  }
  nw = block_sum(nw, dred);
  wzr = block_sum(wzr, dred);
  if (FOURIER) wzi = block_sum(wzi, dred);
  double gamma;
  if constexpr (FOURIER) gamma = c64[0].x; else gamma = c64[0];
  const double d2 = gamma - nw;
  if (!(d2 > 1e-13 * gamma)) {
    if (tid == 0) { st->numeric = 1; st->done = 1; }
    return;
  }
  const double d = sqrt(d2);
  const double invd = 1.0 / d;

  // ---- new row of W: v_k = -(sum_{i>=k} conj(w_i) W(i,k)) / d
  Wd acc[KPT];
#pragma unroll
  for (int q = 0; q < KPT; ++q) acc[q] = vzero(Wd());
  const int nq = (n + L_THREADS - 1) / L_THREADS;
  ls_rows_wh<FOURIER, KPT, L_VB>(W, w, 0, 1, n, nq, tid, acc);
  __syncthreads();   // everyone is done reading g
  Wd* Wn = W + (int64_t)n * (n + 1) / 2;
#pragma unroll
  for (int q = 0; q < KPT; ++q) {
    const int k = tid + q * L_THREADS;
    if (k < n) {
      Wd v;
      if constexpr (FOURIER) v = make_double2(-acc[q].x * invd, -acc[q].y * invd);
      else v = -acc[q] * invd;
      g[k] = v;
      Wn[k] = v;
    }
  }
  Wd b = ((const Wd*)p.h0 + (int64_t)inst * p.inst_h0)[j];
  Wd zt;
  if constexpr (FOURIER) zt = make_double2((b.x - wzr) * invd, (b.y - wzi) * invd);
  else zt = (b - wzr) * invd;
  __syncthreads();

  // ---- x += zt * conj(new row); x_n = zt / d
  for (int k = tid; k < n; k += L_THREADS) {
    if constexpr (FOURIER) {
      const double2 t = cmulc(g[k], zt);
      x[k].x += t.x;
      x[k].y += t.y;
    } else {
      x[k] += g[k] * zt;
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
    lam[n] = (int32_t)j;
    uint32_t* ex = p.excl + (int64_t)inst * p.inst_excl;
    ex[j >> 5] |= 1u << (j & 31);
    st->znorm2 += vmag2(zt);
    st->iterations = t;
    st->last_key = best.key;
    st->min_gap = fmin(st->min_gap, sel_gap(best));
    // optional early stop on the residual norm, ||r||^2 = ||y||^2 - ||z||^2
    if (st->res_tol2 > 0.0 && st->ynorm2 - st->znorm2 <= st->res_tol2 * st->ynorm2) st->done = 1;
  }
  if (p.ord) tap_order_insert(p, inst, n, j);
}

// ---------------------------------------------------------------------------
// The same update split over G workgroups per instance for long supports:
//   ls_ab: identification, Gram column, then for the rows i = gid (mod G),
//          eight at a time: w_i = (W g)_i (two rows per wave) and, while
//          those rows are still in the cache, the partial row
//          sum_i conj(w_i) W(i, k) (thread per column k)
//   ls_c:  d (and the breakdown test), v = -(sum over the G partials, in
//          order)/d, new row of W, z and x
// W is read from memory once per iteration.  Every reduction has a fixed
// order (rows of a partial in increasing order, partials in gid order), so
// results depend on t only.
constexpr int L_RW = 2;      // rows per wave in a batch
constexpr int L_AB = 8;      // rows per step of the partial-row fold (loads in flight)

// NT threads per workgroup (256, or 1024 for launches of few workgroups):
// neither the row-to-wave assignment nor the thread count changes a sum.
//
// Workgroups are dispatched to the eight XCDs round-robin by linear id.  With
// gx > 0 (a batch that is a multiple of 8) the grid is one-dimensional, gx
// workgroups per instance, read so that all the workgroups of instance i run
// on XCD i mod 8: the lines of the kernel vector that each of them gathers
// for the Gram column are then fetched into one L2, not into all eight; the
// split kernel that follows reads the partial rows on that XCD too.
__device__ __forceinline__ void xcd_split(int gx, int& inst, int& part) {
  if (gx > 0) {
    const int L = blockIdx.x, k = L >> 3;
    inst = (L & 7) + 8 * (k / gx);
    part = k % gx;
  } else {
    inst = blockIdx.y;
    part = blockIdx.x;
  }
}

template <bool FOURIER, int KPT, int NT>
__global__ void __launch_bounds__(NT) ls_ab_kernel(LParams p, int gx) {
  using Wd = typename std::conditional<FOURIER, double2, double>::type;
  constexpr int L_BATCH = L_RW * (NT / 64);   // rows per batch
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ Sel red[16];
  __shared__ Wd wl[L_BATCH];
  int inst, gid;
  xcd_split(gx, inst, gid);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int t = p.tofs ? p.t - p.tofs[inst] : p.t;
  const int G = ls_split_groups(t);
  if (G == 1 || gid >= G) return;   // the one-workgroup update takes it / spare workgroup
  const int n = t - 1;
  Status* st = p.status + inst;
  // loads whose addresses do not depend on the outcome go out together: the
  // status, the first partials and the first selected columns
  const int32_t* lam = p.lam + (int64_t)inst * p.inst_lam;
  const Sel* part = p.partial + (int64_t)inst * p.inst_part;
  const Sel s0 = tid < p.npart ? part[tid] : Sel{-1.0, -1, -1.0};
  const int32_t l0 = tid < n ? lam[tid] : 0;
  if (st->done) return;
  if ((p.Kv && t > p.Kv[inst]) ||   // its K selections are made
      (st->res_tol2 > 0.0 && st->ynorm2 - st->znorm2 <= st->res_tol2 * st->ynorm2)) {
    // (or the residual met the tolerance after the previous update; every
    // workgroup of this launch reads the same record and returns)
    if (gid == 0 && threadIdx.x == 0) st->done = 1;
    return;
  }
  Wd* g = (Wd*)smem_raw;
  double bk = -1.0, bk2 = -1.0;
  int64_t bi = -1;
  if (s0.idx >= 0) { bk = s0.key; bi = s0.idx; bk2 = s0.key2; }
  for (int e = tid + NT; e < p.npart; e += NT) {
    const Sel s = part[e];
    if (s.idx >= 0) sel_merge(s.key, s.idx, s.key2, bk, bi, bk2);
  }
  const Sel best = block_sel_reduce(bk, bi, bk2, red);
  if (best.idx < 0 || !(best.key > 0.0)) {
    if (gid == 0 && tid == 0) st->done = 1;
    return;
  }
  const uint32_t j = (uint32_t)best.idx;
  if (gid == 0 && tid == 0) {
    st->cur_j = (int32_t)j;
    st->last_key = best.key;
    st->min_gap = fmin(st->min_gap, sel_gap(best));
  }
  const uint32_t mask = (uint32_t)p.N - 1u;
  const Wd* c64 = (const Wd*)p.c64 + (int64_t)inst * p.inst_c;
  const Wd* W = (const Wd*)p.W + (int64_t)inst * p.inst_W;
  Wd* wout = (Wd*)p.wbuf + (int64_t)inst * p.inst_wbuf;
  if (tid < n) g[tid] = c64[perm_index(FOURIER, (uint32_t)l0, j, mask)];
  for (int i = tid + NT; i < n; i += NT)
    g[i] = c64[perm_index(FOURIER, (uint32_t)lam[i], j, mask)];
  __syncthreads();

  Wd acc[KPT];
#pragma unroll
  for (int q = 0; q < KPT; ++q) acc[q] = vzero(Wd());
  const int nq = (n + NT - 1) / NT;
  for (int b0 = gid; b0 < n; b0 += L_BATCH * G) {
    // ---- w for the wave's rows r_u = b0 + G (L_RW wave + u): lane-strided
    // partial sums over k in increasing order, then a butterfly sum
    int rr[L_RW];
    int rmax = -1;
#pragma unroll
    for (int u = 0; u < L_RW; ++u) {
      rr[u] = b0 + G * (L_RW * wave + u);
      if (rr[u] < n) rmax = rr[u];
    }
    Wd sw[L_RW];
#pragma unroll
    for (int u = 0; u < L_RW; ++u) sw[u] = vzero(Wd());
    for (int k0 = lane; k0 <= rmax; k0 += 64 * L_KU) {
      Wd a[L_KU][L_RW], gk[L_KU];
#pragma unroll
      for (int v = 0; v < L_KU; ++v) {
        const int kc = min(k0 + 64 * v, rmax);
        gk[v] = g[kc];
#pragma unroll
        for (int u = 0; u < L_RW; ++u) {
          const int r = min(rr[u], rmax);
          a[v][u] = W[(int64_t)r * (r + 1) / 2 + min(kc, r)];
        }
      }
#pragma unroll
      for (int v = 0; v < L_KU; ++v) {
        const int k = k0 + 64 * v;
#pragma unroll
        for (int u = 0; u < L_RW; ++u) {
          if (rr[u] < n && k <= rr[u]) {
            if constexpr (FOURIER) {
              const double2 tt = cmul(a[v][u], gk[v]);
              sw[u].x += tt.x;
              sw[u].y += tt.y;
            } else {
              sw[u] += a[v][u] * gk[v];
            }
          }
        }
      }
    }
#pragma unroll
    for (int u = 0; u < L_RW; ++u) {
      if constexpr (FOURIER) { sw[u].x = wave_sum(sw[u].x); sw[u].y = wave_sum(sw[u].y); }
      else sw[u] = wave_sum(sw[u]);
      if (lane == 0) {
        wl[L_RW * wave + u] = sw[u];
        if (rr[u] < n) wout[rr[u]] = sw[u];
      }
    }
    __syncthreads();
    // ---- the batch's rows, in increasing order, into the partial row
#pragma unroll
    for (int q = 0; q < KPT; ++q) {
      const int k = tid + q * NT;
      if (q < nq && k < n) {
        for (int m0 = 0; m0 < L_BATCH && b0 + G * m0 < n; m0 += L_AB) {
          Wd a[L_AB];
#pragma unroll
          for (int u = 0; u < L_AB; ++u) {
            const int r = b0 + G * (m0 + u);
            a[u] = (r < n && k <= r) ? W[(int64_t)r * (r + 1) / 2 + k] : vzero(Wd());
          }
#pragma unroll
          for (int u = 0; u < L_AB; ++u) {
            const int r = b0 + G * (m0 + u);
            if (r < n && k <= r) {
              if constexpr (FOURIER) {
                const double2 tt = cmulc(wl[m0 + u], a[u]);
                acc[q].x += tt.x;
                acc[q].y += tt.y;
              } else {
                acc[q] += wl[m0 + u] * a[u];
              }
            }
          }
        }
      }
    }
    __syncthreads();   // wl is rewritten by the next batch
  }
  Wd* vp = (Wd*)p.vpart + (int64_t)inst * p.inst_vpart + (int64_t)gid * p.vpart_stride;
#pragma unroll
  for (int q = 0; q < KPT; ++q) {
    const int k = tid + q * NT;
    if (q < nq && k < n) vp[k] = acc[q];
  }
}

template <bool FOURIER>
__device__ __forceinline__ bool ls_d(const LParams& p, int inst, int n, double* dred,
                                     double& invd, double& wzr, double& wzi) {
  using Wd = typename std::conditional<FOURIER, double2, double>::type;
  const Wd* w = (const Wd*)p.wbuf + (int64_t)inst * p.inst_wbuf;
  const Wd* z = (const Wd*)p.z + (int64_t)inst * p.inst_z;
  double nw = 0.0;
  wzr = 0.0;
  wzi = 0.0;
  for (int i = threadIdx.x; i < n; i += L_THREADS) {
    const Wd wi = w[i];
    nw += vmag2(wi);
    if constexpr (FOURIER) { const double2 t = cmulc(wi, z[i]); wzr += t.x; wzi += t.y; }
    else wzr += wi * z[i];
  }
  nw = block_sum(nw, dred);
  wzr = block_sum(wzr, dred);
  if (FOURIER) wzi = block_sum(wzi, dred);
  const Wd* c64 = (const Wd*)p.c64 + (int64_t)inst * p.inst_c;
  double gamma;
  if constexpr (FOURIER) gamma = c64[0].x; else gamma = c64[0];
  const double d2 = gamma - nw;
  if (!(d2 > 1e-13 * gamma)) return false;
  invd = 1.0 / sqrt(d2);
  return true;
}

template <bool FOURIER>
__global__ void __launch_bounds__(L_THREADS) ls_c_kernel(LParams p, int Gl, int cx) {
  using Wd = typename std::conditional<FOURIER, double2, double>::type;
  __shared__ double dred[16];
  int inst, cb;
  xcd_split(cx, inst, cb);
  Status* st = p.status + inst;
  if (st->done) return;
  const int t = p.tofs ? p.t - p.tofs[inst] : p.t;
  const int G = p.tofs ? ls_split_groups(t) : Gl;
  if (G == 1) return;
  const int tid = threadIdx.x;
  const int n = t - 1;
  double invd, wzr, wzi;
  if (!ls_d<FOURIER>(p, inst, n, dred, invd, wzr, wzi)) {
    if (cb == 0 && threadIdx.x == 0) { st->numeric = 1; st->done = 1; }
    return;
  }
  const uint32_t j = (uint32_t)st->cur_j;
  Wd b = ((const Wd*)p.h0 + (int64_t)inst * p.inst_h0)[j];
  Wd zt;
  if constexpr (FOURIER) zt = make_double2((b.x - wzr) * invd, (b.y - wzi) * invd);
  else zt = (b - wzr) * invd;
  Wd* W = (Wd*)p.W + (int64_t)inst * p.inst_W;
  Wd* Wn = W + (int64_t)n * (n + 1) / 2;
  Wd* x = (Wd*)p.x + (int64_t)inst * p.inst_x;
  const Wd* vp = (const Wd*)p.vpart + (int64_t)inst * p.inst_vpart;
  const int k = cb * L_THREADS + tid;
  if (k < n) {
    // the G partials in order, eight loads in flight at a time
    Wd s = vzero(Wd());
    int q = 0;
    for (; q + 8 <= G; q += 8) {
      Wd a[8];
#pragma unroll
      for (int v = 0; v < 8; ++v) a[v] = vp[(int64_t)(q + v) * p.vpart_stride + k];
#pragma unroll
      for (int v = 0; v < 8; ++v) {
        if constexpr (FOURIER) { s.x += a[v].x; s.y += a[v].y; } else s += a[v];
      }
    }
    for (; q < G; ++q) {
      const Wd a = vp[(int64_t)q * p.vpart_stride + k];
      if constexpr (FOURIER) { s.x += a.x; s.y += a.y; } else s += a;
    }
    Wd v;
    if constexpr (FOURIER) {
      v = make_double2(-s.x * invd, -s.y * invd);
      const double2 t = cmulc(v, zt);
      x[k].x += t.x;
      x[k].y += t.y;
    } else {
      v = -s * invd;
      x[k] += v * zt;
    }
    Wn[k] = v;
  }
  if (cb == 0 && tid == 0) {
    if constexpr (FOURIER) {
      Wn[n] = make_double2(invd, 0.0);
      x[n] = make_double2(zt.x * invd, zt.y * invd);
    } else {
      Wn[n] = invd;
      x[n] = zt * invd;
    }
    Wd* z = (Wd*)p.z + (int64_t)inst * p.inst_z;
    z[n] = zt;
    int32_t* lam = p.lam + (int64_t)inst * p.inst_lam;
    lam[n] = (int32_t)j;
    uint32_t* ex = p.excl + (int64_t)inst * p.inst_excl;
    ex[j >> 5] |= 1u << (j & 31);
    st->znorm2 += vmag2(zt);
    st->iterations = t;
  }
  if (cb == 0 && p.ord) tap_order_insert(p, inst, n, j);
}

// The XCD-grouped one-dimensional grid (see xcd_split) for a lockstep batch
// that is a multiple of 8.  Not for slot groups: their slots sit at different
// iterations or are free, and pinning each slot's workgroups to one XCD would
// leave the XCDs of short or free slots idle.
static bool ls_xcd_map(const LParams& p, int ninst, int per_inst) {
  return !p.tofs && ninst >= 8 && ninst % 8 == 0 &&
         (int64_t)per_inst * ninst < (int64_t(1) << 31);
}

// Columns per thread of the w^H W product, rounded up to a power of two.
static int ls_kpt(int n) {
  const int nq = (n + L_THREADS - 1) / L_THREADS;
  int k = 1;
  while (k < nq) k *= 2;
  return k;
}

template <bool FOURIER, int KPT>
static hipError_t launch_ls_kpt(const LParams& p, int ninst, int G, bool split, size_t lds,
                                hipStream_t st) {
  if (split) {
    const bool xm = ls_xcd_map(p, ninst, G);
    const dim3 grid = xm ? dim3(G * ninst) : dim3(G, ninst);
    const int gx = xm ? G : 0;
    // few workgroups in all: 1024 threads each (more rows and loads in
    // flight), a quarter of the columns per thread
    if ((int64_t)G * ninst < 512) {
      constexpr int K4 = KPT >= 4 ? KPT / 4 : 1;
      hipError_t e = raise_lds_limit((const void*)ls_ab_kernel<FOURIER, K4, 1024>, lds);
      if (e != hipSuccess) return e;
      hipLaunchKernelGGL((ls_ab_kernel<FOURIER, K4, 1024>), grid, dim3(1024), lds, st, p, gx);
      return hipGetLastError();
    }
    hipError_t e = raise_lds_limit((const void*)ls_ab_kernel<FOURIER, KPT, L_THREADS>, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((ls_ab_kernel<FOURIER, KPT, L_THREADS>), grid, dim3(L_THREADS), lds, st,
                       p, gx);
  } else {
    hipError_t e = raise_lds_limit((const void*)ls_kernel<FOURIER, KPT>, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((ls_kernel<FOURIER, KPT>), dim3(ninst), dim3(L_THREADS), lds, st, p);
  }
  return hipGetLastError();
}

template <bool FOURIER>
static hipError_t launch_ls_by_kpt(const LParams& p, int ninst, int G, bool split, size_t lds,
                                   int n, hipStream_t st) {
  switch (ls_kpt(n)) {
    case 1: return launch_ls_kpt<FOURIER, 1>(p, ninst, G, split, lds, st);
    case 2: return launch_ls_kpt<FOURIER, 2>(p, ninst, G, split, lds, st);
    case 4: return launch_ls_kpt<FOURIER, 4>(p, ninst, G, split, lds, st);
    case 8: return launch_ls_kpt<FOURIER, 8>(p, ninst, G, split, lds, st);
    default: return launch_ls_kpt<FOURIER, 16>(p, ninst, G, split, lds, st);
  }
}

template <bool FOURIER>
static hipError_t launch_ls_split(const LParams& p, int ninst, int G, int n, hipStream_t st) {
  const size_t lds = (size_t)n * (FOURIER ? 16 : 8) + 16;   // the Gram column
  const int cblocks = (n + L_THREADS - 1) / L_THREADS;
  hipError_t e = launch_ls_by_kpt<FOURIER>(p, ninst, G, true, lds, n, st);
  if (e != hipSuccess) return e;
  const bool xm = ls_xcd_map(p, ninst, cblocks);
  hipLaunchKernelGGL(ls_c_kernel<FOURIER>, xm ? dim3(cblocks * ninst) : dim3(cblocks, ninst),
                     dim3(L_THREADS), 0, st, p, G, xm ? cblocks : 0);
  return hipGetLastError();
}

hipError_t launch_ls_update_slots(const LParams& p, int ninst, int t_lo, int t_hi,
                                  hipStream_t st) {
  if (!p.tofs || t_lo < 1 || t_hi < t_lo || !p.wbuf || !p.vpart) return hipErrorInvalidValue;
  const int n_hi = t_hi - 1;
  if (n_hi > L_KPT * L_THREADS) return hipErrorInvalidValue;
  hipError_t e = hipSuccess;
  // instances on the one-workgroup update (t <= 64), sized for the longest
  if (ls_split_groups(t_lo) == 1) {
    const int n1 = std::max(1, std::min(t_hi, 64) - 1);
    const size_t wb = p.fourier ? 16 : 8;
    const size_t lds = 2 * n1 * wb + (size_t)n1 * 4 + 16;
    e = p.fourier ? launch_ls_by_kpt<true>(p, ninst, 1, false, lds, n1, st)
                  : launch_ls_by_kpt<false>(p, ninst, 1, false, lds, n1, st);
    if (e != hipSuccess) return e;
  }
  // instances on the split update, each with its own row split
  const int G = ls_split_groups(t_hi);
  if (G > 1)
    e = p.fourier ? launch_ls_split<true>(p, ninst, G, n_hi, st)
                  : launch_ls_split<false>(p, ninst, G, n_hi, st);
  return e;
}

hipError_t launch_ls_update(const LParams& p, int ninst, hipStream_t st) {
  const int G = ls_split_groups(p.t);
  const int n = p.t - 1;
  if (n > L_KPT * L_THREADS) return hipErrorInvalidValue;
  if (G > 1 && p.wbuf && p.vpart)
    return p.fourier ? launch_ls_split<true>(p, ninst, G, n, st)
                     : launch_ls_split<false>(p, ninst, G, n, st);
  const int n1 = n > 0 ? n : 1;
  const size_t wb = p.fourier ? 16 : 8;
  const size_t lds = 2 * n1 * wb + (size_t)n1 * 4 + 16;
  return p.fourier ? launch_ls_by_kpt<true>(p, ninst, 1, false, lds, n, st)
                   : launch_ls_by_kpt<false>(p, ninst, 1, false, lds, n, st);
}

}  // namespace fcmp
