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
constexpr int L_KPT = 16;     // columns per thread in the w^H W product: K <= 4096

template <bool FOURIER>
__global__ void __launch_bounds__(L_THREADS) ls_kernel(LParams p) {
  using Wd = typename std::conditional<FOURIER, double2, double>::type;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ Sel red[16];
  __shared__ double dred[16];
  const int inst = blockIdx.x;
  Status* st = p.status + inst;
  if (st->done) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int nwaves = L_THREADS / 64;
  const int n = p.t - 1;     // previous selections
  Wd* g = (Wd*)smem_raw;     // g, then the new row of W
  Wd* w = g + (n > 0 ? n : 1);
  int32_t* sl = (int32_t*)(w + (n > 0 ? n : 1));

  // ---- step 3: reduce the per-workgroup partials
  const Sel* part = p.partial + (int64_t)inst * p.inst_part;
  double bk = -1.0;
  int64_t bi = -1;
  for (int e = tid; e < p.npart; e += L_THREADS) {
    const Sel s = part[e];
    if (s.idx >= 0 && sel_better(s.key, s.idx, bk, bi)) { bk = s.key; bi = s.idx; }
  }
  const Sel best = block_sel_reduce(bk, bi, red);
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
  for (int i = wave; i < n; i += nwaves) {
    const Wd* Wi = W + (int64_t)i * (i + 1) / 2;
    Wd s = vzero(Wd());
    for (int k = lane; k <= i; k += 64) {
      if constexpr (FOURIER) { const double2 t = cmul(Wi[k], g[k]); s.x += t.x; s.y += t.y; }
      else s += Wi[k] * g[k];
    }
    if constexpr (FOURIER) { s.x = wave_sum(s.x); s.y = wave_sum(s.y); }
    else s = wave_sum(s);
    if (lane == 0) w[i] = s;
  }
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
  Wd acc[L_KPT];
#pragma unroll
  for (int q = 0; q < L_KPT; ++q) acc[q] = vzero(Wd());
  const int nq = (n + L_THREADS - 1) / L_THREADS;
  for (int i = 0; i < n; ++i) {
    const Wd* Wi = W + (int64_t)i * (i + 1) / 2;
    const Wd wi = w[i];
#pragma unroll
    for (int q = 0; q < L_KPT; ++q) {
      if (q >= nq) break;
      const int k = tid + q * L_THREADS;
      if (k <= i) {
        if constexpr (FOURIER) { const double2 t = cmulc(wi, Wi[k]); acc[q].x += t.x; acc[q].y += t.y; }
        else acc[q] += wi * Wi[k];
      }
    }
  }
  __syncthreads();   // everyone is done reading g
  Wd* Wn = W + (int64_t)n * (n + 1) / 2;
#pragma unroll
  for (int q = 0; q < L_KPT; ++q) {
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
    st->iterations = p.t;
    st->last_key = best.key;
  }
}

hipError_t launch_ls_update(const LParams& p, int ninst, hipStream_t st) {
  const int n = p.t - 1 > 0 ? p.t - 1 : 1;
  const size_t wb = p.fourier ? 16 : 8;
  const size_t lds = 2 * n * wb + (size_t)n * 4 + 16;
  if (p.fourier) {
    if (lds > 65536)
      hipFuncSetAttribute((const void*)ls_kernel<true>,
                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(ls_kernel<true>, dim3(ninst), dim3(L_THREADS), lds, st, p);
  } else {
    if (lds > 65536)
      hipFuncSetAttribute((const void*)ls_kernel<false>,
                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(ls_kernel<false>, dim3(ninst), dim3(L_THREADS), lds, st, p);
  }
  return hipGetLastError();
}

}  // namespace fcmp
