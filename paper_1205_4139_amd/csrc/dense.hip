// Dense FP64 least squares on a support T (the set-based pursuits, SP and
// CoSaMP): Gram G = Phi_T^H Phi_T built from the kernel vector (column
// lambda of Phi^H Phi is P_lambda c, so G[a][b] = c(T_a (-) T_b)), right-hand
// side b = Phi_T^H y = h_0(T), blocked Cholesky G = L L^H, then forward and
// backward substitution.  The order s is padded to a multiple of 64 with an
// identity block, whose solution entries are zero.
#include "kernels.h"

namespace fcmp {

constexpr int NB = 64;

template <class Wd> __device__ __forceinline__ Wd wmul(Wd a, Wd b);
template <> __device__ __forceinline__ double wmul<double>(double a, double b) { return a * b; }
template <> __device__ __forceinline__ double2 wmul<double2>(double2 a, double2 b) { return cmul(a, b); }
// a * conj(b)
template <class Wd> __device__ __forceinline__ Wd wmulc(Wd a, Wd b);
template <> __device__ __forceinline__ double wmulc<double>(double a, double b) { return a * b; }
template <> __device__ __forceinline__ double2 wmulc<double2>(double2 a, double2 b) {
  return make_double2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
template <class Wd> __device__ __forceinline__ Wd wconj(Wd a);
template <> __device__ __forceinline__ double wconj<double>(double a) { return a; }
template <> __device__ __forceinline__ double2 wconj<double2>(double2 a) { return make_double2(a.x, -a.y); }
template <class Wd> __device__ __forceinline__ double wre(Wd a);
template <> __device__ __forceinline__ double wre<double>(double a) { return a; }
template <> __device__ __forceinline__ double wre<double2>(double2 a) { return a.x; }
template <class Wd> __device__ __forceinline__ Wd wreal(double a);
template <> __device__ __forceinline__ double wreal<double>(double a) { return a; }
template <> __device__ __forceinline__ double2 wreal<double2>(double a) { return make_double2(a, 0.0); }

// G (sp x sp, row-major, lower triangle used) and b; padded with identity.
template <class Wd, bool FOURIER>
__global__ void gram_kernel(const Wd* c64, const Wd* h0, const int32_t* T, int s, int sp, int N,
                            Wd* G, Wd* b) {
  const uint32_t mask = (uint32_t)N - 1u;
  const int64_t total = (int64_t)sp * sp;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(e / sp), j = (int)(e % sp);
    Wd v = vzero(Wd());
    if (j <= i) {
      if (i < s) {
        if (j < s) v = c64[perm_index(FOURIER, (uint32_t)T[i], (uint32_t)T[j], mask)];
      } else if (i == j) {
        v = wreal<Wd>(1.0);
      }
    }
    G[e] = v;
  }
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < sp; i += gridDim.x * blockDim.x)
    b[i] = i < s ? h0[T[i]] : vzero(Wd());
}

// Factor the diagonal block p in LDS (unblocked right-looking Cholesky).
template <class Wd>
__global__ void __launch_bounds__(256) potrf_diag_kernel(Wd* G, int sp, int p, int* bad) {
  __shared__ Wd A[NB][NB + 1];
  const int o = p * NB;
  for (int e = threadIdx.x; e < NB * NB; e += 256) {
    const int i = e / NB, j = e % NB;
    A[i][j] = G[(int64_t)(o + i) * sp + o + j];
  }
  __syncthreads();
  for (int k = 0; k < NB; ++k) {
    const double d2 = wre(A[k][k]);
    if (!(d2 > 0.0)) {
      if (threadIdx.x == 0) *bad = 1;
      return;   // uniform: every thread reads the same d2
    }
    const double d = sqrt(d2);
    __syncthreads();
    if (threadIdx.x == 0) A[k][k] = wreal<Wd>(d);
    for (int i = k + 1 + threadIdx.x; i < NB; i += 256) A[i][k] = vscale(A[i][k], 1.0 / d);
    __syncthreads();
    // trailing update of the lower triangle: A[i][j] -= L[i][k] conj(L[j][k])
    const int m = NB - k - 1;
    for (int e = threadIdx.x; e < m * m; e += 256) {
      const int i = k + 1 + e / m, j = k + 1 + e % m;
      if (j <= i) A[i][j] = vsub(A[i][j], wmulc(A[i][k], A[j][k]));
    }
    __syncthreads();
  }
  for (int e = threadIdx.x; e < NB * NB; e += 256) {
    const int i = e / NB, j = e % NB;
    if (j <= i) G[(int64_t)(o + i) * sp + o + j] = A[i][j];
  }
}

// Rows of the panel below block p: X L_pp^H = A  (one workgroup per 64 rows).
template <class Wd>
__global__ void __launch_bounds__(64) trsm_panel_kernel(Wd* G, int sp, int p) {
  __shared__ Wd Lp[NB][NB + 1];
  __shared__ Wd X[NB][NB + 1];
  const int o = p * NB;
  const int r0 = o + NB + blockIdx.x * NB;
  const int t = threadIdx.x;
  for (int e = t; e < NB * NB; e += 64) {
    const int i = e / NB, j = e % NB;
    Lp[i][j] = G[(int64_t)(o + i) * sp + o + j];
    X[i][j] = G[(int64_t)(r0 + i) * sp + o + j];
  }
  __syncthreads();
  // thread t solves row t
  for (int k = 0; k < NB; ++k) {
    Wd a = X[t][k];
    for (int m = 0; m < k; ++m) a = vsub(a, wmulc(X[t][m], Lp[k][m]));
    X[t][k] = vscale(a, 1.0 / wre(Lp[k][k]));
  }
  __syncthreads();
  for (int e = t; e < NB * NB; e += 64) {
    const int i = e / NB, j = e % NB;
    G[(int64_t)(r0 + i) * sp + o + j] = X[i][j];
  }
}

// Trailing update A[I][J] -= L[I][p] L[J][p]^H for block tiles I >= J > p.
template <class Wd>
__global__ void __launch_bounds__(256) syrk_kernel(Wd* G, int sp, int p) {
  const int I = p + 1 + blockIdx.y, J = p + 1 + blockIdx.x;
  if (J > I) return;
  __shared__ Wd Li[NB][NB + 1];
  __shared__ Wd Lj[NB][NB + 1];
  const int o = p * NB;
  for (int e = threadIdx.x; e < NB * NB; e += 256) {
    const int i = e / NB, k = e % NB;
    Li[i][k] = G[(int64_t)(I * NB + i) * sp + o + k];
    Lj[i][k] = G[(int64_t)(J * NB + i) * sp + o + k];
  }
  __syncthreads();
  // 4 x 4 outputs per thread
  const int ti = (threadIdx.x / 16) * 4, tj = (threadIdx.x % 16) * 4;
  Wd acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = vzero(Wd());
  for (int k = 0; k < NB; ++k) {
    Wd x[4], y[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) { x[a] = Li[ti + a][k]; y[a] = Lj[tj + a][k]; }
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) acc[a][b] = vadd(acc[a][b], wmulc(x[a], y[b]));
  }
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int64_t idx = (int64_t)(I * NB + ti + a) * sp + J * NB + tj + b;
      G[idx] = vsub(G[idx], acc[a][b]);
    }
}

__device__ __forceinline__ double wshfl(double v, int src) { return __shfl(v, src, 64); }
__device__ __forceinline__ double2 wshfl(double2 v, int src) {
  return make_double2(__shfl(v.x, src, 64), __shfl(v.y, src, 64));
}

// Forward then backward substitution with L (one workgroup of 1024): x = G^{-1} b.
// Each 64 x 64 diagonal block is solved by wave 0 alone, lane t holding entry
// t and shuffles broadcasting the finished entries; the other blocks' right-hand
// sides are then updated by all threads.
template <class Wd>
__global__ void __launch_bounds__(1024) chol_solve_kernel(const Wd* G, int sp, Wd* b, Wd* x,
                                                          Wd* xout, int s) {
  const int t = threadIdx.x;
  const int nb = sp / NB;
  // forward: L z = b (z overwrites b)
  for (int p = 0; p < nb; ++p) {
    const int o = p * NB;
    if (t < 64) {
      Wd v = b[o + t];
      for (int m = 0; m < NB; ++m) {
        const Wd zm = vscale(wshfl(v, m), 1.0 / wre(G[(int64_t)(o + m) * sp + o + m]));
        if (t == m) v = zm;
        else if (t > m) v = vsub(v, wmul(G[(int64_t)(o + t) * sp + o + m], zm));
      }
      b[o + t] = v;
    }
    __syncthreads();
    for (int i = o + NB + t; i < sp; i += 1024) {
      Wd acc = vzero(Wd());
      const Wd* Li = G + (int64_t)i * sp + o;
      for (int m = 0; m < NB; ++m) acc = vadd(acc, wmul(Li[m], b[o + m]));
      b[i] = vsub(b[i], acc);
    }
    __syncthreads();
  }
  // backward: L^H x = z
  for (int p = nb - 1; p >= 0; --p) {
    const int o = p * NB;
    if (t < 64) {
      Wd v = b[o + t];
      for (int m = NB - 1; m >= 0; --m) {
        const Wd xm = vscale(wshfl(v, m), 1.0 / wre(G[(int64_t)(o + m) * sp + o + m]));
        if (t == m) v = xm;
        else if (t < m) v = vsub(v, wmul(wconj(G[(int64_t)(o + m) * sp + o + t]), xm));
      }
      x[o + t] = v;
    }
    __syncthreads();
    for (int k = t; k < o; k += 1024) {
      Wd acc = vzero(Wd());
      for (int m = 0; m < NB; ++m)
        acc = vadd(acc, wmul(wconj(G[(int64_t)(o + m) * sp + k]), x[o + m]));
      b[k] = vsub(b[k], acc);
    }
    __syncthreads();
  }
  // only the s leading entries belong to the caller (the rest is padding)
  for (int i = t; i < s; i += 1024) xout[i] = x[i];
}

template <class Wd, bool FOURIER>
static hipError_t dense_t(const void* c64, const void* h0, const int32_t* T, int s, int N,
                          void* G, void* b, void* x, int* bad, hipStream_t st) {
  const int sp = (s + NB - 1) / NB * NB;
  const int64_t total = (int64_t)sp * sp;
  const int groups = (int)std::min<int64_t>(4096, (total + 255) / 256);
  hipLaunchKernelGGL((gram_kernel<Wd, FOURIER>), dim3(groups), dim3(256), 0, st, (const Wd*)c64,
                     (const Wd*)h0, T, s, sp, N, (Wd*)G, (Wd*)b);
  const int nb = sp / NB;
  for (int p = 0; p < nb; ++p) {
    hipLaunchKernelGGL(potrf_diag_kernel<Wd>, dim3(1), dim3(256), 0, st, (Wd*)G, sp, p, bad);
    const int rest = nb - p - 1;
    if (rest > 0) {
      hipLaunchKernelGGL(trsm_panel_kernel<Wd>, dim3(rest), dim3(64), 0, st, (Wd*)G, sp, p);
      hipLaunchKernelGGL(syrk_kernel<Wd>, dim3(rest, rest), dim3(256), 0, st, (Wd*)G, sp, p);
    }
  }
  Wd* xs = (Wd*)b + sp;   // padded solution, workspace-owned
  hipLaunchKernelGGL(chol_solve_kernel<Wd>, dim3(1), dim3(1024), 0, st, (const Wd*)G, sp, (Wd*)b,
                     xs, (Wd*)x, s);
  return hipGetLastError();
}

size_t dense_ls_workspace(int s_max, bool fourier) {
  const size_t sp = (size_t)(s_max + NB - 1) / NB * NB;
  const size_t wb = fourier ? 16 : 8;
  return (sp * sp + 3 * sp) * wb + 1024;
}

hipError_t launch_dense_ls(int fourier, const void* c64, const void* h0, const int32_t* T, int s,
                           int N, void* ws, void* x, int* bad, hipStream_t st) {
  const size_t sp = (size_t)(s + NB - 1) / NB * NB;
  const size_t wb = fourier ? 16 : 8;
  char* w = (char*)ws;
  void* G = w;
  void* b = w + sp * sp * wb;
  if (fourier) return dense_t<double2, true>(c64, h0, T, s, N, G, b, x, bad, st);
  return dense_t<double, false>(c64, h0, T, s, N, G, b, x, bad, st);
}

}  // namespace fcmp
