// Small helper kernels: fills, gathers, status initialisation, result copy-out,
// the final reduction of identification partials and measurement noise.
#include "kernels.h"

#include <mutex>
#include <unordered_map>

namespace fcmp {

hipError_t raise_lds_limit(const void* kernel, size_t bytes) {
  if (bytes <= 65536) return hipSuccess;
  static std::mutex mu;
  static std::unordered_map<const void*, size_t> set;
  std::lock_guard<std::mutex> lk(mu);
  size_t& cur = set[kernel];
  if (bytes <= cur) return hipSuccess;
  hipError_t e = hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  if (e == hipSuccess) cur = bytes;
  return e;
}

__global__ void fill_u32_kernel(uint32_t* p, uint32_t v, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ void to_int16_kernel(const double* in, int16_t* out, double mul, int64_t n,
                                int64_t ii, int64_t io) {
  const int inst = blockIdx.y;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    out[inst * io + i] = (int16_t)rint(mul * in[inst * ii + i]);
}

hipError_t launch_to_int16(const double* in, int16_t* out, double mul, int64_t n, int64_t inst_in,
                           int64_t inst_out, int ninst, hipStream_t st) {
  int64_t groups = (n + 255) / 256;
  if (groups > 1024) groups = 1024;
  hipLaunchKernelGGL(to_int16_kernel, dim3((unsigned)groups, ninst), dim3(256), 0, st, in, out, mul,
                     n, inst_in, inst_out);
  return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  int64_t groups = (n + 255) / 256;
  if (groups > 4096) groups = 4096;
  hipLaunchKernelGGL(fill_u32_kernel, dim3((unsigned)groups), dim3(256), 0, st, p, v, n);
  return hipGetLastError();
}

template <class Wd>
__global__ void gather_kernel(const Wd* src, const int32_t* idx, Wd* dst, int64_t n,
                              int64_t is, int64_t ii, int64_t id) {
  const int inst = blockIdx.y;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x)
    dst[inst * id + e] = src[inst * is + idx[inst * ii + e]];
}

hipError_t launch_gather_wide(int vk, const void* src, const int32_t* idx, void* dst,
                              int64_t n, int64_t is, int64_t ii, int64_t id, int ninst,
                              hipStream_t st) {
  if (n <= 0) return hipSuccess;
  int64_t groups = (n + 255) / 256;
  if (groups > 2048) groups = 2048;
  dim3 grid((unsigned)groups, ninst);
  const size_t eb = vbytes(vk);
  if (eb == 16)
    hipLaunchKernelGGL(gather_kernel<double2>, grid, dim3(256), 0, st, (const double2*)src, idx,
                       (double2*)dst, n, is, ii, id);
  else if (eb == 8)
    hipLaunchKernelGGL(gather_kernel<uint64_t>, grid, dim3(256), 0, st, (const uint64_t*)src,
                       idx, (uint64_t*)dst, n, is, ii, id);
  else
    hipLaunchKernelGGL(gather_kernel<uint32_t>, grid, dim3(256), 0, st, (const uint32_t*)src,
                       idx, (uint32_t*)dst, n, is, ii, id);
  return hipGetLastError();
}

template <class Wd>
__global__ void finalize_kernel(const Status* status, const int32_t* lam, const Wd* x, int K,
                                int32_t* sup, Wd* xo) {
  const int it = status->iterations;
  for (int i = threadIdx.x + blockIdx.x * blockDim.x; i < K; i += blockDim.x * gridDim.x) {
    const bool ok = i < it;
    sup[i] = ok ? lam[i] : -1;
    xo[i] = ok ? x[i] : vzero(Wd());
  }
}

hipError_t launch_finalize(int fourier, const Status* status, const int32_t* lam, const void* x,
                           int K, int32_t* sup, void* xo, hipStream_t st) {
  const int groups = (K + 255) / 256;
  if (fourier)
    hipLaunchKernelGGL(finalize_kernel<double2>, dim3(groups), dim3(256), 0, st, status, lam,
                       (const double2*)x, K, sup, (double2*)xo);
  else
    hipLaunchKernelGGL(finalize_kernel<double>, dim3(groups), dim3(256), 0, st, status, lam,
                       (const double*)x, K, sup, (double*)xo);
  return hipGetLastError();
}

__global__ void status_done_kernel(Status* s, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) s[i].done = 1;
}

hipError_t launch_status_done(Status* s, int n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(status_done_kernel, dim3((n + 255) / 256), dim3(256), 0, st, s, n);
  return hipGetLastError();
}

__global__ void reduce_sel_kernel(const Sel* partial, int n, Sel* out) {
  __shared__ Sel red[16];
  double bk = -1.0, bk2 = -1.0;
  int64_t bi = -1;
  for (int e = threadIdx.x; e < n; e += blockDim.x) {
    const Sel s = partial[e];
    if (s.idx >= 0) sel_merge(s.key, s.idx, s.key2, bk, bi, bk2);
  }
  const Sel r = block_sel_reduce(bk, bi, bk2, red);
  if (threadIdx.x == 0) *out = r;
}

hipError_t launch_reduce_sel(const Sel* partial, int n, Sel* out, hipStream_t st) {
  hipLaunchKernelGGL(reduce_sel_kernel, dim3(1), dim3(256), 0, st, partial, n, out);
  return hipGetLastError();
}

// status[inst] = {0...}, ynorm2 = ||y||^2 (one workgroup per instance)
__global__ void init_status_kernel(Status* st, const double* y, int64_t nreal, int64_t inst_y,
                                   const int32_t* Mv, int per_row, double res_tol2) {
  __shared__ double dred[16];
  const int inst = blockIdx.x;
  if (Mv) nreal = (int64_t)Mv[inst] * per_row;
  const double* yi = y + (int64_t)inst * inst_y;
  double s = 0.0;
  for (int64_t e = threadIdx.x; e < nreal; e += blockDim.x) s += yi[e] * yi[e];
  s = block_sum(s, dred);
  if (threadIdx.x == 0) {
    Status z;
    z.done = 0; z.numeric = 0; z.iterations = 0; z.cur_j = -1;
    z.znorm2 = 0.0; z.ynorm2 = s; z.last_key = 0.0; z.t_done = 0.0;
    z.min_gap = __builtin_inf(); z.res_tol2 = res_tol2;
    st[inst] = z;
  }
}

hipError_t launch_init_status(Status* st_dev, const void* y, int M, int fourier, int64_t inst_y,
                              int ninst, hipStream_t st, const int32_t* Mv, double res_tol2) {
  const int64_t nreal = fourier ? 2 * (int64_t)M : M;
  const int64_t istride = fourier ? 2 * inst_y : inst_y;
  hipLaunchKernelGGL(init_status_kernel, dim3(ninst), dim3(256), 0, st, st_dev,
                     (const double*)y, nreal, istride, Mv, fourier ? 2 : 1, res_tol2);
  return hipGetLastError();
}

// y = clean + g * ||clean|| / ||g|| * 10^(-snr/20), one workgroup (M real or complex)
__global__ void noise_kernel(const double* clean, const double* g, double snr_db, double* y,
                             int64_t nreal) {
  __shared__ double dred[16];
  double a = 0.0, b = 0.0;
  for (int64_t e = threadIdx.x; e < nreal; e += blockDim.x) {
    a += clean[e] * clean[e];
    b += g[e] * g[e];
  }
  a = block_sum(a, dred);
  b = block_sum(b, dred);
  const double sc = (b > 0.0) ? sqrt(a / b) * pow(10.0, -snr_db / 20.0) : 0.0;
  for (int64_t e = threadIdx.x; e < nreal; e += blockDim.x) y[e] = clean[e] + g[e] * sc;
}

hipError_t launch_noise(int fourier, const void* clean, const void* noise, double snr_db, void* y,
                        int M, hipStream_t st) {
  const int64_t nreal = fourier ? 2 * (int64_t)M : M;
  hipLaunchKernelGGL(noise_kernel, dim3(1), dim3(1024), 0, st, (const double*)clean,
                     (const double*)noise, snr_db, (double*)y, nreal);
  return hipGetLastError();
}

// dst[b][p] = src_b[idx[b][p]] with src_b = ptrs[b] (per-instance caller buffers)
template <class T>
__global__ void gather_ptr_kernel(const T* const* ptrs, const int32_t* idx, T* dst, int64_t n,
                                  int64_t ii, int64_t id, const int32_t* Mv) {
  const int inst = blockIdx.y;
  const T* src = ptrs[inst];
  if (Mv) n = Mv[inst];
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x)
    dst[inst * id + e] = src[idx[inst * ii + e]];
}

hipError_t launch_gather_ptr(int vk, const void* const* ptrs, const int32_t* idx, void* dst,
                             int64_t n, int64_t ii, int64_t id, int ninst, hipStream_t st,
                             const int32_t* Mv) {
  if (n <= 0) return hipSuccess;
  int64_t groups = (n + 255) / 256;
  if (groups > 1024) groups = 1024;
  dim3 grid((unsigned)groups, ninst);
  if (vbytes(vk) == 16)
    hipLaunchKernelGGL(gather_ptr_kernel<double2>, grid, dim3(256), 0, st,
                       (const double2* const*)ptrs, idx, (double2*)dst, n, ii, id, Mv);
  else
    hipLaunchKernelGGL(gather_ptr_kernel<double>, grid, dim3(256), 0, st,
                       (const double* const*)ptrs, idx, (double*)dst, n, ii, id, Mv);
  return hipGetLastError();
}

template <class Wd>
__global__ void finalize_ptr_kernel(const Status* status, const int32_t* lam, const Wd* x, int K,
                                    int64_t il, int64_t ix, int32_t* const* sup, Wd* const* xo,
                                    const int32_t* Kv) {
  const int inst = blockIdx.y;
  if (Kv) K = Kv[inst];
  const int it = status[inst].iterations;
  int32_t* s = sup[inst];
  Wd* xd = xo[inst];
  for (int i = threadIdx.x + blockIdx.x * blockDim.x; i < K; i += blockDim.x * gridDim.x) {
    const bool ok = i < it;
    s[i] = ok ? lam[inst * il + i] : -1;
    xd[i] = ok ? x[inst * ix + i] : vzero(Wd());
  }
}

hipError_t launch_finalize_ptr(int fourier, const Status* status, const int32_t* lam,
                               const void* x, int K, int64_t il, int64_t ix,
                               int32_t* const* sup, void* const* xo, int ninst, hipStream_t st,
                               const int32_t* Kv) {
  dim3 grid((K + 255) / 256, ninst);
  if (fourier)
    hipLaunchKernelGGL(finalize_ptr_kernel<double2>, grid, dim3(256), 0, st, status, lam,
                       (const double2*)x, K, il, ix, sup, (double2* const*)xo, Kv);
  else
    hipLaunchKernelGGL(finalize_ptr_kernel<double>, grid, dim3(256), 0, st, status, lam,
                       (const double*)x, K, il, ix, sup, (double* const*)xo, Kv);
  return hipGetLastError();
}

}  // namespace fcmp

namespace fcmp {

// bits of the listed columns set in an N-bit map (map cleared first by the caller)
__global__ void set_bits_kernel(uint32_t* bm, const int32_t* idx, int n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const uint32_t j = (uint32_t)idx[i];
    atomicOr(&bm[j >> 5], 1u << (j & 31));
  }
}

hipError_t launch_set_bits(uint32_t* bm, int64_t nwords, const int32_t* idx, int n,
                           hipStream_t st) {
  hipError_t e = launch_fill_u32(bm, 0u, nwords, st);
  if (e != hipSuccess || n <= 0) return e;
  hipLaunchKernelGGL(set_bits_kernel, dim3((n + 255) / 256), dim3(256), 0, st, bm, idx, n);
  return hipGetLastError();
}

// out[0] = Re(sum_i conj(h0[S_i]) a_i), out[1] = Re(a^H G_S a) with
// G_S[i][j] = c(S_i (-) S_j)   (one workgroup)
template <class Wd, bool FOURIER>
__global__ void set_quad_kernel(const Wd* c64, const Wd* h0, const int32_t* S, const Wd* a,
                                int s, int N, double* out) {
  __shared__ double red[16];
  const uint32_t mask = (uint32_t)N - 1u;
  double lin = 0.0, quad = 0.0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < s; i += gridDim.x * blockDim.x) {
    const Wd ai = a[i];
    const Wd hi = h0[S[i]];
    Wd g = vzero(Wd());
    for (int j = 0; j < s; ++j) {
      const Wd cij = c64[perm_index(FOURIER, (uint32_t)S[i], (uint32_t)S[j], mask)];
      if constexpr (FOURIER) { const double2 t = cmul(cij, a[j]); g.x += t.x; g.y += t.y; }
      else g += cij * a[j];
    }
    if constexpr (FOURIER) {
      lin += hi.x * ai.x + hi.y * ai.y;
      quad += ai.x * g.x + ai.y * g.y;
    } else {
      lin += hi * ai;
      quad += ai * g;
    }
  }
  lin = block_sum(lin, red);
  quad = block_sum(quad, red);
  if (threadIdx.x == 0) { out[2 * blockIdx.x] = lin; out[2 * blockIdx.x + 1] = quad; }
}

int set_quad_groups(int s) { return std::max(1, std::min(64, (s + 255) / 256)); }

hipError_t launch_set_quad(int fourier, const void* c64, const void* h0, const int32_t* S,
                           const void* a, int s, int N, double* out, hipStream_t st) {
  const int g = set_quad_groups(s);
  if (fourier)
    hipLaunchKernelGGL((set_quad_kernel<double2, true>), dim3(g), dim3(256), 0, st,
                       (const double2*)c64, (const double2*)h0, S, (const double2*)a, s, N, out);
  else
    hipLaunchKernelGGL((set_quad_kernel<double, false>), dim3(g), dim3(256), 0, st,
                       (const double*)c64, (const double*)h0, S, (const double*)a, s, N, out);
  return hipGetLastError();
}

}  // namespace fcmp
