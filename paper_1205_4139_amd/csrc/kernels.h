// Launch interfaces of the HIP kernels (host side).
#pragma once
#include "common.h"

namespace fcmp {

enum VKind { V_F32 = 0, V_F64 = 1, V_C64 = 2, V_C128 = 3 };

inline size_t vbytes(int vk) { return vk == V_F32 ? 4 : (vk == V_C128 ? 16 : 8); }
inline bool vcomplex(int vk) { return vk >= V_C64; }
inline int vwide(int vk) { return vcomplex(vk) ? V_C128 : V_F64; }
inline int vnarrow_kind(int vk) { return vcomplex(vk) ? V_C64 : V_F32; }

// ------------------------------------------------------------------ transforms
// One kernel runs B length-L transforms per workgroup through LDS.  Element
// (s, i) of a sequence s is read from in[s*in_ss + i*in_es] (dense input) or
// scattered from a list of (k, value) entries (sparse input: the zero-filled
// residual of the correlation step); output element (s, j) goes to
// out[s*out_ss + j*out_es].  The FFT is the in-place decimation-in-time form
// (bit-reversed placement on input, natural order out); the WHT is the
// in-place natural-order form.  The identification argmax can be fused into
// the output loop.
enum InMode { IN_DENSE = 0, IN_SPARSE = 1, IN_SPARSE_ONES = 2, IN_TAPS = 3 };

// Offset of the stage twiddles of span h (a power of two >= 2) in the
// per-span table: span h holds, for k < h and register m = 1..15, the value
// W_{16h}^{rev4(m) k} = e^{2 pi i rev4(m) k / (16 h)} at 15 (h - 2) + 15 k + m - 1.
__host__ __device__ constexpr int64_t stage_tw_offset(int64_t h) { return 15 * (h - 2); }
__host__ __device__ constexpr int64_t stage_tw_count(int64_t hmax) {
  return hmax >= 2 ? 15 * (2 * hmax - 2) : 0;
}

struct XParams {
  int L, logL, B;          // transform length and sequences per workgroup
  int N, logN, twS;        // problem size; twiddle table split
  int sign;                // +1: e^{+2 pi i ...} (U^H), -1: e^{-2 pi i ...} (U)
  int in_mode;
  int in_kind;             // VKind of the input values
  const void* in;
  int64_t in_ss, in_es;
  const int32_t* ent_k;    // sparse: k of each entry (entry order)
  const int32_t* goff;     // sparse: per-workgroup entry ranges; NULL: all entries
  int32_t nent;
  int goff_span, goff2_span;   // table groups per workgroup (a single-workgroup
                               // transform covers every group of the table)
  int logN1;               // sparse: k -> (i = k >> logN1, s = k & (N1-1))
  void* out;  int out_kind;    // -1: none
  void* out2; int out2_kind;   // -1: none
  int64_t out_ss, out_es;
  int inter_tw;            // multiply output (s, j) by W_N^{s j}
  double scale;
  Sel* partial;            // nullable: one (key, idx) per workgroup
  const uint32_t* excl;    // nullable exclusion bitmap (global h index)
  const void* tw_lo;       // twiddles in the transform precision, sign +
  const void* tw_hi;       //   (two-level table, for the inter-pass twiddle)
  const void* tws;         // per-span stage twiddles (lds_fft), sign +
  const Status* status;    // nullable: skip when status[inst].done
  // per-instance strides (blockIdx.y), in elements of each array
  int64_t inst_in, inst_ent, inst_goff, inst_out, inst_out2, inst_part, inst_excl;
  int nthreads;
  int role;                // 0 single workgroup, 1 pass 1, 2 pass 2 (profiler name only)
  // IN_TAPS: the sparse vector S_Lambda^T x from (lam, x) pairs
  const int32_t* taps_lam; const void* taps_x; int ntaps;
  int64_t inst_taps_lam, inst_taps_x;
  // residual output: r[q] = yres[q] - out(k) for the rows k of Omega this
  // workgroup produces (entries [goff2[g], goff2[g+1]) of ent2_k; q = pos1[e])
  int resid;
  const int32_t* ent2_k; const int32_t* goff2; const int32_t* pos1; int nent2;
  const void* yres; int yres_kind; void* rout; int r_kind; int log_out_es;
  int64_t inst_ent2, inst_goff2, inst_yres, inst_rout;
  // staging of exclusion bits: 0 none, 1 contiguous outputs, 2 strided outputs
  int excl_mode;
  // residual output in plans with per-instance row counts: only instances
  // with rsel_M[inst] * rsel_ntaps > rsel_thr take the transform residual
  const int32_t* rsel_M; int rsel_ntaps; double rsel_thr;
};

// vk: VKind of the transform arithmetic; fft: Fourier (else Hadamard)
hipError_t launch_xform(int vk, bool fft, const XParams& p, int groups, int ninst,
                        hipStream_t st);
size_t xform_lds_bytes(int vk, bool fft, const XParams& p);
// Register-resident second pass with the identification fused (rows of
// length 256, 512 or 1024, outputs identified and not stored): xrow_q gives
// Q = L / 256 when the pass qualifies, else 0.
int xrow_q(const XParams& b);
hipError_t launch_xrow(int vk, bool fft, const XParams& b, int ninst, hipStream_t st);
// First pass of an FP64 two-pass transform of a taps input evaluated
// directly (a few taps per column); ok when the tile and tap count suit it.
bool taps_pass1_ok(const XParams& a, int vk);
hipError_t launch_taps_pass1(const XParams& a, int vk, int groups, int ninst, hipStream_t st);

// ------------------------------------------------------------------ fused residual
// The residual r = y - S_Omega U S_Lambda^T x at the rows of one first-pass
// correlation workgroup, computed from the taps in FP64, followed by that
// workgroup's correlation first pass (same geometry and output as pass 1 of
// a two-pass transform).  Taps are read in bucket order: ord lists the tap
// indices sorted by (bucket, index), taps of bucket l at [bstart[l],
// bstart[l+1]); bucket = lam mod N2 (Fourier) or lam >> log2 N1 (Hadamard).
struct RCParams {
  int N, logN, twS;
  int L, logL, B, logN1;   // L = N2 and B columns (k mod N1) per workgroup
  // taps: ord and bstart hold two buffers per instance (the parity of the tap
  // count selects one, ord_half / bstart_half apart)
  const int32_t* lam; const void* x; const int32_t* ord; const int32_t* bstart; int ntaps;
  int64_t inst_lam, inst_x, inst_ord, inst_bstart, ord_half, bstart_half;
  // nullable: per-instance iteration offsets (instance i has ntaps - tofs[i]
  // taps) and K (an instance with K taps made is skipped)
  const int32_t* tofs; const int32_t* Kv;
  const int32_t* ent_k;    // rows of Omega, sorted by column (k mod N1), then by row
  const int32_t* goff;     // entry index of the first row of each column (N1 + 1 values)
  const void* y;           // FP64 (wide) in entry order
  int64_t inst_ent, inst_goff, inst_y;
  double rscale;           // N^{-1/2}
  const void* twr_lo; const void* twr_hi; const void* twr_st;   // FP64 twiddles, sign +
  const void* twc_lo; const void* twc_hi; const void* twc_st;   // correlation precision, sign +
  void* out; int64_t inst_out;   // pass-1 output: out[(s0 + c) + N1 j]
  const Status* status;
  // rows of Omega per column (entries sorted by column, then row): bit m of
  // word m / 32 of column c marks row c + N1 m; cbase holds the entry index of
  // the first marked row at or after 32 (m / 32); N2 / 32 words per column
  const uint32_t* cmask; const int32_t* cbase; int64_t inst_cmask;
};
bool rcorr_ok(int pk, bool fft, const RCParams& p, int nthreads);
hipError_t launch_rcorr(int pk, bool fft, const RCParams& p, int groups, int ninst, int nthreads,
                        hipStream_t st);
// The register-resident variant for N2 = 256 rows per column (N = 2^16 .. 2^18),
// 16 columns per workgroup; needs cmask and cbase.
bool rcorr_reg_ok(int pk, bool fft, const RCParams& p);
hipError_t launch_rcorr_reg(int pk, bool fft, const RCParams& p, int ninst, hipStream_t st);

// ------------------------------------------------------------------ residual
// r[e] = y[e] - sum_tau U(k_e, lam_tau) x_tau for the current support, in FP64,
// stored in the correlation precision (Algorithm 1.1, step 7).
struct RParams {
  int N, logN, twS;
  int fourier;
  int32_t M;
  const int32_t* ent_k;    // entry order
  const void* y;           // FP64 (wide) in entry order
  void* r;  int r_kind;    // output
  const int32_t* lam;      // selected columns
  const void* x;           // FP64 (wide) coefficients
  int ntaps;
  const void* tw_lo;       // FP64 twiddles, sign +
  const void* tw_hi;
  const Status* status;
  int64_t inst_ent, inst_y, inst_r, inst_lam, inst_x;
  // per-instance row counts (nullable: M for all); with Mv, only instances
  // with Mv[inst] * ntaps <= thr are handled here (the rest take the
  // transform residual)
  const int32_t* Mv; double thr;
};
hipError_t launch_residual(const RParams& p, int ninst, hipStream_t st);

// ------------------------------------------------------------------ fast path
// h(j) = h0(j) - sum_tau x_tau c((j - lam_tau) mod N) (Fourier) or
// c(j XOR lam_tau) (Hadamard), eq. (kernelsum); FP64 accumulation.
struct FParams {
  int N, logN;
  int fourier;
  int c_kind;              // VKind of the stored kernel vector
  int c_int16;             // Hadamard: c holds the integers N c as int16 (c_kind ignored)
  int c_half;              // Fourier: read c(m) for m > N/2 as conj(c(N - m))
  double cscale;           //   and c(j) = cscale * (N c)(j), cscale = 1/N (exact)
  const void* h0;          // FP64 (wide)
  const void* c;
  const int32_t* lam;
  const void* x;           // FP64 (wide)
  int ntaps;
  void* h;                 // nullable FP64 (wide) output
  Sel* partial;
  const uint32_t* excl;
  const Status* status;
  int64_t inst_h0, inst_c, inst_lam, inst_x, inst_h, inst_part, inst_excl;
  // set by the launcher: workgroups per instance, and whether the grid is
  // one-dimensional with every workgroup of instance i on XCD i mod 8
  int groups, xcd_map;
};
hipError_t launch_fastcorr(const FParams& p, int ninst, int* groups_out, hipStream_t st);
// The conjugate-symmetric pairing (Fourier, N <= 8192, h0 and x FP64): one
// workgroup per instance, h in LDS, one identification partial per instance.
bool fastpair_ok(const FParams& p);
hipError_t launch_fastpair(const FParams& p, int ninst, int* groups_out, hipStream_t st);
int fastcorr_groups(int N);

// ------------------------------------------------------------------ least squares
// Selects lambda_t from the partials, appends it to the support, extends the
// inverse Cholesky factor W = L^{-1} of the Gram by one row, updates z = W b
// and x = W^H z (Algorithm 1.1, steps 3-6).
struct LParams {
  int N;
  int fourier;
  int t;                   // this call makes selection number t (1-based)
  const int32_t* tofs;     // nullable: instance i makes selection t - tofs[i]
  const Sel* partial;  int npart;
  const void* c64;         // FP64 kernel vector (Gram entries)
  const void* h0;          // FP64 h_0 = Phi^H y (right-hand side b = h0(Lambda))
  void* W;                 // packed rows, t(t+1)/2 entries
  void* z;  void* x;
  int32_t* lam;
  uint32_t* excl;
  Status* status;
  int64_t inst_part, inst_c, inst_h0, inst_W, inst_z, inst_x, inst_lam, inst_excl;
  // scratch for the split update (nullable: then one workgroup per instance)
  void* wbuf; int64_t inst_wbuf;          // w = W g, K values
  void* vpart; int64_t inst_vpart;        // ls_split_groups(K) partial rows of w^H W, K values each
  int64_t vpart_stride;
  const int32_t* Kv;       // nullable: per-instance K; an instance whose K
                           // selections are made is marked done at t = K + 1
  // nullable: bucket order of the taps for the fused residual, two buffers
  // per instance (parity of the tap count); bucket = (lam >> bshift) & (nbuck-1)
  int32_t* ord; int32_t* bstart;
  int64_t inst_ord, inst_bstart, ord_half, bstart_half;
  int nbuck, bshift;
};
hipError_t launch_ls_update(const LParams& p, int ninst, hipStream_t st);
constexpr int LS_MAX_GROUPS = 256;  // most partial rows of w^H W (long supports)
// Workgroups per instance of the least-squares update at iteration t (1: the
// one-workgroup kernel); a function of t only, so every sum's order is too.
__host__ __device__ inline int ls_split_groups(int t) {
  const int n = t - 1;
  if (n < 64) return 1;
  int G = n / 24;
  if (G < 2) G = 2;
  if (G > LS_MAX_GROUPS) G = LS_MAX_GROUPS;
  return G;
}
// Instances at different iterations (tofs set): p.t is the step, instance i
// makes selection p.t - tofs[i], and t_lo / t_hi bound those of the instances
// that are not done.
hipError_t launch_ls_update_slots(const LParams& p, int ninst, int t_lo, int t_hi,
                                  hipStream_t st);

// ------------------------------------------------------------------ utilities
hipError_t launch_fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t st);
// out[i] = round(mul * in[i]) as int16 for n values of ninst instances
// (the Hadamard kernel vector's integers N c)
hipError_t launch_to_int16(const double* in, int16_t* out, double mul, int64_t n, int64_t inst_in,
                           int64_t inst_out, int ninst, hipStream_t st);
hipError_t launch_gather_wide(int vk, const void* src, const int32_t* idx, void* dst,
                              int64_t n, int64_t inst_src, int64_t inst_idx, int64_t inst_dst,
                              int ninst, hipStream_t st);
hipError_t launch_finalize(int fourier, const Status* status, const int32_t* lam,
                           const void* x, int K, int32_t* support_out, void* x_out,
                           hipStream_t st);
hipError_t launch_reduce_sel(const Sel* partial, int n, Sel* out, hipStream_t st);
// Mv / Kv (nullable): per-instance counts, at most M / K; NULL: M / K for all.
// res_tol2: a solve stops once ||r||^2 <= res_tol2 ||y||^2 (0: never)
// Marks n status records done (every later iteration kernel skips them).
hipError_t launch_status_done(Status* s, int n, hipStream_t st);
hipError_t launch_init_status(Status* st_dev, const void* y, int M, int fourier,
                              int64_t inst_y, int ninst, hipStream_t st,
                              const int32_t* Mv = nullptr, double res_tol2 = 0.0);
hipError_t launch_gather_ptr(int vk, const void* const* ptrs, const int32_t* idx, void* dst,
                             int64_t n, int64_t inst_idx, int64_t inst_dst, int ninst,
                             hipStream_t st, const int32_t* Mv = nullptr);
hipError_t launch_finalize_ptr(int fourier, const Status* status, const int32_t* lam,
                               const void* x, int K, int64_t inst_lam, int64_t inst_x,
                               int32_t* const* sup, void* const* xo, int ninst, hipStream_t st,
                               const int32_t* Kv = nullptr);
// top-K by |v|^2 (ties to the lowest index), excluded entries skipped;
// out: K ascending indices (fewer when fewer entries are eligible: then the
// state flag st[4] is set and the tail is unspecified).
size_t topk_workspace(int64_t n);
hipError_t launch_topk(const void* v, int kind, int64_t n, const uint32_t* excl, int64_t K,
                       void* ws, int32_t* out, hipStream_t st);
// Dense FP64 least squares on the support T (s ascending columns):
// x = (Phi_T^H Phi_T)^{-1} Phi_T^H y from the kernel vector and h_0 by a
// blocked Cholesky; *bad (device int) set to 1 on a non-positive pivot.
size_t dense_ls_workspace(int s_max, bool fourier);
hipError_t launch_dense_ls(int fourier, const void* c64, const void* h0, const int32_t* T, int s,
                           int N, void* ws, void* x, int* bad, hipStream_t st);
hipError_t launch_set_bits(uint32_t* bm, int64_t nwords, const int32_t* idx, int n,
                           hipStream_t st);
// per workgroup w: out[2w] = part of Re(h0(S)^H a), out[2w+1] = part of
// Re(a^H G_S a) (squared residual norm pieces); set_quad_groups(s) workgroups
int set_quad_groups(int s);
hipError_t launch_set_quad(int fourier, const void* c64, const void* h0, const int32_t* S,
                           const void* a, int s, int N, double* out, hipStream_t st);
// ------------------------------------------------------------------ persistent batch
// One workgroup runs a whole OMP solve of one instance (N small enough for
// its transform tile to live in LDS); workgroups pull instances from an
// atomic counter in the order given by `order` (largest first).
struct WgDesc {
  int32_t cls;            // FCMP_HADAMARD / FCMP_FOURIER
  int32_t N, logN, M, K;
  int32_t method;         // FCMP_CORR_*
  int32_t switch_t;       // adaptive: last iteration with the fast method
  int32_t pad;
  int64_t off_om;         // int32[M]   rows of Phi (any order, matching off_y)
  int64_t off_y;          // FP64[M]
  int64_t off_c64;        // FP64[N]    kernel vector
  int64_t off_cp;         // corr[N]    kernel vector in the correlation precision
  int64_t off_h0;         // FP64[N]
  int64_t off_W;          // FP64[K(K+1)/2]
  int64_t off_x, off_z;   // FP64[K]
};
struct WgParams {
  const WgDesc* desc;
  const int32_t* order;
  int n;
  int* counter;           // zeroed before the launch
  char* base;             // workspace base for the offsets
  Status* status;         // per instance (indexed like desc)
  void* const* ptrs;      // 3n device pointers indexed like desc: y, support, x
  const double2* tw64;    // two-level twiddles of the fixed table size 2^logT, sign +
  const float2* tw32;
  int logT, twS;          // table size and its lo/hi split (independent of the batch)
  const double2* tws64;   // per-span stage twiddles of the LDS transforms
  const float2* tws32;
  int logNmax;            // largest N in the batch (exclusion bitmap)
  int Kmax;
  const uint64_t* t0;     // device wall-clock ticks at the batch start
  size_t tile_bytes;      // LDS bytes reserved for the transform tile
};
hipError_t launch_omp_wg(const WgParams& p, int precision, int groups, hipStream_t st);
// workgroups of the persistent kernel that fit on one CU at once
int omp_wg_per_cu(const WgParams& p, int precision);
hipError_t launch_stamp(uint64_t* dst, hipStream_t st);
// Raises (never lowers) a kernel's dynamic-LDS limit; safe when several host
// threads launch the same kernel with different LDS sizes.
hipError_t raise_lds_limit(const void* kernel, size_t bytes);
size_t omp_wg_lds_bytes(const WgParams& p);
hipError_t launch_noise(int fourier, const void* clean, const void* noise, double snr_db,
                        void* y, int M, hipStream_t st);

}  // namespace fcmp
