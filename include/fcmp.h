/*
 * fcmp.h -- fast correlation for matching pursuit on AMD MI355X (gfx950).
 *
 * C ABI of libfcmp.so.  The library recovers a K-sparse x from
 * y = Phi x + eta, Phi = S_Omega U (eq. (CSbasic); Sec. I defines S_Omega as
 * the M rows, indexed by Omega, of the N x N identity), for the two unitary
 * classes the paper names: the unitary DFT and the Sylvester-ordered
 * Hadamard matrix.  The hot step of every matching pursuit algorithm is the
 * correlation h = Phi^H r (Algorithm 1.1, step 2); the library computes it
 * either as one N-point transform of the zero-filled residual ("conventional",
 * Sec. III-B) or by the paper's method, h = h_0 - sum_tau x(tau) P_lambda c
 * (eqs. (kernelsum), (kernelsumOMP)), with the identification argmax fused
 * into the kernel that produces h.  Least squares is an FP64 incremental
 * inverse-Cholesky update on the selected columns (Algorithm 1.1, step 6).
 *
 * Conventions (0-based, N a power of two):
 *   Fourier : U[k][n] = exp(-2 pi i ((k n) mod N) / N) / sqrt(N)
 *   Hadamard: U[k][n] = (-1)^popcount(k & n) / sqrt(N)
 *   Identification picks argmax |h(j)|^2 over columns not yet selected; ties
 *   go to the lowest index.
 *
 * Data types on the device:
 *   Hadamard vectors (y, x, h) are float64; Fourier vectors are complex128
 *   stored as interleaved (re, im) float64 pairs.  "Correlation precision"
 *   FP32 means the correlation runs in float32 / complex64 while h_0, the
 *   kernel-vector Gram entries and all least squares stay FP64.
 *
 * Memory ownership: the caller owns every device buffer.  The library never
 * allocates device memory: each call that needs scratch space takes a device
 * workspace whose size the matching *_query_workspace call returns (host-only,
 * no HIP call).  Host arrays passed in (Omega) are read before the call
 * returns.  Opaque handles (plans, servers) are host objects freed by their
 * *_destroy call.
 *
 * Streams: device work is enqueued on the caller's hipStream_t (passed as
 * void*; NULL = the null stream).  Outputs are valid once that stream has
 * been synchronised.  Calls that take a host stats pointer synchronise the
 * stream before returning when that pointer is non-NULL.
 *
 * Errors: every call returns FCMP_OK (0) or a negative status.  Validation is
 * host-only and precedes any device work, so an FCMP_E_INVALID or
 * FCMP_E_WORKSPACE return leaves all outputs untouched.  fcmp_last_error()
 * returns a thread-local description of the most recent failure.
 */
#ifndef FCMP_H
#define FCMP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FCMP_ABI_VERSION 3

/* status codes */
#define FCMP_OK            0
#define FCMP_E_INVALID    -1   /* bad argument (sizes, Omega, enums, pointers) */
#define FCMP_E_WORKSPACE  -2   /* workspace smaller than the query returned */
#define FCMP_E_DEVICE     -3   /* a HIP runtime error; see fcmp_last_error() */
#define FCMP_E_BUSY       -4   /* server queue full */
#define FCMP_E_NUMERIC    -5   /* Cholesky breakdown (Gram not positive) */
#define FCMP_E_NOTFOUND   -6   /* unknown ticket */

/* matrix classes (Sec. I: partial Hadamard, partial Fourier) */
#define FCMP_HADAMARD 0
#define FCMP_FOURIER  1

/* algorithms: OMP is Algorithm 1.1; SP and CoSaMP are the cited MPAs */
#define FCMP_OMP    0
#define FCMP_SP     1
#define FCMP_COSAMP 2

/* correlation methods */
#define FCMP_CORR_CONVENTIONAL 0  /* N-point transform of the zero-filled residual */
#define FCMP_CORR_FAST         1  /* eq. (kernelsumOMP): h_0 - sum x P c          */
#define FCMP_CORR_ADAPTIVE     2  /* fast up to a switch iteration, then conventional
                                     (the adaptive strategy of Sec. IV)           */

/* correlation precision (least squares is always FP64) */
#define FCMP_FP64 0
#define FCMP_FP32 1

/* Problem statement, eq. (CSbasic): Phi = S_Omega U with |Omega| = M.
 * N: power of two in [2, 2^24] (Fourier: [2, 2^22]); M in [1, N]; K in [1, M-1] (K < M, Sec. I).
 * omega: HOST pointer, M strictly increasing indices in [0, N).            */
typedef struct {
  int32_t matrix_class;      /* FCMP_HADAMARD or FCMP_FOURIER */
  int32_t reserved;
  int64_t N, M, K;
  const int32_t* omega;
} fcmp_problem;

typedef struct {
  int32_t algorithm;         /* FCMP_OMP / FCMP_SP / FCMP_COSAMP */
  int32_t corr_method;       /* FCMP_CORR_* */
  int32_t corr_precision;    /* FCMP_FP64 / FCMP_FP32 */
  int32_t max_iter;          /* SP/CoSaMP outer iterations (0 = 50); OMP runs K */
  int32_t switch_t;          /* ADAPTIVE: last iteration that uses the fast method
                                (0 = library's tuned value) */
  uint32_t flags;            /* FCMP_FLAG_* */
  double  res_tol;           /* optional halting rule (Algorithm 1.1 step 8):
                                OMP stops after the first selection whose
                                residual meets ||r|| <= res_tol ||y||; SP and
                                CoSaMP stop their loop once it is met.
                                0 = off; must be in [0, 1). */
} fcmp_options;

/* fcmp_plan_solve recomputes the kernel vector (A1) instead of reusing the
 * one the plan stored at creation. */
#define FCMP_FLAG_RECOMPUTE_KERNEL 1u
/* fcmp_batch_solve runs every problem as a lockstep plan, never in the
 * persistent one-workgroup-per-problem kernel. */
#define FCMP_FLAG_NO_PERSISTENT 2u
/* Hadamard plans with M < 2^15 store the kernel vector's integers N c
 * (|N c(j)| <= M; Sec. III-B notes the few distinct values) as int16 and the
 * fast correlation gathers those, half the bytes of FP32 and a quarter of
 * FP64; c = (N c)/N is exact, so results are bit-identical to the
 * floating-point gathers.  This flag makes a solve gather the floating-point
 * copy instead. */
#define FCMP_FLAG_FLOAT_KERNEL 4u
/* Fourier plans, fast correlation (eq. (kernelsumOMP)): gather only the half
 * c(0..N/2) of the kernel vector and use c(m) = conj(c(N - m)) above N/2,
 * the conjugate symmetry of the Fourier kernel vector (Sec. III-B: it is the
 * DFT of the real 0/1 mask of Omega), so a correlation touches half of c.  The
 * values above N/2 are the conjugated mirror entries rather than the stored
 * ones, so results agree with the full gathers to rounding, not bit for bit.
 * Ignored for the Hadamard class and by the persistent batch kernel. */
#define FCMP_FLAG_HALF_KERNEL 8u
/* Fill the ms_corr / ms_select / ms_ls / ms_resid fields of fcmp_stats:
 * every phase's launch sequence of this solve is bracketed by hipEvents on
 * the solve's stream (a small overhead per launch).  Ignored under graph
 * capture and by the persistent batch kernel. */
#define FCMP_FLAG_PHASE_TIMES 16u
/* Fourier plans with N <= 8192, fast correlation: the conjugate-symmetric
 * pairing of Sec. III-B (complexity of the proposed OMP, partial Fourier).
 * Because c(N - m) = conj(c(m)), the four real products of x c(m) give both
 * x c(m), added at h(lambda + m), and x conj(c(m)), added at h(lambda - m):
 * (N/2)(t - 1) complex multiplications per correlation.  One workgroup per
 * instance holds h in LDS and takes the taps in order.  Like
 * FCMP_FLAG_HALF_KERNEL it reads c only up to N/2, so results agree with the
 * full gathers to rounding, not bit for bit.  FCMP_E_INVALID for the Hadamard
 * class or N > 8192; ignored by the persistent batch kernel. */
#define FCMP_FLAG_CONJ_PAIR 32u

/* Per-solve statistics. */
typedef struct {
  int32_t iterations;        /* OMP: selections made; SP/CoSaMP: outer iterations */
  int32_t status_detail;     /* FCMP_OK or FCMP_E_NUMERIC (Cholesky breakdown) */
  double  res_norm;          /* ||y - Phi_Lambda x|| (from the normal equations) */
  double  min_gap;           /* OMP: smallest identification gap over the solve,
                                (|h|_(1) - |h|_(2)) / |h|_(1) over the columns not
                                yet selected, keys in the correlation precision
                                (1 when a selection had no runner-up, +inf
                                before the first); SP/CoSaMP: NaN (not tracked) */
  float   ms_corr;           /* with FCMP_FLAG_PHASE_TIMES (else 0), device time
                                of this solve's phases, ms: correlation (h_0,
                                conventional incl. a fused residual, fast) */
  float   ms_select;         /*   SP/CoSaMP top-K selection (OMP's argmax is
                                fused into the correlation and least squares) */
  float   ms_ls;             /*   identification merge + least squares */
  float   ms_resid;          /*   residual computed apart from the correlation */
  double  ms_total;          /* device time of the solve (hipEvent), ms; for a
                                problem run by the persistent batch kernel: its
                                completion time from the start of the batch */
} fcmp_stats;

int         fcmp_abi_version(void);
const char* fcmp_status_str(int status);
const char* fcmp_last_error(void);

/* ---- whole solves ---------------------------------------------------- */

/* Device bytes fcmp_solve needs for this problem and options.  Host-only. */
int fcmp_query_workspace(const fcmp_problem* prob, const fcmp_options* opt,
                         size_t* bytes);

/* Recover x from y (Algorithm 1.1 for OMP).
 * y_dev      : device, M values (float64 | complex128)
 * ws_dev     : device workspace of ws_bytes >= fcmp_query_workspace()
 * support_dev: device int32[K]; OMP: selection order; SP/CoSaMP: ascending;
 *              entries past the last selection are -1
 * x_dev      : device, K values (float64 | complex128) aligned with support
 * stats      : host, nullable; when given the call synchronises the stream  */
int fcmp_solve(const fcmp_problem* prob, const fcmp_options* opt,
               const void* y_dev, void* ws_dev, size_t ws_bytes,
               int32_t* support_dev, void* x_dev, fcmp_stats* stats,
               void* hip_stream);

/* fcmp_solve for callers that cannot allocate device memory: code that runs
 * under HIP graph capture, tight serving loops, and harnesses that forbid
 * hipMalloc.  The workspace comes from a static device array of
 * FCMP_NOALLOC_SCRATCH_BYTES inside the library (each GPU the library runs
 * on holds its own copy until the process ends) instead of a caller buffer;
 * the call itself allocates no device memory and creates no events.  The
 * caller still owns y, support and x (layouts as for fcmp_solve).  A problem
 * whose fcmp_query_workspace exceeds FCMP_NOALLOC_SCRATCH_BYTES is refused
 * with FCMP_E_WORKSPACE (OMP fits up to N = 2^20, M = 2^17, K = 1024, which
 * needs 36 MiB).  Every call on one GPU shares that GPU's array: calls that
 * overlap on one GPU (from several host threads or streams) race and must
 * be serialised by the caller.  stats (nullable) are filled after a stream
 * synchronisation, with ms_total = 0 (no device timing).  Results are
 * bit-identical to fcmp_solve's. */
#define FCMP_NOALLOC_SCRATCH_BYTES (64u << 20)
int fcmp_solve_noalloc(const fcmp_problem* prob, const fcmp_options* opt,
                       const void* y_dev, int32_t* support_dev, void* x_dev,
                       fcmp_stats* stats, void* hip_stream);

/* Many independent problems in one call.  OMP problems whose transform fits
 * one workgroup's LDS (N * element size <= 140 KiB, K <= 1024) run whole
 * solves, one workgroup per problem, in one persistent launch after a
 * lockstep prologue (kernel vector and h_0 per (class, N, M) group); the
 * others run as lockstep plans, one per (class, N) for OMP (each problem
 * keeps its own M and K) and one per (class, N, M, K) for SP/CoSaMP.  Arrays are HOST arrays of n
 * entries holding device pointers; stats (nullable) is a host array of n
 * (when given the call synchronises the stream). */
int fcmp_batch_query_workspace(int64_t n, const fcmp_problem* probs,
                               const fcmp_options* opt, size_t* bytes);
int fcmp_batch_solve(int64_t n, const fcmp_problem* probs, const fcmp_options* opt,
                     const void* const* y_dev, void* ws_dev, size_t ws_bytes,
                     int32_t* const* support_dev, void* const* x_dev,
                     fcmp_stats* stats, void* hip_stream);

/* A batch plan fixes a set of n uneven problems (each with its own Omega and
 * shape; one options record): creation builds every table, descriptor and
 * kernel vector once and, for OMP, captures the whole device work of a
 * solve -- the persistent launch with its prologue and every lockstep plan's
 * iterations -- into one hipGraph.  Each fcmp_batch_plan_solve uploads the
 * n (y, support, x) device pointers and replays the graph on the caller's
 * stream.  SP/CoSaMP batch plans run eagerly (their loops read partial
 * results back on the host).  The workspace (from
 * fcmp_batch_plan_query_workspace, host-only) must stay untouched while the
 * plan lives; solves on one plan must not overlap.  Creation synchronises
 * the stream.  Pointer arrays and stats are as for fcmp_batch_solve. */
typedef struct fcmp_batch_plan fcmp_batch_plan;
int fcmp_batch_plan_query_workspace(int64_t n, const fcmp_problem* probs,
                                    const fcmp_options* opt, size_t* bytes);
int fcmp_batch_plan_create(fcmp_batch_plan** out, int64_t n, const fcmp_problem* probs,
                           const fcmp_options* opt, void* ws_dev, size_t ws_bytes,
                           void* hip_stream);
int fcmp_batch_plan_solve(fcmp_batch_plan* plan, const void* const* y_dev,
                          int32_t* const* support_dev, void* const* x_dev,
                          fcmp_stats* stats, void* hip_stream);
int fcmp_batch_plan_destroy(fcmp_batch_plan* plan);

/* ---- plans ------------------------------------------------------------ */

/* A plan holds, in the caller's device workspace, what depends on Omega only
 * -- the rows of Phi in the order the transform kernels consume them and the
 * correlation kernel vector c, which the paper notes is independent of x and
 * "stored in advance" (definition after eq. (kernelsum)) -- plus every
 * per-solve buffer, for n problems of one class and N solved in lockstep:
 * each kernel launch of a solve covers all n instances.  OMP problems may
 * differ in M and K (each makes its own K selections; the loop runs to the
 * largest K); SP/CoSaMP plans need one (M, K).
 * probs: HOST array of n problems (each with its own Omega); the options fix
 * algorithm and correlation precision for the plan's lifetime.  Creation
 * uploads the tables, computes c and synchronises the stream.  Solves on one
 * plan must not overlap (they share the workspace). */
typedef struct fcmp_plan fcmp_plan;
int fcmp_plan_query_workspace(int64_t n, const fcmp_problem* probs, const fcmp_options* opt,
                              size_t* bytes);
int fcmp_plan_create(fcmp_plan** out, int64_t n, const fcmp_problem* probs,
                     const fcmp_options* opt, void* ws_dev, size_t ws_bytes, void* hip_stream);
/* y_dev / support_dev / x_dev: HOST arrays of n device pointers (layouts as
 * for fcmp_solve).  opt may differ from the creation options only in
 * corr_method, switch_t and flags (NULL: creation options).  stats: host
 * array of n (nullable; when given the call synchronises the stream). */
int fcmp_plan_solve(fcmp_plan* plan, const fcmp_options* opt, const void* const* y_dev,
                    int32_t* const* support_dev, void* const* x_dev, fcmp_stats* stats,
                    void* hip_stream);
int fcmp_plan_destroy(fcmp_plan* plan);

/* ---- serving ---------------------------------------------------------- */

/* A solver service with continuous batching.  Requests (problem, options,
 * y on the HOST) queue on submit and are admitted in arrival order whenever
 * request slots and room in the caller's device pool allow:
 *  - slot groups (iteration-granular): OMP requests with the conventional
 *    correlation whose residual is fused with the transform (two-pass N)
 *    join a resident group of slots of their class, N and options between
 *    two iterations, run their own iteration count in lockstep with the
 *    others, and leave as soon as their K selections are made, so a request
 *    never waits for a wave to end.  Each group has its own thread and
 *    stream (at most max_groups); its Omega tables are prepared on host
 *    threads, kept in a cache keyed by (class, N, Omega), and a slot whose
 *    device tables already hold the request's Omega (or another slot's
 *    copy) reuses them with no host work;
 *  - waves, on worker streams: all queued OMP requests the persistent
 *    one-workgroup-per-problem kernel takes, with the same options, in one
 *    persistent launch (at most max_wave); any other request as a lockstep
 *    plan with the queued requests of its class and N (SP/CoSaMP: same M
 *    and K).  With several worker streams, stream 0 runs persistent waves.
 * Work on different streams overlaps on the device.  A request's device
 * state stays in its slot or wave region from admission to completion;
 * results are copied to host memory.  A request's results do not depend on
 * the requests it shares a group or wave with, nor on when it joined.  The
 * library never allocates device memory beyond the pool (pinned host
 * staging is allocated per worker and per group). */
typedef struct fcmp_server fcmp_server;
typedef struct {
  int32_t max_slots;         /* requests on the device at once (0: 4096) */
  int32_t max_pending;       /* queued, not yet admitted (0: 65536); more: FCMP_E_BUSY */
  int32_t n_streams;         /* worker streams, 1..8 (0: 4) */
  int32_t max_wave;          /* requests per persistent wave (0: 1024) */
  int32_t max_groups;        /* slot groups at once, 1..16 (0: 8; -1: none, waves only) */
} fcmp_server_config;
typedef struct {             /* milliseconds on the server's clock (from creation) */
  double t_submit;           /* fcmp_server_submit returned the ticket */
  double t_launch;           /* admitted: its wave started */
  double t_done;             /* results were back in host memory */
} fcmp_times;
typedef struct {
  int64_t submitted, completed, queued, inflight, waves;
  int64_t pool_peak;         /* most pool bytes in use at once */
  int64_t groups;            /* slot groups created */
  int64_t slot_joins;        /* requests that joined a slot group */
  int64_t slot_steps;        /* iterations run by slot groups */
  int64_t tables_built;      /* Omega tables built on the host */
  int64_t tables_cached;     /* ... found in the host table cache instead */
  int64_t tables_resident;   /* joins whose slot already held the tables */
  int64_t tables_copied;     /* joins that copied another slot's tables */
} fcmp_server_info;

/* Device pool bytes one request occupies when admitted alone (solver state
 * plus y, support and x); the admission test uses it.  Host-only. */
int fcmp_server_footprint(const fcmp_problem* prob, const fcmp_options* opt, size_t* bytes);
/* pool_dev / pool_bytes: caller-owned device memory, untouched by anything
 * else while the server lives.  cfg nullable (all defaults).  The current
 * device at creation is the server's device. */
int fcmp_server_create(fcmp_server** out, void* pool_dev, size_t pool_bytes,
                       const fcmp_server_config* cfg);
/* y_host: M values (float64 | complex128), copied before the call returns;
 * omega is copied too.  FCMP_E_WORKSPACE when the request can never fit the
 * pool, FCMP_E_BUSY when max_pending requests are queued. */
int fcmp_server_submit(fcmp_server* srv, const fcmp_problem* prob, const fcmp_options* opt,
                       const void* y_host, uint64_t* ticket);
/* Non-blocking.  *done = 0 while the request runs.  Once done, copies K
 * support entries and K values of x to the host buffers (each nullable),
 * fills stats and times (nullable; stats.ms_total is the completion time
 * from the wave's start), forgets the ticket and returns the request's
 * status (FCMP_E_NOTFOUND for an unknown or already collected ticket). */
int fcmp_server_poll(fcmp_server* srv, uint64_t ticket, int32_t* support_host, void* x_host,
                     fcmp_stats* stats, fcmp_times* times, int32_t* done);
/* Waits until no request is queued or running (timeout_ms <= 0: no limit);
 * FCMP_E_BUSY at the timeout. */
int fcmp_server_drain(fcmp_server* srv, double timeout_ms);
int fcmp_server_get_info(fcmp_server* srv, fcmp_server_info* info);
/* Finishes the running waves, drops queued requests and frees the host
 * objects; the pool may be reused once it returns. */
int fcmp_server_destroy(fcmp_server* srv);

/* ---- adaptive switch autotuning ---------------------------------------- */

/* The adaptive method (FCMP_CORR_ADAPTIVE with switch_t = 0) uses the fast
 * correlation up to a switch iteration.  Without tuning that iteration is the
 * flop-model crossover of Table I (Fourier: 2 + floor(5 log2 N / 6);
 * Hadamard: 1 + log2 N).  fcmp_autotune measures it instead: it builds a
 * lockstep plan of `batch` problems of (class, N, M) in the workspace
 * (bytes from fcmp_autotune_query_workspace, host-only), times the fast and
 * the conventional correlation launch sequences at growing tap counts on the
 * stream, and records the last iteration at which the fast one is no slower
 * in the library's process-wide table; *switch_t receives it.  cache_path
 * (nullable): a text file of "class N precision switch_t" lines; an entry for
 * (class, N, precision) found there is used without measuring, and a new
 * measurement is appended.  The call synchronises the stream. */
int fcmp_autotune_query_workspace(int32_t matrix_class, int64_t N, int64_t M,
                                  int32_t corr_precision, int32_t batch, size_t* bytes);
int fcmp_autotune(int32_t matrix_class, int64_t N, int64_t M, int32_t corr_precision,
                  int32_t batch, const char* cache_path, void* ws_dev, size_t ws_bytes,
                  int32_t* switch_t, void* hip_stream);
/* The measurement behind the autotuner, exposed: the device time of one
 * fast (eq. (kernelsumOMP), t - 1 taps) and one conventional (residual and
 * transform) correlation launch sequence of a lockstep plan of `batch`
 * problems (class, N, M) at each iteration ts[i] (each >= 2 and <= M - 1),
 * written to fast_ms[i] and conv_ms[i] (ms per launch sequence over the whole
 * batch, mean of a few repetitions).  This is the per-iteration cost curve
 * whose crossing is the adaptive strategy's switch (Sec. IV; Table I gives
 * the flop-count version).  flags: FCMP_FLAG_HALF_KERNEL, FCMP_FLAG_CONJ_PAIR
 * or FCMP_FLAG_FLOAT_KERNEL select the fast correlation's variant (others:
 * FCMP_E_INVALID).  The workspace size comes from
 * fcmp_corr_curve_query_workspace with tmax = max ts (host-only).  The call
 * synchronises the stream. */
int fcmp_corr_curve_query_workspace(int32_t matrix_class, int64_t N, int64_t M,
                                    int32_t corr_precision, int32_t batch, int32_t tmax,
                                    size_t* bytes);
int fcmp_corr_curve(int32_t matrix_class, int64_t N, int64_t M, int32_t corr_precision,
                    int32_t batch, uint32_t flags, const int32_t* ts, int32_t nt, void* ws_dev,
                    size_t ws_bytes, float* fast_ms, float* conv_ms, void* hip_stream);
/* Loads every valid entry of a cache file (switch iterations and launch
 * schedules) into the tables (host-only); FCMP_E_NOTFOUND when the file is
 * missing or holds no valid entry. */
int fcmp_autotune_load(const char* cache_path);
/* The switch iteration an adaptive solve with switch_t = 0 uses; *tuned
 * (nullable) is 1 when it comes from the table, 0 for the flop model.
 * Host-only. */
int fcmp_adaptive_switch(int32_t matrix_class, int64_t N, int32_t corr_precision,
                         int32_t* switch_t, int32_t* tuned);

/* ---- launch-schedule autotuning --------------------------------------- */

/* How a plan spreads its transforms over the device: the values per
 * workgroup tile of the two-pass transforms (the B1, B2 sequences per
 * workgroup of the N = N1 N2 split), the most threads of a transform
 * workgroup, and the threads of the generic fused residual + first pass.
 * Zero fields mean the library's defaults.  No field changes a result: each
 * one only splits the same per-element arithmetic and the identification's
 * total order over workgroups and threads differently.  (The least-squares
 * row split and the persistent kernel's workgroup size are not schedule
 * fields: they fix the order of floating-point sums.) */
typedef struct {
  int32_t tile;       /* power of two <= 8192 (0: chosen from the batch size) */
  int32_t threads;    /* 64, 128 or 256 (0: 256) */
  int32_t rthreads;   /* 64, 128 or 256 (0: from the first pass's tile) */
} fcmp_schedule;
/* fcmp_schedule_tune times, for a lockstep plan of `batch` problems (class,
 * N, M) in the workspace (bytes from fcmp_schedule_query_workspace,
 * host-only), one conventional correlation (t = 16) plus the share of the
 * h_0 and kernel-vector transforms of a 256-iteration solve under the
 * default schedule and under every distinct tile, then thread counts at the
 * best tile, and records the fastest in the library's table for (device
 * architecture, class, N, precision, batch bucket: 1, <= 8, <= 32, <= 128,
 * more); plans and batch plans created afterwards for that key use it.
 * ms_default / ms_best (nullable) receive the timed costs.  cache_path
 * (nullable): the same text file as fcmp_autotune, one
 * "sched arch class N precision bucket tile threads rthreads" line per
 * entry; an entry found there is used without measuring, a new one is
 * appended.  The call synchronises the stream. */
int fcmp_schedule_query_workspace(int32_t matrix_class, int64_t N, int64_t M,
                                  int32_t corr_precision, int32_t batch, size_t* bytes);
int fcmp_schedule_tune(int32_t matrix_class, int64_t N, int64_t M, int32_t corr_precision,
                       int32_t batch, const char* cache_path, void* ws_dev, size_t ws_bytes,
                       fcmp_schedule* best, float* ms_default, float* ms_best,
                       void* hip_stream);
/* Sets (s non-NULL) or drops (s NULL) the table entry for the current
 * device's architecture and (class, N, precision, batch bucket). */
int fcmp_schedule_set(int32_t matrix_class, int64_t N, int32_t corr_precision, int32_t batch,
                      const fcmp_schedule* s);
/* The schedule a plan of `batch` problems of (class, N, precision) uses;
 * *tuned (nullable) is 1 when it comes from the table.  Host-only while the
 * table is empty. */
int fcmp_schedule_get(int32_t matrix_class, int64_t N, int32_t corr_precision, int32_t batch,
                      fcmp_schedule* s, int32_t* tuned);

/* ---- phase timing ------------------------------------------------------ */

/* When enabled, every launch sequence of a phase is bracketed by hipEvents on
 * the stream it runs on; fcmp_profile_read synchronises those events and
 * returns the summed device time per phase. */
#define FCMP_PHASE_KERNEL 0   /* kernel vector c (plan time, or RECOMPUTE flag) */
#define FCMP_PHASE_H0     1   /* h_0 = Phi^H y and the first identification      */
#define FCMP_PHASE_CORR   2   /* conventional correlation (all transform passes;
                                 where the residual is fused into the first pass,
                                 the residual too)                                */
#define FCMP_PHASE_FAST   3   /* fast correlation, eq. (kernelsumOMP)            */
#define FCMP_PHASE_RESID  4   /* residual r = y - Phi_t x_t, when computed apart  */
#define FCMP_PHASE_LS     5   /* identification + least-squares update           */
#define FCMP_PHASE_OTHER  6   /* gathers, status, copy-out                        */
#define FCMP_PHASE_SELECT 7   /* SP/CoSaMP top-K selection                        */
#define FCMP_NPHASE       8
typedef struct {
  double  ms[FCMP_NPHASE];
  int64_t launches[FCMP_NPHASE];
} fcmp_profile;
int fcmp_profile_enable(int enable);
int fcmp_profile_read(fcmp_profile* out, int reset);

/* ---- single steps of the hot path (each one launch sequence) ---------- */

/* Kernel vector c = U^H S_Omega^T S_Omega U e_0 (definition after eq.
 * (kernelsum)).  c64_dev: N FP64 values (float64 | complex128); cp_dev
 * (nullable): N values in the correlation precision (float32 | complex64
 * for FCMP_FP32, else float64 | complex128). */
int fcmp_kernel_vector_workspace(const fcmp_problem* prob, size_t* bytes);
int fcmp_kernel_vector(const fcmp_problem* prob, int32_t precision,
                       void* c64_dev, void* cp_dev, void* ws_dev, size_t ws_bytes,
                       void* hip_stream);

/* Conventional correlation h = Phi^H r = U^H S_Omega^T r (Algorithm 1.1
 * step 2) with the identification of step 3 fused.
 * r_dev  : device, M values in the given precision (float64 | complex128 for
 *          FP64; float32 | complex64 for FP32), aligned with omega
 * h_dev  : device (nullable), N values in the same precision
 * excl_dev: device (nullable), uint32[(N+31)/32] bitmap of excluded columns
 * sel_dev: device (nullable), 24 bytes {double |h|^2, int64 index, double
 *          runner-up |h|^2} of the winner (index -1 when every column is
 *          excluded or h vanishes; runner-up -1 when there is none)        */
int fcmp_correlate_workspace(const fcmp_problem* prob, int32_t precision,
                             size_t* bytes);
int fcmp_correlate(const fcmp_problem* prob, int32_t precision,
                   const void* r_dev, void* h_dev, const uint32_t* excl_dev,
                   void* sel_dev, void* ws_dev, size_t ws_bytes, void* hip_stream);

/* Fast correlation, eq. (kernelsum): h = h0 - sum_tau x(tau) P_{lam(tau)} c,
 * with P_lambda the cyclic shift (Fourier) or XOR (Hadamard) permutation of
 * Thm 2-1 / Sec. III-B, and the identification fused.
 * h0_dev : N FP64 values; cp_dev: N values in the precision (FP32 or FP64);
 * lam_dev: int32[ntaps]; xt_dev: ntaps FP64 values; accumulation is FP64.
 * h_dev, excl_dev, sel_dev as for fcmp_correlate (h_dev is FP64 here).    */
int fcmp_fast_correlate_workspace(const fcmp_problem* prob, size_t* bytes);
int fcmp_fast_correlate(const fcmp_problem* prob, int32_t precision,
                        const void* h0_dev, const void* cp_dev,
                        const int32_t* lam_dev, const void* xt_dev, int64_t ntaps,
                        void* h_dev, const uint32_t* excl_dev, void* sel_dev,
                        void* ws_dev, size_t ws_bytes, void* hip_stream);

/* Top-K identification of the set-based pursuits (SP and CoSaMP select the
 * K or 2K largest entries of their proxy h = Phi^H r, the step that
 * Algorithm 1.1 step 3 takes for K = 1): the K indices j of largest |v(j)|^2
 * among the entries whose bit in excl_dev is clear, ties to the lowest
 * index, written to out_dev in ascending index order.  v_dev: n values,
 * float32 | complex64 for FCMP_FP32 and float64 | complex128 for FCMP_FP64,
 * real for FCMP_HADAMARD and complex for FCMP_FOURIER; excl_dev nullable,
 * uint32[(n+31)/32]; out_dev: int32[K].  When fewer than K entries are
 * eligible, the slots after the last eligible index hold -1.  1 <= K <= n,
 * n < 2^31; the workspace size comes from fcmp_topk_workspace (host-only). */
int fcmp_topk_workspace(int64_t n, size_t* bytes);
int fcmp_topk(int32_t matrix_class, int32_t precision, const void* v_dev, int64_t n,
              const uint32_t* excl_dev, int64_t K, int32_t* out_dev, void* ws_dev,
              size_t ws_bytes, void* hip_stream);

/* Forward operator y = Phi x (+ noise scaled to snr_db when noise_dev is not
 * NULL: eta = g ||Phi x|| / ||g|| 10^(-snr/20)).  x_dev: N FP64 values;
 * noise_dev: M values; y_dev: M values (float64 | complex128).             */
int fcmp_measure_workspace(const fcmp_problem* prob, size_t* bytes);
int fcmp_measure(const fcmp_problem* prob, const void* x_dev, const void* noise_dev,
                 double snr_db, void* y_dev, void* ws_dev, size_t ws_bytes,
                 void* hip_stream);

#ifdef __cplusplus
}
#endif
#endif /* FCMP_H */
