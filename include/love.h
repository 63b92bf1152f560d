/*
 * love.h -- C ABI of the LOVE (LanczOs Variance Estimates) library for KISS-GP
 * on AMD Instinct MI355X (gfx950).
 *
 * The method is that of Pleiss, Gardner, Weinberger and Wilson, "Constant-Time
 * Predictive Distributions for Gaussian Processes" (ICML 2018):
 *
 *   training operator   Khat = W K W^T + sigma^2 I          (Sec. 2.3, eq. ski; Alg. 1 input mvm_K_XX)
 *   W                   cubic (Keys) interpolation, 4^d non-zeros per row (Sec. 2.3)
 *   K = K_UU            Toeplitz / Kronecker-of-Toeplitz grid kernel (Sec. 2.3)
 *   cache               k-step Lanczos on Khat with probe b = (1/m) W K 1 and
 *                       full reorthogonalisation (Sec. 3.2, Sec. 5), T = L L^T,
 *                       R = Q^T W K, R' = T^{-1} R (Alg. 1).  The library stores the
 *                       single m x k matrix Rt = (L^{-1} R)^T, for which
 *                       R^T R' = Rt Rt^T, so one gather serves both factors.
 *   mean cache          a = K W^T Khat^{-1} y (Sec. 2.3, eq. pred_mean_ski)
 *   variance            var(x*) = w*^T K w* - ||Rt^T w*||^2 (eq. pred_covar_ski_fast, i = j)
 *   sampling            S = Q' V Lambda_+^{1/2} from Lanczos on K - R^T R' and
 *                       T' = V Lambda V^T (Sec. 3.3, eqs. lancapprox,
 *                       pred_covar_ski_interp_form; S S^T = Q' T' Q'^T when T'
 *                       is positive semidefinite);
 *                       sample = mu(X*) + W_{X*} S z (eq. sample)
 *
 * Conventions shared by every entry point
 *   - All array arguments are DEVICE pointers owned by the caller, except the
 *     love_config structs and the small host arrays of the batched entry
 *     points, which are host memory.  The library owns every love_cache.
 *   - Element type of x, y, x*, mean, var, samples and gradients follows
 *     love_config.precision: LOVE_P_FP64 -> double, otherwise float.
 *     Sampling noise z and the optional dRt gradient are always float.
 *   - Point arrays are row-major n x d (d = cfg->d).  Every coordinate must lie
 *     in [lo_i, hi_i] of its dimension.
 *   - All work is enqueued on `stream` (a hipStream_t, NULL = default stream).
 *     Query entry points never synchronise the host.  love_build_cache
 *     synchronises once at its end (to report device-detected errors) unless
 *     LOVE_FLAG_ASYNC is set.
 *   - Errors are returned as love_status; nothing is thrown across the ABI.
 *     Argument errors are detected on the host before any work is enqueued.
 *     Conditions only visible on the device (a query point outside the domain,
 *     non-finite values) set bits in the cache's status word, reported by
 *     love_cache_info; out-of-domain query points get NaN outputs.
 *   - A built cache is immutable; concurrent queries on different streams are
 *     safe.  Calls that allocate (build, free) are not thread-safe with respect
 *     to the same cache.
 *   - Device memory.  The build, batched build, import and covariance-block
 *     entry points take a `const love_allocator*`.  NULL selects the device's
 *     stream-ordered pool (hipMallocAsync / hipFreeAsync).  Otherwise every
 *     device buffer of the call, the cache and its transient workspace alike,
 *     comes from alloc() and goes back through free(); a cache keeps its
 *     allocator (the struct is copied; ctx must stay valid until
 *     love_cache_free) and the calls on it that need scratch (sampling, the
 *     backward, paired covariances, the operator products) use it as well.
 *     The library allocates each block on a stream and releases it on that same
 *     stream once every other stream that used it has been joined into it, so
 *     a stream-ordered allocator (torch's caching allocator, a hipMallocAsync
 *     pool) may reuse a freed block for later work on that stream at once.
 *     Streams passed to the callbacks may be library-internal (the sampler and
 *     the grid-space mean solve run on side streams).
 *   - Environment.  LOVE_AUTOTUNE=0 replaces the autotuner's timing runs by a
 *     size rule (LOVE_TOEPLITZ_AUTO only).  LOVE_PSUM_MAX_NB=<blocks> sets the
 *     row-block count up to which a Lanczos run adds its partial dot-product
 *     rows inside the consuming kernels instead of separate column-sum launches
 *     (default 160).  Both change only the order of floating-point sums, so
 *     results move at rounding level.
 */
#ifndef LOVE_H_
#define LOVE_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LOVE_ABI_VERSION 4
#define LOVE_MAX_DIM 4
#define LOVE_MAX_K 128

typedef int32_t love_status;
enum {
  LOVE_OK = 0,
  LOVE_EINVAL = -1,        /* bad argument (null pointer, size, dimension, k, ...)          */
  LOVE_EDOMAIN = -2,       /* a training point lies outside [lo, hi]                         */
  LOVE_ENOTPD = -3,        /* the Lanczos tridiagonal T was not positive definite            */
  LOVE_ENOMEM = -4,        /* device allocation failed                                       */
  LOVE_EHIP = -5,          /* a HIP runtime call failed                                      */
  LOVE_ENONFINITE = -6,    /* non-finite training input or Lanczos coefficient               */
  LOVE_EUNSUPPORTED = -7,  /* valid request the library does not support (e.g. no sampler)   */
  LOVE_ELIMIT = -8         /* request exceeds a fixed limit of the call (the static scratch of
                              love_sample_posterior_noalloc)                                    */
};

/* Bytes of the fixed device scratch array behind love_sample_posterior_noalloc
 * (one copy per device, held until the process ends). */
#define LOVE_NOALLOC_SCRATCH_BYTES (8u << 20)

typedef enum { LOVE_RBF = 0, LOVE_MATERN52 = 1 } love_kernel;   /* product over dimensions */

typedef enum {
  LOVE_P_FP64 = 0,          /* all vectors and the cache in double                              */
  LOVE_P_FP32 = 1,          /* float vectors and cache; double tridiagonal work and variance
                               subtraction                                                      */
  LOVE_P_FP32_BF16SPLIT = 2 /* as FP32, but Rt stored as bf16 hi + bf16 lo planes              */
} love_precision;

typedef enum {
  LOVE_TOEPLITZ_AUTO = 0,   /* per-axis choice by the built-in autotuner                       */
  LOVE_TOEPLITZ_DIRECT = 1, /* O(m_i^2) per line, register-blocked, all CUs                    */
  LOVE_TOEPLITZ_FFT = 2     /* circulant embedding, LDS-resident radix-2 FFT, O(m_i log m_i).
                               Available while the circulant length (the power of two
                               >= 2 m_i - 1) is at most 8192; an explicit request beyond
                               that makes the build return LOVE_EUNSUPPORTED            */
} love_toeplitz_mode;

/* Flags (love_config.flags) */
#define LOVE_FLAG_ASYNC 1u          /* build does not synchronise at its end                     */
#define LOVE_FLAG_NO_MEAN 2u        /* skip the mean cache a                                      */
#define LOVE_FLAG_PLAIN_CG 4u       /* mean solve: CG without the Lanczos preconditioner         */
#define LOVE_FLAG_EIG_QL 8u         /* sampler: eigenvectors of T' by implicit QL (slow path)     */
#define LOVE_FLAG_MEAN_KRYLOV 16u   /* mean solve: data-space CG even where the grid-space solve
                                       applies (d >= 2 with every m_i <= 128)                     */
#define LOVE_FLAG_ADDITIVE 32u      /* additive composition (Sec. 3.4, eq.
                                       multi_dimensional_kernel_block):
                                       k(x, x') = outputscale * sum_i k_i(x_i, x'_i), one 1-D
                                       component per dimension on that dimension's grid.  The
                                       grid vectors (Rt rows, the mean cache a, S rows) stack the
                                       axes one after another, axis 0 first: m = sum_i m_i, and
                                       K is block diagonal; every entry point takes the block form
                                       (a query point's interpolation vector has 4 d entries, its
                                       prior is the sum of the axes' terms).  Every GP of a batched
                                       build must agree on this flag (LOVE_EINVAL otherwise).     */
#define LOVE_FLAG_HYPER 64u         /* also keep B = W^T Q L^{-T} (m x k, cache precision) for
                                       love_predict_var_hyper_grad; Rt = K B.  Does not change
                                       any other result of the cache                              */

typedef struct {
  int32_t d;                        /* input dimension, 1..4                                     */
  int32_t m[LOVE_MAX_DIM];          /* grid points per dimension, >= 4.  The grid is padded by
                                       one cell on each side: h_i = (hi_i - lo_i) / (m_i - 3),
                                       node j at lo_i + (j - 1) h_i                              */
  double lo[LOVE_MAX_DIM];          /* data domain per dimension (lo < hi)                       */
  double hi[LOVE_MAX_DIM];
  int32_t kernel;                   /* love_kernel                                               */
  double lengthscale[LOVE_MAX_DIM]; /* > 0                                                       */
  double outputscale;               /* > 0                                                       */
  double noise;                     /* sigma^2 > 0 (a variance)                                  */
  int32_t k;                        /* Lanczos steps, 1..LOVE_MAX_K (k_eff <= k is reported)     */
  int32_t k_sample;                 /* 0: no sampling cache; else second-Lanczos steps (<= 128)  */
  int32_t precision;                /* love_precision                                            */
  int32_t toeplitz;                 /* love_toeplitz_mode                                        */
  double cg_tol;                    /* mean solve tolerance (<= 0: 1e-6 / 1e-12).  Data-space CG:
                                       ||Khat x - y|| <= tol ||y||.  Grid-space solve: residual
                                       <= tol sigma ||y||, so the training-point mean is within
                                       tol ||y|| (2-norm) of the exact solve                     */
  int32_t cg_maxit;                 /* <= 0: 1000                                                */
  uint32_t flags;                   /* LOVE_FLAG_*                                               */
  /* Restart with a new probe (Sec. 5, "Ensuring Lanczos solves are accurate").
   * With restart_tol > 0 the Lanczos solve Q T^{-1} Q^T is checked, after the k
   * steps, on restart_groups averaged columns of W K (column g: W K 1_g / |g|,
   * 1_g the indicator of the g-th of restart_groups runs of consecutive grid
   * nodes).  While the worst relative residual ||c - Khat Q H^{-1} Q^T c|| / ||c||
   * exceeds restart_tol (at most restart_max times), restart_k further Lanczos
   * steps are taken from that residual, orthogonalised against every earlier
   * vector; the cache then uses H = Q^T Khat Q over both blocks (no longer
   * tridiagonal) and its dense Cholesky factor.  Single-GP builds only
   * (love_build_cache_batched: LOVE_EUNSUPPORTED).  k + restart_max restart_k
   * <= LOVE_MAX_K.  The check synchronises the host once per round.         */
  double restart_tol;               /* <= 0: no check                                            */
  int32_t restart_k;                /* steps per restart (>= 1 when restart_tol > 0)             */
  int32_t restart_max;              /* <= 0: 1                                                   */
  int32_t restart_groups;           /* <= 0: 8                                                   */
} love_config;

typedef struct love_cache love_cache;   /* opaque */

/* Caller-supplied device memory (see "Device memory" above).
 *   alloc(bytes, stream, ctx): a device block of at least `bytes` bytes, aligned
 *     to 256 bytes, usable by work enqueued on `stream` (a hipStream_t) after
 *     the call; NULL on failure (the entry point then returns LOVE_ENOMEM).
 *   free(ptr, stream, ctx): release a block from alloc(); work already
 *     enqueued on `stream` may still use it, and the block may be reused by
 *     work enqueued on `stream` afterwards.
 * Both must be non-NULL (LOVE_EINVAL otherwise); they are called from the
 * thread of the entry point, never from a stream callback. */
typedef struct {
  void* (*alloc)(size_t bytes, void* stream, void* ctx);
  void (*free)(void* ptr, void* stream, void* ctx);
  void* ctx;
} love_allocator;

/* Status bits (love_cache_info_t.status_flags) */
#define LOVE_SF_DOMAIN 1u           /* a point outside [lo, hi] was seen                          */
#define LOVE_SF_NONFINITE 2u        /* non-finite x / y / coefficient                              */
#define LOVE_SF_NOTPD 4u            /* T not positive definite; k_eff truncated at the first bad pivot */
#define LOVE_SF_BREAKDOWN 8u        /* Lanczos stopped early (invariant subspace); not an error   */
#define LOVE_SF_CG_NOCONV 16u       /* mean CG hit cg_maxit                                        */
#define LOVE_SF_SAMPLER_TRUNC 32u   /* T' had non-positive eigenvalues, clipped to zero           */

typedef struct {
  int32_t k_eff;                    /* Lanczos steps kept                                         */
  int32_t k_eff_sample;             /* columns of S                                               */
  int32_t cg_iters;                 /* CG iterations of the mean solve                            */
  int32_t d;
  int64_t n, m;                     /* training rows; grid points (product of the m_i, or their
                                       sum for LOVE_FLAG_ADDITIVE: the rows of rt, a and s)       */
  double beta_last;                 /* last Lanczos off-diagonal                                  */
  double ortho_loss;                /* max |Q^T Q - I| of the Lanczos vectors (NaN: not computed,
                                       i.e. without the preconditioned mean solve)                */
  uint32_t status_flags;            /* LOVE_SF_*                                                  */
  uint32_t toeplitz_mode[LOVE_MAX_DIM]; /* backend chosen per axis (1 direct, 2 fft)          */
  uint32_t fft_len[LOVE_MAX_DIM];   /* circulant length per axis when FFT is used                 */
  size_t bytes;                     /* device bytes held by the cache                             */
  int32_t restarts;                 /* restarts taken (love_config.restart_tol)                   */
  double solve_residual;            /* worst relative residual of the last check (NaN: none)      */
} love_cache_info_t;

/* Buffers the cache contents can be copied into (all device, caller-owned, any may be NULL). */
typedef struct {
  double* alpha;                    /* k_eff  : diagonal of T                                      */
  double* beta;                     /* k_eff  : off-diagonal of T (beta[k_eff-1] = last residual)  */
  float* rt;                        /* m x k_eff row-major : Rt (dequantised for the bf16 split)  */
  double* rt64;                     /* m x k_eff row-major : Rt when precision is FP64            */
  void* a;                          /* m      : mean cache (precision's element type)             */
  float* s;                         /* m x k_eff_sample row-major : sampling matrix S             */
} love_export;

/* Cache contents to rebuild a cache from (all device, caller-owned; the
 * layouts are those of love_export, so an exported cache imports as is). */
typedef struct {
  int32_t k_eff;                    /* columns of rt, 1..LOVE_MAX_K                               */
  int32_t k_eff_sample;             /* columns of s, 0..LOVE_MAX_K (0: no sampler)                */
  const double* alpha;              /* k_eff (nullable: then zeros)                               */
  const double* beta;               /* k_eff (nullable: then zeros)                               */
  const float* rt;                  /* m x k_eff row-major (FP32 and BF16-split precisions)       */
  const double* rt64;               /* m x k_eff row-major (FP64 precision)                       */
  const void* a;                    /* m, precision's element type (NULL: zero mean cache)        */
  const float* s;                   /* m x k_eff_sample row-major (NULL iff k_eff_sample = 0)     */
} love_import;

/* ABI version of the loaded library (LOVE_ABI_VERSION). */
int32_t love_abi_version(void);

/* Human-readable name of a status code (static string). */
const char* love_status_string(love_status s);

/* Build the LOVE cache (Alg. 1 precomputation, Sec. 3.2) and, if
 * cfg->k_sample > 0, the sampling matrix S (Sec. 3.3).
 *   x : n x d training inputs, y : n targets (device, precision's type).
 *   alloc : device memory source (NULL: the device's stream-ordered pool).
 *   out : receives the new cache; untouched on error.
 * Errors: EINVAL (arguments), EDOMAIN (x outside [lo, hi]), ENONFINITE (non-finite
 * x, y, or Lanczos breakdown into NaN), ENOMEM, EHIP.  A T that is not positive
 * definite truncates k_eff and sets LOVE_SF_NOTPD (not an error). */
love_status love_build_cache(const love_config* cfg, const void* x, const void* y, int64_t n,
                             const love_allocator* alloc, void* stream, love_cache** out);

/* Build G independent caches (a1-a11 of the build for every GP) with every
 * phase launched once for all GPs, in lock step over the Lanczos and CG
 * steps: each kernel maps its blocks to (GP, local block) through a
 * per-launch work table and reads the GP's arguments from a device array, so
 * small GPs share the device instead of each under-filling it.  cfgs, xs, ys,
 * ns, out are host arrays of length G; all GPs must share precision, d and the
 * LOVE_FLAG_NO_MEAN bit (EINVAL otherwise).  Batches beyond 64 GPs run in
 * groups of 64.  Samplers (k_sample > 0) are built one GP after another on a
 * side stream.  On error no cache is returned.  Each GP's cache equals its
 * single-GP build on the same inputs bit for bit (love_build_cache is the
 * batch of one). */
love_status love_build_cache_batched(int32_t G, const love_config* cfgs, const void* const* xs,
                                     const void* const* ys, const int64_t* ns,
                                     const love_allocator* alloc, void* stream,
                                     love_cache** out);

/* Constant-time predictive mean and variance (eq. pred_mean_ski; eq.
 * pred_covar_ski_fast with i = j).  xs : t x d; mean (nullable) and var : t. */
love_status love_predict_mean_var(const love_cache* c, const void* xs, int64_t t, void* mean,
                                  void* var, void* stream);

/* Same for G caches in one launch (host arrays of length G; means may be
 * NULL, or hold NULL entries).  All caches must share precision and d. */
love_status love_predict_mean_var_batched(int32_t G, const love_cache* const* caches,
                                          const void* const* xs, const int64_t* ts,
                                          void* const* means, void* const* vars, void* stream);

/* Predictive cross-covariance of paired points: cov[i] = k(xa_i, xb_i)
 * (Alg. 1 with w_i != w_j).  xa, xb : t x d; cov : t. */
love_status love_predict_covar_pairs(const love_cache* c, const void* xa, const void* xb,
                                     int64_t t, void* cov, void* stream);

/* Predictive covariance of every pair: cov[i * tb + j] = k(xa_i, xb_j)
 * (Alg. 1 with w_i != w_j, eq. pred_covar_ski_fast):
 * prod_e w_{a,e}^T T_e w_{b,e} - (Rt^T w_a) . (Rt^T w_b), the dot product in
 * double.  xa : ta x d, xb : tb x d (cache precision, device); cov : ta x tb
 * row-major, caller-owned.  ta <= 65535 * 32.  A point outside [lo, hi]
 * gives NaN in its row / column and sets LOVE_SF_DOMAIN.  The call allocates
 * (ta + tb) (kpad + 5 d + 1) doubles of scratch on `stream` from `alloc`
 * (NULL: the cache's own memory source) and frees it on the stream.
 * Errors: EINVAL for bad sizes or NULL buffers, ENOMEM. */
love_status love_predict_covar_block(const love_cache* c, const void* xa, int64_t ta,
                                     const void* xb, int64_t tb, void* cov,
                                     const love_allocator* alloc, void* stream);

/* Posterior samples (eq. sample with S of eq. pred_covar_ski_interp_form):
 * out[i, j] = mu(xs_i) + sum_a w_a(xs_i) (S z_j)[a].
 *   z : k_eff_sample x s row-major standard normals (float; rows beyond
 *       k_eff_sample are ignored, so a k_sample x s array is always valid);
 *   out : t x s row-major.
 * Errors: EUNSUPPORTED if the cache has no sampler. */
love_status love_sample_posterior(const love_cache* c, const void* xs, int64_t t, const float* z,
                                  int64_t s, void* out, void* stream);

/* love_sample_posterior for callers that cannot allocate device memory: code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  Same arguments, kernels and results (bit for bit) as
 * love_sample_posterior, but the t x (kspad + 1) floats of intermediate
 * W_{X*} S and means live in a fixed device array of
 * LOVE_NOALLOC_SCRATCH_BYTES instead of memory from the cache's allocator;
 * no hipMalloc, hipFree or allocating library routine is called.
 *   kspad = 64 if min(k_sample, m) <= 64, else 128, so t may be at most
 *   32263 (kspad 64) or 16256 (kspad 128) points per call; a larger t returns
 *   LOVE_ELIMIT before any device work (split the points over several calls).
 *   The array's address is looked up once per device (hipGetSymbolAddress)
 *   on the first call made with that device current; the call runs on the
 *   current device, which must be the cache's (EINVAL otherwise).
 *   Every call on one device shares that device's array and leaves its
 *   contents behind: calls that overlap on one device (several streams or
 *   threads, or a graph replayed beside another call) race and must be
 *   serialised by the caller.
 * Errors: as love_sample_posterior, plus ELIMIT; EHIP if the symbol lookup
 * fails. */
love_status love_sample_posterior_noalloc(const love_cache* c, const void* xs, int64_t t,
                                          const float* z, int64_t s, void* out, void* stream);

/* Backward of love_predict_mean_var: given upstream gradients g_mean, g_var
 * (t each, either nullable), writes g_xs (t x d) = d(sum g_mean*mean + g_var*var)/d xs,
 * through the derivative interpolation weights, and, if g_rt is not NULL,
 * ADDS d(sum g_var*var)/d Rt = -2 sum_i g_var,i w(x*_i) (Rt^T w(x*_i))^T to g_rt
 * (m x k_eff row-major float; the caller zeroes it).  The g_rt sum is formed
 * per grid node over the query points sorted by stencil cell, in double and in
 * a fixed order, so it is bitwise reproducible; it takes t x kpad floats plus
 * (t, or d t for LOVE_FLAG_ADDITIVE) + cells + 1 32-bit words of scratch from
 * the cache's memory source.  Out-of-domain points contribute nothing.
 * Errors: EINVAL, ENOMEM (scratch), EHIP. */
love_status love_predict_backward(const love_cache* c, const void* xs, int64_t t,
                                  const void* g_mean, const void* g_var, void* g_xs, float* g_rt,
                                  void* stream);

/* Gradient of sum_i g_var[i] var(xs_i) with respect to the hyper-parameters,
 * through the cache (Sec. 3.2: the cache is built during training; eqs.
 * pred_covar_approx, pred_covar_ski_cache, pred_covar_ski_fast).  Every solve
 * Khat^{-1} in the derivative of the variance is taken as the cached Lanczos
 * solve Q T^{-1} Q^T (eq. lanczos_solve), as the cached variance itself does:
 *   d/dtheta sum g_i var_i = sum g_i dp_i/dtheta + <dK/dtheta B, B M - 2 P>
 *                            + [theta = sigma^2] sum g_i ||L^{-T} u_i||^2,
 * with u_i = Rt^T w_i, M = sum g_i u_i u_i^T, P = sum g_i w_i u_i^T (the
 * last term takes Q^T Q = I).  theta order in grad (device, d + 2 doubles):
 * lengthscale_0 .. lengthscale_{d-1}, outputscale, noise sigma^2.  For an
 * additive composition the lengthscale of axis e moves block e only.
 *   xs : t x d, g_var : t (precision's type, device); points outside the
 *   domain contribute nothing.  Scratch: about (t + 3 m) kpad + t d doubles
 *   from the cache's memory source.
 * Errors: EUNSUPPORTED if the cache was built without LOVE_FLAG_HYPER (or
 * imported), EINVAL, ENOMEM, EHIP. */
love_status love_predict_var_hyper_grad(const love_cache* c, const void* xs, int64_t t,
                                        const void* g_var, double* grad, void* stream);

/* out = Khat v = (W K W^T + sigma^2 I) v in the caller's training-row order (n). */
love_status love_apply_khat(const love_cache* c, const void* v, void* out, void* stream);

/* out = K_UU g on the grid (m, row-major grid order, last dimension fastest). */
love_status love_apply_kuu(const love_cache* c, const void* g, void* out, void* stream);

/* Query counters and status (synchronises the stream the cache was built on). */
love_status love_cache_info(const love_cache* c, love_cache_info_t* info);

/* k_eff and k_eff_sample (the rows z of love_sample_posterior needs) without
 * synchronising: the values recorded when a synchronous build (no
 * LOVE_FLAG_ASYNC) or an import returned.  After an asynchronous build the
 * first call reads them like love_cache_info (synchronising the build stream).
 * Out-pointers are host memory; EINVAL on NULL. */
love_status love_cache_keff(const love_cache* c, int32_t* k_eff, int32_t* k_eff_sample);

/* Copy cache contents into caller device buffers (enqueued on `stream`). */
love_status love_cache_export(const love_cache* c, const love_export* e, void* stream);

/* Rebuild a cache from its contents (love_export layout) without the
 * training data: the LOVE query (Alg. 1, eq. pred_covar_ski_fast), the
 * covariance calls, the backward and, with s, the sampler (eq. sample) then
 * work as on the cache that was exported; love_apply_khat needs the training
 * rows and returns LOVE_EUNSUPPORTED.  cfg gives the grid, kernel and
 * precision (cfg->k and cfg->k_sample are replaced by the imported column
 * counts); alloc as for love_build_cache.  For the BF16 split the float Rt is split again into hi + lo,
 * whose sum reproduces it.  Enqueued on `stream`; the imported buffers may be
 * released once the stream has passed this call.
 * Errors: EINVAL (bad config, counts or NULL buffers), ENOMEM, EHIP. */
love_status love_cache_import(const love_config* cfg, const love_import* im,
                              const love_allocator* alloc, void* stream, love_cache** out);

/* Release a cache, stream-ordered on its build stream: work queued on that
 * stream before the call finishes first, and the host does not wait.  Work on
 * other streams that reads the cache must be complete (or ordered before the
 * build stream's current point) when this is called.  The memory goes back
 * through the allocator the cache was built (or imported) with.  NULL is a
 * no-op. */
void love_cache_free(love_cache* c);

/* Per-kernel timing with HIP events recorded around each launch on the
 * launch stream.  enable=1 starts (and clears) collection, 0 stops it.  Timing
 * adds a pair of event records per launch; it does not change the work. */
love_status love_profile_enable(int32_t enable);

/* Restrict timing to the named scopes (comma-separated); NULL or "" = all. */
love_status love_profile_select(const char* names);

/* Read accumulated timings (synchronises).  For each kernel name in
 * `names` (comma-separated, e.g. "cgs_update,gather_dots"), writes the number of
 * launches and the total milliseconds into calls[i] and ms[i]. */
love_status love_profile_read(const char* names, int64_t* calls, double* ms);

#ifdef __cplusplus
}
#endif
#endif /* LOVE_H_ */
