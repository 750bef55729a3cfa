/*
 * ssicov.h - C ABI of the MI355X covariance-driven stochastic subspace
 * identification (SSI-COV) library with randomized SVD.
 *
 * Problem (Section 2.1 of Tomassini, Garcia-Macias, Ubertini, "Fast
 * Stochastic Subspace Identification of Densely Instrumented Bridges Using
 * Randomized SVD"): from l output channels sampled N times at f_s
 * (the discrete model of Eq. (5)), estimate modal frequencies, damping ratios
 * and mode shapes for every model order n2 in [order_min, order_max] and every
 * time-lag step j_b of the 3D stabilization diagram (Section 2.3, step i).
 *
 * Path: correlations R_1..R_{2 j_b,max - 1} (Section 2.1) -> block Toeplitz
 * T_{1|j_b} (Eq. (6)) -> SVD (Eq. (8)) or randomized SVD (Algorithm 1 and
 * Eq. (13)-(18), with oversampling p and q power iterations) -> O = U S^1/2,
 * C and A by shift least squares (Eq. (9)-(10)) -> eig(A) (Eq. (11)) ->
 * lambda, f, xi, phi (Eq. (12) read through Eq. (3)).
 *
 * Conventions for every call:
 *   - Every function returns ssi_status unless stated otherwise; nothing
 *     throws across the ABI.  On failure ssi_last_error() returns a
 *     thread-local message.  The context stays usable after any error.
 *   - "device pointer" means memory on the context's GPU (hipMalloc'd or a
 *     torch CUDA tensor's data_ptr); "host pointer" means ordinary host memory.
 *     All device-pointer arguments are owned by the caller; the library never
 *     frees them and keeps no reference after the call returns.
 *   - All stage and identification calls are asynchronous and ordered on the
 *     context's HIP stream: they return once the work is enqueued.  Call
 *     ssi_synchronize() (or synchronize the stream) before reading outputs.
 *   - Matrices are row-major.  y is channel-major: y[a * ldy + k] is sample k
 *     of channel a.
 *   - Arguments are validated on the host before any launch; invalid sizes or
 *     pointers give SSI_EINVAL and launch nothing.
 */
#ifndef SSICOV_H
#define SSICOV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum ssi_status {
  SSI_OK = 0,
  SSI_EINVAL = 1,     /* invalid argument, shape or order range            */
  SSI_ENOMEM = 2,     /* device workspace could not be allocated            */
  SSI_EDEVICE = 3,    /* HIP runtime error or no usable gfx950 device       */
  SSI_ENOCONV = 4,    /* an iterative kernel hit its iteration limit        */
  SSI_EINTERNAL = 5,
  SSI_EBUSY = 6       /* serving: the request has not finished yet          */
} ssi_status;

typedef enum ssi_svd_mode {
  SSI_SVD_FULL = 0,        /* exact SVD of T (Eq. (8)); for small T          */
  SSI_SVD_RANDOMIZED = 1   /* randomized SVD (Algorithm 1, Eq. (13)-(18))   */
} ssi_svd_mode;

/* Arithmetic of the range-finder products of the randomized SVD (the sketch
 * Y = T Omega and the power-iteration products).  The projection P = Q^T T,
 * every orthonormalization, the small SVD, the shift least squares and the
 * eigen-analysis are FP64 in both modes. */
typedef enum ssi_precision {
  SSI_PREC_FP32 = 0,   /* T as stored (FP32) times FP64 X, FP64 MFMA accumulation */
  SSI_PREC_BF16 = 1,   /* T and X rounded to BF16 (nearest even), FP32 MFMA
                          accumulation, FP64 sum of the K slices.  A lower-accuracy
                          mode: 8 significant bits resolve singular vectors only
                          down to about 2^-9 sigma_1, so poles at orders that need
                          smaller singular values move by more than the
                          reduced-precision tolerance (up to 6e-3 in frequency on a
                          180-channel record at orders 86..200)                  */
  SSI_PREC_BF16X3 = 2, /* T and X split into BF16 hi + lo parts (lo = BF16 of the
                          remainder), three BF16 MFMA products hi hi + hi lo +
                          lo hi with FP32 accumulation: about 16 significant bits
                          per operand.  With one refinement step
                          (ssi_params.refine = 1) it keeps frequencies within 1e-3,
                          damping within 2e-3 and MAC above 0.99 of the FP64
                          computation at every order of the 180-channel record at
                          lags 20..100 (worst 1.3e-4); without refinement the
                          products' FP32 accumulation leaves 4e-3 at lag 20    */
  SSI_PREC_BF16X6 = 3, /* T (FP32 as stored) and X (rounded to FP32) split
                          exactly into three BF16 parts each by truncation; the six
                          products of weight >= 2^-16 on v_mfma_f32_16x16x32_bf16,
                          each exact in FP32, FP32 accumulation: FP32-operand
                          products at the BF16 matrix rate, FP32 accumulation
                          (1.4e-3 in frequency at lag 20 without refinement,
                          5e-5 with one refinement step)                         */
  SSI_PREC_FP8 = 4     /* T and X block-scaled FP8 E4M3 along the contraction
                          index (32 elements per power-of-two E8M0 scale; the
                          block maximum scaled into [128, 256), nearest even),
                          v_mfma_scale_f32_16x16x128_f8f6f4 with FP32
                          accumulation, FP64 sum of the K slices.  T is quantized
                          twice per randomized SVD (along rows for T X, along
                          columns for T^T X), X before each product.  A
                          lower-accuracy mode: 3 mantissa bits per operand leave
                          frequencies within about 1e-2 of the FP64 computation
                          on a 180-channel record with one refinement step
                          (ssi_params.refine), the form it is meant to run in   */
} ssi_precision;

/* Arithmetic of the correlation products (Section 2.1), a context option.
 * All accumulate FP32 products in FP32 over 32-sample steps, fold into FP64
 * every 256 samples and sum the time splits in FP64. */
typedef enum ssi_corr_mode {
  SSI_CORR_FP32 = 0,   /* FP32 samples on v_mfma_f32_16x16x4f32                   */
  SSI_CORR_BF16X6 = 1, /* each FP32 sample split exactly into three BF16 parts
                          (hi + mid + lo, by truncation); the six cross products of
                          weight >= 2^-16 on v_mfma_f32_16x16x32_bf16, each exact in
                          FP32; the three dropped terms are below 2^-23 |y_a y_b|.
                          Needs 6 l' N' bytes of workspace for the parts (l', N':
                          channels and samples rounded up); falls back to
                          SSI_CORR_FP32 when a tile would not fit (tiny lag counts
                          with many channels).                                    */
  SSI_CORR_F16X3 = 2   /* each channel scaled by a power of two 2^e_a that puts its
                          largest |sample| in [2^13, 2^14); each scaled sample x
                          split into two FP16 parts, hi = FP16(x) and
                          lo = FP16(x - hi) (nearest even), so hi + lo equals x to
                          2^-22 |x|; the three cross products hi hi, hi lo, lo hi
                          on v_mfma_f32_16x16x32_f16, each exact in FP32, the
                          dropped lo lo below 2^-22 |x_a x_b|; the sums scaled back
                          by 2^-(e_a + e_b) exactly.  Per product the error is at
                          most about 2^-21 |y_a y_b|, below the worst-case rounding
                          of the 256-sample FP32 accumulation that every mode
                          shares.  Needs 4 l' N' + 36 l' bytes of workspace; falls
                          back to SSI_CORR_FP32 like SSI_CORR_BF16X6.  The
                          default.                                                */
} ssi_corr_mode;

/* Identification parameters (Section 2.1 and 2.3 control parameters). */
typedef struct ssi_params {
  double fs;                  /* sampling frequency f_s in Hz, > 0                  */
  const int32_t *lags;        /* host pointer: n_lags time-lag steps j_b,
                                 strictly increasing, j_b >= 2, 2 j_b - 1 < N       */
  int32_t n_lags;             /* >= 1                                               */
  int32_t order_min;          /* model orders order_min, +order_step, .. <= max     */
  int32_t order_max;
  int32_t order_step;         /* >= 1                                               */
  int32_t svd;                /* ssi_svd_mode                                       */
  int32_t rank;               /* randomized: k >= order_max (Section 2.2 end);
                                 full: ignored (order_max singular triplets kept)   */
  int32_t oversample;         /* randomized: p >= 0; sketch width ell = k + p <= m  */
  int32_t power_iters;        /* randomized: q >= 0                                 */
  uint64_t seed;              /* Gaussian sketch seed (Philox-4x32-10 key)          */
  int32_t prec;               /* ssi_precision of the range-finder products;
                                 other than SSI_PREC_FP32 needs
                                 svd = SSI_SVD_RANDOMIZED                          */
  const float *omega;         /* optional caller sketch (Eq. (14)): device pointer,
                                 m_max x (k + p) floats, row-major, ld omega_ld,
                                 m_max = max(j_b) l; lag i uses its leading j_b,i l
                                 rows.  NULL: drawn from `seed` (Philox stream i for
                                 lag i).  Randomized SVD only.  Read during the
                                 call's device work (stream-ordered).               */
  int64_t omega_ld;           /* >= k + p when omega is given                       */
  int32_t refine;             /* reduced-precision products only: the last `refine`
                                 power iterations (both products) run as in
                                 SSI_PREC_FP32 (refinement steps); 0 <= refine <= q  */
} ssi_params;

/* Sizes of the device output buffers of ssi_identify, from ssi_output_layout. */
typedef struct ssi_layout {
  int32_t n_lags;
  int32_t n_orders;           /* number of model orders in the sweep                */
  int32_t sigma_per_lag;      /* singular values stored per lag                     */
  int32_t pole_cap;           /* pole slots per lag: sum over orders of n2 / 2      */
  int32_t l;                  /* channels                                           */
  int32_t n_corr;             /* correlation blocks computed: 2 max(j_b) - 1        */
} ssi_layout;

/* Device output buffers of ssi_identify (all device pointers, caller-owned).
 * Poles of (lag i, order o) occupy slots [off(o), off(o) + count[i][o]) of lag
 * i, with off(o) = sum over earlier orders of n2 / 2 (see ssi_pole_offset);
 * within an order they are sorted by (f, xi); the remaining slots of the
 * order, up to off(o) + n2 / 2, are written with zeros.  One pole is kept per
 * complex conjugate pair (Im mu > 0); real eigenvalues are dropped.       */
typedef struct ssi_output {
  double *sigma;      /* [n_lags][sigma_per_lag], descending                      */
  int32_t *count;     /* [n_lags][n_orders] poles per (lag, order)                */
  double *f;          /* [n_lags][pole_cap] natural frequency, Hz                 */
  double *xi;         /* [n_lags][pole_cap] damping ratio                         */
  double *mu;         /* [n_lags][pole_cap][2] discrete eigenvalue (re, im)       */
  float *phi;         /* [n_lags][pole_cap][l][2] mode shape (re, im), unit
                         2-norm, largest-modulus entry real and positive          */
  int32_t *flags;     /* [n_lags][n_orders] 0 = converged, 1 = eig iteration
                         limit reached (poles of that order unreliable)           */
} ssi_output;

typedef struct ssi_ctx ssi_ctx;

/* ---------------------------------------------------------------- context */

/* Create a context on HIP device `device`.  `hip_stream` is the hipStream_t
 * to order all work on; NULL is the device's default (null) stream, as
 * everywhere in HIP.  Returns SSI_EDEVICE when the device is absent or not
 * gfx950.  *out is set only on SSI_OK.  Device workspace is allocated lazily
 * and grows on demand. */
ssi_status ssi_create(int device, void *hip_stream, ssi_ctx **out);
/* Free the context and its workspace.  NULL is ignored. */
void ssi_destroy(ssi_ctx *ctx);
/* Block until all work enqueued by this context has finished, then report
 * (and clear) what the kernels flagged on the device:
 *   SSI_EINVAL   the record held non-finite samples (NaN or Inf);
 *   SSI_ENOCONV  a Cholesky factorization broke down, or the QR iteration of
 *                an order hit its sweep limit (ssi_set_eig_max_sweeps; the
 *                order's output flag is 1), or a pole's wait for its order's
 *                eigenvalues timed out (that pole is skipped);
 *   SSI_EINTERNAL the eigen-analysis work loop hit its pass cap.
 * The kernels finish normally in every case. */
ssi_status ssi_synchronize(ssi_ctx *ctx);
/* Bytes of device workspace currently held by the context. */
size_t ssi_workspace_bytes(const ssi_ctx *ctx);

/* Stage timing.  When enabled, the context records a pair of HIP events on
 * its stream around every stage it enqueues; ssi_profile_read synchronizes,
 * adds the elapsed times into per-stage totals and returns them.  Stage ids:
 * SSI_STAGE_* below.  ms[i] (milliseconds) and calls[i] are accumulated since
 * the last read; n_stages is the length of both caller arrays (host). */
enum {
  SSI_STAGE_CORR_MFMA = 0,   /* correlation contraction kernel          */
  SSI_STAGE_CORR_REDUCE,     /* split-K reduction of the correlations   */
  SSI_STAGE_TOEPLITZ,        /* block-Toeplitz assembly                 */
  SSI_STAGE_SKETCH,          /* Gaussian sketch                         */
  SSI_STAGE_PRODUCTS,        /* T X and T^T X products (incl. reduce)   */
  SSI_STAGE_ORTH,            /* CholeskyQR orthonormalisations          */
  SSI_STAGE_SMALL_SVD,       /* P P^T, eigen-decomposition, U = Q U~    */
  SSI_STAGE_SHIFT_LS,        /* Gram matrices, Cholesky, W, X_n and their
                                Hessenberg forms (per lag)              */
  SSI_STAGE_EIG,             /* QR iterations, poles and sorting of every
                                (lag, order), one launch                */
  SSI_STAGE_CORR_SPLIT,      /* split parts of the record (BF16x6, FP16x3) */
  SSI_STAGE_COUNT
};
ssi_status ssi_set_profiling(ssi_ctx *ctx, int enable);
ssi_status ssi_profile_read(ssi_ctx *ctx, double *ms, int32_t *calls, int32_t n_stages);

/* Lag sweep of the 3D stabilization diagram (Section 2.3, step i) over n
 * streams (1 <= n <= 4, default 1).  ssi_identify computes the correlations
 * once on the context stream and prepares every lag (Toeplitz, SVD, shift
 * least squares, Hessenberg forms); with n > 1 lag i is prepared on internal
 * stream i % n, each with its own buffers, and the context stream waits for
 * all of them.  The eigen-analysis, poles and sorting of every (lag, order)
 * then run in one persistent launch on the context stream.  Results are
 * identical for every n; lags of different streams overlap on the device.
 * The internal streams are created here (default priority, non-blocking).
 * Synchronizes the context stream. */
ssi_status ssi_set_lag_streams(ssi_ctx *ctx, int32_t n);
/* Graph mode for ssi_identify (default off).  When on, every ssi_identify
 * call with a device record is keyed by all its arguments (pointers, sizes,
 * parameters, lag streams).  The first call with a key runs eagerly, waits
 * for completion, and captures the whole identification - all lags and
 * orders - into one HIP graph; later calls with the same key launch that
 * graph on the context stream.  The context keeps the 8 most recently used
 * graphs (a ninth key evicts the least recently used, after synchronizing),
 * so graph mode pays off for callers that reuse their record and output
 * buffers.  Graphs are dropped when the workspace grows, the lag-stream count
 * or another option changes, or graph mode is turned off.  Calls with a host
 * record always run eagerly.  Stage profiling is not recorded for graph
 * launches.  The output buffers and y must stay allocated while a graph that
 * names them may be launched. */
ssi_status ssi_set_graphs(ssi_ctx *ctx, int enable);
/* Autotuning of the range-finder products (default off).  When on, the
 * first product of each (precision, orientation, M, N, K) times candidate
 * launch configurations with HIP events on the context stream: K-slice
 * counts (the planner's own choice, then 2, 4, 6, 8, 12, 16) and, for the
 * FP32 x FP64 products, each of them on 128-row and on 64-row output tiles
 * (each candidate computes the full product, so results are unaffected), and
 * keeps the fastest for the life of the context.  Tuning synchronizes the
 * stream once per new shape and never runs inside a graph capture. */
ssi_status ssi_set_autotune(ssi_ctx *ctx, int enable);
/* Output-tile height of the FP32 x FP64 range-finder products for products
 * the autotuner has not tuned: 0 (default) or 128 for 128-row tiles, 64 for
 * 64-row tiles (pins the configuration, e.g. for timing or testing one tile
 * shape).  SSI_EINVAL for other values.  Drops captured graphs. */
ssi_status ssi_set_product_tile_rows(ssi_ctx *ctx, int32_t rows);
/* Workgroups of the identification's eigen-analysis launch (Eq. (11) for
 * every order in one persistent launch): 0 (default) for one per CU; n > 0
 * for n workgroups, raised to the number of (lag, order) items when smaller
 * and capped at one per CU.  Fewer workgroups leave CUs to the kernels of
 * other windows running on other streams at the same time; results are
 * unaffected.  SSI_EINVAL for n < 0.  Drops captured graphs. */
ssi_status ssi_set_eig_workgroups(ssi_ctx *ctx, int32_t n);
/* Sweep limit of the eigen-analysis (Eq. (11)): the QR iteration of an order
 * of size n stops after sweeps_per_row * max(10, n) sweeps (default 30, as
 * LAPACK's Hessenberg QR), marks the order in the output flags and makes the
 * next ssi_synchronize return SSI_ENOCONV.  0 <= sweeps_per_row <= 1000; 0
 * fails every order that needs a sweep (orders of size 1 and 2 need none).
 * The iteration runs inside the kernel and always ends at the limit.  Drops
 * captured graphs. */
ssi_status ssi_set_eig_max_sweeps(ssi_ctx *ctx, int32_t sweeps_per_row);
/* Device memory for the context's workspace and ssi_identify_result's output
 * buffers from the caller's allocator (for example a framework's caching
 * allocator) instead of hipMalloc/hipFree.  alloc(bytes, user) returns a
 * device pointer on the context's device, or NULL when it cannot (the call
 * that needed it then fails with SSI_ENOMEM); release(ptr, user) takes back
 * what alloc returned, after all work that used it has finished.  Pass NULL
 * for both to return to hipMalloc.  Memory held from the previous allocator is
 * released to it first (after synchronizing).  Drops captured graphs. */
ssi_status ssi_set_allocator(ssi_ctx *ctx, void *(*alloc)(size_t bytes, void *user),
                             void (*release)(void *ptr, void *user), void *user);
/* Correlation product arithmetic (ssi_corr_mode) for later ssi_correlate,
 * ssi_identify and serving calls on this context; default SSI_CORR_F16X3.
 * SSI_EINVAL for an unknown mode.  Drops captured graphs. */
ssi_status ssi_set_corr_mode(ssi_ctx *ctx, int32_t mode);
/* Launch configuration chosen by the autotuner for a product, 0 if not
 * tuned: the K-slice count, plus 100 when the FP32 x FP64 product runs on
 * 64-row output tiles instead of 128-row ones.
 * kind: 0 = FP32 x FP64 product, 1 = BF16 product, 3 = split BF16 product, 6 = three-way
 * split BF16 product;
 * trans: 1 for T^T X. */
int32_t ssi_tuned_splits(const ssi_ctx *ctx, int32_t kind, int32_t trans, int32_t m,
                         int32_t n, int32_t k);

/* ----------------------------------------------- host-only helpers (no GPU) */

/* Check parameters against l channels and n samples: 2 <= j_b, 2 j_b - 1 < n,
 * 1 <= order_min <= order_max <= min(l (j_b - 1), 448) for every lag; for the
 * randomized mode order_max <= k and k + p <= min(j_b l, 1024); for the full
 * SVD j_b l <= 1024.  Host-only. */
ssi_status ssi_validate(const ssi_params *p, int32_t l, int64_t n);
/* Output buffer sizes for ssi_identify.  Host-only. */
ssi_status ssi_output_layout(const ssi_params *p, int32_t l, int64_t n,
                             ssi_layout *out);
/* Slot offset of order index o (0-based) within one lag's pole arrays. */
int32_t ssi_pole_offset(const ssi_params *p, int32_t order_index);
/* Device workspace bytes ssi_identify will need for these sizes.  Host-only. */
ssi_status ssi_workspace_estimate(const ssi_params *p, int32_t l, int64_t n,
                                  size_t *bytes);
/* Eq. (20): tau = (2 j_b - 1) / f_s. */
double ssi_tau(int32_t jb, double fs);
/* Eq. (22) with factor 10 (and the lower lag of Eq. (23) with factor 9):
 * ceil(factor f_s / (2 f0)); 'int' in the paper read as rounding up. */
int32_t ssi_lag_rule(double fs, double f0, double factor);
/* Eq. (21): minimum rank ceil(max(30 - 0.00156 T, 25) T / 100) for Toeplitz
 * size T = j_b l. */
int32_t ssi_default_rank(int64_t t_size);
const char *ssi_status_string(ssi_status s);
const char *ssi_last_error(void);

/* ---------------------------------------------------- whole identification */

/* Full identification of one record for every (lag, order) (Section 2.1,
 * Section 2.3 step i).
 * y: l x n floats, channel-major with leading dimension ldy (>= n); a device
 * pointer, or a host pointer (pinned or pageable), which is first copied into
 * the workspace (l n 4 more bytes) on the context stream; with pageable
 * memory that copy may return only once the data is staged.  out: device
 * buffers sized by ssi_output_layout.  Enqueued on the context stream;
 * results are valid after ssi_synchronize(), which also reports a record
 * with non-finite samples (SSI_EINVAL) and non-convergence (SSI_ENOCONV). */
ssi_status ssi_identify(ssi_ctx *ctx, const float *y, int32_t l, int64_t n,
                        int64_t ldy, const ssi_params *p, const ssi_output *out);

/* Host results.  An ssi_result holds host copies of one identification's
 * outputs; the library owns it and every pointer its accessors return, all
 * valid until ssi_result_free. */
typedef struct ssi_result ssi_result;
/* Synchronous identification: runs ssi_identify into output buffers the
 * context owns (kept and reused; from the allocator of ssi_set_allocator
 * when set), waits for it and copies the outputs to a new host result.
 * y: device or host pointer as for ssi_identify.  Returns the status of
 * ssi_synchronize; on SSI_ENOCONV or SSI_EINVAL from the device checks *res is
 * still set (per-order flags tell which orders failed). */
ssi_status ssi_identify_result(ssi_ctx *ctx, const float *y, int32_t l, int64_t n,
                               int64_t ldy, const ssi_params *p, ssi_result **res);
/* Waits for the context (ssi_synchronize, whose status it returns) and
 * copies the device outputs `out` of an identification with parameters p and
 * l channels into a new host result, set on every status but a failed copy. */
ssi_status ssi_result_fetch(ssi_ctx *ctx, const ssi_params *p, int32_t l,
                            const ssi_output *out, ssi_result **res);
ssi_status ssi_result_dims(const ssi_result *res, int32_t *n_lags, int32_t *n_orders,
                           int32_t *l);
/* Poles of (lag index, order index): model order n2, pole count, and arrays
 * of n_poles entries sorted by (f, xi): f in Hz, damping ratio, discrete
 * eigenvalue (re, im) pairs, mode shapes (n_poles x l complex, (re, im)
 * interleaved); flag 1 when that order's QR iteration hit its limit.  Any
 * output pointer may be NULL. */
ssi_status ssi_result_poles(const ssi_result *res, int32_t lag_i, int32_t order_i,
                            int32_t *order, int32_t *n_poles, const double **f_hz,
                            const double **zeta, const double **mu_reim,
                            const float **phi_reim, int32_t *flag);
/* Singular values of lag lag_i (descending; *n = sigma_per_lag). */
ssi_status ssi_result_singular_values(const ssi_result *res, int32_t lag_i, int32_t *n,
                                      const double **sigma);
/* Frees a result (NULL is ignored). */
void ssi_result_free(ssi_result *res);

/* ------------------------------------- stages on device buffers (parity) */

/* Section 2.1: R[j-1][a][b] = (1/n) sum_{k=0}^{n-1-j} y[a][k+j] y[b][k],
 * j = 1..n_corr.  y: device, l x n (ld ldy).  r: device, n_corr x l x l
 * floats.  Accumulates in FP32 on MFMA over short sample blocks and in FP64
 * across blocks.  1 <= n_corr < n. */
ssi_status ssi_correlate(ssi_ctx *ctx, const float *y, int32_t l, int64_t n,
                         int64_t ldy, int32_t n_corr, float *r);

/* Eq. (6): T[r_ l + a][c l + b] = R_{jb + r_ - c}[a][b] for 0 <= r_, c < jb.
 * r: device, at least 2 jb - 1 blocks of l x l floats (R_1 first).
 * t: device, (jb l) x ldt floats, ldt >= jb l. */
ssi_status ssi_toeplitz(ssi_ctx *ctx, const float *r, int32_t l, int32_t jb,
                        float *t, int64_t ldt);

/* Eq. (14): Gaussian test matrix.  omega: device, m x ell floats (ld ldo).
 * Entry e = i ell + c uses Philox-4x32-10 counter (lo(e/2), hi(e/2), stream,
 * 0) and key (lo(seed), hi(seed)); uniforms (top 52 bits + 1/2) 2^-52 of the
 * word pairs (x0, x1), (x2, x3); Box-Muller cosine branch for even e and sine
 * branch for odd e, computed in FP64 and rounded to FP32. */
ssi_status ssi_sketch(ssi_ctx *ctx, uint64_t seed, uint32_t stream, int64_t m,
                      int32_t ell, float *omega, int64_t ldo);

/* Randomized SVD of the m x m matrix T (Algorithm 1, Eq. (13)-(18)):
 * Y = T Omega; Q = orth(Y); q times: Q = orth(T^T Q), Q = orth(T Q);
 * P = Q^T T; P = U~ S V^T; U = Q U~.  The range-finder products follow
 * `prec` (ssi_precision), except the last `refine` power iterations, which
 * run as SSI_PREC_FP32 (0 <= refine <= q; refinement steps of a
 * reduced-precision range finder); the projection multiplies FP32 T by FP64
 * Q with FP64 MFMA accumulation; orthonormal bases (shifted CholeskyQR), the
 * small SVD and U are FP64.
 * t: device m x ldt floats.  omega: device m x (k+p) floats (ld k+p), or NULL
 * to draw it with ssi_sketch(seed, stream).  u: device m x k doubles
 * (row-major, ld k).  sigma: device k doubles, descending. */
ssi_status ssi_rsvd(ssi_ctx *ctx, const float *t, int64_t m, int64_t ldt,
                    int32_t k, int32_t p, int32_t q, int32_t prec, int32_t refine,
                    const float *omega, uint64_t seed, uint32_t stream, double *u,
                    double *sigma);

/* Exact SVD of the m x m matrix T (Eq. (8)): leading k left singular vectors
 * u (device m x k doubles) and singular values sigma (device, k doubles),
 * via the FP64 symmetric eigen-decomposition of T T^T.  m <= 1024. */
ssi_status ssi_svd_full(ssi_ctx *ctx, const float *t, int64_t m, int64_t ldt,
                        int32_t k, double *u, double *sigma);

/* Modal stage for one lag (Eq. (9)-(12)): for every order n of p, O = U_n
 * S_n^1/2, C = first l rows, A = pinv(O_top) O_bot, eig(A), poles.  Computed
 * through the similar matrix pinv(U_top,n) U_bot,n, which has the same
 * eigenvalues, with phi = U[0:l, :n] psi (so sigma only scales and is not
 * read).  u: device m x k doubles (ld k), sigma: device k doubles, m = jb l,
 * order_max <= min(k, m - l, 448).  Writes lag slot `lag_index` of `out`
 * (out->sigma is not written). */
ssi_status ssi_modal(ssi_ctx *ctx, const double *u, const double *sigma,
                     int64_t m, int32_t k, int32_t l, const ssi_params *p,
                     int32_t lag_index, const ssi_output *out);

/* ------------------------------------------------- stability analysis */

/* Thresholds of the hard criteria (Section 2.1 end) and of the soft
 * criteria of the 3D stabilization diagram (Eq. (19)).  The paper's 3D
 * analysis of the frame uses xi_max 0.10, mpc_min 0.60, mpd_max 0.50,
 * alpha_f 0.01, alpha_xi 0.03, alpha_mac 0.02. */
typedef struct ssi_stability_params {
  double xi_max;      /* keep 0 < xi <= xi_max                                  */
  double mpc_min;     /* keep MPC > mpc_min                                     */
  double mpd_max;     /* keep MPD < mpd_max (MPD normalized to [0, 1])          */
  double alpha_f;     /* |f_i - f_j| / max(f_i, f_j) <= alpha_f                 */
  double alpha_xi;    /* |xi_i - xi_j| / max(xi_i, xi_j) <= alpha_xi            */
  double alpha_mac;   /* 1 - MAC(phi_i, phi_j) <= alpha_mac                      */
} ssi_stability_params;

enum {
  SSI_POLE_HC = 1,          /* passes the hard criteria                         */
  SSI_POLE_STABLE_ORDER = 2,/* matches a pole of the previous order, same lag   */
  SSI_POLE_STABLE_LAG = 4,  /* matches a pole of the previous lag, same order   */
  SSI_POLE_STABLE = 8       /* hard criteria and (order or lag match), Eq. (19) */
};

/* Stability of every pole of an identification (device buffers `out` of
 * ssi_identify with the same p and l).  Per pole slot [lag][pole_cap]:
 *   mpc: modal phase collinearity ((Sxx - Syy)^2 + 4 Sxy^2) / (Sxx + Syy)^2
 *        with Sxx = |Re phi|^2, Syy = |Im phi|^2, Sxy = Re phi . Im phi;
 *   mpd: mean phase deviation: the |phi_a|-weighted mean angle between the
 *        components phi_a and the principal line of the points
 *        (Re phi_a, Im phi_a), over pi/2;
 *   flags: SSI_POLE_* bits.  A pole matches a neighbour (previous order of
 *        the same lag, or same order of the previous lag) when that
 *        neighbour passes the hard criteria and all three soft thresholds
 *        hold for the pair.  Empty slots get 0.
 * mpc, mpd: device doubles, flags: device bytes, each n_lags * pole_cap.
 * FP64 throughout (mode shapes widened from FP32).  Stream-ordered. */
ssi_status ssi_stability(ssi_ctx *ctx, const ssi_params *p, int32_t l,
                         const ssi_output *out, const ssi_stability_params *sp,
                         double *mpc, double *mpd, uint8_t *flags);

/* For callers that cannot allocate device memory (work under HIP graph
 * capture, serving loops or harnesses that forbid hipMalloc): ssi_stability
 * with the same arguments and results, but its per-slot scratch (the
 * hard-criteria verdict, one byte per pole slot) lives in a fixed static
 * device array of ssi_stability_noalloc_max_slots() bytes (4 MiB) instead of
 * the context workspace.  Calls no hipMalloc, hipFree or other allocating
 * routine.  SSI_EINVAL, before any launch, when n_lags * pole_cap exceeds the
 * array.  The array is one per GPU and shared by every call on that GPU from
 * any context: calls that overlap on one GPU race (order them on one stream
 * or synchronize between them).  The array keeps the last call's contents;
 * every slot a call reads is written by that call first, so nothing needs
 * clearing.  Its device address is looked up at ssi_create, once per device. */
ssi_status ssi_stability_noalloc(ssi_ctx *ctx, const ssi_params *p, int32_t l,
                                 const ssi_output *out, const ssi_stability_params *sp,
                                 double *mpc, double *mpd, uint8_t *flags);
/* Pole slots the static scratch of ssi_stability_noalloc holds.  Host-only. */
int64_t ssi_stability_noalloc_max_slots(void);

/* ------------------------------------------------------------- serving */

/* Continuous batching of identifications on one GPU, for monitoring many
 * structures at once (one request = one window of one record).  Requests
 * are queued by ssi_server_submit and admitted, in arrival order with
 * skip-ahead past a request that does not fit, to free slots while the device
 * memory the slots hold stays within the budget.  Each slot owns a context on
 * its own non-blocking stream and device buffers that grow on demand and are
 * kept; slots run concurrently, so work of different requests overlaps on the
 * device.  A request's result does not depend on what else runs (every
 * kernel is deterministic and the work of a request stays on its slot).
 * All functions are thread-safe. */
typedef struct ssi_server ssi_server;

typedef struct ssi_server_config {
  int32_t device;          /* HIP device                                        */
  int32_t max_inflight;    /* slots: requests on the GPU at once, 1..64         */
  size_t hbm_budget;       /* bytes the slots may hold in total; 0 = 80 % of the
                              free device memory at creation                     */
} ssi_server_config;

/* Timestamps in microseconds since the server was created (-1: not yet). */
typedef struct ssi_request_info {
  ssi_status status;       /* of the identification, once finished             */
  int32_t slot;            /* slot that ran it, -1 while queued                 */
  double t_submit_us, t_start_us, t_done_us;
  size_t footprint;        /* bytes charged at admission (ssi_footprint)        */
} ssi_request_info;

/* Host copies of one request's outputs, in the ssi_output layout of
 * `layout`.  Owned by the server until ssi_server_release. */
typedef struct ssi_host_result {
  ssi_layout layout;
  const double *sigma;
  const int32_t *count;
  const double *f, *xi, *mu;
  const float *phi;
  const int32_t *flags;
} ssi_host_result;

typedef struct ssi_server_stats {
  uint64_t submitted, completed, failed;
  int32_t queued, running;
  int32_t peak_inflight;   /* most requests running at once                     */
  uint64_t peak_bytes;     /* most device bytes held or reserved by the slots   */
  uint64_t held_bytes;     /* bytes held now                                    */
  uint64_t budget;
} ssi_server_stats;

/* Device bytes one identification of these sizes holds: the context
 * workspace (with its growth margin), y and the output buffers.  Host-only. */
ssi_status ssi_footprint(const ssi_params *p, int32_t l, int64_t n, size_t *bytes);
ssi_status ssi_server_create(const ssi_server_config *cfg, ssi_server **out);
/* Waits for every submitted request to finish, then frees all slots. */
void ssi_server_destroy(ssi_server *srv);
/* Queue one identification.  y: host pointer, l x n floats, channel-major
 * (ld ldy); copied before returning, as are the parameters (lags included).
 * Returns at once with a ticket.  SSI_EINVAL for invalid parameters (as
 * ssi_validate), SSI_ENOMEM if the request alone exceeds the budget. */
ssi_status ssi_server_submit(ssi_server *srv, const float *y, int32_t l, int64_t n,
                             int64_t ldy, const ssi_params *p, uint64_t *ticket);
/* SSI_EBUSY while queued or running, SSI_OK once finished (the request's own
 * status is info->status).  info may be NULL. */
ssi_status ssi_server_poll(ssi_server *srv, uint64_t ticket, ssi_request_info *info);
/* Blocks until the request has finished. */
ssi_status ssi_server_wait(ssi_server *srv, uint64_t ticket, ssi_request_info *info);
/* Host result of a finished request; its status if it failed. */
ssi_status ssi_server_result(ssi_server *srv, uint64_t ticket, const ssi_host_result **res);
/* Forget a finished request and free its host result. */
ssi_status ssi_server_release(ssi_server *srv, uint64_t ticket);
ssi_status ssi_server_get_stats(ssi_server *srv, ssi_server_stats *out);
/* Thread-local message for the last failed server call. */
const char *ssi_server_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* SSICOV_H */
