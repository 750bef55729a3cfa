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
  SSI_EINTERNAL = 5
} ssi_status;

typedef enum ssi_svd_mode {
  SSI_SVD_FULL = 0,        /* exact SVD of T (Eq. (8)); for small T          */
  SSI_SVD_RANDOMIZED = 1   /* randomized SVD (Algorithm 1, Eq. (13)-(18))   */
} ssi_svd_mode;

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
 * within an order they are sorted by (f, xi).  One pole is kept per complex
 * conjugate pair (Im mu > 0); real eigenvalues are dropped.               */
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
/* Block until all work enqueued by this context has finished. */
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
  SSI_STAGE_SHIFT_LS,        /* Gram matrices, Cholesky, W              */
  SSI_STAGE_EIG,             /* per-order Hessenberg, QR, poles         */
  SSI_STAGE_COUNT
};
ssi_status ssi_set_profiling(ssi_ctx *ctx, int enable);
ssi_status ssi_profile_read(ssi_ctx *ctx, double *ms, int32_t *calls, int32_t n_stages);

/* ----------------------------------------------- host-only helpers (no GPU) */

/* Check parameters against l channels and n samples: 2 <= j_b, 2 j_b - 1 < n,
 * 1 <= order_min <= order_max <= min(l (j_b - 1), 224) for every lag; for the
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

/* Full identification of one record for every (lag, order).
 * y: device pointer, l x n floats, channel-major with leading dimension ldy
 * (>= n).  out: device buffers sized by ssi_output_layout.  Enqueued on the
 * context stream; results are valid after ssi_synchronize(). */
ssi_status ssi_identify(ssi_ctx *ctx, const float *y, int32_t l, int64_t n,
                        int64_t ldy, const ssi_params *p, const ssi_output *out);

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
 * P = Q^T T; P = U~ S V^T; U = Q U~.  Products on FP32 MFMA; orthonormal
 * bases, the small SVD and U in FP64.
 * t: device m x ldt floats.  omega: device m x (k+p) floats (ld k+p), or NULL
 * to draw it with ssi_sketch(seed, stream).  u: device m x k doubles
 * (row-major, ld k).  sigma: device k doubles, descending. */
ssi_status ssi_rsvd(ssi_ctx *ctx, const float *t, int64_t m, int64_t ldt,
                    int32_t k, int32_t p, int32_t q, const float *omega,
                    uint64_t seed, uint32_t stream, double *u, double *sigma);

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
 * order_max <= min(k, m - l, 224).  Writes lag slot `lag_index` of `out`
 * (out->sigma is not written). */
ssi_status ssi_modal(ssi_ctx *ctx, const double *u, const double *sigma,
                     int64_t m, int32_t k, int32_t l, const ssi_params *p,
                     int32_t lag_index, const ssi_output *out);

#ifdef __cplusplus
}
#endif
#endif /* SSICOV_H */
