// Internal launcher declarations shared by the host API and the kernel files.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <algorithm>

namespace ssi {

// Bits of the context's device status word (kernels OR them in; the host
// reads and clears the word in ssi_synchronize).
enum : int {
  kStatusChol = 1,          // a Cholesky factorization broke down
  kStatusEigLimit = 8,      // an order's QR iteration hit its sweep limit
  kStatusClaimCap = 16,     // the eigen-analysis claim loop hit its pass cap
  kStatusNonFinite = 256    // the record held non-finite samples
};

// ---- correlations (correlate.hip)
struct CorrPlan {
  int grid_rows, grid_cols, splits;
  int64_t split_len;
  int sa_stride, na_max;
  size_t lds_bytes;
  size_t partial_elems;
  int mode;                     // ssi_corr_mode of the path taken
  int lp;                       // split paths: channel rows of each plane (multiple of 64)
  int64_t np;                   // split paths: samples per plane row
  int copy_stride;              // split paths: elements between the shifted A-window copies
  size_t planes_elems;          // BF16x6: 3 lp np bf16 elements of split planes;
                                // FP16x3: 2 lp np fp16 elements, then lp int32 exponents
                                // and 8 lp FP32 partial maxima;
                                // FP32: 0
};
// mode: the requested path; the split paths fall back to FP32 where their
// tiles do not fit two workgroups per CU.
CorrPlan plan_correlate(int l, int64_t n, int L, int num_cus, int mode);
hipError_t launch_correlate(const CorrPlan &p, const float *y, int l, int64_t n, int64_t ldy,
                            int L, double *partial, uint16_t *planes, float *r, int *status,
                            hipStream_t st);
// BF16x6: the record's three BF16 parts into planes; FP16x3: the channel
// scales and the two FP16 parts; no-op for FP32
hipError_t launch_correlate_split(const CorrPlan &p, const float *y, int l, int64_t n,
                                  int64_t ldy, uint16_t *planes, hipStream_t st);
hipError_t launch_correlate_mfma(const CorrPlan &p, const float *y, int l, int64_t n, int64_t ldy,
                                 int L, double *partial, const uint16_t *planes, hipStream_t st);
// Sets kStatusNonFinite in *status when a correlation is not finite (a
// non-finite sample makes at least one of them so).
hipError_t launch_correlate_reduce(const CorrPlan &p, int l, int64_t n, int L,
                                   const double *partial, const uint16_t *planes, float *r,
                                   int *status, hipStream_t st);

// ---- Toeplitz (toeplitz.hip)
hipError_t launch_toeplitz(const float *r, int l, int jb, float *t, int64_t ldt,
                           hipStream_t st);

// ---- sketch (sketch.hip)
hipError_t launch_sketch(uint64_t seed, uint32_t stream, int64_t m, int ell, float *omega,
                         int64_t ldo, hipStream_t st);
hipError_t launch_sketch(uint64_t seed, uint32_t stream, int64_t m, int ell, double *omega,
                         int64_t ldo, hipStream_t st);

// ---- dense products (gemm.hip)
struct GemmPlan {
  int gm, gn, splits, k_per_split;
  int bm;                        // rows of an output tile (FP32 x FP64 products: 128 or 64)
  int64_t ldc, split_stride;     // partial-sum layout: [splits][M][ldc]
  size_t part_elems() const { return (size_t)splits * (size_t)split_stride; }
};
// splits > 0 forces the number of K slices (autotuning); 0 picks it from the
// shape and the CU count.  bm: output-tile rows, 128 (default) or 64.
GemmPlan plan_gemm_tf64(int M, int N, int K, int num_cus, int splits = 0, int bm = 128);
GemmPlan plan_gemm_f64(int M, int N, int K, int num_cus);
hipError_t launch_gemm_tf64(const GemmPlan &p, bool trans_a, const float *A, int64_t lda,
                            const double *B, int64_t ldb, int M, int N, int K, double *part,
                            hipStream_t st);
hipError_t launch_gemm_f64(const GemmPlan &p, bool trans_a, const double *A, int64_t lda,
                           const double *B, int64_t ldb, int M, int N, int K, double *part,
                           hipStream_t st);
hipError_t launch_reduce(const GemmPlan &p, const double *part, int M, int N, double scale,
                         double *out, int64_t ldo, float *out32, int64_t ld32, hipStream_t st);
hipError_t launch_convert(const double *in, int64_t ldi, int M, int N, float *out, int64_t ldo,
                          hipStream_t st);

// ---- reduced-precision range-finder products (gemm_bf16.hip)
struct BfPlan {
  int gm, gn, splits, k_per_split;
  int64_t ldc, split_stride;     // FP32 partial sums: [splits][M][ldc]
  int n_pad, k_pad;              // BF16 operand X^T: n_pad x k_pad (ld ldx), zero-padded
  int64_t ldx;
  int nt;                        // 1: one BF16 product; 3: split (hi + lo) operands;
                                 // 6: exact three-way splits, six products
  size_t part_elems() const { return (size_t)splits * (size_t)split_stride; }
  size_t plane() const { return (size_t)n_pad * (size_t)ldx; }
  size_t xt_elems() const { return plane() * (nt == 1 ? 1 : (nt == 3 ? 2 : 3)); }
};
BfPlan plan_gemm_tbf16(int M, int N, int K, int num_cus, int splits = 0, int nt = 1);
hipError_t launch_pack_bf16(const BfPlan &p, const double *x, int64_t ldx, int K, int N,
                            uint16_t *xt, hipStream_t st);
hipError_t launch_gemm_tbf16(const BfPlan &p, bool trans_a, const float *A, int64_t lda,
                             const uint16_t *xt, int M, int N, int K, float *part,
                             hipStream_t st);
hipError_t launch_reduce_f32(const BfPlan &p, const float *part, int M, int N, double *out,
                             int64_t ldo, hipStream_t st);

// ---- FP8 range-finder products (gemm_fp8.hip): C = A B^T, A (M x K) and B
// (N x K) block-scaled FP8 E4M3 along K (32 elements per power-of-two scale)
struct Fp8Plan {
  int gm, gn, splits, k_per_split;
  int kp;                        // K rounded up to the 128-deep step (bytes per row)
  int n_pad;                     // rows of the quantized B (a multiple of the 224-row tile)
  int64_t ldc, split_stride;     // FP32 partial sums: [splits][M][ldc]
  size_t part_elems() const { return (size_t)splits * (size_t)split_stride; }
  size_t scale_bytes(int rows) const { return (size_t)rows * (size_t)(kp / 32); }
};
Fp8Plan plan_gemm_fp8(int M, int N, int K, int num_cus, int splits = 0);
// q[r][0:kp] (E4M3) and s[r][0:kp/32] (E8M0) of a[r][0:cols] (zero past cols)
hipError_t launch_quant_rows_f32(const float *a, int64_t lda, int rows, int cols, int kp,
                                 uint8_t *q, uint8_t *s, hipStream_t st);
// q[j][k] of a[k][j] (the transpose) for j < out_rows, k < kp (zero past the
// rows x cols input)
hipError_t launch_quant_cols_f32(const float *a, int64_t lda, int rows, int cols, int kp,
                                 int out_rows, uint8_t *q, uint8_t *s, hipStream_t st);
hipError_t launch_quant_cols_f64(const double *a, int64_t lda, int rows, int cols, int kp,
                                 int out_rows, uint8_t *q, uint8_t *s, hipStream_t st);
hipError_t launch_gemm_fp8(const Fp8Plan &p, const uint8_t *qa, const uint8_t *sa,
                           const uint8_t *qb, const uint8_t *sb, int M, int N, float *part,
                           hipStream_t st);

hipError_t launch_convert_f32_f64(const float *in, int64_t ldi, int M, int N, double *out,
                                  int64_t ldo, hipStream_t st);
hipError_t launch_sqrt_clamp(const double *ev, int k, double *sigma, hipStream_t st);
hipError_t launch_transpose_f32_f64(const float *in, int64_t ldi, int M, int N, double *out,
                                    int64_t ldo, hipStream_t st);

// ---- small dense FP64 (dense.hip), one workgroup, n <= dense_max_n()
int dense_max_n();
// scratch (doubles) shared by launch_chol_inv and launch_sym_eig for size n
size_t dense_ws_doubles(int n);
hipError_t launch_chol_inv(const double *G, int64_t ldg, int n, double shift_rel, double *Rinv,
                           int64_t ldr, double *Lws, double *ws, int *status, hipStream_t st);
// all n eigenvalues (descending) and the eigenvectors of the leading nvec
// (columns 0..nvec-1 of evecs; the others are left unspecified)
hipError_t launch_sym_eig(const double *G, int64_t ldg, int n, int nvec, double *evals,
                          double *evecs, int64_t ldv, double *ws, int *status, hipStream_t st);

// ---- modal stage (modal.hip)
int modal_max_order();
struct ModalSizes {
  int n_orders;
  int64_t sq, vec, poles;       // sums over orders of n^2, n, n/2
  int64_t vref, taus;           // doubles
  int64_t francis_glb;
  int64_t queue_ints;           // work counters and deferred list of the eig launch
};
ModalSizes modal_sizes(int nmin, int nmax, int step, int l);
// Per-lag element strides of the modal buffers of a multi-lag launch: lag g's
// Hessenberg matrices at hbuf + g sq, reflectors at vref + g vref, ..., the
// transposed first l rows of its U at u + g u.
struct ModalStrides {
  int64_t sq, vec, poles, vref, taus, u;
};
struct ModalArgs {
  ModalSizes sizes;
  int nmin, step, l;
  int n_lags;                   // lags of the eigen-analysis launch
  int ldw;                      // leading dimension of rinv and w
  int ldu;                      // columns of U: u holds, per lag, U[0:l, :ldu] transposed
                                // (ldu rows of l entries)
  double fs;
  const double *u, *rinv, *w;
  double *xbuf, *hbuf, *vref, *taus, *evbuf, *gscr;
  double *tf, *txi, *tmu, *tphi;
  int *npole, *pidx, *flags_tmp;
  int *queue, *done;            // work counters and per-order flags of the eig launch
  int *status;                  // context status word
  int eig_grid;                 // workgroups of the eigen-analysis launch, 0: one per CU
  int sweeps_per_row;           // QR sweep limit per order: sweeps_per_row * max(10, n)
  int32_t *count, *flags;       // outputs of the first lag of the launch
  double *f, *xi, *mu;
  float *phi;
};
ModalStrides modal_strides(const ModalSizes &s, int l, int ldu);
// X_n for every order (form_x) and their Hessenberg forms into lag slot `lag`
// (uses rinv, w, xbuf, hbuf, vref, taus).
hipError_t launch_modal_prep(const ModalArgs &a, int lag, hipStream_t st);
// U[0:l, :k] (U: row-major, ld k) transposed into dst (k rows of l entries),
// the layout the mode-shape products of the eigen-analysis read.
hipError_t launch_mode_head(const double *u, int k, int l, double *dst, hipStream_t st);
// QR iterations, poles and sorting of all n_lags lags in one launch; outputs
// of lag g at the output pointers plus g times the per-lag layout sizes.
hipError_t launch_modal_eig(const ModalArgs &a, hipStream_t st);

// ---- stability analysis (stability.hip)
struct StabilityArgs {
  int n_lags, n_orders, nmin, step, pole_cap, l;
  const int32_t *count;
  const double *f, *xi;
  const float *phi;
  double xi_max, mpc_min, mpd_max, alpha_f, alpha_xi, alpha_mac;
  double *mpc, *mpd;
  uint8_t *hc;                  // workspace: hard-criteria verdict per slot
  uint8_t *flags;
};
hipError_t launch_stability(const StabilityArgs &a, hipStream_t st);
// Static device scratch of the allocation-free stability entry point:
// capacity in pole slots, and its device address on `device` (which must be
// current; looked up with hipGetSymbolAddress once per device).
size_t noalloc_stability_slots();
hipError_t noalloc_scratch(int device, uint8_t **ptr);

}  // namespace ssi
