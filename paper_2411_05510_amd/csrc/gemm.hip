// Dense products of the randomized SVD and the modal stage.
//
// gemm_tf64: C = op(T) X with T in FP32 (the Toeplitz matrix as stored) and X
//   in FP64, on v_mfma_f64_16x16x4f64 with FP64 accumulation: the sketch,
//   power-iteration and projection products Y = T X, Z = T^T X.  T is
//   converted exactly to FP64 in registers, so the only rounding is FP64
//   accumulation.  Tile 64 x 224 x 16: the thin side (ell = k + p columns)
//   fits one column block, the long side is split across workgroups and
//   along K.  The flat grid is decoded split-fastest, so with 8 splits the
//   workgroups of one K slice land on one XCD (dispatch is round-robin over
//   the 8 XCDs) and that XCD's L2 holds the slice of X they all read.
//   Partial sums (FP64) are added by reduce_splits in a fixed order.
// gemm_f64: FP64 operands on v_mfma_f64_16x16x4f64 (Gram matrices, basis
//   updates, small triangular products).  Tile 64 x 64 x 16.
#include "common.h"
#include "kernels.h"

namespace {

constexpr int tBM = 64, tBN = 224, tKT = 16;
constexpr int tLA = tKT + 4;    // FP32 A row stride in LDS (floats), A stored [i][k]
constexpr int tLB = tBN + 4;    // FP64 B row stride in LDS (doubles), B stored [k][j]

constexpr int dBM = 64, dBN = 64, dKT = 16, dLS = dKT + 2;    // fp64 tiles

// Guarded 4-float load of row `row` (< rows) starting at column c (< cols).
template <bool VEC>
SSI_DEV float4 load4(const float *__restrict__ p, int64_t ld, int64_t row, int64_t rows,
                     int64_t c, int64_t cols) {
  float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
  if (row >= rows) return v;
  const float *q = p + row * ld + c;
  if (VEC && c + 3 < cols) return *reinterpret_cast<const float4 *>(q);
  if (c < cols) v.x = q[0];
  if (c + 1 < cols) v.y = q[1];
  if (c + 2 < cols) v.z = q[2];
  if (c + 3 < cols) v.w = q[3];
  return v;
}

SSI_DEV float f4get(const float4 &v, int s) {
  return s == 0 ? v.x : s == 1 ? v.y : s == 2 ? v.z : v.w;
}

}  // namespace

// C_part[split][i][j] = sum_{k in split} op(A)[i][k] B[k][j]
//   TA = false: A is M x K (lda);  TA = true: A is K x M (lda), op(A) = A^T.
//   A FP32, B FP64 K x N (ldb).  VEC: lda % 4 == 0 and A 16-byte aligned;
//   BVEC: ldb even and B 16-byte aligned.
// Each K tile (16) is loaded into registers with all loads in flight at once
// (out-of-range rows and columns read a clamped in-range address and are
// zeroed by select), then written to LDS.  In MFMA step s of K sub-tile h the
// 16-lane group g of a wave supplies k = 16 h + 4 g + s.
template <bool TA, bool VEC, bool BVEC>
__global__ void __launch_bounds__(256, 2)
gemm_tf64_mfma(const float *__restrict__ A, int64_t lda, const double *__restrict__ B,
               int64_t ldb, double *__restrict__ C, int64_t ldc, int64_t split_stride, int M,
               int N, int K, int k_per_split, int gm, int splits) {
  __shared__ __attribute__((aligned(16))) float As[tBM * tLA];
  __shared__ __attribute__((aligned(16))) double Bs[tKT * tLB];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave & 1, wc = wave >> 1;
  const int split = blockIdx.x % splits;
  const int rest = blockIdx.x / splits;
  const int m0 = (rest % gm) * tBM, n0 = (rest / gm) * tBN;
  const int kb = split * k_per_split;
  const int ke = min(K, kb + k_per_split);

  f64x4 acc[2][7];
#pragma unroll
  for (int rt = 0; rt < 2; ++rt)
#pragma unroll
    for (int ct = 0; ct < 7; ++ct) acc[rt][ct] = f64x4{0.0, 0.0, 0.0, 0.0};
  bool colok[7];
#pragma unroll
  for (int ct = 0; ct < 7; ++ct) colok[ct] = n0 + wc * 112 + ct * 16 < N;

  for (int k0 = kb; k0 < ke; k0 += tKT) {
    // ---- A tile (64 x 16 FP32): one float4 per thread
    float4 ra[1];
#pragma unroll
    for (int h = 0; h < 1; ++h) {
      const int idx = tid + 256 * h;
      if (!TA) {
        const int r = idx >> 2, c4 = idx & 3;              // row, 4-column group of k
        const int gi = m0 + r, gk = k0 + 4 * c4;
        const float *p = A + (int64_t)min(gi, M - 1) * lda;
        float4 v;
        if (VEC && gk + 3 < ke) v = *reinterpret_cast<const float4 *>(p + gk);
        else v = load4<false>(p, 0, 0, 1, gk, ke);
        ra[h] = gi < M ? v : make_float4(0.f, 0.f, 0.f, 0.f);
      } else {
        const int kr = idx >> 4, c4 = idx & 15;            // k row, 4-column group of i
        const int gk = k0 + kr, gi = m0 + 4 * c4;
        const float *p = A + (int64_t)min(gk, ke - 1) * lda;
        float4 v;
        if (VEC && gi + 3 < M) v = *reinterpret_cast<const float4 *>(p + gi);
        else v = load4<false>(p, 0, 0, 1, gi, M);
        ra[h] = gk < ke ? v : make_float4(0.f, 0.f, 0.f, 0.f);
      }
    }
    // ---- B tile (16 x 224 FP64): seven double pairs per thread
    double2 rbv[7];
#pragma unroll
    for (int h = 0; h < 7; ++h) {
      const int idx = tid + 256 * h;
      const int kr = idx / 112, c2 = idx - kr * 112;
      const int gk = k0 + kr, gj = n0 + 2 * c2;
      const double *q = B + (int64_t)min(gk, ke - 1) * ldb;
      double2 v;
      if (BVEC && gj + 1 < N) {
        v = *reinterpret_cast<const double2 *>(q + gj);
      } else {
        v.x = q[min(gj, N - 1)];
        v.y = q[min(gj + 1, N - 1)];
        if (gj >= N) v.x = 0.0;
        if (gj + 1 >= N) v.y = 0.0;
      }
      rbv[h] = gk < ke ? v : make_double2(0.0, 0.0);
    }
    __syncthreads();                      // previous tile's reads are done
#pragma unroll
    for (int h = 0; h < 1; ++h) {
      const int idx = tid + 256 * h;
      if (!TA) {
        const int r = idx >> 2, c4 = idx & 3;
        *reinterpret_cast<float4 *>(&As[r * tLA + 4 * c4]) = ra[h];
      } else {
        const int kr = idx >> 4, c4 = idx & 15;
        As[(4 * c4 + 0) * tLA + kr] = ra[h].x;
        As[(4 * c4 + 1) * tLA + kr] = ra[h].y;
        As[(4 * c4 + 2) * tLA + kr] = ra[h].z;
        As[(4 * c4 + 3) * tLA + kr] = ra[h].w;
      }
    }
#pragma unroll
    for (int h = 0; h < 7; ++h) {
      const int idx = tid + 256 * h;
      const int kr = idx / 112, c2 = idx - kr * 112;
      *reinterpret_cast<double2 *>(&Bs[kr * tLB + 2 * c2]) = rbv[h];
    }
    __syncthreads();

#pragma unroll
    for (int hk = 0; hk < tKT / 16; ++hk) {
      const int ko = 16 * hk + 4 * (lane >> 4);
      float4 a4[2];
#pragma unroll
      for (int rt = 0; rt < 2; ++rt)
        a4[rt] = *reinterpret_cast<const float4 *>(
            &As[(wr * 32 + rt * 16 + (lane & 15)) * tLA + ko]);
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        double bv[7];
#pragma unroll
        for (int ct = 0; ct < 7; ++ct) bv[ct] = Bs[(ko + s) * tLB + wc * 112 + ct * 16 + (lane & 15)];
#pragma unroll
        for (int ct = 0; ct < 7; ++ct) {
          if (!colok[ct]) continue;
#pragma unroll
          for (int rt = 0; rt < 2; ++rt)
            acc[rt][ct] = __builtin_amdgcn_mfma_f64_16x16x4f64((double)f4get(a4[rt], s),
                                                               bv[ct], acc[rt][ct], 0, 0, 0);
        }
      }
    }
  }

  // D layout of 16x16x4f64: lane holds rows (lane/16) + 4 q, column lane%16.
  double *dst = C + (int64_t)split * split_stride;
#pragma unroll
  for (int rt = 0; rt < 2; ++rt)
#pragma unroll
    for (int ct = 0; ct < 7; ++ct) {
      const int col = n0 + wc * 112 + ct * 16 + (lane & 15);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int row = m0 + wr * 32 + rt * 16 + (lane >> 4) + 4 * q;
        if (row < M && col < N) dst[(int64_t)row * ldc + col] = acc[rt][ct][q];
      }
    }
}

// C_part[split][i][j] = sum_{k in split} op(A)[i][k] B[k][j], FP64 operands.
template <bool TA>
__global__ void __launch_bounds__(256)
gemm_f64_mfma(const double *__restrict__ A, int64_t lda, const double *__restrict__ B,
              int64_t ldb, double *__restrict__ C, int64_t ldc, int64_t split_stride, int M,
              int N, int K, int k_per_split) {
  __shared__ double As[dBM * dLS];
  __shared__ double Bs[dBN * dLS];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave & 1, wc = wave >> 1;
  const int m0 = blockIdx.x * dBM, n0 = blockIdx.y * dBN;
  const int kb = blockIdx.z * k_per_split;
  const int ke = min(K, kb + k_per_split);

  f64x4 acc[2][2];
#pragma unroll
  for (int rt = 0; rt < 2; ++rt)
#pragma unroll
    for (int ct = 0; ct < 2; ++ct) acc[rt][ct] = f64x4{0.0, 0.0, 0.0, 0.0};

  for (int k0 = kb; k0 < ke; k0 += dKT) {
    __syncthreads();
#pragma unroll
    for (int h = 0; h < 4; ++h) {
      const int idx = tid + 256 * h;          // 1024 elements per tile
      if (!TA) {
        const int r = idx >> 4, kr = idx & 15;
        const int gi = m0 + r, gk = k0 + kr;
        As[r * dLS + kr] = (gi < M && gk < ke) ? A[(int64_t)gi * lda + gk] : 0.0;
      } else {
        const int kr = idx >> 6, c = idx & 63;
        const int gi = m0 + c, gk = k0 + kr;
        As[c * dLS + kr] = (gi < M && gk < ke) ? A[(int64_t)gk * lda + gi] : 0.0;
      }
      {
        const int kr = idx >> 6, c = idx & 63;
        const int gj = n0 + c, gk = k0 + kr;
        Bs[c * dLS + kr] = (gj < N && gk < ke) ? B[(int64_t)gk * ldb + gj] : 0.0;
      }
    }
    __syncthreads();
#pragma unroll
    for (int s = 0; s < dKT / 4; ++s) {
      const int ko = 4 * s + (lane >> 4);
      double av[2], bv[2];
#pragma unroll
      for (int rt = 0; rt < 2; ++rt) av[rt] = As[(wr * 32 + rt * 16 + (lane & 15)) * dLS + ko];
#pragma unroll
      for (int ct = 0; ct < 2; ++ct) bv[ct] = Bs[(wc * 32 + ct * 16 + (lane & 15)) * dLS + ko];
#pragma unroll
      for (int rt = 0; rt < 2; ++rt)
#pragma unroll
        for (int ct = 0; ct < 2; ++ct)
          acc[rt][ct] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[rt], bv[ct], acc[rt][ct], 0, 0, 0);
    }
  }

  // D layout of 16x16x4f64: lane holds rows (lane/16) + 4 q, column lane%16.
  double *dst = C + (int64_t)blockIdx.z * split_stride;
#pragma unroll
  for (int rt = 0; rt < 2; ++rt)
#pragma unroll
    for (int ct = 0; ct < 2; ++ct) {
      const int col = n0 + wc * 32 + ct * 16 + (lane & 15);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int row = m0 + wr * 32 + rt * 16 + (lane >> 4) + 4 * q;
        if (row < M && col < N) dst[(int64_t)row * ldc + col] = acc[rt][ct][q];
      }
    }
}

// out[i][j] = scale * sum_s part[s][i][j]; optional FP32 copy.
__global__ void __launch_bounds__(256)
reduce_splits(const double *__restrict__ part, int splits, int64_t split_stride, int64_t ldp,
              int M, int N, double scale, double *__restrict__ out, int64_t ldo,
              float *__restrict__ out32, int64_t ld32) {
  const int64_t total = (int64_t)M * N;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = idx / N, j = idx - i * N;
    double s = 0.0;
    for (int sp = 0; sp < splits; ++sp) s += part[sp * split_stride + i * ldp + j];
    s *= scale;
    if (out) out[i * ldo + j] = s;
    if (out32) out32[i * ld32 + j] = (float)s;
  }
}

// out32[i][j] = (float) in[i][j]
__global__ void __launch_bounds__(256)
convert_f64_f32(const double *__restrict__ in, int64_t ldi, int M, int N,
                float *__restrict__ out, int64_t ldo) {
  const int64_t total = (int64_t)M * N;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = idx / N, j = idx - i * N;
    out[i * ldo + j] = (float)in[i * ldi + j];
  }
}

// out[i][j] = (double) in[i][j]
__global__ void __launch_bounds__(256)
convert_f32_f64(const float *__restrict__ in, int64_t ldi, int M, int N,
                double *__restrict__ out, int64_t ldo) {
  const int64_t total = (int64_t)M * N;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = idx / N, j = idx - i * N;
    out[i * ldo + j] = (double)in[i * ldi + j];
  }
}

// sigma[i] = sqrt(max(evals[i], 0)), i < k
__global__ void sqrt_clamp_kernel(const double *__restrict__ ev, int k, double *__restrict__ sigma) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < k) sigma[i] = sqrt(fmax(ev[i], 0.0));
}

// out[j][i] = (double) in[i][j]  (FP32 -> FP64 transpose, m x n -> n x m)
__global__ void __launch_bounds__(256)
transpose_f32_f64(const float *__restrict__ in, int64_t ldi, int M, int N,
                  double *__restrict__ out, int64_t ldo) {
  const int64_t total = (int64_t)M * N;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t j = idx / M, i = idx - j * M;
    out[j * ldo + i] = (double)in[i * ldi + j];
  }
}

namespace ssi {

namespace {
int grid_cap(int64_t work) {
  int64_t b = ceil_div<int64_t>(work, 256);
  if (b > 16384) b = 16384;
  if (b < 1) b = 1;
  return (int)b;
}
}  // namespace

GemmPlan plan_gemm_tf64(int M, int N, int K, int num_cus, int force_splits) {
  GemmPlan p{};
  p.gm = ceil_div(M, tBM);
  p.gn = ceil_div(N, tBN);
  // Eight K slices (one per XCD) once K is long enough for each to keep its
  // workgroups busy; fewer for short K.
  const int64_t tiles = (int64_t)p.gm * p.gn;
  int64_t splits = 8;
  if (tiles * 8 < (int64_t)num_cus) splits = ceil_div<int64_t>((int64_t)num_cus * 2, tiles);
  const int64_t max_splits = ceil_div<int64_t>(K, 512);
  splits = std::max<int64_t>(1, std::min(splits, max_splits));
  if (force_splits > 0) splits = std::min<int64_t>(force_splits, ceil_div<int64_t>(K, tKT));
  int64_t kps = ceil_div<int64_t>(K, splits);
  kps = ceil_div<int64_t>(kps, tKT) * tKT;
  p.k_per_split = (int)kps;
  p.splits = (int)ceil_div<int64_t>(K, kps);
  p.ldc = N;
  p.split_stride = (int64_t)M * N;
  return p;
}

GemmPlan plan_gemm_f64(int M, int N, int K, int num_cus) {
  GemmPlan p{};
  p.gm = ceil_div(M, dBM);
  p.gn = ceil_div(N, dBN);
  const int64_t tiles = (int64_t)p.gm * p.gn;
  int64_t splits = ceil_div<int64_t>((int64_t)num_cus * 2, tiles);
  const int64_t max_splits = ceil_div<int64_t>(K, 128);
  splits = std::max<int64_t>(1, std::min(splits, max_splits));
  int64_t kps = ceil_div<int64_t>(K, splits);
  kps = ceil_div<int64_t>(kps, dKT) * dKT;
  p.k_per_split = (int)kps;
  p.splits = (int)ceil_div<int64_t>(K, kps);
  p.ldc = N;
  p.split_stride = (int64_t)M * N;
  return p;
}

template <bool TA>
static void launch_tf64_variant(const GemmPlan &p, bool vec, bool bvec, const float *A,
                                int64_t lda, const double *B, int64_t ldb, int M, int N, int K,
                                double *part, hipStream_t st) {
  const dim3 grid((unsigned)((int64_t)p.gm * p.gn * p.splits));
#define SSI_TF64(V, BV)                                                                      \
  hipLaunchKernelGGL((gemm_tf64_mfma<TA, V, BV>), grid, dim3(256), 0, st, A, lda, B, ldb, part, \
                     p.ldc, p.split_stride, M, N, K, p.k_per_split, p.gm, p.splits)
  if (vec && bvec) SSI_TF64(true, true);
  else if (vec) SSI_TF64(true, false);
  else if (bvec) SSI_TF64(false, true);
  else SSI_TF64(false, false);
#undef SSI_TF64
}

hipError_t launch_gemm_tf64(const GemmPlan &p, bool trans_a, const float *A, int64_t lda,
                            const double *B, int64_t ldb, int M, int N, int K, double *part,
                            hipStream_t st) {
  const bool vec = (lda % 4 == 0) && ((uintptr_t)A % 16 == 0);
  const bool bvec = (ldb % 2 == 0) && ((uintptr_t)B % 16 == 0);
  if (trans_a) launch_tf64_variant<true>(p, vec, bvec, A, lda, B, ldb, M, N, K, part, st);
  else launch_tf64_variant<false>(p, vec, bvec, A, lda, B, ldb, M, N, K, part, st);
  return hipGetLastError();
}

hipError_t launch_gemm_f64(const GemmPlan &p, bool trans_a, const double *A, int64_t lda,
                           const double *B, int64_t ldb, int M, int N, int K, double *part,
                           hipStream_t st) {
  dim3 grid(p.gm, p.gn, p.splits);
  if (trans_a)
    hipLaunchKernelGGL((gemm_f64_mfma<true>), grid, dim3(256), 0, st, A, lda, B, ldb, part,
                       p.ldc, p.split_stride, M, N, K, p.k_per_split);
  else
    hipLaunchKernelGGL((gemm_f64_mfma<false>), grid, dim3(256), 0, st, A, lda, B, ldb, part,
                       p.ldc, p.split_stride, M, N, K, p.k_per_split);
  return hipGetLastError();
}

hipError_t launch_reduce(const GemmPlan &p, const double *part, int M, int N, double scale,
                         double *out, int64_t ldo, float *out32, int64_t ld32, hipStream_t st) {
  hipLaunchKernelGGL(reduce_splits, dim3(grid_cap((int64_t)M * N)), dim3(256), 0, st, part,
                     p.splits, p.split_stride, p.ldc, M, N, scale, out, ldo, out32, ld32);
  return hipGetLastError();
}

hipError_t launch_convert(const double *in, int64_t ldi, int M, int N, float *out, int64_t ldo,
                          hipStream_t st) {
  hipLaunchKernelGGL(convert_f64_f32, dim3(grid_cap((int64_t)M * N)), dim3(256), 0, st, in,
                     ldi, M, N, out, ldo);
  return hipGetLastError();
}

hipError_t launch_convert_f32_f64(const float *in, int64_t ldi, int M, int N, double *out,
                                  int64_t ldo, hipStream_t st) {
  hipLaunchKernelGGL(convert_f32_f64, dim3(grid_cap((int64_t)M * N)), dim3(256), 0, st, in,
                     ldi, M, N, out, ldo);
  return hipGetLastError();
}

hipError_t launch_sqrt_clamp(const double *ev, int k, double *sigma, hipStream_t st) {
  hipLaunchKernelGGL(sqrt_clamp_kernel, dim3(ceil_div(k, 256)), dim3(256), 0, st, ev, k, sigma);
  return hipGetLastError();
}

hipError_t launch_transpose_f32_f64(const float *in, int64_t ldi, int M, int N, double *out,
                                    int64_t ldo, hipStream_t st) {
  hipLaunchKernelGGL(transpose_f32_f64, dim3(grid_cap((int64_t)M * N)), dim3(256), 0, st, in,
                     ldi, M, N, out, ldo);
  return hipGetLastError();
}

}  // namespace ssi
