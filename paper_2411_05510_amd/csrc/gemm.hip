// Dense products of the randomized SVD and the modal stage.
//
// gemm_f32: C = op(A) B with FP32 operands on v_mfma_f32_16x16x4f32 (the
//   sketch, power-iteration and projection products Y = T X, Z = T^T X).
//   Tile 64 x 224 x 32: the thin side (ell = k + p columns) fits one or two
//   column blocks, the long side is split across workgroups and along K
//   (split-K); each workgroup folds its fp32 accumulators into fp64 every 256
//   k and writes fp64 partial sums, added by reduce_splits in a fixed order.
//   LDS holds both tiles k-contiguous so every lane fetches four consecutive
//   k of its row with one 16-byte read and feeds four MFMA steps from it.
// gemm_f64: the same with FP64 operands on v_mfma_f64_16x16x4f64 (Gram
//   matrices, basis updates, small triangular products).  Tile 64 x 64 x 16.
#include "common.h"
#include "kernels.h"

namespace {

constexpr int kBM = 64, kBN = 224, kKT = 32, kLS = kKT + 4;   // fp32 tiles
constexpr int kFlush = 8;                                    // K-tiles per fp64 fold

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

}  // namespace

// C_part[split][i][j] = sum_{k in split} op(A)[i][k] B[k][j]
//   TA = false: A is M x K (lda);  TA = true: A is K x M (lda), op(A) = A^T.
//   B is K x N (ldb).
template <bool TA, bool VEC>
__global__ void __launch_bounds__(256, 2)
gemm_f32_mfma(const float *__restrict__ A, int64_t lda, const float *__restrict__ B,
              int64_t ldb, double *__restrict__ C, int64_t ldc, int64_t split_stride, int M,
              int N, int K, int k_per_split) {
  __shared__ __attribute__((aligned(16))) float As[kBM * kLS];
  __shared__ __attribute__((aligned(16))) float Bs[kBN * kLS];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave & 1, wc = wave >> 1;
  const int m0 = blockIdx.x * kBM, n0 = blockIdx.y * kBN;
  const int kb = blockIdx.z * k_per_split;
  const int ke = min(K, kb + k_per_split);

  f32x4 acc[2][7];
  double accd[2][7][4];
#pragma unroll
  for (int rt = 0; rt < 2; ++rt)
#pragma unroll
    for (int ct = 0; ct < 7; ++ct) {
      acc[rt][ct] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int q = 0; q < 4; ++q) accd[rt][ct][q] = 0.0;
    }
  bool colok[7];
#pragma unroll
  for (int ct = 0; ct < 7; ++ct) colok[ct] = n0 + wc * 112 + ct * 16 < N;

  int tiles = 0;
  for (int k0 = kb; k0 < ke; k0 += kKT) {
    __syncthreads();
    // ---- A tile -> As[i][k]
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int idx = tid + 256 * h;
      if (!TA) {
        const int r = idx >> 3, c4 = idx & 7;
        const float4 v = load4<VEC>(A, lda, m0 + r, M, k0 + 4 * c4, ke);
        *reinterpret_cast<float4 *>(&As[r * kLS + 4 * c4]) = v;
      } else {
        const int kr = idx >> 4, c4 = idx & 15;
        const float4 v = (k0 + kr < ke) ? load4<VEC>(A, lda, k0 + kr, ke, m0 + 4 * c4, M)
                                        : make_float4(0.f, 0.f, 0.f, 0.f);
        As[(4 * c4 + 0) * kLS + kr] = v.x;
        As[(4 * c4 + 1) * kLS + kr] = v.y;
        As[(4 * c4 + 2) * kLS + kr] = v.z;
        As[(4 * c4 + 3) * kLS + kr] = v.w;
      }
    }
    // ---- B tile -> Bs[j][k]
#pragma unroll
    for (int h = 0; h < 7; ++h) {
      const int idx = tid + 256 * h;
      const int kr = idx / 56, c4 = idx - kr * 56;
      const float4 v = (k0 + kr < ke) ? load4<VEC>(B, ldb, k0 + kr, ke, n0 + 4 * c4, N)
                                      : make_float4(0.f, 0.f, 0.f, 0.f);
      Bs[(4 * c4 + 0) * kLS + kr] = v.x;
      Bs[(4 * c4 + 1) * kLS + kr] = v.y;
      Bs[(4 * c4 + 2) * kLS + kr] = v.z;
      Bs[(4 * c4 + 3) * kLS + kr] = v.w;
    }
    __syncthreads();

#pragma unroll
    for (int g = 0; g < kKT / 16; ++g) {
      const int ko = g * 16 + 4 * (lane >> 4);
      float4 a4[2], b4[7];
#pragma unroll
      for (int rt = 0; rt < 2; ++rt)
        a4[rt] = *reinterpret_cast<const float4 *>(&As[(wr * 32 + rt * 16 + (lane & 15)) * kLS + ko]);
#pragma unroll
      for (int ct = 0; ct < 7; ++ct)
        b4[ct] = *reinterpret_cast<const float4 *>(&Bs[(wc * 112 + ct * 16 + (lane & 15)) * kLS + ko]);
#pragma unroll
      for (int t = 0; t < 4; ++t) {
#pragma unroll
        for (int ct = 0; ct < 7; ++ct) {
          if (!colok[ct]) continue;
          const float bv = t == 0 ? b4[ct].x : t == 1 ? b4[ct].y : t == 2 ? b4[ct].z : b4[ct].w;
#pragma unroll
          for (int rt = 0; rt < 2; ++rt) {
            const float av = t == 0 ? a4[rt].x : t == 1 ? a4[rt].y : t == 2 ? a4[rt].z : a4[rt].w;
            acc[rt][ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv, acc[rt][ct], 0, 0, 0);
          }
        }
      }
    }
    if (++tiles == kFlush || k0 + kKT >= ke) {
      tiles = 0;
#pragma unroll
      for (int rt = 0; rt < 2; ++rt)
#pragma unroll
        for (int ct = 0; ct < 7; ++ct) {
#pragma unroll
          for (int q = 0; q < 4; ++q) accd[rt][ct][q] += (double)acc[rt][ct][q];
          acc[rt][ct] = f32x4{0.f, 0.f, 0.f, 0.f};
        }
    }
  }

  double *dst = C + (int64_t)blockIdx.z * split_stride;
#pragma unroll
  for (int rt = 0; rt < 2; ++rt)
#pragma unroll
    for (int ct = 0; ct < 7; ++ct) {
      const int col = n0 + wc * 112 + ct * 16 + (lane & 15);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int row = m0 + wr * 32 + rt * 16 + 4 * (lane >> 4) + q;
        if (row < M && col < N) dst[(int64_t)row * ldc + col] = accd[rt][ct][q];
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

GemmPlan plan_gemm_f32(int M, int N, int K, int num_cus) {
  GemmPlan p{};
  p.gm = ceil_div(M, kBM);
  p.gn = ceil_div(N, kBN);
  const int64_t tiles = (int64_t)p.gm * p.gn;
  int64_t splits = ceil_div<int64_t>((int64_t)num_cus * 2, tiles);
  const int64_t max_splits = ceil_div<int64_t>(K, 256);
  splits = std::max<int64_t>(1, std::min(splits, max_splits));
  int64_t kps = ceil_div<int64_t>(K, splits);
  kps = ceil_div<int64_t>(kps, kKT) * kKT;
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

hipError_t launch_gemm_f32(const GemmPlan &p, bool trans_a, const float *A, int64_t lda,
                           const float *B, int64_t ldb, int M, int N, int K, double *part,
                           hipStream_t st) {
  dim3 grid(p.gm, p.gn, p.splits);
  const bool vec = (lda % 4 == 0) && (ldb % 4 == 0) && ((uintptr_t)A % 16 == 0) &&
                   ((uintptr_t)B % 16 == 0);
  if (trans_a) {
    if (vec)
      hipLaunchKernelGGL((gemm_f32_mfma<true, true>), grid, dim3(256), 0, st, A, lda, B, ldb,
                         part, p.ldc, p.split_stride, M, N, K, p.k_per_split);
    else
      hipLaunchKernelGGL((gemm_f32_mfma<true, false>), grid, dim3(256), 0, st, A, lda, B, ldb,
                         part, p.ldc, p.split_stride, M, N, K, p.k_per_split);
  } else {
    if (vec)
      hipLaunchKernelGGL((gemm_f32_mfma<false, true>), grid, dim3(256), 0, st, A, lda, B, ldb,
                         part, p.ldc, p.split_stride, M, N, K, p.k_per_split);
    else
      hipLaunchKernelGGL((gemm_f32_mfma<false, false>), grid, dim3(256), 0, st, A, lda, B, ldb,
                         part, p.ldc, p.split_stride, M, N, K, p.k_per_split);
  }
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
