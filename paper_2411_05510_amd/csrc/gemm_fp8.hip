// FP8 range-finder products: C = A B^T with A (M x K) and B (N x K) both
// block-scaled FP8 E4M3 along the contraction index (32 elements per E8M0
// power-of-two scale), on v_mfma_scale_f32_16x16x128_f8f6f4 with FP32
// accumulation; the K slices' FP32 partial sums are added in FP64.
//
// Quantization (the same reading as the checker's): the FP32 value (FP64
// operands are rounded to FP32 first) is divided by the block scale 2^(E - 7),
// E = floor(log2(max |v|)) over the block, so the block maximum lands in
// [128, 256) and nothing saturates (an all-zero block takes 2^0); the quotient
// is rounded to the nearest E4M3 value, ties to the even mantissa.  E4M3 is
// the OCP format (bias 7, 3 mantissa bits, largest finite 448, subnormals
// m 2^-9), the matrix instruction's FP8 input on this target.
//
// Quantized operand: rows of kp bytes (kp a multiple of 128, zero past the
// true length) and kp / 32 scale bytes per row.  T enters twice, quantized
// along its rows (for T X) and along its columns (for T^T X), once per
// randomized SVD; X (FP64) is quantized along its columns before each
// product.
//
// Operand layout of the 16 x 16 x 128 instruction (measured): lane l serves
// row l % 16 of its 16-row tile; its 32 bytes hold k = 16 g .. 16 g + 15 and
// k = 64 + 16 g .. 64 + 16 g + 15 of the 128-deep step (g = l / 16), and its
// scale byte is the scale of the 32-element block k = 32 g .. 32 g + 31.
#include <algorithm>

#include "common.h"
#include "kernels.h"

namespace {

constexpr int fBM = 128, fBN = 224, fKS = 128;   // workgroup tile, K step
constexpr int kBlk = 32;                         // elements per scale

typedef int i32x8 __attribute__((ext_vector_type(8)));
typedef float f32x4v __attribute__((ext_vector_type(4)));

// E4M3 code of y, |y| < 256 (a scaled element), nearest value, ties to even.
SSI_DEV uint32_t e4m3_code(float y) {
  const uint32_t sign = (__float_as_uint(y) >> 31) << 7;
  const float a = fabsf(y);
  uint32_t code;
  if (a < 0.015625f) {                 // below 2^-6: the subnormal grid m 2^-9
    code = (uint32_t)rintf(a * 512.0f); // exact product, round to nearest even
  } else {
    uint32_t b = __float_as_uint(a);
    b += 0x7FFFFu + ((b >> 20) & 1u); // keep 3 mantissa bits, ties to even
    const int e = (int)(b >> 23) - 127;
    code = ((uint32_t)(e + 7) << 3) | ((b >> 20) & 7u);
  }
  code = min(code, 0x7Eu);
  return code == 0u ? 0u : (code | sign);
}

// Scale exponent of a block from its largest magnitude.
SSI_DEV int block_exp(float amax) {
  if (!(amax > 0.0f)) return 0;
  int x;
  (void)frexpf(amax, &x);              // amax = f 2^x, f in [0.5, 1)
  return max(x - 1 - 7, -127);
}

// Quantizes 32 values (in v) with their block scale; writes 32 codes and the
// scale byte.
SSI_DEV void quant_block(const float (&v)[kBlk], uint8_t *__restrict__ q, uint8_t *__restrict__ s) {
  float amax = 0.0f;
#pragma unroll
  for (int i = 0; i < kBlk; ++i) amax = fmaxf(amax, fabsf(v[i]));
  const int e = block_exp(amax);
  uint32_t w[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    uint32_t c = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) c |= e4m3_code(ldexpf(v[4 * i + j], -e)) << (8 * j);
    w[i] = c;
  }
  *reinterpret_cast<uint4 *>(q) = make_uint4(w[0], w[1], w[2], w[3]);
  *reinterpret_cast<uint4 *>(q + 16) = make_uint4(w[4], w[5], w[6], w[7]);
  *s = (uint8_t)(e + 127);
}

}  // namespace

// Row quantization: q[r][k] from a[r][k] (k < cols, zero up to kp).  Eight
// lanes share a 32-element block, four elements each (one 16-byte load when
// rows are 16-byte aligned, VEC), so a wave reads 1 KiB of a row at once and
// writes 256 contiguous code bytes; the block maximum is a maximum over the
// eight lanes.  Lanes past the last block work on block 0 and store nothing.
template <bool VEC>
__global__ void __launch_bounds__(256)
quant_rows_f32(const float *__restrict__ a, int64_t lda, int rows, int cols, int kp,
               uint8_t *__restrict__ q, uint8_t *__restrict__ s) {
  const int nb = kp / kBlk;
  const int64_t blk = ((int64_t)blockIdx.x * 256 + threadIdx.x) >> 3;
  const int sub = threadIdx.x & 7;
  const bool live = blk < (int64_t)rows * nb;
  const int64_t bc = live ? blk : 0;
  const int r = (int)(bc / nb), b = (int)(bc - (int64_t)r * nb);
  const float *src = a + (int64_t)r * lda;
  const int k0 = b * kBlk + 4 * sub;
  float v[4];
  if (VEC && k0 + 3 < cols) {
    const f32x4v x = *reinterpret_cast<const f32x4v *>(src + k0);
    v[0] = x.x; v[1] = x.y; v[2] = x.z; v[3] = x.w;
  } else {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int k = k0 + i;
      const float x = src[min(k, cols - 1)];
      v[i] = k < cols ? x : 0.0f;
    }
  }
  float amax = fmaxf(fmaxf(fabsf(v[0]), fabsf(v[1])), fmaxf(fabsf(v[2]), fabsf(v[3])));
  amax = fmaxf(amax, __shfl_xor(amax, 1, 64));
  amax = fmaxf(amax, __shfl_xor(amax, 2, 64));
  amax = fmaxf(amax, __shfl_xor(amax, 4, 64));
  const int e = block_exp(amax);
  uint32_t c = 0;
#pragma unroll
  for (int j = 0; j < 4; ++j) c |= e4m3_code(ldexpf(v[j], -e)) << (8 * j);
  if (live) {
    *reinterpret_cast<uint32_t *>(q + (int64_t)r * kp + k0) = c;
    if (sub == 0) s[(int64_t)r * nb + b] = (uint8_t)(e + 127);
  }
}

// Column quantization (the transpose): q[j][k] from a[k][j] for j < cols and
// k < rows (zero past them, up to out_rows x kp).  A workgroup takes 64
// columns and 8 consecutive blocks of k, wave w block w: the lanes of a wave
// take consecutive j, so every one of the 32 loads is coalesced, and the
// eight waves write adjacent 32-byte pieces of each column's codes, 256
// contiguous bytes per column.
constexpr int kQcCols = 64, kQcBlocks = 8;
template <typename T>
__global__ void __launch_bounds__(64 * kQcBlocks)
quant_cols(const T *__restrict__ a, int64_t lda, int rows, int cols, int kp, int out_rows,
           uint8_t *__restrict__ q, uint8_t *__restrict__ s) {
  const int nb = kp / kBlk;
  const int njt = (out_rows + kQcCols - 1) / kQcCols;
  const int jt = blockIdx.x % njt, bg = blockIdx.x / njt;
  const int j = jt * kQcCols + (threadIdx.x & (kQcCols - 1));
  const int b = bg * kQcBlocks + (threadIdx.x >> 6);
  if (j >= out_rows || b >= nb) return;
  const int jc = min(j, cols - 1);
  float v[kBlk];
#pragma unroll
  for (int i = 0; i < kBlk; ++i) {
    const int k = b * kBlk + i;
    const float x = (float)a[(int64_t)min(k, rows - 1) * lda + jc];
    v[i] = (k < rows && j < cols) ? x : 0.0f;
  }
  quant_block(v, q + (int64_t)j * kp + b * kBlk, s + (int64_t)j * nb + b);
}

// C_part[split][i][j] = sum_{k in split} A[i][k] B[j][k] (dequantized), FP32.
// 8 waves (4 x 2), each 32 x 112 (2 x 7 tiles of 16 x 16), on a 128 x 224
// tile.  Each 128-deep K step of A (128 rows) and B (224 rows), codes and
// scales, is staged in LDS by the whole workgroup (rows padded to 144 bytes,
// so the 16 rows a fragment read touches start in different banks), double
// buffered: the next step's global loads are in registers while the current
// step's products run, with one barrier per step.  Every global load is
// issued at an index clamped into its array, so none sits under a branch.
namespace {
constexpr int fLS = fKS + 16;                    // LDS row stride (bytes)
constexpr int fAT = fBM * fLS, fBT = fBN * fLS;  // one buffer of A / B codes
constexpr int kFThreads = 512;
// codes, one scale word per thread (rows of A, then of B, then unused), and a
// 16-byte dummy slot per thread for the B chunks past the tile
constexpr int fBuf = fAT + fBT + 4 * kFThreads + 16 * kFThreads;
static_assert(fBM * fKS / 16 == 2 * kFThreads, "two A chunks per thread");
static_assert(fBN * fKS / 16 <= 4 * kFThreads, "at most four B chunks per thread");
}  // namespace

__global__ void __launch_bounds__(kFThreads)
gemm_fp8_mfma(const uint8_t *__restrict__ qa, const uint8_t *__restrict__ sa,
              const uint8_t *__restrict__ qb, const uint8_t *__restrict__ sb, int kp, int M,
              int N, int n_pad, float *__restrict__ C, int64_t ldc, int64_t split_stride,
              int k_per_split, int gm, int splits) {
  extern __shared__ __align__(16) uint8_t lds8[];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wr = wave & 3, wc = wave >> 2;
  const int split = blockIdx.x % splits, rest = blockIdx.x / splits;
  const int m0 = (rest % gm) * fBM, n0 = (rest / gm) * fBN;
  const int kb = split * k_per_split, ke = min(kp, kb + k_per_split);
  const int steps = (ke - kb) / fKS;
  const int r = lane & 15, g = lane >> 4;
  const int nb = kp / kBlk;

  // global chunks of this thread: A rows ar[h] (h < 2), B rows br[h] (h < 4)
  const uint8_t *ga[2], *gb[4];
  int la[2], lb[4];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int idx = tid + kFThreads * h, row = idx >> 3, ch = idx & 7;
    ga[h] = qa + (int64_t)min(m0 + row, M - 1) * kp + 16 * ch;
    la[h] = row * fLS + 16 * ch;
  }
#pragma unroll
  for (int h = 0; h < 4; ++h) {
    const int idx = tid + kFThreads * h;
    const bool ok = idx < fBN * fKS / 16;
    const int row = ok ? idx >> 3 : 0, ch = idx & 7;
    gb[h] = qb + (int64_t)min(n0 + row, n_pad - 1) * kp + 16 * ch;
    // chunks past the tile land in this thread's dummy slot: no store branch
    lb[h] = ok ? fAT + row * fLS + 16 * ch : fAT + fBT + 4 * kFThreads + 16 * tid;
  }
  // scale words (the 4 blocks of a step): A rows for tid < 128, B rows for
  // 128 <= tid < 352; the other threads load a valid word and store it unused
  const int srow = tid < fBM ? tid : tid - fBM;
  const uint8_t *gs = tid < fBM ? sa + (int64_t)min(m0 + srow, M - 1) * nb
                                : sb + (int64_t)min(n0 + min(srow, fBN - 1), n_pad - 1) * nb;

  // the next step's chunks (plain registers: arrays captured by a lambda
  // end up in scratch memory)
  uint4 ra0, ra1, rb0, rb1, rb2, rb3;
  uint32_t rs = 0;
#define SSI_FP8_GLOAD(k0)                                                       \
  do {                                                                          \
    ra0 = *reinterpret_cast<const uint4 *>(ga[0] + (k0));                       \
    ra1 = *reinterpret_cast<const uint4 *>(ga[1] + (k0));                       \
    rb0 = *reinterpret_cast<const uint4 *>(gb[0] + (k0));                       \
    rb1 = *reinterpret_cast<const uint4 *>(gb[1] + (k0));                       \
    rb2 = *reinterpret_cast<const uint4 *>(gb[2] + (k0));                       \
    rb3 = *reinterpret_cast<const uint4 *>(gb[3] + (k0));                       \
    rs = *reinterpret_cast<const uint32_t *>(gs + (k0) / kBlk);                 \
  } while (0)
#define SSI_FP8_LSTORE(buf)                                                     \
  do {                                                                          \
    *reinterpret_cast<uint4 *>((buf) + la[0]) = ra0;                            \
    *reinterpret_cast<uint4 *>((buf) + la[1]) = ra1;                            \
    *reinterpret_cast<uint4 *>((buf) + lb[0]) = rb0;                            \
    *reinterpret_cast<uint4 *>((buf) + lb[1]) = rb1;                            \
    *reinterpret_cast<uint4 *>((buf) + lb[2]) = rb2;                            \
    *reinterpret_cast<uint4 *>((buf) + lb[3]) = rb3;                            \
    reinterpret_cast<uint32_t *>((buf) + fAT + fBT)[tid] = rs;                  \
  } while (0)

  f32x4v acc[2][7];
#pragma unroll
  for (int rt = 0; rt < 2; ++rt)
#pragma unroll
    for (int ct = 0; ct < 7; ++ct) acc[rt][ct] = f32x4v{0.f, 0.f, 0.f, 0.f};

  auto frag = [](const uint8_t *p) {
    const uint4 lo = *reinterpret_cast<const uint4 *>(p);
    const uint4 hi = *reinterpret_cast<const uint4 *>(p + 64);
    i32x8 f;
    f[0] = (int)lo.x; f[1] = (int)lo.y; f[2] = (int)lo.z; f[3] = (int)lo.w;
    f[4] = (int)hi.x; f[5] = (int)hi.y; f[6] = (int)hi.z; f[7] = (int)hi.w;
    return f;
  };
  const int klast = ke - fKS;                    // a valid step start
  if (steps > 0) {
    SSI_FP8_GLOAD(kb);
    SSI_FP8_LSTORE(lds8);
  }
  __syncthreads();
  for (int s = 0; s < steps; ++s) {
    const uint8_t *buf = lds8 + (s & 1) * fBuf;
    SSI_FP8_GLOAD(min(kb + (s + 1) * fKS, klast));   // the next step, in flight
    const uint8_t *As = buf, *Bs = buf + fAT;
    const uint32_t *Ss = reinterpret_cast<const uint32_t *>(buf + fAT + fBT);
    i32x8 fa[2], fb[7];
    int sa_[2], sb_[7];
#pragma unroll
    for (int rt = 0; rt < 2; ++rt) {
      const int row = wr * 32 + rt * 16 + r;
      fa[rt] = frag(As + row * fLS + 16 * g);
      sa_[rt] = (int)((Ss[row] >> (8 * g)) & 0xFFu);
    }
#pragma unroll
    for (int ct = 0; ct < 7; ++ct) {
      const int row = wc * 112 + ct * 16 + r;
      fb[ct] = frag(Bs + row * fLS + 16 * g);
      sb_[ct] = (int)((Ss[fBM + row] >> (8 * g)) & 0xFFu);
    }
#pragma unroll
    for (int ct = 0; ct < 7; ++ct)
#pragma unroll
      for (int rt = 0; rt < 2; ++rt)
        acc[rt][ct] = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(
            fa[rt], fb[ct], acc[rt][ct], 0, 0, 0, sa_[rt], 0, sb_[ct]);
    // the other buffer was last read before the previous barrier
    SSI_FP8_LSTORE(lds8 + ((s + 1) & 1) * fBuf);
    __syncthreads();
  }
#undef SSI_FP8_GLOAD
#undef SSI_FP8_LSTORE

  // D layout of 16x16 MFMA: lane holds rows 4 (lane / 16) + q, column lane % 16.
  float *dst = C + (int64_t)split * split_stride;
#pragma unroll
  for (int rt = 0; rt < 2; ++rt)
#pragma unroll
    for (int ct = 0; ct < 7; ++ct) {
      const int col = n0 + wc * 112 + ct * 16 + r;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int row = m0 + wr * 32 + rt * 16 + 4 * g + q;
        if (row < M && col < N) dst[(int64_t)row * ldc + col] = acc[rt][ct][q];
      }
    }
}

namespace ssi {

Fp8Plan plan_gemm_fp8(int M, int N, int K, int num_cus, int force_splits) {
  Fp8Plan p{};
  p.kp = ceil_div(K, fKS) * fKS;
  p.gm = ceil_div(M, fBM);
  p.gn = ceil_div(N, fBN);
  p.n_pad = p.gn * fBN;
  // one workgroup per CU; fill about two rounds, at least 4 K steps a slice
  const int64_t tiles = (int64_t)p.gm * p.gn;
  const int64_t steps = p.kp / fKS;
  int64_t splits = ceil_div<int64_t>((int64_t)num_cus * 2, tiles);
  splits = std::max<int64_t>(1, std::min<int64_t>({splits, 16, ceil_div<int64_t>(steps, 4)}));
  if (force_splits > 0) splits = std::min<int64_t>(force_splits, steps);
  const int64_t sps = ceil_div<int64_t>(steps, splits);          // steps per slice
  p.k_per_split = (int)(sps * fKS);
  p.splits = (int)ceil_div<int64_t>(steps, sps);
  p.ldc = N;
  p.split_stride = (int64_t)M * N;
  return p;
}

hipError_t launch_quant_rows_f32(const float *a, int64_t lda, int rows, int cols, int kp,
                                 uint8_t *q, uint8_t *s, hipStream_t st) {
  const int64_t lanes = (int64_t)rows * (kp / kBlk) * 8;
  const dim3 grid((unsigned)ceil_div<int64_t>(lanes, 256));
  if (lda % 4 == 0 && (uintptr_t)a % 16 == 0)
    hipLaunchKernelGGL(quant_rows_f32<true>, grid, dim3(256), 0, st, a, lda, rows, cols, kp, q, s);
  else
    hipLaunchKernelGGL(quant_rows_f32<false>, grid, dim3(256), 0, st, a, lda, rows, cols, kp, q,
                       s);
  return hipGetLastError();
}

namespace {
dim3 quant_cols_grid(int out_rows, int kp) {
  const int64_t njt = ceil_div(out_rows, kQcCols), nbg = ceil_div(kp / kBlk, kQcBlocks);
  return dim3((unsigned)(njt * nbg));
}
}  // namespace

hipError_t launch_quant_cols_f32(const float *a, int64_t lda, int rows, int cols, int kp,
                                 int out_rows, uint8_t *q, uint8_t *s, hipStream_t st) {
  hipLaunchKernelGGL(quant_cols<float>, quant_cols_grid(out_rows, kp), dim3(64 * kQcBlocks), 0,
                     st, a, lda, rows, cols, kp, out_rows, q, s);
  return hipGetLastError();
}

hipError_t launch_quant_cols_f64(const double *a, int64_t lda, int rows, int cols, int kp,
                                 int out_rows, uint8_t *q, uint8_t *s, hipStream_t st) {
  hipLaunchKernelGGL(quant_cols<double>, quant_cols_grid(out_rows, kp), dim3(64 * kQcBlocks), 0,
                     st, a, lda, rows, cols, kp, out_rows, q, s);
  return hipGetLastError();
}

hipError_t launch_gemm_fp8(const Fp8Plan &p, const uint8_t *qa, const uint8_t *sa,
                           const uint8_t *qb, const uint8_t *sb, int M, int N, float *part,
                           hipStream_t st) {
  const dim3 grid((unsigned)((int64_t)p.gm * p.gn * p.splits));
  const size_t lds = 2 * (size_t)fBuf;
  hipError_t e = hipFuncSetAttribute((const void *)gemm_fp8_mfma,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(gemm_fp8_mfma, grid, dim3(kFThreads), lds, st, qa, sa, qb, sb, p.kp, M, N,
                     p.n_pad, part, p.ldc, p.split_stride, p.k_per_split, p.gm, p.splits);
  return hipGetLastError();
}

}  // namespace ssi
