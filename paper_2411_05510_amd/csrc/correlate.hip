// Output correlations R_j = (1/N) sum_{k=0}^{N-1-j} y_{k+j} y_k^T, j = 1..L
// (Section 2.1 of the paper; estimator as stated in the library header).
//
// All L lags form one sliding-window contraction over time:
//   C[(a, j)][b] = sum_s y[a][s + j] * y[b][s],  rows (a, j) flattened as
//   r = a L + (j - 1), columns b, contraction over the sample index s.
// Every row of the A operand is a shifted window of one channel, so one LDS
// tile of y (a few channels plus an L-sample halo) feeds all lags, and the
// flattened rows need no padding to a lag multiple.  The B operand is a plain
// tile of y.  Products run on v_mfma_f32_16x16x4f32; fp32 accumulators are
// folded into fp64 every FLUSH_TILES tiles to bound the rounding growth over
// long records, and the time axis is split across workgroups (split-K) whose
// fp64 partial sums are added by a second kernel in a fixed order.
#include "common.h"
#include "kernels.h"

namespace {

constexpr int kThreads = 512;        // 8 waves: 4 row blocks x 2 column halves
constexpr int kRowsPerWave = 64;     // 4 MFMA row tiles of 16
constexpr int kColsPerWave = 32;     // 2 MFMA column tiles of 16
constexpr int kRowsPerWG = 4 * kRowsPerWave;
constexpr int kColsPerWG = 2 * kColsPerWave;
constexpr int kST = 128;             // samples per LDS tile
constexpr int kSB = kST + 4;         // LDS row stride of the B tile (floats): rows stay
                                     // 16-byte aligned and the 16 rows a fragment
                                     // read touches start in distinct banks
constexpr int kFlushTiles = 2;       // fold fp32 into fp64 every 256 samples

// Four consecutive samples s..s+3 of one channel row p, zero at and past lim.
template <bool VEC>
SSI_DEV float4 load4(const float *__restrict__ p, int64_t s, int64_t lim) {
  if (VEC && s + 3 < lim) return *reinterpret_cast<const float4 *>(p + s);
  float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
  if (s < lim) v.x = p[s];
  if (s + 1 < lim) v.y = p[s + 1];
  if (s + 2 < lim) v.z = p[s + 2];
  if (s + 3 < lim) v.w = p[s + 3];
  return v;
}

SSI_DEV float4 zero4() { return make_float4(0.f, 0.f, 0.f, 0.f); }

}  // namespace

// One workgroup: rows [r0, r0 + 256) x columns [c0, c0 + 64) over samples
// [s_begin, s_end); wave w owns rows 64 (w % 4).. and columns 32 (w / 4)...
// Tiles are loaded with 16-byte loads (VEC: ldy % 4 == 0 and y 16-byte
// aligned), all issued before the first is written to LDS; tiles that lie
// inside the split (B) or the record (A window) skip the per-sample guards.
// Writes fp64 partial sums partial[split][r][b].
template <bool VEC>
__global__ void __launch_bounds__(kThreads, 2)
correlate_mfma(const float *__restrict__ y, int l, int64_t n, int64_t ldy, int L,
               int64_t split_len, double *__restrict__ partial, int sa_stride,
               int na_max) {
  extern __shared__ float lds[];
  const int rows_total = l * L;
  const int r0 = blockIdx.x * kRowsPerWG;
  const int c0 = blockIdx.y * kColsPerWG;
  const int split = blockIdx.z;
  const int64_t s_begin = (int64_t)split * split_len;
  const int64_t s_end = min(n, s_begin + split_len);
  if (s_begin >= s_end) return;

  float *yb = lds;                         // [64][kSB]   y[c0 + bb][s0 + t]
  float *ya = lds + kColsPerWG * kSB;      // [na][sa_stride] y[a_first + i][s0 + t]

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wr = wave & 3, wc = wave >> 2;
  const int a_first = r0 / L;
  const int a_last = min(l - 1, (min(r0 + kRowsPerWG, rows_total) - 1) / L);
  const int na = a_last - a_first + 1;     // <= na_max by construction
  const int wa4 = (kST + L + 3) / 4;       // A window length per channel (float4)
  const int na4 = na * wa4;

  // Per-lane LDS offsets of the A rows (4 row tiles) and B columns (2 tiles).
  int offA[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int r = min(r0 + wr * kRowsPerWave + t * 16 + (lane & 15), rows_total - 1);
    const int a = r / L, j = r - a * L + 1;
    offA[t] = (a - a_first) * sa_stride + j + (lane >> 4);
  }
  int offB[2];
#pragma unroll
  for (int u = 0; u < 2; ++u)
    offB[u] = (wc * kColsPerWave + u * 16 + (lane & 15)) * kSB + (lane >> 4);

  f32x4 acc[4][2];
  double accd[4][2][4];
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      acc[t][u] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int q = 0; q < 4; ++q) accd[t][u][q] = 0.0;
    }

  // this thread's B elements: rows bb = tid / 32 + 16 h, float4 column tid % 32
  const int bb0 = tid >> 5, bc4 = tid & 31;
  int tile_count = 0;
  for (int64_t s0 = s_begin; s0 < s_end; s0 += kST) {
    // B tile: y[c0 + bb][s0 + t] for s in the split, zero elsewhere
    float4 rb[4];
    const bool full_b = s0 + kST <= s_end;
#pragma unroll
    for (int h = 0; h < 4; ++h) {
      const int b = c0 + bb0 + 16 * h;
      const float *row = y + (int64_t)min(b, l - 1) * ldy;
      float4 v;
      if (VEC && full_b) v = *reinterpret_cast<const float4 *>(row + s0 + 4 * bc4);
      else v = load4<VEC>(row, s0 + 4 * bc4, s_end);
      rb[h] = b < l ? v : zero4();
    }
    // A window: y[a][s0 + t] for t < kST + L, zero past the record
    float4 ra;
    int ia = 0, ca = 0;
    const bool full_a = s0 + 4 * wa4 <= n;
    if (tid < na4) {
      ia = tid / wa4;
      ca = tid - ia * wa4;
      const float *row = y + (int64_t)(a_first + ia) * ldy;
      if (VEC && full_a) ra = *reinterpret_cast<const float4 *>(row + s0 + 4 * ca);
      else ra = load4<VEC>(row, s0 + 4 * ca, n);
    }
    __syncthreads();                       // previous tile's reads are done
#pragma unroll
    for (int h = 0; h < 4; ++h)
      *reinterpret_cast<float4 *>(&yb[(bb0 + 16 * h) * kSB + 4 * bc4]) = rb[h];
    if (tid < na4) *reinterpret_cast<float4 *>(&ya[ia * sa_stride + 4 * ca]) = ra;
    for (int idx = tid + kThreads; idx < na4; idx += kThreads) {   // wide windows (small L)
      const int i = idx / wa4, c4 = idx - i * wa4;
      *reinterpret_cast<float4 *>(&ya[i * sa_stride + 4 * c4]) =
          load4<VEC>(y + (int64_t)(a_first + i) * ldy, s0 + 4 * c4, n);
    }
    __syncthreads();

#pragma unroll 4
    for (int kk = 0; kk < kST; kk += 4) {
      float af[4], bf[2];
#pragma unroll
      for (int t = 0; t < 4; ++t) af[t] = ya[offA[t] + kk];
#pragma unroll
      for (int u = 0; u < 2; ++u) bf[u] = yb[offB[u] + kk];
#pragma unroll
      for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int u = 0; u < 2; ++u)
          acc[t][u] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[t], bf[u], acc[t][u], 0, 0, 0);
    }

    if (++tile_count == kFlushTiles || s0 + kST >= s_end) {
      tile_count = 0;
#pragma unroll
      for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int u = 0; u < 2; ++u) {
#pragma unroll
          for (int q = 0; q < 4; ++q) accd[t][u][q] += (double)acc[t][u][q];
          acc[t][u] = f32x4{0.f, 0.f, 0.f, 0.f};
        }
    }
  }

  // D layout of 16x16x4f32: lane holds rows 4*(lane/16)+q, column lane%16.
  double *dst = partial + (int64_t)split * rows_total * l;
#pragma unroll
  for (int t = 0; t < 4; ++t) {
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int b = c0 + wc * kColsPerWave + u * 16 + (lane & 15);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int r = r0 + wr * kRowsPerWave + t * 16 + 4 * (lane >> 4) + q;
        if (r < rows_total && b < l) dst[(int64_t)r * l + b] = accd[t][u][q];
      }
    }
  }
  (void)na_max;
}

// R[j-1][a][b] = (float)(sum_split partial[split][a L + j - 1][b] / n)
__global__ void __launch_bounds__(256)
correlate_reduce(const double *__restrict__ partial, int l, int L, int splits,
                 double inv_n, float *__restrict__ r) {
  const int64_t total = (int64_t)l * L * l;
  const int64_t plane = total;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int b = (int)(idx % l);
    const int64_t ja = idx / l;
    const int a = (int)(ja % l);
    const int j = (int)(ja / l);                 // j - 1
    const int64_t src = ((int64_t)a * L + j) * l + b;
    double s = 0.0;
    for (int sp = 0; sp < splits; ++sp) s += partial[sp * plane + src];
    r[idx] = (float)(s * inv_n);
  }
}

// ------------------------------------------------------------------ launch
namespace ssi {

CorrPlan plan_correlate(int l, int64_t n, int L, int num_cus) {
  CorrPlan p{};
  const int rows_total = l * L;
  p.grid_rows = ceil_div(rows_total, kRowsPerWG);
  p.grid_cols = ceil_div(l, kColsPerWG);
  const int tiles = p.grid_rows * p.grid_cols;
  // Aim for about four resident rounds of two workgroups per CU, with at
  // least 1024 samples per split.
  const int64_t target = (int64_t)num_cus * 2 * 4;
  int64_t splits = ceil_div<int64_t>(target, tiles);
  const int64_t max_splits = ceil_div<int64_t>(n, 1024);
  if (splits > max_splits) splits = max_splits;
  if (splits < 1) splits = 1;
  int64_t len = ceil_div<int64_t>(n, splits);
  len = ceil_div<int64_t>(len, kST) * kST;
  p.split_len = len;
  p.splits = (int)ceil_div<int64_t>(n, len);
  // A window rows: channels spanned by 256 flattened rows.
  p.na_max = kRowsPerWG / L + 2;
  if (p.na_max > l) p.na_max = l;
  // A window row stride: whole float4s, not a multiple of 32 floats
  p.sa_stride = (kST + L + 3) / 4 * 4;
  if ((p.sa_stride & 31) == 0) p.sa_stride += 4;
  p.lds_bytes = sizeof(float) * ((size_t)kColsPerWG * kSB + (size_t)p.na_max * p.sa_stride);
  p.partial_elems = (size_t)p.splits * rows_total * l;
  return p;
}

hipError_t launch_correlate_mfma(const CorrPlan &p, const float *y, int l, int64_t n, int64_t ldy,
                                 int L, double *partial, hipStream_t st) {
  dim3 grid(p.grid_rows, p.grid_cols, p.splits);
  const bool vec = (ldy % 4 == 0) && ((uintptr_t)y % 16 == 0);
  const void *fn = vec ? (const void *)correlate_mfma<true> : (const void *)correlate_mfma<false>;
  if (p.lds_bytes > 65536) {
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)p.lds_bytes);
    if (e != hipSuccess) return e;
  }
  if (vec)
    hipLaunchKernelGGL(correlate_mfma<true>, grid, dim3(kThreads), p.lds_bytes, st, y, l, n,
                       ldy, L, p.split_len, partial, p.sa_stride, p.na_max);
  else
    hipLaunchKernelGGL(correlate_mfma<false>, grid, dim3(kThreads), p.lds_bytes, st, y, l, n,
                       ldy, L, p.split_len, partial, p.sa_stride, p.na_max);
  return hipGetLastError();
}

hipError_t launch_correlate_reduce(const CorrPlan &p, int l, int64_t n, int L,
                                   const double *partial, float *r, hipStream_t st) {
  const int64_t total = (int64_t)l * L * l;
  int blocks = (int)ceil_div<int64_t>(total, 256);
  if (blocks > 65535 * 8) blocks = 65535 * 8;
  hipLaunchKernelGGL(correlate_reduce, dim3(blocks), dim3(256), 0, st, partial, l, L,
                     p.splits, 1.0 / (double)n, r);
  return hipGetLastError();
}

hipError_t launch_correlate(const CorrPlan &p, const float *y, int l, int64_t n, int64_t ldy,
                            int L, double *partial, float *r, hipStream_t st) {
  hipError_t e = launch_correlate_mfma(p, y, l, n, ldy, L, partial, st);
  if (e != hipSuccess) return e;
  return launch_correlate_reduce(p, l, n, L, partial, r, st);
}

}  // namespace ssi
