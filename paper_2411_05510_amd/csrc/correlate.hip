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

constexpr int kWaves = 4;            // waves per workgroup
constexpr int kRowsPerWave = 64;     // 4 MFMA row tiles of 16
constexpr int kRowsPerWG = kWaves * kRowsPerWave;
constexpr int kColsPerWG = 64;       // 4 MFMA column tiles of 16, shared by waves
constexpr int kST = 128;             // samples per LDS tile
constexpr int kSB = kST + 2;         // LDS row stride of the B tile (floats)
constexpr int kFlushTiles = 2;       // fold fp32 into fp64 every 256 samples

}  // namespace

// One workgroup: rows [r0, r0 + 256) x columns [c0, c0 + 64) over samples
// [s_begin, s_end).  Writes fp64 partial sums partial[split][r][b].
__global__ void __launch_bounds__(256, 2)
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
  const int a_first = r0 / L;
  const int a_last = min(l - 1, (min(r0 + kRowsPerWG, rows_total) - 1) / L);
  const int na = a_last - a_first + 1;     // <= na_max by construction
  const int wa = kST + L;                  // A window length per channel

  // Per-lane LDS offsets of the A rows (4 row tiles) and B columns (4 tiles).
  int offA[4];
  bool rowok[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int r = r0 + wave * kRowsPerWave + t * 16 + (lane & 15);
    rowok[t] = r < rows_total;
    const int rr = rowok[t] ? r : r0;
    const int a = rr / L, j = rr - a * L + 1;
    offA[t] = (a - a_first) * sa_stride + j + (lane >> 4);
  }
  int offB[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) offB[u] = (u * 16 + (lane & 15)) * kSB + (lane >> 4);

  f32x4 acc[4][4];
  double accd[4][4][4];
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      acc[t][u] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int q = 0; q < 4; ++q) accd[t][u][q] = 0.0;
    }

  int tile_count = 0;
  for (int64_t s0 = s_begin; s0 < s_end; s0 += kST) {
    __syncthreads();
    // B tile: y[c0 + bb][s0 + t] for s in the split, zero elsewhere.
    for (int idx = tid; idx < kColsPerWG * kST; idx += 256) {
      const int bb = idx / kST, t = idx - bb * kST;
      const int b = c0 + bb;
      const int64_t s = s0 + t;
      float v = 0.f;
      if (b < l && s < s_end) v = y[(int64_t)b * ldy + s];
      yb[bb * kSB + t] = v;
    }
    // A window: y[a][s0 + t] for t < kST + L, zero past the record.
    for (int idx = tid; idx < na * wa; idx += 256) {
      const int i = idx / wa, t = idx - i * wa;
      const int64_t s = s0 + t;
      float v = 0.f;
      if (s < n) v = y[(int64_t)(a_first + i) * ldy + s];
      ya[i * sa_stride + t] = v;
    }
    __syncthreads();

#pragma unroll 4
    for (int kk = 0; kk < kST; kk += 4) {
      float af[4], bf[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) af[t] = ya[offA[t] + kk];
#pragma unroll
      for (int u = 0; u < 4; ++u) bf[u] = yb[offB[u] + kk];
#pragma unroll
      for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int u = 0; u < 4; ++u)
          acc[t][u] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[t], bf[u], acc[t][u], 0, 0, 0);
    }

    if (++tile_count == kFlushTiles || s0 + kST >= s_end) {
      tile_count = 0;
#pragma unroll
      for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int u = 0; u < 4; ++u) {
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
    for (int u = 0; u < 4; ++u) {
      const int b = c0 + u * 16 + (lane & 15);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int r = r0 + wave * kRowsPerWave + t * 16 + 4 * (lane >> 4) + q;
        if (r < rows_total && b < l) dst[(int64_t)r * l + b] = accd[t][u][q];
      }
    }
  }
  (void)rowok;
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
  p.sa_stride = kST + L + 2;
  if ((p.sa_stride & 31) == 0) p.sa_stride += 2;
  p.lds_bytes = sizeof(float) * ((size_t)kColsPerWG * kSB + (size_t)p.na_max * p.sa_stride);
  p.partial_elems = (size_t)p.splits * rows_total * l;
  return p;
}

hipError_t launch_correlate_mfma(const CorrPlan &p, const float *y, int l, int64_t n, int64_t ldy,
                                 int L, double *partial, hipStream_t st) {
  dim3 grid(p.grid_rows, p.grid_cols, p.splits);
  if (p.lds_bytes > 65536) {
    hipError_t e = hipFuncSetAttribute((const void *)correlate_mfma,
                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)p.lds_bytes);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(correlate_mfma, grid, dim3(256), p.lds_bytes, st, y, l, n, ldy, L,
                     p.split_len, partial, p.sa_stride, p.na_max);
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
