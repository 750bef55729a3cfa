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
//
// Two product paths share the tiling, the split-K partials and the reduction:
//   FP32   v_mfma_f32_16x16x4f32 on the FP32 samples;
//   BF16x6 each FP32 sample is split exactly into three BF16 parts,
//          y = hi + mid + lo (truncation: hi keeps the top 8 significant bits,
//          mid the next 8, lo the last 8), and y_a y_b is formed from the six
//          cross products whose weight is at least 2^-16 of the leading one
//          (hi hi, hi mid, mid hi, hi lo, lo hi, mid mid) on
//          v_mfma_f32_16x16x32_bf16.  Each BF16 product is exact in FP32, the
//          dropped terms are below 2^-23 of |y_a y_b|, and accumulation is FP32
//          with the same FP64 folding, so the sums carry FP32-product accuracy
//          at the BF16 matrix rate.
#include <algorithm>

#include "common.h"
#include "kernels.h"
#include "ssicov.h"

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

// Tile of a workgroup of the one-dimensional grid.  Workgroup p runs on XCD
// p mod 8 (the dispatcher deals workgroups round-robin over the eight XCDs,
// each with its own L2), so each XCD gets one contiguous run of tiles in
// (row tile, column tile, split) order, row tiles fastest: the workgroups
// resident on one XCD at a time share their B tile (one column tile of one
// split) instead of every XCD streaming every B tile.
struct CorrTile { int rt, ct, split; };
SSI_DEV CorrTile corr_tile(int grid_rows, int grid_cols, int total) {
  constexpr int kXcd = 8;
  const int p = blockIdx.x;
  const int xcd = p % kXcd, k = p / kXcd;
  const int base = total / kXcd, rem = total % kXcd;
  const int t = xcd * base + min(xcd, rem) + k;
  const int rt = t % grid_rows, rest = t / grid_rows;
  return {rt, rest % grid_cols, rest / grid_cols};
}

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
               int na_max, int grid_rows, int grid_cols, int n_splits) {
  extern __shared__ float lds[];
  const int rows_total = l * L;
  const CorrTile tile = corr_tile(grid_rows, grid_cols, grid_rows * grid_cols * n_splits);
  const int r0 = tile.rt * kRowsPerWG;
  const int c0 = tile.ct * kColsPerWG;
  const int split = tile.split;
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

// ------------------------------------------------------------ BF16x6 path
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

namespace {
constexpr int kSB6 = kST + 8;        // B tile row stride (bf16): 272 bytes, 16-byte
                                     // rows whose 16 fragment reads hit distinct banks

// Top 8 significant bits of x (truncation toward zero), as BF16 bits and as FP32.
SSI_DEV uint32_t bf16_trunc_bits(float x) { return __float_as_uint(x) >> 16; }
SSI_DEV float bf16_trunc_val(float x) { return __uint_as_float(__float_as_uint(x) & 0xffff0000u); }
}  // namespace

// planes[q][c][s] (q = hi, mid, lo; c < lp; s < np) from y (l x n, ld ldy);
// zero past the record and for channels c >= l.  hi + mid + lo == y exactly.
__global__ void __launch_bounds__(256)
split3_kernel(const float *__restrict__ y, int l, int64_t n, int64_t ldy, int lp, int64_t np,
              uint16_t *__restrict__ planes) {
  const int64_t per_row = np / 4;
  const int64_t total = (int64_t)lp * per_row;
  const int64_t plane = (int64_t)lp * np;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int c = (int)(idx / per_row);
    const int64_t s = (idx - (int64_t)c * per_row) * 4;
    float v[4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
      v[i] = (c < l && s + i < n) ? y[(int64_t)c * ldy + s + i] : 0.0f;
    uint32_t h[2], m[2], w[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      uint32_t hb[2], mb[2], lb[2];
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        const float x = v[2 * i + k];
        const float hv = bf16_trunc_val(x);
        const float r1 = x - hv;                 // exact: the low 16 significant bits
        const float mv = bf16_trunc_val(r1);
        const float r2 = r1 - mv;                // exact, at most 8 significant bits
        hb[k] = bf16_trunc_bits(x);
        mb[k] = bf16_trunc_bits(r1);
        lb[k] = bf16_trunc_bits(r2);
      }
      h[i] = hb[0] | (hb[1] << 16);
      m[i] = mb[0] | (mb[1] << 16);
      w[i] = lb[0] | (lb[1] << 16);
    }
    const int64_t o = (int64_t)c * np + s;
    *reinterpret_cast<uint2 *>(planes + o) = make_uint2(h[0], h[1]);
    *reinterpret_cast<uint2 *>(planes + plane + o) = make_uint2(m[0], m[1]);
    *reinterpret_cast<uint2 *>(planes + 2 * plane + o) = make_uint2(w[0], w[1]);
  }
}

// FP16x3 path, step 1: partial maxima of |sample| per channel row, kScaleParts
// workgroups per channel, each over one contiguous part of the record (zero
// for the padding channels c >= l).  fmaxf drops NaN; a NaN or Inf sample
// still reaches the products and makes a correlation non-finite.
constexpr int kScaleParts = 8;

__global__ void __launch_bounds__(256)
chan_max_kernel(const float *__restrict__ y, int l, int64_t n, int64_t ldy,
                float *__restrict__ pmax) {
  __shared__ float part[4];
  const int c = blockIdx.x, g = blockIdx.y;
  const int64_t len = (n + kScaleParts - 1) / kScaleParts;
  const int64_t s_end = min(n, (g + 1) * len);
  float mx = 0.0f;
  if (c < l) {
    const float *row = y + (int64_t)c * ldy;
    int64_t s = g * len + threadIdx.x;
    for (; s + 3 * 256 < s_end; s += 4 * 256) {
      const float a = row[s], b = row[s + 256], d = row[s + 512], e = row[s + 768];
      mx = fmaxf(mx, fmaxf(fmaxf(fabsf(a), fabsf(b)), fmaxf(fabsf(d), fabsf(e))));
    }
    for (; s < s_end; s += 256) mx = fmaxf(mx, fabsf(row[s]));
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) mx = fmaxf(mx, __shfl_xor(mx, off));
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = mx;
  __syncthreads();
  if (threadIdx.x == 0)
    pmax[c * kScaleParts + g] = fmaxf(fmaxf(part[0], part[1]), fmaxf(part[2], part[3]));
}

// The channel's scale exponent e: 2^e brings its largest |sample| into
// [2^13, 2^14), well inside the FP16 range; e = 0 for an all-zero or
// non-finite channel and for the padding channels.
SSI_DEV int chan_exponent(const float *__restrict__ pmax, int c) {
  float mx = 0.0f;
#pragma unroll
  for (int g = 0; g < kScaleParts; ++g) mx = fmaxf(mx, pmax[c * kScaleParts + g]);
  if (!(mx > 0.0f) || !isfinite(mx)) return 0;
  int ex;
  (void)frexpf(mx, &ex);                         // mx = m 2^ex, m in [1/2, 1)
  return 14 - ex;
}

// FP16x3 path, step 2: planes[q][c][s] (q = hi, lo) of x = y 2^e_c, and
// the exponents e_c:
// hi = FP16(x), lo = FP16(x - hi) (round to nearest even; x - hi is exact in
// FP32), so |x - hi - lo| <= 2^-22 |x| for normal FP16 parts, and below
// 2^-25 absolutely (2^-38 of the channel maximum) for the smallest samples.
// Zero past the record and for channels c >= l.
__global__ void __launch_bounds__(256)
split2h_kernel(const float *__restrict__ y, int l, int64_t n, int64_t ldy, int lp, int64_t np,
               const float *__restrict__ pmax, int *__restrict__ exps,
               uint16_t *__restrict__ planes) {
  const int64_t per_row = np / 4;
  const int64_t total = (int64_t)lp * per_row;
  const int64_t plane = (int64_t)lp * np;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int c = (int)(idx / per_row);
    const int64_t s = (idx - (int64_t)c * per_row) * 4;
    const int e = chan_exponent(pmax, c);
    if (s == 0) exps[c] = e;                     // for the reduction's scale-back
    uint32_t hb[4], lb[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const float x = (c < l && s + i < n) ? ldexpf(y[(int64_t)c * ldy + s + i], e) : 0.0f;
      const _Float16 h = (_Float16)x;
      const _Float16 w = (_Float16)(x - (float)h);
      hb[i] = __builtin_bit_cast(uint16_t, h);
      lb[i] = __builtin_bit_cast(uint16_t, w);
    }
    const int64_t o = (int64_t)c * np + s;
    *reinterpret_cast<uint2 *>(planes + o) = make_uint2(hb[0] | (hb[1] << 16), hb[2] | (hb[3] << 16));
    *reinterpret_cast<uint2 *>(planes + plane + o) =
        make_uint2(lb[0] | (lb[1] << 16), lb[2] | (lb[3] << 16));
  }
}

// Same tiling and outputs as correlate_mfma, on the three BF16 planes.  One
// K step covers 32 samples.  An A fragment of rows (a, j) is, in lane (row, g),
// the 8 samples s + 8 g + j .. + 7 of channel a's window: they start at any
// sample, so the window is kept in LDS as eight copies shifted by 0..7 samples
// and the fragment is one aligned 16-byte read of copy j mod 8.  B fragments
// are aligned 16-byte reads of the B tile.  The next tile's global loads are
// issued before the current tile's products.  The planes are zero past the
// record and past the channels, so no load needs a guard; split_len is a
// multiple of the tile, so a tile never reaches past its split except at the
// end of the record.
template <int NP>
SSI_DEV __forceinline__ void
correlate_split_body(const uint16_t *__restrict__ planes, int l, int64_t n, int lp, int64_t np,
                     int L, int64_t split_len, double *__restrict__ partial, int sa_stride,
                     int na_max, int copy_stride, int grid_rows, int grid_cols, int n_splits) {
  extern __shared__ __align__(16) uint16_t lds6[];
  const int rows_total = l * L;
  const CorrTile tile = corr_tile(grid_rows, grid_cols, grid_rows * grid_cols * n_splits);
  const int r0 = tile.rt * kRowsPerWG;
  const int c0 = tile.ct * kColsPerWG;
  const int split = tile.split;
  const int64_t s_begin = (int64_t)split * split_len;
  const int64_t s_end = min(n, s_begin + split_len);
  if (s_begin >= s_end) return;
  const int64_t plane = (int64_t)lp * np;

  // [NP][64][kSB6] B tile, then 8 copies (stride copy_stride) of the
  // [NP][na_max][sa_stride] A window, copy c holding window sample t + c at t
  uint16_t *yb = lds6;
  uint16_t *ya = lds6 + NP * kColsPerWG * kSB6;
  const int pa = na_max * sa_stride;                    // elements per plane of a copy

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wr = wave & 3, wc = wave >> 2;
  const int a_first = r0 / L;
  const int a_last = min(l - 1, (min(r0 + kRowsPerWG, rows_total) - 1) / L);
  const int na = a_last - a_first + 1;
  const int wa8 = sa_stride / 8;                        // window chunks of 8 samples per row

  int offA[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int r = min(r0 + wr * kRowsPerWave + t * 16 + (lane & 15), rows_total - 1);
    const int a = r / L, j = r - a * L + 1;
    offA[t] = (j & 7) * copy_stride + (a - a_first) * sa_stride + 8 * (lane >> 4) + (j & ~7);
  }
  int offB[2];
#pragma unroll
  for (int u = 0; u < 2; ++u)
    offB[u] = (wc * kColsPerWave + u * 16 + (lane & 15)) * kSB6 + 8 * (lane >> 4);

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

  // B tile: NP planes x 64 rows x 16 chunks of 8 samples = NP x 1024 chunks,
  // 2 NP per thread.  A window: NP planes x na rows x wa8 chunks; a thread
  // takes chunk c8 and the one after it and writes the eight shifted copies of
  // chunk c8.
  const int nA = NP * na * wa8;
  u32x4 rb[2 * NP], ra0 = u32x4{0u, 0u, 0u, 0u}, ra1 = ra0;
  int qa = 0, ia = 0, ca = 0;
  if (tid < nA) {
    qa = tid / (na * wa8);
    const int rem = tid - qa * na * wa8;
    ia = rem / wa8;
    ca = rem - ia * wa8;
  }
  auto load_tile = [&](int64_t s0) {
#pragma unroll
    for (int h = 0; h < 2 * NP; ++h) {
      const int idx = tid + kThreads * h;
      const int q = idx >> 10, rem = idx & 1023, row = rem >> 4, ch = rem & 15;
      rb[h] = *reinterpret_cast<const u32x4 *>(planes + q * plane + (int64_t)(c0 + row) * np +
                                               s0 + 8 * ch);
    }
    if (tid < nA) {
      const uint16_t *src = planes + qa * plane + (int64_t)(a_first + ia) * np + s0 + 8 * ca;
      ra0 = *reinterpret_cast<const u32x4 *>(src);
      ra1 = *reinterpret_cast<const u32x4 *>(src + 8);
    }
  };
  // the eight shifted copies of one window chunk: copy c, chunk c8 holds
  // samples 8 c8 + c .. + 7, i.e. bytes 2c .. 2c + 15 of the chunk pair
  auto store_shifted = [&](int q, int i, int c8, const u32x4 &lo, const u32x4 &hi) {
    const uint32_t d[8] = {lo.x, lo.y, lo.z, lo.w, hi.x, hi.y, hi.z, hi.w};
    uint16_t *dst = ya + (q * na_max + i) * sa_stride + 8 * c8;
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      u32x4 w;
      const int k = c >> 1, sh = (c & 1) * 2;
      w.x = __builtin_amdgcn_alignbyte(d[k + 1], d[k], sh);
      w.y = __builtin_amdgcn_alignbyte(d[k + 2], d[k + 1], sh);
      w.z = __builtin_amdgcn_alignbyte(d[k + 3], d[k + 2], sh);
      w.w = __builtin_amdgcn_alignbyte(d[k + 4], d[k + 3], sh);
      *reinterpret_cast<u32x4 *>(dst + c * copy_stride) = w;
    }
  };
  auto store_tile = [&](int64_t s0) {
#pragma unroll
    for (int h = 0; h < 2 * NP; ++h) {
      const int idx = tid + kThreads * h;
      const int q = idx >> 10, rem = idx & 1023, row = rem >> 4, ch = rem & 15;
      *reinterpret_cast<u32x4 *>(&yb[(q * kColsPerWG + row) * kSB6 + 8 * ch]) = rb[h];
    }
    if (tid < nA) store_shifted(qa, ia, ca, ra0, ra1);
    for (int idx = tid + kThreads; idx < nA; idx += kThreads) {   // wide windows (small L)
      const int q = idx / (na * wa8), rem = idx - q * na * wa8;
      const int i = rem / wa8, c8 = rem - i * wa8;
      const uint16_t *src = planes + q * plane + (int64_t)(a_first + i) * np + s0 + 8 * c8;
      store_shifted(q, i, c8, *reinterpret_cast<const u32x4 *>(src),
                    *reinterpret_cast<const u32x4 *>(src + 8));
    }
  };
  load_tile(s_begin);
  int tile_count = 0;
  for (int64_t s0 = s_begin; s0 < s_end; s0 += kST) {
    __syncthreads();                       // the previous tile's reads are done
    store_tile(s0);
    __syncthreads();
    if (s0 + kST < s_end) load_tile(s0 + kST);

#pragma unroll 2
    for (int kk = 0; kk < kST; kk += 32) {
      if constexpr (NP == 3) {
        bf16x8 bf[2][3];
#pragma unroll
        for (int u = 0; u < 2; ++u)
#pragma unroll
          for (int q = 0; q < 3; ++q)
            bf[u][q] = *reinterpret_cast<const bf16x8 *>(&yb[q * kColsPerWG * kSB6 + offB[u] + kk]);
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          bf16x8 af[3];
#pragma unroll
          for (int q = 0; q < 3; ++q)
            af[q] = *reinterpret_cast<const bf16x8 *>(&ya[offA[t] + q * pa + kk]);
#pragma unroll
          for (int u = 0; u < 2; ++u) {
            f32x4 c = acc[t][u];
            c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[2], bf[u][0], c, 0, 0, 0);   // lo hi
            c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[0], bf[u][2], c, 0, 0, 0);   // hi lo
            c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[1], bf[u][1], c, 0, 0, 0);   // mid mid
            c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[1], bf[u][0], c, 0, 0, 0);   // mid hi
            c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[0], bf[u][1], c, 0, 0, 0);   // hi mid
            c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[0], bf[u][0], c, 0, 0, 0);   // hi hi
            acc[t][u] = c;
          }
        }
      } else {
        f16x8 bf[2][2];
#pragma unroll
        for (int u = 0; u < 2; ++u)
#pragma unroll
          for (int q = 0; q < 2; ++q)
            bf[u][q] = *reinterpret_cast<const f16x8 *>(&yb[q * kColsPerWG * kSB6 + offB[u] + kk]);
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          f16x8 af[2];
#pragma unroll
          for (int q = 0; q < 2; ++q)
            af[q] = *reinterpret_cast<const f16x8 *>(&ya[offA[t] + q * pa + kk]);
#pragma unroll
          for (int u = 0; u < 2; ++u) {
            f32x4 c = acc[t][u];
            c = __builtin_amdgcn_mfma_f32_16x16x32_f16(af[1], bf[u][0], c, 0, 0, 0);    // lo hi
            c = __builtin_amdgcn_mfma_f32_16x16x32_f16(af[0], bf[u][1], c, 0, 0, 0);    // hi lo
            c = __builtin_amdgcn_mfma_f32_16x16x32_f16(af[0], bf[u][0], c, 0, 0, 0);    // hi hi
            acc[t][u] = c;
          }
        }
      }
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

  // D layout of 16x16x32 bf16 and f16: lane holds rows 4*(lane/16)+q, column lane%16.
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
}

__global__ void __launch_bounds__(kThreads, 2)
correlate_b6(const uint16_t *__restrict__ planes, int l, int64_t n, int lp, int64_t np, int L,
             int64_t split_len, double *__restrict__ partial, int sa_stride, int na_max,
             int copy_stride, int grid_rows, int grid_cols, int n_splits) {
  correlate_split_body<3>(planes, l, n, lp, np, L, split_len, partial, sa_stride, na_max,
                          copy_stride, grid_rows, grid_cols, n_splits);
}

// FP16x3: the same tiling on the two FP16 planes of the scaled record.
__global__ void __launch_bounds__(kThreads, 2)
correlate_h3(const uint16_t *__restrict__ planes, int l, int64_t n, int lp, int64_t np, int L,
             int64_t split_len, double *__restrict__ partial, int sa_stride, int na_max,
             int copy_stride, int grid_rows, int grid_cols, int n_splits) {
  correlate_split_body<2>(planes, l, n, lp, np, L, split_len, partial, sa_stride, na_max,
                          copy_stride, grid_rows, grid_cols, n_splits);
}

// R[j-1][a][b] = (float)(sum_split partial[split][a L + j - 1][b] / n), times
// 2^-(e_a + e_b) when the FP16x3 path scaled the channels (exps not null).
// A non-finite sample makes some correlation non-finite (every sample enters
// at least one product, and NaN or Inf times anything stays non-finite or
// gives NaN), so checking the results here flags such a record without a
// separate pass over it.
__global__ void __launch_bounds__(256)
correlate_reduce(const double *__restrict__ partial, int l, int L, int splits,
                 double inv_n, const int *__restrict__ exps, float *__restrict__ r,
                 int *__restrict__ status) {
  const int64_t total = (int64_t)l * L * l;
  const int64_t plane = total;
  int bad = 0;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int b = (int)(idx % l);
    const int64_t ja = idx / l;
    const int a = (int)(ja % l);
    const int j = (int)(ja / l);                 // j - 1
    const int64_t src = ((int64_t)a * L + j) * l + b;
    double s = 0.0;
    for (int sp = 0; sp < splits; ++sp) s += partial[sp * plane + src];
    s *= inv_n;
    if (exps) s = ldexp(s, -(exps[a] + exps[b]));   // undo the FP16x3 channel scales (exact)
    const float v = (float)s;
    bad |= !isfinite(v);
    r[idx] = v;
  }
  if (__any(bad) && (threadIdx.x & 63) == 0) atomicOr(status, ssi::kStatusNonFinite);
}

// ------------------------------------------------------------------ launch
namespace ssi {

namespace {
// FP16x3: the channel exponents stored after the two planes
int *corr_exps(const CorrPlan &p, const uint16_t *planes) {
  return reinterpret_cast<int *>(const_cast<uint16_t *>(planes) + (size_t)2 * p.lp * p.np);
}
}  // namespace

CorrPlan plan_correlate(int l, int64_t n, int L, int num_cus, int mode) {
  CorrPlan p{};
  const int rows_total = l * L;
  p.grid_rows = ceil_div(rows_total, kRowsPerWG);
  p.grid_cols = ceil_div(l, kColsPerWG);
  const int tiles = p.grid_rows * p.grid_cols;
  // Aim for about four resident rounds of workgroups, with at least 1024
  // samples per split: two workgroups per CU for the FP32 path, one for the
  // split paths (their registers allow one eight-wave workgroup per CU), so
  // that the split paths write half as many FP64 partials.
  const bool split_mode = mode == SSI_CORR_BF16X6 || mode == SSI_CORR_F16X3;
  const int64_t target = (int64_t)num_cus * (split_mode ? 1 : 2) * 4;
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
  p.partial_elems = (size_t)p.splits * rows_total * l;
  p.mode = SSI_CORR_FP32;
  if (mode == SSI_CORR_BF16X6 || mode == SSI_CORR_F16X3) {
    const int nplanes = mode == SSI_CORR_BF16X6 ? 3 : 2;
    // window row: samples up to 127 + L past the tile start, whole 16-byte chunks
    const int sa = (kST + L + 7) / 8 * 8;
    // copy stride: whole chunks, 5 chunks (20 dwords) past a multiple of 64
    // dwords; the lanes of a fragment read take consecutive lags, i.e. copies
    // 0..7 at two or three chunk positions, and an odd chunk offset between
    // copies spreads them over the banks (measured: 6.3 ms against 6.75 ms
    // for an offset of 2 chunks and 9.5 ms for none on the 180-channel record)
    int cs = nplanes * p.na_max * sa;
    cs = (cs + 127) / 128 * 128 + 40;
    const size_t lds =
        sizeof(uint16_t) * ((size_t)nplanes * kColsPerWG * kSB6 + (size_t)8 * cs);
    if (lds <= 160 * 1024) {
      p.mode = mode;
      p.sa_stride = sa;
      p.copy_stride = cs;
      p.lds_bytes = lds;
      p.lp = p.grid_cols * kColsPerWG;
      p.np = (n + 2 * kST + L + 64 + 7) / 8 * 8;   // every window and tile read stays inside
      // FP16x3: the lp channel exponents (int32) and the kScaleParts partial
      // maxima per channel (FP32) follow the two planes
      p.planes_elems = (size_t)nplanes * p.lp * p.np +
                       (mode == SSI_CORR_F16X3 ? (size_t)2 * p.lp * (1 + kScaleParts) : 0);
    }
  }
  if (p.mode == SSI_CORR_FP32) {
    // A window row stride: whole float4s, not a multiple of 32 floats
    p.sa_stride = (kST + L + 3) / 4 * 4;
    if ((p.sa_stride & 31) == 0) p.sa_stride += 4;
    p.lds_bytes = sizeof(float) * ((size_t)kColsPerWG * kSB + (size_t)p.na_max * p.sa_stride);
  }
  return p;
}

hipError_t launch_correlate_split(const CorrPlan &p, const float *y, int l, int64_t n,
                                  int64_t ldy, uint16_t *planes, hipStream_t st) {
  if (p.mode == SSI_CORR_FP32) return hipSuccess;
  const int64_t chunks = (int64_t)p.lp * (p.np / 4);
  const int blocks = (int)std::min<int64_t>(ceil_div<int64_t>(chunks, 256), 65535 * 4);
  if (p.mode == SSI_CORR_BF16X6) {
    hipLaunchKernelGGL(split3_kernel, dim3(blocks), dim3(256), 0, st, y, l, n, ldy, p.lp, p.np,
                       planes);
    return hipGetLastError();
  }
  int *exps = corr_exps(p, planes);
  float *pmax = reinterpret_cast<float *>(exps + p.lp);
  hipLaunchKernelGGL(chan_max_kernel, dim3(p.lp, kScaleParts), dim3(256), 0, st, y, l, n, ldy,
                     pmax);
  hipLaunchKernelGGL(split2h_kernel, dim3(blocks), dim3(256), 0, st, y, l, n, ldy, p.lp, p.np,
                     pmax, exps, planes);
  return hipGetLastError();
}

hipError_t launch_correlate_mfma(const CorrPlan &p, const float *y, int l, int64_t n, int64_t ldy,
                                 int L, double *partial, const uint16_t *planes, hipStream_t st) {
  const dim3 grid((unsigned)(p.grid_rows * p.grid_cols * p.splits));
  if (p.mode == SSI_CORR_BF16X6 || p.mode == SSI_CORR_F16X3) {
    const auto fn = p.mode == SSI_CORR_BF16X6 ? correlate_b6 : correlate_h3;
    hipError_t e = hipFuncSetAttribute((const void *)fn,
                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)p.lds_bytes);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(fn, grid, dim3(kThreads), p.lds_bytes, st, planes, l, n, p.lp, p.np, L,
                       p.split_len, partial, p.sa_stride, p.na_max, p.copy_stride, p.grid_rows,
                       p.grid_cols, p.splits);
    return hipGetLastError();
  }
  const bool vec = (ldy % 4 == 0) && ((uintptr_t)y % 16 == 0);
  const void *fn = vec ? (const void *)correlate_mfma<true> : (const void *)correlate_mfma<false>;
  if (p.lds_bytes > 65536) {
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)p.lds_bytes);
    if (e != hipSuccess) return e;
  }
  if (vec)
    hipLaunchKernelGGL(correlate_mfma<true>, grid, dim3(kThreads), p.lds_bytes, st, y, l, n,
                       ldy, L, p.split_len, partial, p.sa_stride, p.na_max, p.grid_rows,
                       p.grid_cols, p.splits);
  else
    hipLaunchKernelGGL(correlate_mfma<false>, grid, dim3(kThreads), p.lds_bytes, st, y, l, n,
                       ldy, L, p.split_len, partial, p.sa_stride, p.na_max, p.grid_rows,
                       p.grid_cols, p.splits);
  return hipGetLastError();
}

hipError_t launch_correlate_reduce(const CorrPlan &p, int l, int64_t n, int L,
                                   const double *partial, const uint16_t *planes, float *r,
                                   int *status, hipStream_t st) {
  const int64_t total = (int64_t)l * L * l;
  int blocks = (int)ceil_div<int64_t>(total, 256);
  if (blocks > 65535 * 8) blocks = 65535 * 8;
  hipLaunchKernelGGL(correlate_reduce, dim3(blocks), dim3(256), 0, st, partial, l, L,
                     p.splits, 1.0 / (double)n,
                     p.mode == SSI_CORR_F16X3 ? corr_exps(p, planes) : (const int *)nullptr, r,
                     status);
  return hipGetLastError();
}

hipError_t launch_correlate(const CorrPlan &p, const float *y, int l, int64_t n, int64_t ldy,
                            int L, double *partial, uint16_t *planes, float *r, int *status,
                            hipStream_t st) {
  hipError_t e = launch_correlate_split(p, y, l, n, ldy, planes, st);
  if (e == hipSuccess) e = launch_correlate_mfma(p, y, l, n, ldy, L, partial, planes, st);
  if (e != hipSuccess) return e;
  return launch_correlate_reduce(p, l, n, L, partial, planes, r, status, st);
}

}  // namespace ssi
