// Block-Toeplitz assembly, Eq. (6):
//   T[r l + a][c l + b] = R_{jb + r - c}[a][b],  0 <= r, c < jb,
// with R_j stored at r_stack[(j - 1) l l + a l + b].
//
// A pure HBM write stream (m^2 floats) whose source, the 2 jb - 1 blocks of R,
// stays in L2 / Infinity Cache.  A workgroup covers 2048 floats of one row;
// in each of its two 16-byte store instructions the lanes of a wave write
// consecutive float4s, so every store instruction of a wave is one contiguous
// 1 KiB run of full cache lines.  Measured at m = 10800 with 256 threads: two
// stores per thread 6.0-6.4 TB/s, four 5.5-5.6, one 4.9-5.1.  The stores carry
// the nontemporal hint: T is written once and read back only by the next
// kernel, after far more data than the caches hold has passed (4.1 TB/s
// without it).  The vector path needs l, ldt and both
// pointers 16-byte aligned (a float4 then never straddles two blocks);
// otherwise a scalar path is used.
#include "common.h"
#include "kernels.h"

namespace {

constexpr int kVecPerThread = 2;                 // float4 stores per thread
constexpr int kThreads = 256;
constexpr int kFloatsPerBlock = kThreads * kVecPerThread * 4;

}  // namespace

__global__ void __launch_bounds__(kThreads)
toeplitz_vec4(const float *__restrict__ r, int l, int jb, float *__restrict__ t,
              int64_t ldt, int blocks_per_row) {
  const int m = jb * l;
  const int row = blockIdx.x / blocks_per_row;
  const int cblk = blockIdx.x - row * blocks_per_row;
  const int rb = row / l, a = row - rb * l;
  const float *rrow = r + (int64_t)a * l;       // row a of every block
  float *dst = t + (int64_t)row * ldt;
#pragma unroll
  for (int v = 0; v < kVecPerThread; ++v) {
    const int x = cblk * kFloatsPerBlock + (v * kThreads + (int)threadIdx.x) * 4;
    if (x < m) {
      const int cb = x / l, b = x - cb * l;
      const int blk = jb + rb - cb - 1;          // R_{jb + r - c} -> index j - 1
      const f32x4 val = *reinterpret_cast<const f32x4 *>(rrow + (int64_t)blk * l * l + b);
      __builtin_nontemporal_store(val, reinterpret_cast<f32x4 *>(dst + x));
    }
  }
}

__global__ void __launch_bounds__(kThreads)
toeplitz_scalar(const float *__restrict__ r, int l, int jb, float *__restrict__ t,
                int64_t ldt) {
  const int m = jb * l;
  const int row = blockIdx.x;
  const int rb = row / l, a = row - rb * l;
  for (int x = threadIdx.x; x < m; x += kThreads) {
    const int cb = x / l, b = x - cb * l;
    t[(int64_t)row * ldt + x] = r[(int64_t)(jb + rb - cb - 1) * l * l + (int64_t)a * l + b];
  }
}

namespace ssi {

hipError_t launch_toeplitz(const float *r, int l, int jb, float *t, int64_t ldt,
                           hipStream_t st) {
  const int m = jb * l;
  const bool vec = (l % 4 == 0) && (ldt % 4 == 0) &&
                   ((uintptr_t)r % 16 == 0) && ((uintptr_t)t % 16 == 0);
  if (vec) {
    const int bpr = ceil_div(m, kFloatsPerBlock);
    hipLaunchKernelGGL(toeplitz_vec4, dim3((unsigned)((int64_t)bpr * m)), dim3(kThreads), 0,
                       st, r, l, jb, t, ldt, bpr);
  } else {
    hipLaunchKernelGGL(toeplitz_scalar, dim3(m), dim3(kThreads), 0, st, r, l, jb, t, ldt);
  }
  return hipGetLastError();
}

}  // namespace ssi
