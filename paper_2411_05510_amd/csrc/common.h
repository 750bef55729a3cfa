// Shared device/host helpers for the SSI-COV kernels (gfx950 only).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

#define SSI_DEV __device__ __forceinline__

// Integer ceiling division on host and device.
template <typename T>
__host__ __device__ __forceinline__ T ceil_div(T a, T b) {
  return (a + b - 1) / b;
}

// Cross-lane reductions on DPP (VALU operand permutations inside a row of
// 16 lanes) rather than LDS-routed shuffles.  All lanes of the wave must be
// active.  dpp_d / dpp_i: the value of the lane that the DPP control CTRL
// selects within the caller's row: quad_perm [1,0,3,2] (0xB1) and [2,3,0,1]
// (0x4E) exchange lanes differing in bit 0 and bit 1, row_half_mirror (0x141)
// pairs the two quads of each half-row, row_mirror (0x140) the two halves.
template <int CTRL>
SSI_DEV int dpp_i(int v) {
  return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, false);
}
template <int CTRL>
SSI_DEV double dpp_d(double v) {
  const int lo = dpp_i<CTRL>(__double2loint(v)), hi = dpp_i<CTRL>(__double2hiint(v));
  return __hiloint2double(hi, lo);
}
// Sum over the 16 lanes of each row (lanes equal in bits 4..5); every lane of
// the row gets the same value.
SSI_DEV double row16_sum(double v) {
  v += dpp_d<0xB1>(v);
  v += dpp_d<0x4E>(v);
  v += dpp_d<0x141>(v);
  v += dpp_d<0x140>(v);
  return v;
}
// Sum over the four rows of the wave at this lane's position in its row
// (lanes l, l ^ 16, l ^ 32, l ^ 48); every lane gets its column's sum.
// v_permlane16_swap exchanges rows 0 <-> 1 and 2 <-> 3, v_permlane32_swap the
// two halves (VALU moves, no LDS); an FP64 value moves as two dwords.  With
// both operands equal, the swap's two results hold v and its partner.
SSI_DEV double rows4_sum(double v) {
  unsigned lo = __double2loint(v), hi = __double2hiint(v);
  const auto a = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
  const auto b = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
  const double s = __hiloint2double(b[0], a[0]) + __hiloint2double(b[1], a[1]);
  lo = __double2loint(s);
  hi = __double2hiint(s);
  const auto c = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
  const auto d = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
  return __hiloint2double(d[0], c[0]) + __hiloint2double(d[1], c[1]);
}
SSI_DEV double row16_max(double v) {
  v = fmax(v, dpp_d<0xB1>(v));
  v = fmax(v, dpp_d<0x4E>(v));
  v = fmax(v, dpp_d<0x141>(v));
  v = fmax(v, dpp_d<0x140>(v));
  return v;
}
SSI_DEV double row16_min(double v) {
  v = fmin(v, dpp_d<0xB1>(v));
  v = fmin(v, dpp_d<0x4E>(v));
  v = fmin(v, dpp_d<0x141>(v));
  v = fmin(v, dpp_d<0x140>(v));
  return v;
}
SSI_DEV int row16_max_i(int v) {
  v = max(v, dpp_i<0xB1>(v));
  v = max(v, dpp_i<0x4E>(v));
  v = max(v, dpp_i<0x141>(v));
  v = max(v, dpp_i<0x140>(v));
  return v;
}
SSI_DEV double lane_read_d(double v, int src) {
  return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), src),
                          __builtin_amdgcn_readlane(__double2loint(v), src));
}
// Wave-wide (64-lane) reductions: row reductions, then the four row results
// read from lanes 0, 16, 32, 48.  The result is wave-uniform.
SSI_DEV double wave_sum(double v) {
  v = row16_sum(v);
  return (lane_read_d(v, 0) + lane_read_d(v, 16)) + (lane_read_d(v, 32) + lane_read_d(v, 48));
}
SSI_DEV double wave_max(double v) {
  v = row16_max(v);
  return fmax(fmax(lane_read_d(v, 0), lane_read_d(v, 16)),
              fmax(lane_read_d(v, 32), lane_read_d(v, 48)));
}
SSI_DEV double wave_min(double v) {
  v = row16_min(v);
  return fmin(fmin(lane_read_d(v, 0), lane_read_d(v, 16)),
              fmin(lane_read_d(v, 32), lane_read_d(v, 48)));
}
SSI_DEV int wave_max_i(int v) {
  v = row16_max_i(v);
  return max(max(__builtin_amdgcn_readlane(v, 0), __builtin_amdgcn_readlane(v, 16)),
             max(__builtin_amdgcn_readlane(v, 32), __builtin_amdgcn_readlane(v, 48)));
}
// Block-wide sum over blockDim.x threads (multiple of 64, <= 1024) using a
// 16-entry shared scratch.  Every thread gets the total.
SSI_DEV double block_sum(double v, double *scratch16) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nw = blockDim.x >> 6;
  v = wave_sum(v);
  __syncthreads();
  if (lane == 0) scratch16[wave] = v;
  __syncthreads();
  double t = 0.0;
  for (int w = 0; w < nw; ++w) t += scratch16[w];
  return t;
}
