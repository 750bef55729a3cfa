// Gaussian test matrix Omega (Eq. (14)), drawn on the device.
//
// Philox-4x32-10 (Salmon et al., SC'11): 4-word counter, 2-word key, ten
// rounds of two 32x32->64-bit multiplies with word permutation and key XOR,
// key bumped by the Weyl constants between rounds.  Element e = i ell + c
// uses counter (lo(e/2), hi(e/2), stream, 0) and key (lo(seed), hi(seed)).
// Uniforms are (top 52 bits of a word pair + 1/2) * 2^-52, exact in FP64;
// Box-Muller gives r cos(2 pi u2) for even e and r sin(2 pi u2) for odd e.
#include "common.h"
#include "kernels.h"

namespace {

struct U4 { uint32_t x0, x1, x2, x3; };

SSI_DEV U4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                         uint32_t k0, uint32_t k1) {
  constexpr uint32_t kM0 = 0xD2511F53u, kM1 = 0xCD9E8D57u;
  constexpr uint32_t kW0 = 0x9E3779B9u, kW1 = 0xBB67AE85u;
#pragma unroll
  for (int rnd = 0; rnd < 10; ++rnd) {
    if (rnd) { k0 += kW0; k1 += kW1; }
    const uint32_t hi0 = __umulhi(kM0, c0), lo0 = kM0 * c0;
    const uint32_t hi1 = __umulhi(kM1, c2), lo1 = kM1 * c2;
    const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
  }
  return U4{c0, c1, c2, c3};
}

SSI_DEV double uniform52(uint32_t lo, uint32_t hi) {
  const uint64_t w = (((uint64_t)hi << 32) | lo) >> 12;
  return ((double)w + 0.5) * 0x1.0p-52;
}

}  // namespace

template <typename T>
__global__ void __launch_bounds__(256)
sketch_philox(uint64_t seed, uint32_t stream, int64_t m, int ell, T *__restrict__ omega,
              int64_t ldo) {
  const int64_t total = m * (int64_t)ell;
  const int64_t pairs = (total + 1) / 2;
  const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < pairs;
       g += (int64_t)gridDim.x * blockDim.x) {
    const U4 x = philox4x32_10((uint32_t)g, (uint32_t)((uint64_t)g >> 32), stream, 0u, k0, k1);
    const double u1 = uniform52(x.x0, x.x1), u2 = uniform52(x.x2, x.x3);
    const double rad = sqrt(-2.0 * log(u1));
    double sn, cs;
    sincos(2.0 * M_PI * u2, &sn, &cs);
    const int64_t e0 = 2 * g;
    {
      const int64_t i = e0 / ell, c = e0 - i * ell;
      omega[i * ldo + c] = (T)(rad * cs);
    }
    if (e0 + 1 < total) {
      const int64_t e1 = e0 + 1;
      const int64_t i = e1 / ell, c = e1 - i * ell;
      omega[i * ldo + c] = (T)(rad * sn);
    }
  }
}

namespace ssi {

namespace {
template <typename T>
hipError_t sketch_launch(uint64_t seed, uint32_t stream, int64_t m, int ell, T *omega,
                         int64_t ldo, hipStream_t st) {
  const int64_t pairs = (m * (int64_t)ell + 1) / 2;
  int64_t blocks = ceil_div<int64_t>(pairs, 256);
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(sketch_philox<T>, dim3((unsigned)blocks), dim3(256), 0, st, seed, stream, m,
                     ell, omega, ldo);
  return hipGetLastError();
}
}  // namespace

hipError_t launch_sketch(uint64_t seed, uint32_t stream, int64_t m, int ell, float *omega,
                         int64_t ldo, hipStream_t st) {
  return sketch_launch(seed, stream, m, ell, omega, ldo, st);
}

hipError_t launch_sketch(uint64_t seed, uint32_t stream, int64_t m, int ell, double *omega,
                         int64_t ldo, hipStream_t st) {
  return sketch_launch(seed, stream, m, ell, omega, ldo, st);
}

}  // namespace ssi
