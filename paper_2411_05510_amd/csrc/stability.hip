// Stability analysis of the 3D stabilization diagram (Section 2.1 end and
// Section 2.3 step ii, Eq. (19)) on the poles ssi_identify wrote.
//
// quality_kernel (one wave per pole slot):
//   MPC = ((Sxx - Syy)^2 + 4 Sxy^2) / (Sxx + Syy)^2 with Sxx = |Re phi|^2,
//   Syy = |Im phi|^2, Sxy = Re phi . Im phi (1 for a mode whose components
//   are collinear in the complex plane);
//   MPD = mean over components, weighted by |phi_a|, of the angle between
//   phi_a and the principal line of the points (Re phi_a, Im phi_a) (the
//   first right singular vector of [Re phi, Im phi]), divided by pi/2 so
//   that it lies in [0, 1];
//   hard criteria: 0 < xi <= xi_max, MPC > mpc_min, MPD < mpd_max.
// soft_kernel (one wave per pole slot that passed the hard criteria):
//   stable along the order axis if some pole of the previous order of the
//   same lag that passed the hard criteria has relative f and xi differences
//   (|a - b| / max(a, b)) within alpha_f and alpha_xi and 1 - MAC within
//   alpha_mac; along the lag axis likewise with the same order of the
//   previous lag.  Stable: hard criteria and (order axis or lag axis).
// Everything is FP64 (mode shapes are widened from their FP32 storage).
#include <mutex>

#include "common.h"
#include "kernels.h"

namespace {

// Fixed device array for ssi_stability_noalloc: the hard-criteria verdict of
// every pole slot (one byte per slot), for callers that cannot allocate.
// Each GPU the library runs on holds its own copy until the process ends.
constexpr size_t kNoAllocSlots = size_t(4) << 20;
__device__ __align__(256) uint8_t scratch[kNoAllocSlots];

// Device address of `scratch` per device, from hipGetSymbolAddress.  In host
// code the array's name is only a host-side stand-in, never a device address.
constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
uint8_t *g_scratch_dev[kMaxScratchDevices] = {};

constexpr double kHalfPi = 1.5707963267948966;

SSI_DEV int pole_offset_of(int o, int nmin, int step) {
  int off = 0;
  for (int i = 0; i < o; ++i) off += (nmin + i * step) / 2;
  return off;
}

// Decode a flat slot index of one lag into (order, pole) by scanning the
// order offsets; returns false for slots beyond the order's count.
SSI_DEV bool slot_order(int s, int n_orders, int nmin, int step, const int32_t *count, int *o_out,
                        int *p_out) {
  int off = 0;
  for (int o = 0; o < n_orders; ++o) {
    const int cap = (nmin + o * step) / 2;
    if (s < off + cap) {
      *o_out = o;
      *p_out = s - off;
      return s - off < count[o];
    }
    off += cap;
  }
  return false;
}

}  // namespace

__global__ void __launch_bounds__(256)
quality_kernel(int n_lags, int n_orders, int nmin, int step, int pole_cap, int l,
               const int32_t *__restrict__ count, const double *__restrict__ xi,
               const float *__restrict__ phi, double xi_max, double mpc_min, double mpd_max,
               double *__restrict__ mpc_out, double *__restrict__ mpd_out,
               uint8_t *__restrict__ hc_out) {
  const int lane = threadIdx.x & 63;
  const int64_t total = (int64_t)n_lags * pole_cap;
  const int64_t waves = (int64_t)gridDim.x * (blockDim.x >> 6);
  for (int64_t w = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); w < total;
       w += waves) {
    const int lag = (int)(w / pole_cap), s = (int)(w - (int64_t)lag * pole_cap);
    int o, p;
    if (!slot_order(s, n_orders, nmin, step, count + (int64_t)lag * n_orders, &o, &p)) {
      if (lane == 0) {                 // empty slot
        mpc_out[w] = 0.0;
        mpd_out[w] = 0.0;
        hc_out[w] = 0;
      }
      continue;
    }
    const float *ph = phi + (size_t)w * l * 2;
    double sxx = 0.0, syy = 0.0, sxy = 0.0;
    for (int a = lane; a < l; a += 64) {
      const double re = ph[2 * a], im = ph[2 * a + 1];
      sxx += re * re;
      syy += im * im;
      sxy += re * im;
    }
    sxx = wave_sum(sxx);
    syy = wave_sum(syy);
    sxy = wave_sum(sxy);
    const double tr = sxx + syy;
    const double mpc = tr > 0.0 ? ((sxx - syy) * (sxx - syy) + 4.0 * sxy * sxy) / (tr * tr) : 0.0;
    // principal direction of the 2 x 2 Gram matrix [[sxx, sxy], [sxy, syy]]
    const double half = 0.5 * (sxx - syy);
    const double lam = 0.5 * tr + sqrt(half * half + sxy * sxy);
    double dx, dy;
    if (sxy == 0.0) {
      dx = sxx >= syy ? 1.0 : 0.0;
      dy = sxx >= syy ? 0.0 : 1.0;
    } else if (sxx >= syy) {
      dx = lam - syy;
      dy = sxy;
    } else {
      dx = sxy;
      dy = lam - sxx;
    }
    const double dn = sqrt(dx * dx + dy * dy);
    dx /= dn;
    dy /= dn;
    double wsum = 0.0, asum = 0.0;
    for (int a = lane; a < l; a += 64) {
      const double re = ph[2 * a], im = ph[2 * a + 1];
      const double r = sqrt(re * re + im * im);
      if (r > 0.0) {
        const double c = fmin(1.0, fabs(re * dx + im * dy) / r);
        wsum += r;
        asum += r * acos(c);
      }
    }
    wsum = wave_sum(wsum);
    asum = wave_sum(asum);
    const double mpd = wsum > 0.0 ? asum / wsum / kHalfPi : 1.0;
    if (lane == 0) {
      const double x = xi[w];
      const bool hc = x > 0.0 && x <= xi_max && mpc > mpc_min && mpd < mpd_max;
      mpc_out[w] = mpc;
      mpd_out[w] = mpd;
      hc_out[w] = hc ? 1 : 0;
    }
  }
}

__global__ void __launch_bounds__(256)
soft_kernel(int n_lags, int n_orders, int nmin, int step, int pole_cap, int l,
            const int32_t *__restrict__ count, const double *__restrict__ f,
            const double *__restrict__ xi, const float *__restrict__ phi, double alpha_f,
            double alpha_xi, double alpha_mac, const uint8_t *__restrict__ hc,
            uint8_t *__restrict__ flags) {
  const int lane = threadIdx.x & 63;
  const int64_t total = (int64_t)n_lags * pole_cap;
  const int64_t waves = (int64_t)gridDim.x * (blockDim.x >> 6);
  for (int64_t w = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); w < total;
       w += waves) {
    const int lag = (int)(w / pole_cap), s = (int)(w - (int64_t)lag * pole_cap);
    int o, p;
    const bool valid = slot_order(s, n_orders, nmin, step, count + (int64_t)lag * n_orders, &o, &p);
    const uint8_t mine = valid ? hc[w] : 0;
    if (!(mine & 1)) {
      if (lane == 0) flags[w] = mine;
      continue;
    }
    const double fi = f[w], xii = xi[w];
    const float *pi = phi + (size_t)w * l * 2;
    double nii = 0.0;
    for (int a = lane; a < l; a += 64) {
      const double re = pi[2 * a], im = pi[2 * a + 1];
      nii += re * re + im * im;
    }
    nii = wave_sum(nii);
    bool axis[2] = {false, false};
    for (int ax = 0; ax < 2; ++ax) {
      // ax 0: previous order, same lag; ax 1: same order, previous lag
      const int lj = ax == 0 ? lag : lag - 1;
      const int oj = ax == 0 ? o - 1 : o;
      if (lj < 0 || oj < 0) continue;
      const int cnt = count[(int64_t)lj * n_orders + oj];
      const int64_t base = (int64_t)lj * pole_cap + pole_offset_of(oj, nmin, step);
      for (int q = 0; q < cnt && !axis[ax]; ++q) {
        const int64_t j = base + q;
        if (!(hc[j] & 1)) continue;
        const double fj = f[j], xj = xi[j];
        if (fabs(fi - fj) / fmax(fi, fj) > alpha_f) continue;
        if (fabs(xii - xj) / fmax(xii, xj) > alpha_xi) continue;
        const float *pj = phi + (size_t)j * l * 2;
        double cr = 0.0, ci = 0.0, njj = 0.0;
        for (int a = lane; a < l; a += 64) {
          const double ar = pi[2 * a], ai = pi[2 * a + 1];
          const double br = pj[2 * a], bi = pj[2 * a + 1];
          cr += ar * br + ai * bi;       // conj(a) b
          ci += ar * bi - ai * br;
          njj += br * br + bi * bi;
        }
        cr = wave_sum(cr);
        ci = wave_sum(ci);
        njj = wave_sum(njj);
        const double mac = (cr * cr + ci * ci) / (nii * njj);
        if (1.0 - mac <= alpha_mac) axis[ax] = true;
      }
    }
    if (lane == 0)
      flags[w] = (uint8_t)(mine | (axis[0] ? 2 : 0) | (axis[1] ? 4 : 0) |
                           ((axis[0] || axis[1]) ? 8 : 0));
  }
}

namespace ssi {

size_t noalloc_stability_slots() { return kNoAllocSlots; }

// The caller has made `device` current.  Looks the address up once per
// device; later calls return the cached pointer.
hipError_t noalloc_scratch(int device, uint8_t **ptr) {
  if (device < 0 || device >= kMaxScratchDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[device]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_dev[device] = static_cast<uint8_t *>(p);
  }
  *ptr = g_scratch_dev[device];
  return hipSuccess;
}

hipError_t launch_stability(const StabilityArgs &a, hipStream_t st) {
  const int64_t total = (int64_t)a.n_lags * a.pole_cap;
  const int blocks = (int)std::max<int64_t>(1, std::min<int64_t>(ceil_div<int64_t>(total, 4), 4096));
  hipLaunchKernelGGL(quality_kernel, dim3(blocks), dim3(256), 0, st, a.n_lags, a.n_orders,
                     a.nmin, a.step, a.pole_cap, a.l, a.count, a.xi, a.phi, a.xi_max, a.mpc_min,
                     a.mpd_max, a.mpc, a.mpd, a.hc);
  hipLaunchKernelGGL(soft_kernel, dim3(blocks), dim3(256), 0, st, a.n_lags, a.n_orders, a.nmin,
                     a.step, a.pole_cap, a.l, a.count, a.f, a.xi, a.phi, a.alpha_f, a.alpha_xi,
                     a.alpha_mac, a.hc, a.flags);
  return hipGetLastError();
}

}  // namespace ssi
