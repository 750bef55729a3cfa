// Small dense FP64 factorizations on one workgroup.
//
// An n x n FP64 matrix of the sizes used here (ell = k + p around 220, up to
// 392 KiB) does not fit in the 160 KiB LDS of a CU, so it is distributed over
// 512 threads that form a 16 x 32 grid: thread (tr, tc) owns the entries
// (tr + 16 p, tc + 32 q).  The 16 threads of one grid column are 16
// consecutive lanes, so sums along a matrix column are lane shuffles, and LDS
// only broadcasts one row or column per step.  Two storage policies share the
// code:
//   registers   (n <= 224): 14 x 7 entries per thread, the fast path;
//   global      (n <= 1024): 64 x 32 entries per thread in thread-private,
//               lane-interleaved (coalesced) scratch, for the full SVD of
//               larger Toeplitz matrices.
// All per-entry guards are selects on loads that are always in bounds, so the
// register tile stays in registers.
//
//   chol + tri_inv:  (G + s I) = L L^T, then R^{-1} = (L^{-1})^T (upper).
//                    Used by CholeskyQR and the shift least squares.
//   sym_eig:         symmetric eigen-decomposition: Householder
//                    tridiagonalisation, eigenvalues by Sturm bisection,
//                    eigenvectors by inverse iteration on the tridiagonal,
//                    reflectors applied back.  Eigenvalues descending.
#include "common.h"
#include "kernels.h"

namespace {

constexpr int kThreads = 512;
constexpr int kWaves = kThreads / 64;

SSI_DEV int row_of(int tr, int p) { return tr + 16 * p; }
SSI_DEV int col_of(int tc, int q) { return tc + 32 * q; }

SSI_DEV double sel(bool c, double v) { return c ? v : 0.0; }

// Sum over the 16 lanes of a grid column (lanes differ only in bits 0..3).
SSI_DEV double col_group_sum(double v) {
  v += __shfl_xor(v, 1, 64);
  v += __shfl_xor(v, 2, 64);
  v += __shfl_xor(v, 4, 64);
  v += __shfl_xor(v, 8, 64);
  return v;
}

SSI_DEV double block_sum_all(double v, double *red) {
  v = wave_sum(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double t = 0.0;
#pragma unroll
  for (int w = 0; w < kWaves; ++w) t += red[w];
  return t;
}

// Entries owned by one thread: registers or lane-interleaved global scratch.
template <int TP, int TQ, bool GM>
struct Tile {
  double r[GM ? 1 : TP][GM ? 1 : TQ];
  double *gp;   // GM: slot (p, q) at gp[(p * TQ + q) * kThreads]
  // (p, q) must be compile-time after unrolling in register mode
  SSI_DEV double &operator()(int p, int q) {
    if constexpr (GM) return gp[(size_t)(p * TQ + q) * kThreads];
    else return r[p][q];
  }
  // column index qr known only at run time: select, never index registers
  SSI_DEV double getq(int p, int qr) {
    if constexpr (GM) return gp[(size_t)(p * TQ + qr) * kThreads];
    double v = 0.0;
#pragma unroll
    for (int q = 0; q < TQ; ++q) v = (q == qr) ? r[p][q] : v;
    return v;
  }
  SSI_DEV void setq(int p, int qr, double v) {
    if constexpr (GM) {
      gp[(size_t)(p * TQ + qr) * kThreads] = v;
    } else {
#pragma unroll
      for (int q = 0; q < TQ; ++q) r[p][q] = (q == qr) ? v : r[p][q];
    }
  }
  // row index pr known only at run time
  SSI_DEV double getp(int pr, int q) {
    if constexpr (GM) return gp[(size_t)(pr * TQ + q) * kThreads];
    double v = 0.0;
#pragma unroll
    for (int p = 0; p < TP; ++p) v = (p == pr) ? r[p][q] : v;
    return v;
  }
  SSI_DEV void setp(int pr, int q, double v) {
    if constexpr (GM) {
      gp[(size_t)(pr * TQ + q) * kThreads] = v;
    } else {
#pragma unroll
      for (int p = 0; p < TP; ++p) r[p][q] = (p == pr) ? v : r[p][q];
    }
  }
};

template <int TP, int TQ>
struct Geo {
  static constexpr int kN = (16 * TP < 32 * TQ) ? 16 * TP : 32 * TQ;
};

}  // namespace

// ---------------------------------------------------------------- Cholesky
// Lower Cholesky factor L (into Lws, ld n) of G + shift_rel tr(G) I.
// status bit 0 is set on a non-positive pivot.
template <int TP, int TQ, bool GM>
__global__ void __launch_bounds__(kThreads)
chol_kernel(const double *__restrict__ G, int64_t ldg, int n, double shift_rel,
            double *__restrict__ Lws, double *__restrict__ tile_ws, int *__restrict__ status) {
  constexpr int kN = Geo<TP, TQ>::kN;
  constexpr int UP = GM ? 1 : TP, UQ = GM ? 1 : TQ;
  __shared__ double colbuf[kN];
  __shared__ double red[kWaves];
  __shared__ double piv;
  __shared__ int bad;
  const int t = threadIdx.x, tr = t & 15, tc = t >> 4;
  Tile<TP, TQ, GM> g;
  g.gp = tile_ws + t;
  double trace_part = 0.0;
#pragma unroll UP
  for (int p = 0; p < TP; ++p)
#pragma unroll UQ
    for (int q = 0; q < TQ; ++q) {
      const int i = row_of(tr, p), j = col_of(tc, q);
      const double v = G[(int64_t)min(i, n - 1) * ldg + min(j, n - 1)];
      g(p, q) = sel(i < n && j < n, v);
      trace_part += sel(i == j && i < n, v);
    }
  if (t == 0) bad = 0;
  const double shift = shift_rel * block_sum_all(trace_part, red);
#pragma unroll UP
  for (int p = 0; p < TP; ++p)
#pragma unroll UQ
    for (int q = 0; q < TQ; ++q)
      g(p, q) += sel(row_of(tr, p) == col_of(tc, q) && row_of(tr, p) < n, shift);

  for (int k = 0; k < n; ++k) {
    const int kq = k >> 5;
    if (tr == (k & 15) && tc == (k & 31)) {
      double d = 0.0;
#pragma unroll UP
      for (int p = 0; p < TP; ++p) d += sel(row_of(tr, p) == k, g.getq(p, kq));
      if (!(d > 0.0)) {
        bad = 1;
        d = 1e-300;
      }
      piv = sqrt(d);
    }
    __syncthreads();
    const double pv = piv, rpv = 1.0 / pv;
    if (tc == (k & 31)) {
#pragma unroll UP
      for (int p = 0; p < TP; ++p) {
        const int i = row_of(tr, p);
        const double nv = (i == k) ? pv : g.getq(p, kq) * rpv;
        if (i >= k && i < n) {
          g.setq(p, kq, nv);
          colbuf[i] = nv;
        }
      }
    }
    __syncthreads();
    double cj[TQ];
#pragma unroll UQ
    for (int q = 0; q < TQ; ++q) {
      const int j = col_of(tc, q);
      cj[q] = sel(j > k && j < n, colbuf[min(j, kN - 1)]);
    }
#pragma unroll UP
    for (int p = 0; p < TP; ++p) {
      const int i = row_of(tr, p);
      if (GM && (i <= k || i >= n)) continue;
      const double ci = sel(i > k && i < n, colbuf[min(i, kN - 1)]);
#pragma unroll UQ
      for (int q = 0; q < TQ; ++q) g(p, q) -= ci * cj[q];
    }
  }
#pragma unroll UP
  for (int p = 0; p < TP; ++p)
#pragma unroll UQ
    for (int q = 0; q < TQ; ++q) {
      const int i = row_of(tr, p), j = col_of(tc, q);
      if (i < n && j <= i) Lws[(int64_t)i * n + j] = g(p, q);
    }
  if (t == 0 && bad) atomicOr(status, 1);
}

// X = L^{-1} for the lower-triangular L in Lws (ld n); writes Rinv = X^T.
template <int TP, int TQ, bool GM>
__global__ void __launch_bounds__(kThreads)
tri_inv_kernel(int n, const double *__restrict__ Lws, double *__restrict__ Rinv, int64_t ldr,
               double *__restrict__ tile_ws) {
  constexpr int kN = Geo<TP, TQ>::kN;
  constexpr int UP = GM ? 1 : TP, UQ = GM ? 1 : TQ;
  __shared__ double rowbuf[kN];
  __shared__ double lcol[8][kN];
  const int t = threadIdx.x, tr = t & 15, tc = t >> 4;
  Tile<TP, TQ, GM> g;
  g.gp = tile_ws + t;
#pragma unroll UP
  for (int p = 0; p < TP; ++p)
#pragma unroll UQ
    for (int q = 0; q < TQ; ++q)
      g(p, q) = sel(row_of(tr, p) == col_of(tc, q) && row_of(tr, p) < n, 1.0);
  for (int k = 0; k < n; ++k) {
    const int kp = k >> 4, kk = k & 7;
    if (kk == 0) {
      for (int idx = t; idx < 8 * kN; idx += kThreads) {
        const int c = idx / kN, i = idx - c * kN;
        const int col = k + c;
        lcol[c][i] = sel(col < n && i >= col && i < n,
                         Lws[(int64_t)min(i, n - 1) * n + min(col, n - 1)]);
      }
      __syncthreads();
    }
    const double rlkk = 1.0 / lcol[kk][k];
    if (tr == (k & 15)) {
#pragma unroll UQ
      for (int q = 0; q < TQ; ++q) {
        const int j = col_of(tc, q);
        const double v = g.getp(kp, q) * rlkk;
        g.setp(kp, q, v);
        if (j < n) rowbuf[j] = v;
      }
    }
    __syncthreads();
    double rj[TQ];
#pragma unroll UQ
    for (int q = 0; q < TQ; ++q) {
      const int j = col_of(tc, q);
      rj[q] = sel(j <= k && j < n, rowbuf[min(j, kN - 1)]);
    }
#pragma unroll UP
    for (int p = 0; p < TP; ++p) {
      const int i = row_of(tr, p);
      if (GM && (i <= k || i >= n)) continue;
      const double li = sel(i > k && i < n, lcol[kk][min(i, kN - 1)]);
#pragma unroll UQ
      for (int q = 0; q < TQ; ++q) g(p, q) -= li * rj[q];
    }
    __syncthreads();
  }
#pragma unroll UP
  for (int p = 0; p < TP; ++p)
#pragma unroll UQ
    for (int q = 0; q < TQ; ++q) {
      const int i = row_of(tr, p), j = col_of(tc, q);
      if (i < n && j < n) Rinv[(int64_t)j * ldr + i] = (i >= j) ? g(p, q) : 0.0;
    }
}

// ------------------------------------------------------------ sym eigen
// Scratch layout (doubles): vref[kN][kN] | tau[kN] | d[kN] | e[kN] | lu[5][kN][kN]
template <int TP, int TQ, bool GM>
__global__ void __launch_bounds__(kThreads)
sym_tridiag_kernel(const double *__restrict__ G, int64_t ldg, int n, double *__restrict__ ws,
                   double *__restrict__ tile_ws) {
  constexpr int kN = Geo<TP, TQ>::kN;
  constexpr int UP = GM ? 1 : TP, UQ = GM ? 1 : TQ;
  __shared__ double vbuf[kN];
  __shared__ double pbuf[kN];
  __shared__ double red[kWaves];
  __shared__ double stau;
  const int t = threadIdx.x, tr = t & 15, tc = t >> 4;
  double *vref = ws;
  double *tauv = ws + (size_t)kN * kN;
  double *dd = tauv + kN;
  double *ee = dd + kN;
  Tile<TP, TQ, GM> g;
  g.gp = tile_ws + t;
#pragma unroll UP
  for (int p = 0; p < TP; ++p)
#pragma unroll UQ
    for (int q = 0; q < TQ; ++q) {
      const int i = row_of(tr, p), j = col_of(tc, q);
      g(p, q) = sel(i < n && j < n, G[(int64_t)min(i, n - 1) * ldg + min(j, n - 1)]);
    }

  for (int k = 0; k + 2 < n; ++k) {
    const int kq = k >> 5;
    if (tc == (k & 31)) {
      // Householder vector of column k below the diagonal
      double s2 = 0.0, x1 = 0.0, dk = 0.0;
#pragma unroll UP
      for (int p = 0; p < TP; ++p) {
        const int i = row_of(tr, p);
        const double v = g.getq(p, kq);
        x1 += sel(i == k + 1, v);
        s2 += sel(i > k + 1 && i < n, v * v);
        dk += sel(i == k, v);
      }
      s2 = col_group_sum(s2);
      x1 = col_group_sum(x1);
      dk = col_group_sum(dk);
      double tau = 0.0, alpha = x1, v1 = 0.0;
      if (s2 > 0.0) {
        alpha = -copysign(sqrt(x1 * x1 + s2), x1);
        v1 = x1 - alpha;
        tau = 2.0 / (s2 + v1 * v1);
      }
#pragma unroll UP
      for (int p = 0; p < TP; ++p) {
        const int i = row_of(tr, p);
        if (i < n) {
          const double v = (i == k + 1) ? v1 : sel(i > k + 1, g.getq(p, kq));
          vbuf[i] = v;
          vref[(size_t)k * kN + i] = v;
        }
      }
      if (tr == 0) {
        stau = tau;
        tauv[k] = tau;
        dd[k] = dk;
        ee[k] = alpha;
      }
    }
    __syncthreads();
    const double tau = stau;
    if (tau != 0.0) {
      // p = tau G v by column sums (G symmetric); K = v^T p
      double sq[TQ];
#pragma unroll UQ
      for (int q = 0; q < TQ; ++q) sq[q] = 0.0;
#pragma unroll UP
      for (int p = 0; p < TP; ++p) {
        const int i = row_of(tr, p);
        if (GM && (i <= k || i >= n)) continue;
        const double vi = sel(i > k && i < n, vbuf[min(i, kN - 1)]);
#pragma unroll UQ
        for (int q = 0; q < TQ; ++q) sq[q] += g(p, q) * vi;
      }
      double kpart = 0.0;
#pragma unroll UQ
      for (int q = 0; q < TQ; ++q) {
        const double s = tau * col_group_sum(sq[q]);
        const int j = col_of(tc, q);
        if (tr == 0 && j < n) {
          pbuf[j] = s;
          kpart += s * sel(j > k, vbuf[j]);
        }
      }
      const double K = block_sum_all(kpart, red);
      const double c = 0.5 * tau * K;
      // G -= v w^T + w v^T with w = p - c v
      double vj[TQ], wj[TQ];
#pragma unroll UQ
      for (int q = 0; q < TQ; ++q) {
        const int j = col_of(tc, q);
        vj[q] = sel(j > k && j < n, vbuf[min(j, kN - 1)]);
        wj[q] = sel(j < n, pbuf[min(j, kN - 1)] - c * vj[q]);
      }
#pragma unroll UP
      for (int p = 0; p < TP; ++p) {
        const int i = row_of(tr, p);
        if (GM && i >= n) continue;
        const double vi = sel(i > k && i < n, vbuf[min(i, kN - 1)]);
        const double wi = sel(i < n, pbuf[min(i, kN - 1)] - c * vi);
#pragma unroll UQ
        for (int q = 0; q < TQ; ++q) g(p, q) -= vi * wj[q] + wi * vj[q];
      }
    }
    __syncthreads();
  }
  // trailing 2 x 2 (or 1 x 1) block
#pragma unroll UP
  for (int p = 0; p < TP; ++p)
#pragma unroll UQ
    for (int q = 0; q < TQ; ++q) {
      const int i = row_of(tr, p), j = col_of(tc, q);
      if (i < n && i == j && i >= n - 2) dd[i] = g(p, q);
      if (n >= 2 && i == n - 1 && j == n - 2) ee[n - 2] = g(p, q);
    }
}

namespace {

// Number of eigenvalues of the tridiagonal (d, e2 = e^2) smaller than x.
SSI_DEV int sturm_count(const double *d, const double *e2, int n, double x, double pivmin) {
  int cnt = 0;
  double q = d[0] - x;
  if (fabs(q) < pivmin) q = -pivmin;
  cnt += q < 0.0;
  for (int j = 1; j < n; ++j) {
    q = d[j] - x - e2[j - 1] / q;
    if (fabs(q) < pivmin) q = -pivmin;
    cnt += q < 0.0;
  }
  return cnt;
}

SSI_DEV double hash_unit(uint32_t a, uint32_t b) {
  uint32_t h = a * 0x9E3779B1u ^ (b + 0x7F4A7C15u) * 0x85EBCA77u;
  h ^= h >> 15;
  h *= 0x2C1B3C6Du;
  h ^= h >> 12;
  return 0.5 + (double)(h & 0xFFFF) * (1.0 / 65536.0);   // in [0.5, 1.5)
}

SSI_DEV double block_max_n(double v, double *red, int nt) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double r = red[0];
  for (int w = 1; w < (nt >> 6); ++w) r = fmax(r, red[w]);
  return r;
}

}  // namespace

// Eigenpairs of the tridiagonal (d, e): eigenvalue t (descending) by
// bisection, its eigenvector by inverse iteration; one thread per eigenvalue.
template <int KN>
__global__ void __launch_bounds__(1024)
sym_tridiag_eig_kernel(int n, double *__restrict__ evals, double *__restrict__ evecs,
                       int64_t ldv, double *__restrict__ ws) {
  __shared__ double dd[KN];
  __shared__ double ee[KN];
  __shared__ double e2[KN];
  __shared__ double red[16];
  const int t0 = threadIdx.x, nt = blockDim.x;
  const double *tauv = ws + (size_t)KN * KN;
  double *lu = ws + (size_t)KN * KN + 3 * KN;
  for (int i = t0; i < n; i += nt) {
    dd[i] = tauv[KN + i];
    ee[i] = tauv[2 * KN + i];
  }
  __syncthreads();
  for (int i = t0; i < n; i += nt) e2[i] = (i < n - 1) ? ee[i] * ee[i] : 0.0;
  __syncthreads();
  double lo_part = 1e300, hi_part = -1e300, emax_part = 0.0;
  for (int i = t0; i < n; i += nt) {
    const double r = (i > 0 ? fabs(ee[i - 1]) : 0.0) + (i < n - 1 ? fabs(ee[i]) : 0.0);
    lo_part = fmin(lo_part, dd[i] - r);
    hi_part = fmax(hi_part, dd[i] + r);
    if (i < n - 1) emax_part = fmax(emax_part, e2[i]);
  }
  const double glo = -block_max_n(-lo_part, red, nt);
  const double ghi = block_max_n(hi_part, red, nt);
  const double e2max = block_max_n(emax_part, red, nt);
  const double gnorm = fmax(fabs(glo), fabs(ghi));
  const double pivmin = 2.2250738585072014e-308 * fmax(1.0, e2max);
  const double span = ghi - glo;
  double *u0 = lu, *u1 = lu + (size_t)KN * KN, *u2 = lu + 2 * (size_t)KN * KN;
  double *ml = lu + 3 * (size_t)KN * KN, *xv = lu + 4 * (size_t)KN * KN;
  const double tiny = 2.220446049250313e-16 * fmax(gnorm, 1e-300);
  for (int t = t0; t < n; t += nt) {
    const int target = n - 1 - t;              // ascending index of the t-th largest
    double lo = glo - 1e-14 * span - 2.0 * pivmin, hi = ghi + 1e-14 * span + 2.0 * pivmin;
    for (int it = 0; it < 128; ++it) {
      const double mid = 0.5 * (lo + hi);
      if (hi - lo <= 2.0 * 2.220446049250313e-16 * fmax(fabs(lo), fabs(hi)) + pivmin ||
          mid <= lo || mid >= hi)
        break;
      if (sturm_count(dd, e2, n, mid, pivmin) > target) hi = mid;
      else lo = mid;
    }
    const double lam = 0.5 * (lo + hi);
    evals[t] = lam;

    // inverse iteration: LU with partial pivoting of T - lam I (a row swap is
    // marked by adding 4 to the multiplier, which is at most 1 in magnitude)
    double a = dd[0] - lam, b = (n > 1) ? ee[0] : 0.0, c = 0.0;
    for (int j = 0; j + 1 < n; ++j) {
      const double sub = ee[j];
      const double an = dd[j + 1] - lam;
      const double cn = (j + 2 < n) ? ee[j + 1] : 0.0;
      if (fabs(a) >= fabs(sub)) {
        const double aa = (fabs(a) < tiny) ? copysign(tiny, a == 0.0 ? 1.0 : a) : a;
        const double m = sub / aa;
        u0[(size_t)j * KN + t] = aa;
        u1[(size_t)j * KN + t] = b;
        u2[(size_t)j * KN + t] = c;
        ml[(size_t)j * KN + t] = m;
        a = an - m * b;
        b = cn - m * c;
        c = 0.0;
      } else {
        const double m = a / sub;
        u0[(size_t)j * KN + t] = sub;
        u1[(size_t)j * KN + t] = an;
        u2[(size_t)j * KN + t] = cn;
        ml[(size_t)j * KN + t] = m + 4.0;
        const double na = b - m * an, nb = c - m * cn;
        a = na;
        b = nb;
        c = 0.0;
      }
    }
    if (fabs(a) < tiny) a = copysign(tiny, a == 0.0 ? 1.0 : a);
    u0[(size_t)(n - 1) * KN + t] = a;
    u1[(size_t)(n - 1) * KN + t] = 0.0;
    u2[(size_t)(n - 1) * KN + t] = 0.0;
    for (int j = 0; j < n; ++j) xv[(size_t)j * KN + t] = hash_unit(t, j);
    for (int it = 0; it < 3; ++it) {
      for (int j = 0; j + 1 < n; ++j) {
        double m = ml[(size_t)j * KN + t];
        double bj = xv[(size_t)j * KN + t], bn = xv[(size_t)(j + 1) * KN + t];
        if (m > 2.0) {
          m -= 4.0;
          const double tmp = bj;
          bj = bn;
          bn = tmp;
        }
        xv[(size_t)j * KN + t] = bj;
        xv[(size_t)(j + 1) * KN + t] = bn - m * bj;
      }
      double x1 = 0.0, x2 = 0.0, nrm = 0.0;
      for (int j = n - 1; j >= 0; --j) {
        const double xj = (xv[(size_t)j * KN + t] - u1[(size_t)j * KN + t] * x1 -
                           u2[(size_t)j * KN + t] * x2) / u0[(size_t)j * KN + t];
        xv[(size_t)j * KN + t] = xj;
        x2 = x1;
        x1 = xj;
        nrm = fmax(nrm, fabs(xj));
      }
      const double inv = 1.0 / nrm;
      for (int j = 0; j < n; ++j) xv[(size_t)j * KN + t] *= inv;
    }
    double s = 0.0;
    for (int j = 0; j < n; ++j) s += xv[(size_t)j * KN + t] * xv[(size_t)j * KN + t];
    const double inv = 1.0 / sqrt(s);
    for (int j = 0; j < n; ++j) evecs[(int64_t)j * ldv + t] = xv[(size_t)j * KN + t] * inv;
  }
}

// V <- H_0 H_1 ... H_{n-3} V for the reflectors stored by sym_tridiag_kernel.
template <int TP, int TQ, bool GM>
__global__ void __launch_bounds__(kThreads)
sym_backtransform_kernel(int n, double *__restrict__ evecs, int64_t ldv,
                         const double *__restrict__ ws, double *__restrict__ tile_ws) {
  constexpr int kN = Geo<TP, TQ>::kN;
  constexpr int UP = GM ? 1 : TP, UQ = GM ? 1 : TQ;
  __shared__ double vbuf[kN];
  const int t = threadIdx.x, tr = t & 15, tc = t >> 4;
  const double *vref = ws;
  const double *tauv = ws + (size_t)kN * kN;
  Tile<TP, TQ, GM> g;
  g.gp = tile_ws + t;
#pragma unroll UP
  for (int p = 0; p < TP; ++p)
#pragma unroll UQ
    for (int q = 0; q < TQ; ++q) {
      const int i = row_of(tr, p), j = col_of(tc, q);
      g(p, q) = sel(i < n && j < n, evecs[(int64_t)min(i, n - 1) * ldv + min(j, n - 1)]);
    }
  for (int k = n - 3; k >= 0; --k) {
    for (int i = t; i < n; i += kThreads) vbuf[i] = (i > k) ? vref[(size_t)k * kN + i] : 0.0;
    __syncthreads();
    const double tau = tauv[k];
    if (tau != 0.0) {
      double sq[TQ];
#pragma unroll UQ
      for (int q = 0; q < TQ; ++q) sq[q] = 0.0;
#pragma unroll UP
      for (int p = 0; p < TP; ++p) {
        const int i = row_of(tr, p);
        if (GM && (i <= k || i >= n)) continue;
        const double vi = sel(i > k && i < n, vbuf[min(i, kN - 1)]);
#pragma unroll UQ
        for (int q = 0; q < TQ; ++q) sq[q] += vi * g(p, q);
      }
#pragma unroll UQ
      for (int q = 0; q < TQ; ++q) sq[q] = tau * col_group_sum(sq[q]);
#pragma unroll UP
      for (int p = 0; p < TP; ++p) {
        const int i = row_of(tr, p);
        if (GM && (i <= k || i >= n)) continue;
        const double vi = sel(i > k && i < n, vbuf[min(i, kN - 1)]);
#pragma unroll UQ
        for (int q = 0; q < TQ; ++q) g(p, q) -= vi * sq[q];
      }
    }
    __syncthreads();
  }
#pragma unroll UP
  for (int p = 0; p < TP; ++p)
#pragma unroll UQ
    for (int q = 0; q < TQ; ++q) {
      const int i = row_of(tr, p), j = col_of(tc, q);
      if (i < n && j < n) evecs[(int64_t)i * ldv + j] = g(p, q);
    }
}

namespace ssi {

namespace {
constexpr int kRegP = 14, kRegQ = 7;      // n <= 224
constexpr int kGlbP = 64, kGlbQ = 32;     // n <= 1024
constexpr int kRegN = Geo<kRegP, kRegQ>::kN;
constexpr int kGlbN = Geo<kGlbP, kGlbQ>::kN;

double *glb_tile(double *ws) {
  return ws + (size_t)kGlbN * kGlbN + 3 * kGlbN + 5 * (size_t)kGlbN * kGlbN;
}
}  // namespace

int dense_max_n() { return kGlbN; }

size_t dense_ws_doubles(int n) {
  const size_t kn = n <= kRegN ? kRegN : kGlbN;
  const size_t tile = n <= kRegN ? 0 : (size_t)kGlbP * kGlbQ * kThreads;
  return kn * kn + 3 * kn + 5 * kn * kn + tile;
}

hipError_t launch_chol_inv(const double *G, int64_t ldg, int n, double shift_rel, double *Rinv,
                           int64_t ldr, double *Lws, double *ws, int *status, hipStream_t st) {
  if (n <= kRegN) {
    hipLaunchKernelGGL((chol_kernel<kRegP, kRegQ, false>), dim3(1), dim3(kThreads), 0, st, G,
                       ldg, n, shift_rel, Lws, ws, status);
    hipLaunchKernelGGL((tri_inv_kernel<kRegP, kRegQ, false>), dim3(1), dim3(kThreads), 0, st, n,
                       Lws, Rinv, ldr, ws);
  } else {
    double *tile = glb_tile(ws);
    hipLaunchKernelGGL((chol_kernel<kGlbP, kGlbQ, true>), dim3(1), dim3(kThreads), 0, st, G,
                       ldg, n, shift_rel, Lws, tile, status);
    hipLaunchKernelGGL((tri_inv_kernel<kGlbP, kGlbQ, true>), dim3(1), dim3(kThreads), 0, st, n,
                       Lws, Rinv, ldr, tile);
  }
  return hipGetLastError();
}

hipError_t launch_sym_eig(const double *G, int64_t ldg, int n, double *evals, double *evecs,
                          int64_t ldv, double *ws, int *status, hipStream_t st) {
  (void)status;
  if (n <= kRegN) {
    hipLaunchKernelGGL((sym_tridiag_kernel<kRegP, kRegQ, false>), dim3(1), dim3(kThreads), 0,
                       st, G, ldg, n, ws, ws);
    hipLaunchKernelGGL((sym_tridiag_eig_kernel<kRegN>), dim3(1), dim3(256), 0, st, n, evals,
                       evecs, ldv, ws);
    hipLaunchKernelGGL((sym_backtransform_kernel<kRegP, kRegQ, false>), dim3(1),
                       dim3(kThreads), 0, st, n, evecs, ldv, ws, ws);
  } else {
    double *tile = glb_tile(ws);
    hipLaunchKernelGGL((sym_tridiag_kernel<kGlbP, kGlbQ, true>), dim3(1), dim3(kThreads), 0,
                       st, G, ldg, n, ws, tile);
    hipLaunchKernelGGL((sym_tridiag_eig_kernel<kGlbN>), dim3(1), dim3(1024), 0, st, n, evals,
                       evecs, ldv, ws);
    hipLaunchKernelGGL((sym_backtransform_kernel<kGlbP, kGlbQ, true>), dim3(1),
                       dim3(kThreads), 0, st, n, evecs, ldv, ws, tile);
  }
  return hipGetLastError();
}

}  // namespace ssi
