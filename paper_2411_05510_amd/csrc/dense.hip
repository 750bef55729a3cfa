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
//   mid         (n <= 448): the matrix in global memory (L2-resident), coalesced
//               column passes and MFMA block updates (kernels below);
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
SSI_DEV double col_group_sum(double v) { return row16_sum(v); }

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
  // (p, q) must be compile-time after unrolling in register mode: a run-time
  // index into the register array would move it to scratch memory
  SSI_DEV double &operator()(int p, int q) {
    if constexpr (GM) return gp[(size_t)(p * TQ + q) * kThreads];
    else return r[p][q];
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
  __shared__ double colbuf[2][kN];
  __shared__ double red[kWaves];
  __shared__ int bad;
  const int t = threadIdx.x, tr = t & 15, tc = t >> 4;
  // blocks that hold entries of the n x n matrix (the global tile is sized
  // for n up to 1024; the register tile always covers all of its blocks)
  const int NPB = GM ? min(TP, (n + 15) / 16) : TP, NQB = GM ? min(TQ, (n + 31) / 32) : TQ;
  Tile<TP, TQ, GM> g;
  g.gp = tile_ws + t;
  double trace_part = 0.0;
#pragma unroll UP
  for (int p = 0; p < NPB; ++p)
#pragma unroll UQ
    for (int q = 0; q < NQB; ++q) {
      const int i = row_of(tr, p), j = col_of(tc, q);
      const double v = G[(int64_t)min(i, n - 1) * ldg + min(j, n - 1)];
      g(p, q) = sel(i < n && j < n, v);
      trace_part += sel(i == j && i < n, v);
    }
  if (t == 0) bad = 0;
  const double shift = shift_rel * block_sum_all(trace_part, red);
#pragma unroll UP
  for (int p = 0; p < NPB; ++p)
#pragma unroll UQ
    for (int q = 0; q < NQB; ++q)
      g(p, q) += sel(row_of(tr, p) == col_of(tc, q) && row_of(tr, p) < n, shift);

  // Column k lives in column block kq = k / 32.  The block loop is unrolled in
  // register mode, so the pivot column's registers are compile-time indices;
  // row blocks above the pivot and blocks strictly above the diagonal are
  // never touched again and are skipped.  The 16 lanes that own column k (one
  // row of one wave) take the diagonal entry by a row sum, scale the column
  // and publish it in colbuf[k & 1]: one workgroup barrier per column, the
  // other buffer still being read by threads finishing column k - 1.
#pragma unroll UQ
  for (int kq = 0; kq < NQB; ++kq) {
    const int k0 = 32 * kq, k1 = min(k0 + 32, n);
    for (int k = k0; k < k1; ++k) {
      double *cb = colbuf[k & 1];
      if (tc == (k & 31)) {
        double dpart = 0.0;
#pragma unroll UP
        for (int p = 0; p < NPB; ++p) {
          if (p < 2 * kq) continue;
          dpart += sel(row_of(tr, p) == k, g(p, kq));
        }
        double d = row16_sum(dpart);           // the diagonal entry, in all 16 lanes
        if (!(d > 0.0)) {
          bad = 1;
          d = 1e-300;
        }
        const double pv = sqrt(d), rpv = 1.0 / pv;
#pragma unroll UP
        for (int p = 0; p < NPB; ++p) {
          if (p < 2 * kq) continue;
          const int i = row_of(tr, p);
          const double nv = (i == k) ? pv : g(p, kq) * rpv;
          if (i >= k && i < n) {
            g(p, kq) = nv;
            cb[i] = nv;
          }
        }
      }
      __syncthreads();
      double cj[TQ];
#pragma unroll UQ
      for (int q = 0; q < NQB; ++q) {
        const int j = col_of(tc, q);
        cj[q] = sel(q >= kq && j > k && j < n, cb[min(j, kN - 1)]);
      }
#pragma unroll UP
      for (int p = 0; p < NPB; ++p) {
        const int i = row_of(tr, p);
        if (p < 2 * kq || (GM && (i <= k || i >= n))) continue;
        const double ci = sel(i > k && i < n, cb[min(i, kN - 1)]);
#pragma unroll UQ
        for (int q = 0; q < NQB; ++q) {
          if (q < kq || 32 * q > 16 * p + 15) continue;
          g(p, q) -= ci * cj[q];
        }
      }
    }
  }
#pragma unroll UP
  for (int p = 0; p < NPB; ++p)
#pragma unroll UQ
    for (int q = 0; q < NQB; ++q) {
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
  // blocks that hold entries of the n x n matrix (the global tile is sized
  // for n up to 1024; the register tile always covers all of its blocks)
  const int NPB = GM ? min(TP, (n + 15) / 16) : TP, NQB = GM ? min(TQ, (n + 31) / 32) : TQ;
  Tile<TP, TQ, GM> g;
  g.gp = tile_ws + t;
#pragma unroll UP
  for (int p = 0; p < NPB; ++p)
#pragma unroll UQ
    for (int q = 0; q < NQB; ++q)
      g(p, q) = sel(row_of(tr, p) == col_of(tc, q) && row_of(tr, p) < n, 1.0);
  // Row k lives in row block kp = k / 16.  The block loop is unrolled in
  // register mode, so the pivot row's registers are compile-time indices; X is
  // lower triangular, so finished row blocks and the column blocks right of
  // the current row block are skipped.
#pragma unroll UP
  for (int kp = 0; kp < NPB; ++kp) {
    const int k0 = 16 * kp, k1 = min(k0 + 16, n);
    for (int k = k0; k < k1; ++k) {
      const int kk = k & 7;
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
        for (int q = 0; q < NQB; ++q) {
          if (32 * q > k0 + 15) continue;
          const int j = col_of(tc, q);
          const double v = g(kp, q) * rlkk;
          g(kp, q) = v;
          if (j < n) rowbuf[j] = v;
        }
      }
      __syncthreads();
      double rj[TQ];
#pragma unroll UQ
      for (int q = 0; q < NQB; ++q) {
        const int j = col_of(tc, q);
        rj[q] = sel(32 * q <= k0 + 15 && j <= k && j < n, rowbuf[min(j, kN - 1)]);
      }
#pragma unroll UP
      for (int p = 0; p < NPB; ++p) {
        const int i = row_of(tr, p);
        if (p < kp || (GM && (i <= k || i >= n))) continue;
        const double li = sel(i > k && i < n, lcol[kk][min(i, kN - 1)]);
#pragma unroll UQ
        for (int q = 0; q < NQB; ++q) {
          if (32 * q > k0 + 15) continue;
          g(p, q) -= li * rj[q];
        }
      }
      __syncthreads();
    }
  }
#pragma unroll UP
  for (int p = 0; p < NPB; ++p)
#pragma unroll UQ
    for (int q = 0; q < NQB; ++q) {
      const int i = row_of(tr, p), j = col_of(tc, q);
      if (i < n && j < n) Rinv[(int64_t)j * ldr + i] = (i >= j) ? g(p, q) : 0.0;
    }
}

// ------------------------------------------------------------ sym eigen
// Scratch layout (doubles): vref[kN][kN] | tau[kN] | d[kN] | e[kN]
template <int TP, int TQ, bool GM>
__global__ void __launch_bounds__(kThreads)
sym_tridiag_kernel(const double *__restrict__ G, int64_t ldg, int n, double *__restrict__ ws,
                   double *__restrict__ tile_ws) {
  constexpr int kN = Geo<TP, TQ>::kN;
  constexpr int UP = GM ? 1 : TP, UQ = GM ? 1 : TQ;
  __shared__ double vbufs[2][kN];
  __shared__ double pbufs[2][kN];
  __shared__ double red[kWaves];
  __shared__ double staus[2];
  const int t = threadIdx.x, tr = t & 15, tc = t >> 4;
  // blocks that hold entries of the n x n matrix (the global tile is sized
  // for n up to 1024; the register tile always covers all of its blocks)
  const int NPB = GM ? min(TP, (n + 15) / 16) : TP, NQB = GM ? min(TQ, (n + 31) / 32) : TQ;
  double *vref = ws;
  double *tauv = ws + (size_t)kN * kN;
  double *dd = tauv + kN;
  double *ee = dd + kN;
  Tile<TP, TQ, GM> g;
  g.gp = tile_ws + t;
#pragma unroll UP
  for (int p = 0; p < NPB; ++p)
#pragma unroll UQ
    for (int q = 0; q < NQB; ++q) {
      const int i = row_of(tr, p), j = col_of(tc, q);
      g(p, q) = sel(i < n && j < n, G[(int64_t)min(i, n - 1) * ldg + min(j, n - 1)]);
    }

  // Column k lives in column block kq = k / 32; the unrolled block loop makes
  // the owner's registers compile-time indices.  Rows and columns at or above
  // the pivot are final (d, e are recorded), so blocks before kq (columns) and
  // before 2 kq (rows) are skipped.
#pragma unroll UQ
  for (int kq = 0; kq < NQB; ++kq) {
    const int k0 = 32 * kq, k1 = min(k0 + 32, n - 2);
    for (int k = k0; k < k1; ++k) {
      // column k's vector, p and tau alternate between two buffers, so the
      // next column's owner may publish before every thread is done with k
      double *vbuf = vbufs[k & 1], *pbuf = pbufs[k & 1];
      if (tc == (k & 31)) {
        // Householder vector of column k below the diagonal
        double s2 = 0.0, x1 = 0.0, dk = 0.0;
#pragma unroll UP
        for (int p = 0; p < NPB; ++p) {
          const int i = row_of(tr, p);
          const double v = g(p, kq);
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
        for (int p = 0; p < NPB; ++p) {
          const int i = row_of(tr, p);
          if (i < n) {
            const double v = (i == k + 1) ? v1 : sel(i > k + 1, g(p, kq));
            vbuf[i] = v;
            vref[(size_t)k * kN + i] = v;
          }
        }
        if (tr == 0) {
          staus[k & 1] = tau;
          tauv[k] = tau;
          dd[k] = dk;
          ee[k] = alpha;
        }
      }
      __syncthreads();
      const double tau = staus[k & 1];
      if (tau != 0.0) {
        // p = tau G v by column sums (G symmetric); K = v^T p
        double sq[TQ];
#pragma unroll UQ
        for (int q = 0; q < NQB; ++q) sq[q] = 0.0;
#pragma unroll UP
        for (int p = 0; p < NPB; ++p) {
          const int i = row_of(tr, p);
          if (p < 2 * kq || (GM && (i <= k || i >= n))) continue;
          const double vi = sel(i > k && i < n, vbuf[min(i, kN - 1)]);
#pragma unroll UQ
          for (int q = 0; q < NQB; ++q) {
            if (q < kq) continue;
            sq[q] += g(p, q) * vi;
          }
        }
        double kpart = 0.0;
#pragma unroll UQ
        for (int q = 0; q < NQB; ++q) {
          if (q < kq) continue;
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
        for (int q = 0; q < NQB; ++q) {
          const int j = col_of(tc, q);
          vj[q] = sel(q >= kq && j > k && j < n, vbuf[min(j, kN - 1)]);
          wj[q] = sel(q >= kq && j < n, pbuf[min(j, kN - 1)] - c * vj[q]);
        }
#pragma unroll UP
        for (int p = 0; p < NPB; ++p) {
          const int i = row_of(tr, p);
          if (p < 2 * kq || (GM && i >= n)) continue;
          const double vi = sel(i > k && i < n, vbuf[min(i, kN - 1)]);
          const double wi = sel(i < n, pbuf[min(i, kN - 1)] - c * vi);
#pragma unroll UQ
          for (int q = 0; q < NQB; ++q) {
            if (q < kq) continue;
            g(p, q) -= vi * wj[q] + wi * vj[q];
          }
        }
      }
    }
  }
  // trailing 2 x 2 (or 1 x 1) block
#pragma unroll UP
  for (int p = 0; p < NPB; ++p)
#pragma unroll UQ
    for (int q = 0; q < NQB; ++q) {
      const int i = row_of(tr, p), j = col_of(tc, q);
      if (i < n && i == j && i >= n - 2) dd[i] = g(p, q);
      if (n >= 2 && i == n - 1 && j == n - 2) ee[n - 2] = g(p, q);
    }
}

namespace {

// 1 / q from the hardware estimate refined by two Newton steps (r <- r (2 -
// q r)): within an ulp or two of the rounded quotient, half the dependent
// instructions of the IEEE division sequence.
SSI_DEV double rcp_nr(double q) {
  double r = __builtin_amdgcn_rcp(q);
  r = r * (2.0 - q * r);
  return r * (2.0 - q * r);
}

// Number of eigenvalues of the tridiagonal (d, e2 = e^2) smaller than x.  The
// pivots q carry a relative error of a few ulps from the refined reciprocal,
// a backward perturbation of the same order that the bisection tolerance
// absorbs.
SSI_DEV int sturm_count(const double *d, const double *e2, int n, double x, double pivmin) {
  int cnt = 0;
  double q = d[0] - x;
  if (fabs(q) < pivmin) q = -pivmin;
  cnt += q < 0.0;
  for (int j = 1; j < n; ++j) {
    q = d[j] - x - e2[j - 1] * rcp_nr(q);
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

SSI_DEV double wave_min_d(double v) { return wave_min(v); }
SSI_DEV double wave_max_d(double v) { return wave_max(v); }

}  // namespace

// LU with partial pivoting of the tridiagonal T - lam I (diagonal dd, off-
// diagonal ee), run by one lane.  A row swap is marked by adding 4 to the
// multiplier (at most 1 in magnitude); u0 holds 1 / pivot, pivots below tiny
// are raised to tiny.
SSI_DEV void inv_iter_lu(const double *dd, const double *ee, int n, double lam, double tiny,
                         double *u0, double *u1, double *u2, double *ml) {
  double a = dd[0] - lam, b = (n > 1) ? ee[0] : 0.0, c = 0.0;
  for (int j = 0; j + 1 < n; ++j) {
    const double sub = ee[j];
    const double an = dd[j + 1] - lam;
    const double cn = (j + 2 < n) ? ee[j + 1] : 0.0;
    if (fabs(a) >= fabs(sub)) {
      const double aa = (fabs(a) < tiny) ? copysign(tiny, a == 0.0 ? 1.0 : a) : a;
      const double m = sub / aa;
      u0[j] = 1.0 / aa;
      u1[j] = b;
      u2[j] = c;
      ml[j] = m;
      a = an - m * b;
      b = cn - m * c;
    } else {
      const double m = a / sub;
      u0[j] = 1.0 / sub;
      u1[j] = an;
      u2[j] = cn;
      ml[j] = m + 4.0;
      a = b - m * an;
      b = c - m * cn;
    }
    c = 0.0;
  }
  if (fabs(a) < tiny) a = copysign(tiny, a == 0.0 ? 1.0 : a);
  u0[n - 1] = 1.0 / a;
  u1[n - 1] = 0.0;
  u2[n - 1] = 0.0;
}

// One inverse-iteration step x <- (T - lam I)^-1 x with the factors of
// inv_iter_lu, scaled to max |x_j| = 1; run by one lane.
SSI_DEV void inv_iter_solve(int n, const double *u0, const double *u1, const double *u2,
                            const double *ml, double *xv) {
  double bj = xv[0];
  for (int j = 0; j + 1 < n; ++j) {
    double m = ml[j];
    double bn = xv[j + 1];
    if (m > 2.0) {
      m -= 4.0;
      const double tmp = bj;
      bj = bn;
      bn = tmp;
    }
    xv[j] = bj;
    bj = bn - m * bj;
  }
  xv[n - 1] = bj;
  double x1 = 0.0, x2 = 0.0, nrm = 0.0;
  for (int j = n - 1; j >= 0; --j) {
    const double xj = (xv[j] - u1[j] * x1 - u2[j] * x2) * u0[j];
    xv[j] = xj;
    x2 = x1;
    x1 = xj;
    nrm = fmax(nrm, fabs(xj));
  }
  const double inv = 1.0 / nrm;
  for (int j = 0; j < n; ++j) xv[j] *= inv;
}

// Eigenpairs of the tridiagonal (d, e), one wave per eigenvalue; wave t of the
// grid takes the t-th largest, and its eigenvector when t < nvec.  The eigenvalue comes from multisection of the
// Sturm count: each round the 64 lanes count at 64 interior points of the
// bracket [lo, hi] (invariant: count(lo) <= target < count(hi)) and the
// bracket shrinks to the pair of neighbouring points that straddles the
// target, a factor 65 per round.  The eigenvector comes from inverse
// iteration (three solves) with the LU factors of T - lambda I, partial
// pivoting, held in the wave's slice of LDS and run by lane 0.
template <int KN, int EPW>
__global__ void __launch_bounds__(64 * EPW)
sym_tridiag_eig_kernel(int n, int nvec, double *__restrict__ evals, double *__restrict__ evecs,
                       int64_t ldv, const double *__restrict__ ws) {
  __shared__ double dd[KN];
  __shared__ double ee[KN];
  __shared__ double e2[KN];
  __shared__ double lu[EPW][5][KN];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int t = blockIdx.x * EPW + wv;
  const double *tauv = ws + (size_t)KN * KN;
  for (int i = threadIdx.x; i < n; i += 64 * EPW) {
    dd[i] = tauv[KN + i];
    const double e = (i < n - 1) ? tauv[2 * KN + i] : 0.0;
    ee[i] = e;
    e2[i] = e * e;
  }
  __syncthreads();
  double lo_part = 1e300, hi_part = -1e300, emax_part = 0.0;
  for (int i = lane; i < n; i += 64) {
    const double r = (i > 0 ? fabs(ee[i - 1]) : 0.0) + fabs(ee[i]);
    lo_part = fmin(lo_part, dd[i] - r);
    hi_part = fmax(hi_part, dd[i] + r);
    emax_part = fmax(emax_part, e2[i]);
  }
  const double glo = wave_min_d(lo_part), ghi = wave_max_d(hi_part);
  const double e2max = wave_max_d(emax_part);
  const double gnorm = fmax(fabs(glo), fabs(ghi));
  const double pivmin = 2.2250738585072014e-308 * fmax(1.0, e2max);
  const double span = ghi - glo;
  const double eps = 2.220446049250313e-16;
  const double tiny = eps * fmax(gnorm, 1e-300);
  double *u0 = lu[wv][0], *u1 = lu[wv][1], *u2 = lu[wv][2], *ml = lu[wv][3], *xv = lu[wv][4];
  if (t < n) {
    const int target = n - 1 - t;              // ascending index of the t-th largest
    double lo = glo - 1e-14 * span - 2.0 * pivmin, hi = ghi + 1e-14 * span + 2.0 * pivmin;
    for (int round = 0; round < 64; ++round) {
      if (hi - lo <= 2.0 * eps * fmax(fabs(lo), fabs(hi)) + pivmin) break;
      const double x = lo + (hi - lo) * ((double)(lane + 1) * (1.0 / 65.0));
      const bool above = sturm_count(dd, e2, n, x, pivmin) > target;
      const uint64_t mask = __ballot(above);
      const int f = mask ? __ffsll((unsigned long long)mask) - 1 : 64;
      const double nhi = (f < 64) ? __shfl(x, f, 64) : hi;
      const double nlo = (f > 0) ? __shfl(x, f - 1, 64) : lo;
      if (!(nhi < hi || nlo > lo)) break;      // points no longer separate
      hi = fmin(hi, nhi);
      lo = fmax(lo, nlo);
    }
    const double lam = 0.5 * (lo + hi);
    if (lane == 0) evals[t] = lam;
    if (lane == 0 && t < nvec) {
      inv_iter_lu(dd, ee, n, lam, tiny, u0, u1, u2, ml);
      for (int j = 0; j < n; ++j) xv[j] = hash_unit(t, j);
      for (int it = 0; it < 3; ++it) inv_iter_solve(n, u0, u1, u2, ml, xv);
    }
  }
  __syncthreads();
  if (t < nvec) {
    double s = 0.0;
    for (int j = lane; j < n; j += 64) s += xv[j] * xv[j];
    const double inv = 1.0 / sqrt(wave_sum(s));
    for (int j = lane; j < n; j += 64) evecs[(int64_t)j * ldv + t] = xv[j] * inv;
  }
}

// Eigenvalues closer than kClusterTol ||T|| are a cluster: inverse iteration
// run on each of them alone converges to nearly the same vector (for an exact
// multiple or zero eigenvalue, to nearly parallel ones), so their vectors are
// recomputed here one after another with every iterate orthogonalized against
// the cluster's earlier vectors (modified Gram-Schmidt), as LAPACK's xSTEIN
// does; the vectors of isolated eigenvalues are left as they are.  Inverse
// iteration from an isolated eigenvalue with absolute gap g gives a vector
// within about eps ||T|| / g of the true one, so outside clusters the vectors
// are orthogonal to about 2e-4 or better.  The tolerance is far below
// LAPACK's 1e-3 ||T||: the spectra here are graded down to 1e-8 ||T|| and
// below, and a looser one chains their tails into one cluster of hundreds of
// vectors, each a sequential inverse iteration; at this one, clusters are
// the exactly multiple and the (numerically) zero eigenvalues.  Evals are
// descending (column t holds the t-th largest).  One wave takes whole
// clusters, W waves share them round robin; the LU and the solves run on
// lane 0 as in sym_tridiag_eig_kernel, the projections on the whole wave.
// Only the vectors t < nvec are wanted: a cluster's members are recomputed up
// to nvec - 1 (each is orthogonalized against the earlier ones only).
constexpr double kClusterTol = 1e-12;

template <int KN, int W>
__global__ void __launch_bounds__(64 * W)
sym_cluster_kernel(int n, int nvec, const double *__restrict__ evals,
                   double *__restrict__ evecs, int64_t ldv, const double *__restrict__ ws) {
  __shared__ double dd[KN];
  __shared__ double ee[KN];
  __shared__ double lu[W][5][KN];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const double *tauv = ws + (size_t)KN * KN;
  for (int i = threadIdx.x; i < n; i += 64 * W) {
    dd[i] = tauv[KN + i];
    ee[i] = (i < n - 1) ? tauv[2 * KN + i] : 0.0;
  }
  __syncthreads();
  double nrm_part = 0.0;
  for (int i = lane; i < n; i += 64)
    nrm_part = fmax(nrm_part, fabs(dd[i]) + (i > 0 ? fabs(ee[i - 1]) : 0.0) + fabs(ee[i]));
  const double gnorm = wave_max_d(nrm_part);           // Gershgorin bound of ||T||
  const double tol = kClusterTol * gnorm;
  const double tiny = 2.220446049250313e-16 * fmax(gnorm, 1e-300);
  double *u0 = lu[wv][0], *u1 = lu[wv][1], *u2 = lu[wv][2], *ml = lu[wv][3], *xv = lu[wv][4];
  int ordinal = 0;
  for (int s0 = 0; s0 < nvec;) {
    int e0 = s0 + 1;
    while (e0 < n && evals[e0 - 1] - evals[e0] <= tol) ++e0;
    if (e0 - s0 >= 2 && (ordinal++ % W) == wv) {
      for (int j = s0; j < min(e0, nvec); ++j) {
        if (lane == 0) {
          inv_iter_lu(dd, ee, n, evals[j], tiny, u0, u1, u2, ml);
          for (int i = 0; i < n; ++i) xv[i] = hash_unit(j, i);
        }
        for (int it = 0; it < 3; ++it) {
          if (lane == 0) inv_iter_solve(n, u0, u1, u2, ml, xv);
          __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
          __builtin_amdgcn_wave_barrier();
          for (int p = s0; p < j; ++p) {
            double d = 0.0;
            for (int i = lane; i < n; i += 64) d += xv[i] * evecs[(int64_t)i * ldv + p];
            d = wave_sum(d);
            for (int i = lane; i < n; i += 64) xv[i] -= d * evecs[(int64_t)i * ldv + p];
          }
          double mx = 0.0;
          for (int i = lane; i < n; i += 64) mx = fmax(mx, fabs(xv[i]));
          mx = wave_max_d(mx);
          // an iterate wholly inside the earlier vectors' span (it cannot be,
          // short of rounding) would leave nothing: restart from another vector
          const double inv = mx > 0.0 ? 1.0 / mx : 0.0;
          for (int i = lane; i < n; i += 64) xv[i] = mx > 0.0 ? xv[i] * inv : hash_unit(j + n, i);
          __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
          __builtin_amdgcn_wave_barrier();
        }
        double s2 = 0.0;
        for (int i = lane; i < n; i += 64) s2 += xv[i] * xv[i];
        const double inv = 1.0 / sqrt(wave_sum(s2));
        // each lane writes and later reads the same rows of the column, so
        // the wave's own later projections see these values
        for (int i = lane; i < n; i += 64) evecs[(int64_t)i * ldv + j] = xv[i] * inv;
        __threadfence_block();
      }
    }
    s0 = e0;
  }
}

// V <- H_0 H_1 ... H_{n-3} V for the reflectors stored by sym_tridiag_kernel.
template <int TP, int TQ, bool GM>
__global__ void __launch_bounds__(kThreads)
sym_backtransform_kernel(int n, double *__restrict__ evecs, int64_t ldv,
                         const double *__restrict__ ws, double *__restrict__ tile_ws) {
  constexpr int kN = Geo<TP, TQ>::kN;
  constexpr int UP = GM ? 1 : TP, UQ = GM ? 1 : TQ;
  __shared__ double vbufs[2][kN];
  const int t = threadIdx.x, tr = t & 15, tc = t >> 4;
  // blocks that hold entries of the n x n matrix (the global tile is sized
  // for n up to 1024; the register tile always covers all of its blocks)
  const int NPB = GM ? min(TP, (n + 15) / 16) : TP, NQB = GM ? min(TQ, (n + 31) / 32) : TQ;
  const double *vref = ws;
  const double *tauv = ws + (size_t)kN * kN;
  Tile<TP, TQ, GM> g;
  g.gp = tile_ws + t;
#pragma unroll UP
  for (int p = 0; p < NPB; ++p)
#pragma unroll UQ
    for (int q = 0; q < NQB; ++q) {
      const int i = row_of(tr, p), j = col_of(tc, q);
      g(p, q) = sel(i < n && j < n, evecs[(int64_t)min(i, n - 1) * ldv + min(j, n - 1)]);
    }
  // Reflector k touches rows > k only: row blocks before k / 16 are skipped.
  // Reflectors run k = n-3 .. 0; the next one's vector entry (one per thread,
  // n <= kThreads) and tau are loaded into registers while the current one is
  // applied, and vectors alternate between two LDS buffers, so each reflector
  // takes one barrier and no global round trip.
  static_assert(Geo<TP, TQ>::kN <= kThreads || GM, "one vector entry per thread");
  double nv = 0.0, ntau = 0.0;
  if (n >= 3) {
    nv = vref[(size_t)(n - 3) * kN + min(t, n - 1)];
    ntau = tauv[n - 3];
  }
#pragma unroll UP
  for (int kb = NPB - 1; kb >= 0; --kb) {
    const int k0 = 16 * kb, k1 = min(k0 + 16, n - 2);
    for (int k = k1 - 1; k >= k0; --k) {
      double *vbuf = vbufs[k & 1];
      for (int i = t; i < n; i += kThreads) {
        const double v = (i == t) ? nv : vref[(size_t)k * kN + i];
        vbuf[i] = (i > k) ? v : 0.0;
      }
      const double tau = ntau;
      __syncthreads();
      if (k > 0) {
        nv = vref[(size_t)(k - 1) * kN + min(t, n - 1)];
        ntau = tauv[k - 1];
      }
      if (tau != 0.0) {
        double sq[TQ];
#pragma unroll UQ
        for (int q = 0; q < NQB; ++q) sq[q] = 0.0;
#pragma unroll UP
        for (int p = 0; p < NPB; ++p) {
          const int i = row_of(tr, p);
          if (p < kb || (GM && (i <= k || i >= n))) continue;
          const double vi = sel(i > k && i < n, vbuf[min(i, kN - 1)]);
#pragma unroll UQ
          for (int q = 0; q < NQB; ++q) sq[q] += vi * g(p, q);
        }
#pragma unroll UQ
        for (int q = 0; q < NQB; ++q) sq[q] = tau * col_group_sum(sq[q]);
#pragma unroll UP
        for (int p = 0; p < NPB; ++p) {
          const int i = row_of(tr, p);
          if (p < kb || (GM && (i <= k || i >= n))) continue;
          const double vi = sel(i > k && i < n, vbuf[min(i, kN - 1)]);
#pragma unroll UQ
          for (int q = 0; q < NQB; ++q) g(p, q) -= vi * sq[q];
        }
      }
    }
  }
#pragma unroll UP
  for (int p = 0; p < NPB; ++p)
#pragma unroll UQ
    for (int q = 0; q < NQB; ++q) {
      const int i = row_of(tr, p), j = col_of(tc, q);
      if (i < n && j < n) evecs[(int64_t)i * ldv + j] = g(p, q);
    }
}

// Lower Cholesky factor L (into Lws, ld n, lower triangle) of G + shift_rel
// tr(G) I, n <= 16 kCbMax, by 16 x 16 blocks (right-looking).  The blocks
// (i, j), i >= j, of the lower triangle live in registers as MFMA
// accumulator tiles (lane l: rows l / 16 + 4 q, column l % 16), block
// id = i (i + 1) / 2 + j in slot id / 16 of wave id % 16.  For each block column k: its
// blocks go to an LDS panel; wave 0 factors the diagonal block (lane r holds
// row r, column steps through lane reads); every thread solves one panel row
// against it; then each wave subtracts P_i P_j^T from its blocks (i, j), k <
// j <= i, on v_mfma_f64_16x16x4f64.  Rows and columns past n are those of
// the identity.  status bit 0 is set on a non-positive pivot.
constexpr int kCbMax = 14;
constexpr int kCbWaves = 16;
constexpr int kCbSlots = (kCbMax * (kCbMax + 1) / 2 + kCbWaves - 1) / kCbWaves;
__global__ void __launch_bounds__(64 * kCbWaves)
chol_blk_kernel(const double *__restrict__ G, int64_t ldg, int n, double shift_rel,
                double *__restrict__ Lws, int *__restrict__ status) {
  __shared__ double panel[16 * kCbMax][17];           // rows of block column k, from block row k
  __shared__ double lkk[16][17];
  __shared__ double rdiag[16];
  __shared__ double red[kCbWaves];
  __shared__ int bad;
  const int nb = (n + 15) >> 4, nblk = nb * (nb + 1) / 2;
  const int t = threadIdx.x, lane = t & 63;
  const int wave = __builtin_amdgcn_readfirstlane(t >> 6);
  int bi[kCbSlots], bj[kCbSlots];
#pragma unroll
  for (int s = 0; s < kCbSlots; ++s) {
    const int id = kCbWaves * s + wave;
    int i = 0;
    while ((i + 1) * (i + 2) / 2 <= id) ++i;          // uniform: block row of id
    bi[s] = id < nblk ? i : -1;
    bj[s] = id - i * (i + 1) / 2;
  }
  // load G (identity past n) and the trace of its leading n x n part
  f64x4 acc[kCbSlots];
  double tr_part = 0.0;
#pragma unroll
  for (int s = 0; s < kCbSlots; ++s) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int r = 16 * bi[s] + (lane >> 4) + 4 * q, c = 16 * bj[s] + (lane & 15);
      const double v = G[(int64_t)min(max(r, 0), n - 1) * ldg + min(c, n - 1)];
      const bool in = bi[s] >= 0 && r < n && c < n;
      acc[s][q] = in ? v : (bi[s] >= 0 && r == c ? 1.0 : 0.0);
      tr_part += (in && r == c) ? v : 0.0;
    }
  }
  if (t == 0) bad = 0;
  {
    const double w = wave_sum(tr_part);
    if (lane == 0) red[wave] = w;
    __syncthreads();
    double tr = 0.0;
#pragma unroll
    for (int w8 = 0; w8 < kCbWaves; ++w8) tr += red[w8];
    const double shift = shift_rel * tr;
#pragma unroll
    for (int s = 0; s < kCbSlots; ++s)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int r = 16 * bi[s] + (lane >> 4) + 4 * q, c = 16 * bj[s] + (lane & 15);
        if (bi[s] >= 0 && r == c && r < n) acc[s][q] += shift;
      }
  }
  for (int k = 0; k < nb; ++k) {
    __syncthreads();                                   // the previous panel's readers are done
#pragma unroll
    for (int s = 0; s < kCbSlots; ++s)
      if (bj[s] == k && bi[s] >= k) {
#pragma unroll
        for (int q = 0; q < 4; ++q)
          panel[16 * (bi[s] - k) + (lane >> 4) + 4 * q][lane & 15] = acc[s][q];
      }
    __syncthreads();
    if (wave == 0) {
      // diagonal block: lane r < 16 holds row r
      double a[16];
      const int r = lane & 15;
#pragma unroll
      for (int c = 0; c < 16; ++c) a[c] = panel[r][c];
#pragma unroll
      for (int c = 0; c < 16; ++c) {
        double piv = lane_read_d(a[c], c);
        if (!(piv > 0.0)) {
          if (lane == 0) bad = 1;
          piv = 1e-300;
        }
        const double d = sqrt(piv), rd = 1.0 / d;
        a[c] = (r == c) ? d : a[c] * rd;
        if (lane == 0) rdiag[c] = rd;
#pragma unroll
        for (int j = c + 1; j < 16; ++j) {
          const double xj = lane_read_d(a[c], j);
          if (r >= j) a[j] -= a[c] * xj;
        }
      }
      if (lane < 16) {
#pragma unroll
        for (int c = 0; c < 16; ++c) lkk[r][c] = (c <= r) ? a[c] : 0.0;
        const int gr = 16 * k + r;
        if (gr < n)
#pragma unroll
          for (int c = 0; c < 16; ++c)
            if (c <= r && 16 * k + c < n) Lws[(int64_t)gr * n + 16 * k + c] = a[c];
      }
    }
    __syncthreads();
    // panel rows below the diagonal block: x L_kk^T = a
    const int pr = 16 + t;
    if (pr < 16 * (nb - k)) {
      double x[16];
#pragma unroll
      for (int c = 0; c < 16; ++c) {
        double v = panel[pr][c];
#pragma unroll
        for (int m = 0; m < c; ++m) v -= x[m] * lkk[c][m];
        x[c] = v * rdiag[c];
      }
      const int gr = 16 * k + pr;
#pragma unroll
      for (int c = 0; c < 16; ++c) panel[pr][c] = x[c];
      if (gr < n)
#pragma unroll
        for (int c = 0; c < 16; ++c)
          if (16 * k + c < n) Lws[(int64_t)gr * n + 16 * k + c] = x[c];
    }
    __syncthreads();
    // trailing blocks (i, j), k < j <= i: acc -= P_i P_j^T
#pragma unroll
    for (int s = 0; s < kCbSlots; ++s)
      if (bj[s] > k && bi[s] >= bj[s]) {
        const int ri = 16 * (bi[s] - k) + (lane & 15), rj = 16 * (bj[s] - k) + (lane & 15);
#pragma unroll
        for (int st = 0; st < 4; ++st) {
          const int kk = 4 * st + (lane >> 4);
          acc[s] = __builtin_amdgcn_mfma_f64_16x16x4f64(-panel[ri][kk], panel[rj][kk], acc[s],
                                                        0, 0, 0);
        }
      }
  }
  if (t == 0 && bad) atomicOr(status, 1);
}

// X = L^{-1} for the lower-triangular L in Lws (ld n), n <= 16 IB, by 16 x
// 16 blocks: workgroup b takes block column b.  The inverses D_i of the
// diagonal blocks i >= b come first (one 16-lane group per block, lane c a
// forward substitution for column c, blocks staged in LDS); then block row by
// block row, X_bb = D_b and X_ib = -D_i sum_{b <= j < i} L_ij X_jb, the sum on
// v_mfma_f64_16x16x4f64 with its 16 (i - b) terms split over the four waves
// and the partial products added through LDS.  The chain is nb - b block
// steps instead of n - 16 b row steps.  Rows and columns past n are those of
// the identity.  Writes Rinv = X^T (upper, zero below the diagonal) for rows
// 16 b .. 16 b + 15.  LDS (dynamic): D [IB][256], X [IB][256] (the
// diagonal blocks of L before D exists), partials [4][256].  IB = 14 (n <= 224)
// or 28 (n <= 448, 120 KiB of LDS).
constexpr int kIbMax = 14;
template <int IB>
__global__ void __launch_bounds__(256)
tri_inv_blk_kernel(int n, const double *__restrict__ Lws, double *__restrict__ Rinv,
                   int64_t ldr) {
  extern __shared__ double tib[];
  double *dinv = tib;                                  // [IB][16][16]
  double *xc = tib + IB * 256;                     // [IB][16][16]
  double *sp = tib + 2 * IB * 256;                 // [4][16][16]
  const int nb = (n + 15) >> 4, b = blockIdx.x;
  const int t = threadIdx.x, lane = t & 63;
  const int wave = __builtin_amdgcn_readfirstlane(t >> 6);
  // entry (r, j) of L padded with the identity; the load is unconditional
  auto lg = [&](int r, int j) -> double {
    const double v = Lws[(int64_t)min(r, n - 1) * n + min(j, n - 1)];
    return (r < n && j < n) ? v : (r == j ? 1.0 : 0.0);
  };
  // stage the diagonal blocks i = b.. of L (entry t of each block)
  {
    double v[IB];
#pragma unroll
    for (int g = 0; g < IB; ++g) {
      const int i = b + g;
      v[g] = lg(16 * i + (t >> 4), 16 * i + (t & 15));
    }
#pragma unroll
    for (int g = 0; g < IB; ++g)
      if (b + g < nb) xc[g * 256 + t] = v[g];
  }
  __syncthreads();
  {
    const int c = t & 15;                              // block b + g, column c
    for (int g = t >> 4; g < IB && b + g < nb; g += 16) {
      const double *l = xc + g * 256;
      double x[16];
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        double s = (r == c) ? 1.0 : 0.0;
#pragma unroll
        for (int j = 0; j < r; ++j) s -= l[r * 16 + j] * x[j];
        x[r] = s / l[r * 16 + r];
      }
#pragma unroll
      for (int r = 0; r < 16; ++r) dinv[g * 256 + r * 16 + c] = x[r];
    }
  }
  __syncthreads();
  const int r = t >> 4, c = t & 15;
  const int row = 16 * b + c;                          // row of Rinv written by this thread
  {
    const double x = dinv[t];
    xc[t] = x;
    if (row < n && 16 * b + r < n) Rinv[(int64_t)row * ldr + 16 * b + r] = x;
    if (row < n)
      for (int i = r; i < 16 * b; i += 16) Rinv[(int64_t)row * ldr + i] = 0.0;
  }
  __syncthreads();
  for (int i = b + 1; i < nb; ++i) {
    const int ks = 4 * (i - b);                        // MFMA steps of 4 terms
    double av[IB];
#pragma unroll
    for (int u = 0; u < IB; ++u) {
      const int kk = 4 * (wave + 4 * u) + (lane >> 4);
      av[u] = lg(16 * i + (lane & 15), 16 * b + kk);
    }
    f64x4 acc = f64x4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int u = 0; u < IB; ++u) {
      const int st = wave + 4 * u;
      if (st < ks) {
        const int kk = 4 * st + (lane >> 4);
        const double bv = xc[(kk >> 4) * 256 + (kk & 15) * 16 + (lane & 15)];
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u], bv, acc, 0, 0, 0);
      }
    }
    // D layout: lane holds rows (lane / 16) + 4 q, column lane % 16
#pragma unroll
    for (int q = 0; q < 4; ++q) sp[wave * 256 + ((lane >> 4) + 4 * q) * 16 + (lane & 15)] = acc[q];
    __syncthreads();
    double x = 0.0;
    const double *d = dinv + (i - b) * 256;
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      const int e = k * 16 + c;
      x += d[r * 16 + k] * ((sp[e] + sp[256 + e]) + (sp[512 + e] + sp[768 + e]));
    }
    x = -x;
    xc[(i - b) * 256 + t] = x;
    if (row < n && 16 * i + r < n) Rinv[(int64_t)row * ldr + 16 * i + r] = x;
    __syncthreads();
  }
}

// ---------------------------------------------------------------- mid sizes
namespace {
// Orders the LDS accesses of one wave (its lanes run in lockstep; the fence
// keeps the compiler from moving accesses across).
SSI_DEV void mid_wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
  __builtin_amdgcn_wave_barrier();
}
}  // namespace

// 224 < n <= kMidN: the matrix stays in global memory (n^2 doubles, at most
// 1.6 MiB, so it lives in L2) and the kernels are organized so that every
// access is coalesced and many are in flight, instead of one thread walking
// its slots of the global tile.
constexpr int kMidN = 448;
constexpr int kMidU = kMidN / 64;        // rows of a column per lane
constexpr int kMidKN = 1024;             // row stride of the reflectors (the global layout)

// Lower Cholesky factor L (into Lws, ld n, lower triangle) of G + shift_rel
// tr(G) I for n <= kMidN, by 16 x 16 blocks, right-looking, the trailing
// matrix kept in Lws itself.  For block column k: wave 0 factors the diagonal
// block (adding the shift to its diagonal: the shift commutes with the
// trailing updates), each thread solves one panel row against it (the panel
// is kept in LDS), then the kMidCT / 64 waves subtract P_i P_j^T from the
// trailing blocks (i, j), k < j <= i, four blocks per wave at a time (their
// loads in flight together) on v_mfma_f64_16x16x4f64.  Rows and columns past n: loads
// are clamped, such entries are never stored, and their panel rows are zero.
// status bit 0 is set on a non-positive pivot.
constexpr int kMidCT = 512;              // threads (one panel row each: n - 16 < kMidCT)
__global__ void __launch_bounds__(kMidCT)
chol_mid_kernel(const double *__restrict__ G, int64_t ldg, int n, double shift_rel,
                double *__restrict__ Lws, int *__restrict__ status) {
  __shared__ double panel[kMidN][17];
  __shared__ double lkk[16][17];
  __shared__ double rdiag[16];
  __shared__ double red[kMidCT / 64];
  __shared__ int bad;
  const int t = threadIdx.x, lane = t & 63;
  const int wave = __builtin_amdgcn_readfirstlane(t >> 6);
  const int nb = (n + 15) >> 4;
  // the lower triangle of G into Lws, and the trace
  double tr_part = 0.0;
  for (int idx = t; idx < n * n; idx += kMidCT) {
    const int i = idx / n, j = idx - i * n;
    if (j <= i) {
      const double v = G[(int64_t)i * ldg + j];
      Lws[idx] = v;
      tr_part += (i == j) ? v : 0.0;
    }
  }
  if (t == 0) bad = 0;
  tr_part = wave_sum(tr_part);
  if (lane == 0) red[wave] = tr_part;
  __syncthreads();
  double trace = 0.0;
#pragma unroll
  for (int w = 0; w < kMidCT / 64; ++w) trace += red[w];
  const double shift = shift_rel * trace;
  for (int k = 0; k < nb; ++k) {
    const int r0 = 16 * k;
    if (wave == 0) {
      // diagonal block, factored in LDS by wave 0 (zero above the diagonal,
      // the identity past n)
      for (int e = lane; e < 256; e += 64) {
        const int r = e >> 4, c = e & 15;
        const int gi = r0 + r, gj = r0 + c;
        const double v = Lws[(int64_t)min(gi, n - 1) * n + min(gj, n - 1)];
        const bool in = gi < n && gj < n && c <= r;
        lkk[r][c] = in ? v + (r == c ? shift : 0.0) : (r == c ? 1.0 : 0.0);
      }
      mid_wave_sync();
      for (int c = 0; c < 16; ++c) {
        double piv = lkk[c][c];
        if (!(piv > 0.0)) {
          if (lane == 0) bad = 1;
          piv = 1e-300;
        }
        const double d = sqrt(piv), rd = 1.0 / d;
        mid_wave_sync();                      // every lane has read the pivot
        if (lane == c) lkk[c][c] = d;
        if (lane > c && lane < 16) lkk[lane][c] *= rd;
        if (lane == 0) rdiag[c] = rd;
        mid_wave_sync();
        for (int e = lane; e < 256; e += 64) {
          const int r = e >> 4, j = e & 15;
          if (j > c && r >= j) lkk[r][j] -= lkk[r][c] * lkk[j][c];
        }
        mid_wave_sync();
      }
      for (int e = lane; e < 256; e += 64) {
        const int r = e >> 4, c = e & 15;
        if (r0 + r < n && r0 + c < n)
          Lws[(int64_t)(r0 + r) * n + r0 + c] = (c <= r) ? lkk[r][c] : 0.0;
      }
    }
    __syncthreads();
    // panel rows below the diagonal block: x L_kk^T = w
    const int prow = r0 + 16 + t;
    if (prow < 16 * nb) {
      double x[16];
#pragma unroll
      for (int c = 0; c < 16; ++c)
        x[c] = Lws[(int64_t)min(prow, n - 1) * n + min(r0 + c, n - 1)];
#pragma unroll
      for (int c = 0; c < 16; ++c) {
        double v = (prow < n && r0 + c < n) ? x[c] : 0.0;
#pragma unroll
        for (int m = 0; m < c; ++m) v -= x[m] * lkk[c][m];
        x[c] = v * rdiag[c];
        // one row of L_kk at a time in registers: the compiler would
        // otherwise load all 136 entries up front
        __asm__ volatile("" ::: "memory");
      }
#pragma unroll
      for (int c = 0; c < 16; ++c) panel[t][c] = x[c];
      if (prow < n)
#pragma unroll
        for (int c = 0; c < 16; ++c)
          if (r0 + c < n) Lws[(int64_t)prow * n + r0 + c] = x[c];
    }
    __syncthreads();
    // trailing blocks (i, j) = (k + 1 + ii, k + 1 + jj), jj <= ii < m, as
    // T = m (m + 1) / 2 ids, four per wave per round
    const int m = nb - 1 - k, T = m * (m + 1) / 2;
    for (int id0 = 4 * wave; id0 < T; id0 += 4 * (kMidCT / 64)) {
      f64x4 acc[4];
      int bi[4], bj[4];
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const int id = min(id0 + b, T - 1);
        // row of id in the triangle: the float root is off by at most one
        int ii = (int)((sqrtf(8.0f * id + 1.0f) - 1.0f) * 0.5f);
        ii -= (ii * (ii + 1) / 2 > id) ? 1 : 0;
        ii += ((ii + 1) * (ii + 2) / 2 <= id) ? 1 : 0;
        bi[b] = ii;
        bj[b] = id - ii * (ii + 1) / 2;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int gr = r0 + 16 + 16 * bi[b] + (lane >> 4) + 4 * q;
          const int gc = r0 + 16 + 16 * bj[b] + (lane & 15);
          acc[b][q] = Lws[(int64_t)min(gr, n - 1) * n + min(gc, n - 1)];
        }
      }
#pragma unroll
      for (int b = 0; b < 4; ++b) {
#pragma unroll
        for (int st = 0; st < 4; ++st) {
          const int kk = 4 * st + (lane >> 4);
          acc[b] = __builtin_amdgcn_mfma_f64_16x16x4f64(-panel[16 * bi[b] + (lane & 15)][kk],
                                                        panel[16 * bj[b] + (lane & 15)][kk],
                                                        acc[b], 0, 0, 0);
        }
      }
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        if (id0 + b >= T) continue;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int gr = r0 + 16 + 16 * bi[b] + (lane >> 4) + 4 * q;
          const int gc = r0 + 16 + 16 * bj[b] + (lane & 15);
          if (gr < n && gc < n && gc <= gr) Lws[(int64_t)gr * n + gc] = acc[b][q];
        }
      }
    }
    __syncthreads();
  }
  if (t == 0 && bad) atomicOr(status, 1);
}

namespace {
constexpr int kMidT = 512, kMidW = kMidT / 64;

// Sum over the workgroup (kMidT threads); red holds kMidW doubles.
SSI_DEV double mid_sum(double a, double *red) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  a = wave_sum(a);
  __syncthreads();                        // red is free
  if (lane == 0) red[wave] = a;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int w = 0; w < kMidW; ++w) s += red[w];
  return s;
}
}  // namespace

// Householder tridiagonalization of the symmetric G for n <= kMidN, in place
// in global memory: G is copied by columns into A (n x n) and reduced there;
// the reflectors, tau, d and e go to ws in the layout of the global path (row
// stride kMidKN).  With v, tau the reflector of step k and p = tau B v (B the
// trailing block as step k - 1 left it), the update is B - v w^T - w v^T,
// w = p - (tau / 2) (v . p) v.  The next step needs column k + 1 as this step
// leaves it, so each step first updates that column alone (its diagonal entry
// is then d[k + 1]) and forms the next reflector from it; the pass that then
// updates the trailing columns k + 2 .. n - 1 (rows from k + 2) accumulates
// the next p, column by column (B is symmetric).  One read and one write of
// the trailing block per step.
__global__ void __launch_bounds__(kMidT)
sym_tridiag_mid_kernel(const double *__restrict__ G, int64_t ldg, int n,
                       double *__restrict__ ws, double *__restrict__ A) {
  __shared__ double sv[2][kMidN];        // reflector of this step, of the next
  __shared__ double sp[2][kMidN];        // p (by column), then w, of this step / the next
  __shared__ double red[kMidW];
  __shared__ double stau[2];
  double *vref = ws;
  double *tauv = ws + (size_t)kMidKN * kMidKN;
  double *dd = tauv + kMidKN;
  double *ee = dd + kMidKN;
  const int t = threadIdx.x, lane = t & 63;
  const int wave = __builtin_amdgcn_readfirstlane(t >> 6);
  // A(i, j) = G(j, i): column j of A is row j of G (coalesced; G is symmetric)
  for (int idx = t; idx < n * n; idx += kMidT) {
    const int j = idx / n, i = idx - j * n;
    A[idx] = G[(int64_t)j * ldg + i];
  }
  __syncthreads();
  if (n < 3) {
    if (t < n) dd[t] = A[(int64_t)t * n + t];
    if (t == 0 && n == 2) ee[0] = A[1];
    return;
  }
  // Reflector of step c from column c (x: entry (t, c), rows t > c used):
  // writes v to sv[slot] and row c of vref, tau, d[c] (= dc) and e[c].
  auto reflector = [&](double x, int c, int slot, double dc) {
    double s2 = (t > c + 1 && t < n) ? x * x : 0.0;
    s2 = mid_sum(s2, red);
    double x1 = (t == c + 1) ? x : 0.0;
    x1 = mid_sum(x1, red);
    double tau = 0.0, alpha = x1, v1 = 0.0;
    if (s2 > 0.0) {
      alpha = -copysign(sqrt(x1 * x1 + s2), x1);
      v1 = x1 - alpha;
      tau = 2.0 / (s2 + v1 * v1);
    }
    if (t < n) {
      const double v = (t == c + 1) ? v1 : (t > c + 1 ? x : 0.0);
      sv[slot][t] = v;
      vref[(size_t)c * kMidKN + t] = v;
    }
    if (t == 0) {
      stau[slot] = tau;
      tauv[c] = tau;
      dd[c] = dc;
      ee[c] = alpha;
    }
  };
  // One pass over columns jbeg..n-1, rows from jbeg: with UPD, x -= v_i w_j +
  // w_i v_j and store; then pn[j] = sum_i vn_i x(i, j) (the next p before tau).
  auto pass = [&](int jbeg, bool upd, const double *v, const double *w, const double *vn,
                  double *pn) {
    double vi[kMidU], wi[kMidU], vni[kMidU];
#pragma unroll
    for (int u = 0; u < kMidU; ++u) {
      const int i = lane + 64 * u, ic = min(i, n - 1);
      const bool act = i >= jbeg && i < n;
      vi[u] = act ? v[ic] : 0.0;
      wi[u] = act ? w[ic] : 0.0;
      vni[u] = act ? vn[ic] : 0.0;
    }
    for (int j0 = jbeg + wave; j0 < n; j0 += 2 * kMidW) {
      const int j1 = j0 + kMidW;
      const bool has1 = j1 < n;
      double *c0 = A + (int64_t)j0 * n, *c1 = A + (int64_t)min(j1, n - 1) * n;
      double x0[kMidU], x1[kMidU];
#pragma unroll
      for (int u = 0; u < kMidU; ++u) {
        const int ic = min(lane + 64 * u, n - 1);
        x0[u] = c0[ic];
        x1[u] = c1[ic];
      }
      if (upd) {
        const double vj0 = v[j0], wj0 = w[j0];
        const double vj1 = has1 ? v[j1] : 0.0, wj1 = has1 ? w[j1] : 0.0;
#pragma unroll
        for (int u = 0; u < kMidU; ++u) {
          x0[u] -= vi[u] * wj0 + wi[u] * vj0;
          x1[u] -= vi[u] * wj1 + wi[u] * vj1;
        }
#pragma unroll
        for (int u = 0; u < kMidU; ++u) {
          const int i = lane + 64 * u;
          if (i >= jbeg && i < n) {
            c0[i] = x0[u];
            if (has1) c1[i] = x1[u];
          }
        }
      }
      double s0 = 0.0, s1 = 0.0;
#pragma unroll
      for (int u = 0; u < kMidU; ++u) {
        s0 += vni[u] * x0[u];
        s1 += vni[u] * x1[u];
      }
      s0 = wave_sum(s0);
      s1 = wave_sum(s1);
      if (lane == 0) {
        pn[j0] = s0;
        if (has1) pn[j1] = s1;
      }
    }
  };
  // p <- tau p, then w = p - (tau / 2) (v . p) v over rows from jbeg
  auto finish = [&](int jbeg, int slot) {
    __syncthreads();
    const double tau = stau[slot];
    const bool act = t >= jbeg && t < n;
    const double p = act ? tau * sp[slot][t] : 0.0;
    const double vt = act ? sv[slot][t] : 0.0;
    const double K = mid_sum(vt * p, red);
    if (act) sp[slot][t] = p - 0.5 * tau * K * vt;
    __syncthreads();
  };
  {
    const double x = t < n ? A[t] : 0.0;
    const double d0 = A[0];
    reflector(x, 0, 0, d0);
    __syncthreads();
    pass(1, false, sv[0], sp[0], sv[0], sp[0]);
    finish(1, 0);
  }
  int cur = 0;
  for (int k = 0; k <= n - 3; ++k) {
    const int nx = cur ^ 1;
    // column k + 1 (rows from k + 1) under step k
    const int64_t ck = (int64_t)(k + 1) * n;
    double x = 0.0;
    const bool act = t >= k + 1 && t < n;
    if (act) {
      x = A[ck + t];
      x -= sv[cur][t] * sp[cur][k + 1] + sp[cur][t] * sv[cur][k + 1];
    }
    const double dk1 = (t == k + 1) ? x : 0.0;
    if (k + 1 <= n - 3) {
      const double d1 = mid_sum(dk1, red);
      reflector(x, k + 1, nx, d1);
      __syncthreads();
      if (stau[cur] != 0.0)
        pass(k + 2, true, sv[cur], sp[cur], sv[nx], sp[nx]);
      else
        pass(k + 2, false, sv[cur], sp[cur], sv[nx], sp[nx]);
      finish(k + 2, nx);
    } else {
      // k + 1 = n - 2: the last column pair; d[n-2], e[n-2] from column n - 2
      // as updated, d[n-1] from the last column's update
      if (t == n - 2) dd[n - 2] = x;
      if (t == n - 1) {
        ee[n - 2] = x;
        const double y = A[(int64_t)(n - 1) * n + n - 1];
        const double vl = sv[cur][n - 1], wl = sp[cur][n - 1];
        dd[n - 1] = y - 2.0 * vl * wl;
      }
    }
    cur = nx;
  }
}

// V <- H_0 H_1 ... H_{n-3} V for n <= kMidN (reflectors in the layout of
// sym_tridiag_mid_kernel): one wave per column of V, which it keeps in
// registers (row lane + 64 u in slot u); the reflector rows arrive through a
// register ring kMidRing steps ahead (raw values, masked when used).  Only
// the columns j < nvec are transformed.
constexpr int kMidRing = 4;
__global__ void __launch_bounds__(256)
sym_backtransform_mid_kernel(int n, int nvec, double *__restrict__ evecs, int64_t ldv,
                             const double *__restrict__ ws) {
  const int lane = threadIdx.x & 63;
  const int j = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (j >= nvec) return;
  const double *vref = ws;
  const double *tauv = ws + (size_t)kMidKN * kMidKN;
  double x[kMidU];
#pragma unroll
  for (int u = 0; u < kMidU; ++u) {
    const int i = lane + 64 * u;
    const double v = evecs[(int64_t)min(i, n - 1) * ldv + j];
    x[u] = i < n ? v : 0.0;
  }
  double vq[kMidRing][kMidU], tq[kMidRing];
#pragma unroll
  for (int d = 0; d < kMidRing; ++d) {
    const int k = max(n - 3 - d, 0);
#pragma unroll
    for (int u = 0; u < kMidU; ++u) vq[d][u] = vref[(size_t)k * kMidKN + min(lane + 64 * u, n - 1)];
    tq[d] = tauv[k];
  }
  for (int k0 = n - 3; k0 >= 0; k0 -= kMidRing) {
#pragma unroll
    for (int d = 0; d < kMidRing; ++d) {
      const int k = k0 - d;
      if (k < 0) break;
      const double tau = tq[d];
      double vk[kMidU], s = 0.0;
#pragma unroll
      for (int u = 0; u < kMidU; ++u) {
        vk[u] = (lane + 64 * u < n) ? vq[d][u] : 0.0;
        s += vk[u] * x[u];
      }
      s = tau * wave_sum(s);
#pragma unroll
      for (int u = 0; u < kMidU; ++u) x[u] -= s * vk[u];
      const int kn = max(k - kMidRing, 0);
#pragma unroll
      for (int u = 0; u < kMidU; ++u)
        vq[d][u] = vref[(size_t)kn * kMidKN + min(lane + 64 * u, n - 1)];
      tq[d] = tauv[kn];
    }
  }
#pragma unroll
  for (int u = 0; u < kMidU; ++u) {
    const int i = lane + 64 * u;
    if (i < n) evecs[(int64_t)i * ldv + j] = x[u];
  }
}

namespace ssi {

namespace {
constexpr int kRegP = 14, kRegQ = 7;      // n <= 224
static_assert(kIbMax >= kRegP && kCbMax >= kRegP, "block kernels cover the register path");
constexpr int kGlbP = 64, kGlbQ = 32;     // n <= 1024
constexpr int kRegN = Geo<kRegP, kRegQ>::kN;
constexpr int kGlbN = Geo<kGlbP, kGlbQ>::kN;

constexpr int kRegEpw = 4, kGlbEpw = 1;   // eigenvalues (waves) per workgroup

static_assert(kMidKN == kGlbN, "mid-size kernels write the global path's layout");

double *glb_tile(double *ws) { return ws + (size_t)kGlbN * kGlbN + 3 * kGlbN; }
}  // namespace

int dense_max_n() { return kGlbN; }

size_t dense_ws_doubles(int n) {
  const size_t kn = n <= kRegN ? kRegN : kGlbN;
  const size_t tile = n <= kRegN ? 0 : (size_t)kGlbP * kGlbQ * kThreads;
  return kn * kn + 3 * kn + tile;
}

hipError_t launch_chol_inv(const double *G, int64_t ldg, int n, double shift_rel, double *Rinv,
                           int64_t ldr, double *Lws, double *ws, int *status, hipStream_t st) {
  if (n <= kRegN) {
    hipLaunchKernelGGL(chol_blk_kernel, dim3(1), dim3(64 * kCbWaves), 0, st, G, ldg, n,
                       shift_rel, Lws, status);
    const size_t lds = sizeof(double) * (size_t)(2 * kIbMax + 4) * 256;
    hipError_t e = hipFuncSetAttribute((const void *)tri_inv_blk_kernel<kIbMax>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(tri_inv_blk_kernel<kIbMax>, dim3(ceil_div(n, 16)), dim3(256), lds, st, n,
                       Lws, Rinv, ldr);
  } else if (n <= kMidN) {
    hipLaunchKernelGGL(chol_mid_kernel, dim3(1), dim3(kMidCT), 0, st, G, ldg, n, shift_rel, Lws,
                       status);
    constexpr int kIb = kMidN / 16;
    const size_t lds = sizeof(double) * (size_t)(2 * kIb + 4) * 256;
    hipError_t e = hipFuncSetAttribute((const void *)tri_inv_blk_kernel<kIb>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(tri_inv_blk_kernel<kIb>, dim3(ceil_div(n, 16)), dim3(256), lds, st, n,
                       Lws, Rinv, ldr);
  } else {
    double *tile = glb_tile(ws);
    hipLaunchKernelGGL((chol_kernel<kGlbP, kGlbQ, true>), dim3(1), dim3(kThreads), 0, st, G,
                       ldg, n, shift_rel, Lws, tile, status);
    hipLaunchKernelGGL((tri_inv_kernel<kGlbP, kGlbQ, true>), dim3(1), dim3(kThreads), 0, st, n,
                       Lws, Rinv, ldr, tile);
  }
  return hipGetLastError();
}

hipError_t launch_sym_eig(const double *G, int64_t ldg, int n, int nvec, double *evals,
                          double *evecs, int64_t ldv, double *ws, int *status, hipStream_t st) {
  (void)status;
  if (n <= kRegN) {
    hipLaunchKernelGGL((sym_tridiag_kernel<kRegP, kRegQ, false>), dim3(1), dim3(kThreads), 0,
                       st, G, ldg, n, ws, ws);
    hipLaunchKernelGGL((sym_tridiag_eig_kernel<kRegN, kRegEpw>), dim3(ceil_div(n, kRegEpw)),
                       dim3(64 * kRegEpw), 0, st, n, nvec, evals, evecs, ldv, ws);
    hipLaunchKernelGGL((sym_cluster_kernel<kRegN, 4>), dim3(1), dim3(256), 0, st, n, nvec, evals,
                       evecs, ldv, ws);
    hipLaunchKernelGGL((sym_backtransform_kernel<kRegP, kRegQ, false>), dim3(1),
                       dim3(kThreads), 0, st, n, evecs, ldv, ws, ws);
  } else if (n <= kMidN) {
    hipLaunchKernelGGL(sym_tridiag_mid_kernel, dim3(1), dim3(kMidT), 0, st, G, ldg, n, ws,
                       glb_tile(ws));
    hipLaunchKernelGGL((sym_tridiag_eig_kernel<kGlbN, kGlbEpw>), dim3(ceil_div(n, kGlbEpw)),
                       dim3(64 * kGlbEpw), 0, st, n, nvec, evals, evecs, ldv, ws);
    hipLaunchKernelGGL((sym_cluster_kernel<kGlbN, 2>), dim3(1), dim3(128), 0, st, n, nvec, evals,
                       evecs, ldv, ws);
    hipLaunchKernelGGL(sym_backtransform_mid_kernel, dim3(ceil_div(nvec, 4)), dim3(256), 0, st,
                       n, nvec, evecs, ldv, ws);
  } else {
    double *tile = glb_tile(ws);
    hipLaunchKernelGGL((sym_tridiag_kernel<kGlbP, kGlbQ, true>), dim3(1), dim3(kThreads), 0,
                       st, G, ldg, n, ws, tile);
    hipLaunchKernelGGL((sym_tridiag_eig_kernel<kGlbN, kGlbEpw>), dim3(ceil_div(n, kGlbEpw)),
                       dim3(64 * kGlbEpw), 0, st, n, nvec, evals, evecs, ldv, ws);
    hipLaunchKernelGGL((sym_cluster_kernel<kGlbN, 2>), dim3(1), dim3(128), 0, st, n, nvec, evals,
                       evecs, ldv, ws);
    hipLaunchKernelGGL((sym_backtransform_kernel<kGlbP, kGlbQ, true>), dim3(1),
                       dim3(kThreads), 0, st, n, evecs, ldv, ws, tile);
  }
  return hipGetLastError();
}

}  // namespace ssi
