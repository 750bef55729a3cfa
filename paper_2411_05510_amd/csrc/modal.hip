// Modal stage for one lag, every model order at once (Eq. (9)-(12)).
//
// With O = U_n S_n^1/2 (Eq. (9)), the shift least squares of Eq. (10) gives
//   A_n = S^-1/2 X_n S^1/2,  X_n = pinv(U_top,n) U_bot,n,
// so A_n and X_n have the same eigenvalues and phi = C psi_A = U[0:l, :n] psi_X.
// All orders share one Cholesky factorisation: with U_top^T U_top = R^T R and
// W = R^-T U_top^T U_bot (both leading blocks nest because R^-1 is upper
// triangular), X_n = R^-1[:n, :n] W[:n, :n].
//
// Per order n (one workgroup each):
//   form_x      X_n = Rinv[:n,:n] W[:n,:n]
//   hess        Householder reduction X_n = Q H Q^T (H upper Hessenberg),
//               matrix held in registers over a 16 x 32 thread grid (n <= 224)
//               or reduced in place in global memory (n <= 448)
//   francis     eigenvalues of H by the Francis double-shift QR iteration with
//               deflation, H packed in LDS (n <= 200) or in global scratch
//   vec         per pole (Im mu > 0): inverse iteration on H - mu I in complex
//               arithmetic (column elimination with adjacent pivoting, one
//               wave per pole, 4 or 7 rows of a column per lane), psi_H, then
//               psi_X = Q psi_H by the Hessenberg reflectors and phi =
//               U[0:l, :n] psi_X, normalised; lambda = ln(mu) f_s, f, xi
//   francis and vec run in one persistent launch (eig_persistent_kernel):
//   whole orders first, largest first, then poles, smallest orders first;
//   a pole whose order has not finished is deferred to pole_tail_kernel
//   sort        poles of the order sorted by (f, xi) into the output slots
#include "common.h"
#include "kernels.h"

namespace {

constexpr int kT = 512;                 // threads of the register-tile kernels
constexpr int kTP = 14, kTQ = 7;        // 16 x 32 grid, n <= 224
constexpr int kNR = 224;                // largest order of the register-tile reduction
constexpr int kNMax = 448;              // largest order of the modal stage

SSI_DEV int row_of(int tr, int p) { return tr + 16 * p; }
SSI_DEV int col_of(int tc, int q) { return tc + 32 * q; }
SSI_DEV double sel(bool c, double v) { return c ? v : 0.0; }

SSI_DEV double col_group_sum(double v) { return row16_sum(v); }

struct OrderGeo {
  int n;          // model order
  int64_t sq;     // sum of n'^2 over earlier orders
  int64_t vec;    // sum of n' over earlier orders
  int pole;       // sum of n'/2 over earlier orders
};

SSI_DEV OrderGeo order_geo(int o, int nmin, int step) {
  OrderGeo g{nmin + o * step, 0, 0, 0};
  for (int i = 0; i < o; ++i) {
    const int m = nmin + i * step;
    g.sq += (int64_t)m * m;
    g.vec += m;
    g.pole += m / 2;
  }
  return g;
}

}  // namespace

// ------------------------------------------------------------------ form_x
// X_n[i][j] = sum_{r=i}^{n-1} Rinv[i][r] W[r][j] for every order n at once:
// the sums of the orders are prefixes of one running sum per (i, j) over r,
// written out at each order boundary n = r + 1 with n > j (n > i holds from
// r >= i).  One thread per (i, j) of the largest order; the running offset
// of the next order's matrix in xbuf advances with r.
__global__ void __launch_bounds__(256)
form_x_kernel(const double *__restrict__ rinv, const double *__restrict__ w, int k, int nmin,
              int step, int no, double *__restrict__ xbuf) {
  const int nmax = nmin + (no - 1) * step;
  const int idx = blockIdx.x * 256 + threadIdx.x;
  if (idx >= nmax * nmax) return;
  const int i = idx / nmax, j = idx - i * nmax;
  int nn = nmin, o = 0;          // next order boundary, its index
  int64_t sq = 0;                // offset of order o's matrix
  double s = 0.0;
  for (int r = i; r < nmax; ++r) {
    s += rinv[(int64_t)i * k + r] * w[(int64_t)r * k + j];
    const int n = r + 1;
    while (nn < n) {
      sq += (int64_t)nn * nn;
      nn += step;
      ++o;
    }
    if (nn == n && n > j && o < no) xbuf[sq + (int64_t)i * n + j] = s;
  }
}

// ------------------------------------------------------------------ hess
// Householder reduction of X_n (n <= 224) to upper Hessenberg form.  Writes H
// (n x n, by columns: H(i, j) at j n + i) to hbuf, the reflector vectors to
// vref (v_k in row k of an n x n block at the order's offset sq) and their
// scalars to taus (at the order's offset vec).  TP row blocks of 16 cover
// n <= 16 TP (13 for n <= 208 keeps the register tile clear of scratch
// spills; 14 for n <= 224).
template <int TP>
__global__ void __launch_bounds__(kT)
hess_kernel(const double *__restrict__ xbuf, int nmin, int step, double *__restrict__ hbuf,
            double *__restrict__ vref, double *__restrict__ taus) {
  __shared__ double vbuf[kNR];
  __shared__ double ypart[8][kNR];
  __shared__ double ybuf[kNR];
  __shared__ double stau[2];
  const OrderGeo geo = order_geo(blockIdx.x, nmin, step);
  const int n = geo.n;
  const double *X = xbuf + geo.sq;
  double *H = hbuf + geo.sq;
  double *vr = vref + geo.sq;
  double *tv = taus + geo.vec;
  const int t = threadIdx.x, tr = t & 15, tc = t >> 4, lane = t & 63, wave = t >> 6;
  double g[TP][kTQ];
#pragma unroll
  for (int p = 0; p < TP; ++p)
#pragma unroll
    for (int q = 0; q < kTQ; ++q) {
      const int i = row_of(tr, p), j = col_of(tc, q);
      g[p][q] = sel(i < n && j < n, X[(int64_t)min(i, n - 1) * n + min(j, n - 1)]);
    }
  // Column k lives in column block kq = k / 32; the unrolled block loop makes
  // the owner's registers compile-time indices.  The left update touches rows
  // > k and (up to rounding residue that is never read again) columns >= k;
  // the right update touches columns > k of every row.
#pragma unroll kTQ
  for (int kq = 0; kq < kTQ; ++kq) {
    const int k0 = 32 * kq, k1 = min(k0 + 32, n - 2);
    for (int k = k0; k < k1; ++k) {
      if (tc == (k & 31)) {
        double s2 = 0.0, x1 = 0.0;
#pragma unroll
        for (int p = 0; p < TP; ++p) {
          const int i = row_of(tr, p);
          const double v = g[p][kq];
          x1 += sel(i == k + 1, v);
          s2 += sel(i > k + 1 && i < n, v * v);
        }
        s2 = col_group_sum(s2);
        x1 = col_group_sum(x1);
        double tau = 0.0, v1 = 0.0;
        if (s2 > 0.0) {
          const double alpha = -copysign(sqrt(x1 * x1 + s2), x1);
          v1 = x1 - alpha;
          tau = 2.0 / (s2 + v1 * v1);
        }
#pragma unroll
        for (int p = 0; p < TP; ++p) {
          const int i = row_of(tr, p);
          if (i < n) {
            const double v = (i == k + 1) ? v1 : sel(i > k + 1, g[p][kq]);
            vbuf[i] = v;
            vr[(size_t)k * n + i] = v;
          }
        }
        if (tr == 0) {
          stau[k & 1] = tau;
          tv[k] = tau;
        }
      }
      __syncthreads();
      const double tau = stau[k & 1];
      if (tau != 0.0) {
        // left: X -= tau v (v^T X)
        double zq[kTQ];
#pragma unroll
        for (int q = 0; q < kTQ; ++q) zq[q] = 0.0;
#pragma unroll
        for (int p = 0; p < TP; ++p) {
          if (p < 2 * kq) continue;
          const int i = row_of(tr, p);
          const double vi = sel(i > k && i < n, vbuf[min(i, kNR - 1)]);
#pragma unroll
          for (int q = 0; q < kTQ; ++q) {
            if (q < kq) continue;
            zq[q] += vi * g[p][q];
          }
        }
#pragma unroll
        for (int q = 0; q < kTQ; ++q) zq[q] = (q < kq) ? 0.0 : tau * col_group_sum(zq[q]);
        double vj[kTQ];
#pragma unroll
        for (int q = 0; q < kTQ; ++q) {
          const int j = col_of(tc, q);
          vj[q] = sel(q >= kq && j > k && j < n, vbuf[min(j, kNR - 1)]);
        }
#pragma unroll
        for (int p = 0; p < TP; ++p) {
          const int i = row_of(tr, p);
          const double vi = sel(i > k && i < n, vbuf[min(i, kNR - 1)]);
          double acc = 0.0;
#pragma unroll
          for (int q = 0; q < kTQ; ++q) {
            if (q < kq) continue;
            if (p >= 2 * kq) g[p][q] -= vi * zq[q];
            acc += g[p][q] * vj[q];
          }
          // right: y = X v (row sums over all 32 grid columns)
          acc = rows4_sum(acc);
          if ((lane >> 4) == 0) ypart[wave][i] = acc;
        }
        __syncthreads();
        // y_i = tau sum_w ypart[w][i], reduced once per row
        if (t < n) {
          double y = 0.0;
#pragma unroll
          for (int w = 0; w < 8; ++w) y += ypart[w][t];
          ybuf[t] = y * tau;
        }
        __syncthreads();
#pragma unroll
        for (int p = 0; p < TP; ++p) {
          const int i = row_of(tr, p);
          const double y = sel(i < n, ybuf[min(i, kNR - 1)]);
#pragma unroll
          for (int q = 0; q < kTQ; ++q) {
            if (q < kq) continue;
            g[p][q] -= y * vj[q];
          }
        }
      }
      // No closing barrier: every read of vbuf for column k precedes the
      // barriers above, ypart and ybuf are rewritten only after the next
      // column's first barrier, and tau alternates between two slots.
    }
  }
#pragma unroll
  for (int p = 0; p < TP; ++p)
#pragma unroll
    for (int q = 0; q < kTQ; ++q) {
      const int i = row_of(tr, p), j = col_of(tc, q);
      if (i < n && j < n) H[(int64_t)j * n + i] = (j >= i - 1) ? g[p][q] : 0.0;
    }
}

// ------------------------------------------------------------------ hess (global)
// Householder reduction of X_n for kNR < n <= kNMax, in place in global
// memory: X_n is copied into H by columns and reduced there; the reflectors
// and their scalars are written as by hess_kernel.  One workgroup of kHG
// threads per order; in a pass over columns, wave w takes the columns
// j = w (mod kHW) and lane a holds rows a + 64 u (u < kHU) of each.
//
// With v, tau the reflector of step k, z = X^T v and p = X v (X as step
// k - 1 left it), the two-sided update P X P (P = I - tau v v^T) is
//   X - tau v z^T - w v^T,   w = tau (p - tau (z . v) v),
// since (P X) v = p - tau (z . v) v.  The next step's z and p need column
// k + 1 as this step leaves it, so each step first updates column k + 1
// alone and forms the next reflector from it; the pass that then updates
// columns k + 2 .. n - 1 accumulates the next z (per column) and p (per row)
// from the values it writes.  Each active column is read and written once
// per step.
constexpr int kHG = 512, kHW = kHG / 64, kHU = kNMax / 64;
static_assert(kNMax <= kHG, "one row per thread in the column steps");

namespace {

// Sums of a and b over the workgroup (kHG threads); red holds 2 kHW doubles.
SSI_DEV void hg_sum2(double &a, double &b, double *red) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  a = wave_sum(a);
  b = wave_sum(b);
  __syncthreads();                       // red is free
  if (lane == 0) {
    red[wave] = a;
    red[kHW + wave] = b;
  }
  __syncthreads();
  a = 0.0;
  b = 0.0;
#pragma unroll
  for (int w = 0; w < kHW; ++w) {
    a += red[w];
    b += red[kHW + w];
  }
}

// Reflector of step c from column c; thread t < n holds entry (t, c) in x.
// Writes v to sv and to row c of vr, tau to *stau and tv[c]; returns the
// thread's entry of the reduced column (alpha at row c + 1, zero below).
SSI_DEV double hg_reflector(double x, int c, int n, double *sv, double *stau, double *vr,
                            double *tv, double *red) {
  const int t = threadIdx.x;
  double s2 = (t > c + 1 && t < n) ? x * x : 0.0;
  double x1 = (t == c + 1) ? x : 0.0;
  hg_sum2(s2, x1, red);
  double tau = 0.0, v1 = 0.0, alpha = 0.0;
  if (s2 > 0.0) {
    alpha = -copysign(sqrt(x1 * x1 + s2), x1);
    v1 = x1 - alpha;
    tau = 2.0 / (s2 + v1 * v1);
  }
  if (t < n) {
    const double v = (t == c + 1) ? v1 : (t > c + 1 ? x : 0.0);
    sv[t] = v;
    vr[(size_t)c * n + t] = v;
  }
  if (t == 0) {
    *stau = tau;
    tv[c] = tau;
  }
  return (tau != 0.0 && t > c) ? (t == c + 1 ? alpha : 0.0) : x;
}

// One pass over columns jbeg..n-1: with UPD, x -= tau v_i z_j + w_i v_j and
// store; with ACC, zn[j] = sum_i vn_i x(i, j) and pacc_i += x(i, j) vn_j.
// Two columns per wave are in flight together.
template <bool UPD, bool ACC>
SSI_DEV void hg_pass(double *H, int n, int jbeg, double tau, const double *v, const double *z,
                     const double *w, const double *vn, double *zn, double (&pacc)[kHU]) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double vi[kHU], wi[kHU], vni[kHU];
#pragma unroll
  for (int u = 0; u < kHU; ++u) {
    const int i = lane + 64 * u, ic = min(i, n - 1);
    vi[u] = (UPD && i < n) ? v[ic] : 0.0;
    wi[u] = (UPD && i < n) ? w[ic] : 0.0;
    vni[u] = (ACC && i < n) ? vn[ic] : 0.0;
    pacc[u] = 0.0;
  }
  for (int j0 = jbeg + wave; j0 < n; j0 += 2 * kHW) {
    const int j1 = j0 + kHW;
    const bool has1 = j1 < n;
    double *c0 = H + (int64_t)j0 * n, *c1 = H + (int64_t)min(j1, n - 1) * n;
    double x0[kHU], x1[kHU];
#pragma unroll
    for (int u = 0; u < kHU; ++u) {
      const int ic = min(lane + 64 * u, n - 1);
      x0[u] = c0[ic];
      x1[u] = c1[ic];
    }
    if (UPD) {
      const double tz0 = tau * z[j0], vj0 = v[j0];
      const double tz1 = has1 ? tau * z[j1] : 0.0, vj1 = has1 ? v[j1] : 0.0;
#pragma unroll
      for (int u = 0; u < kHU; ++u) {
        x0[u] -= vi[u] * tz0 + wi[u] * vj0;
        x1[u] -= vi[u] * tz1 + wi[u] * vj1;
      }
#pragma unroll
      for (int u = 0; u < kHU; ++u) {
        const int i = lane + 64 * u;
        if (i < n) {
          c0[i] = x0[u];
          if (has1) c1[i] = x1[u];
        }
      }
    }
    if (ACC) {
      const double vn0 = vn[j0], vn1 = has1 ? vn[j1] : 0.0;
      double s0 = 0.0, s1 = 0.0;
#pragma unroll
      for (int u = 0; u < kHU; ++u) {
        s0 += vni[u] * x0[u];
        s1 += vni[u] * x1[u];
        pacc[u] += x0[u] * vn0 + x1[u] * vn1;
      }
      s0 = wave_sum(s0);
      s1 = wave_sum(s1);
      if (lane == 0) {
        zn[j0] = s0;
        if (has1) zn[j1] = s1;
      }
    }
  }
}

// p of the next step from the per-wave partials, then its w:
// w_i = tau (p_i - tau (z . v) v_i), z . v over the columns from jbeg.
SSI_DEV void hg_finish(int n, int jbeg, const double (&pacc)[kHU], double (*pp)[kNMax],
                       double tau, const double *v, const double *z, double *w, double *red) {
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
#pragma unroll
  for (int u = 0; u < kHU; ++u) {
    const int i = lane + 64 * u;
    if (i < n) pp[wave][i] = pacc[u];
  }
  __syncthreads();
  double p = 0.0;
  if (t < n) {
#pragma unroll
    for (int q = 0; q < kHW; ++q) p += pp[q][t];
  }
  double zv = (t >= jbeg && t < n) ? z[t] * v[t] : 0.0, unused = 0.0;
  hg_sum2(zv, unused, red);
  if (t < n) w[t] = tau * (p - tau * zv * v[t]);
  __syncthreads();
}

}  // namespace

__global__ void __launch_bounds__(kHG)
hess_glb_kernel(const double *__restrict__ xbuf, int nmin, int step, int o0,
                double *__restrict__ hbuf, double *__restrict__ vref, double *__restrict__ taus) {
  __shared__ double sv[2][kNMax];        // reflector of this step, of the next
  __shared__ double sz[2][kNMax];        // z of this step, of the next (by column)
  __shared__ double sw[kNMax];           // w of this step (by row)
  __shared__ double pp[kHW][kNMax];      // per-wave partial sums of the next p
  __shared__ double red[2 * kHW];
  __shared__ double stau[2];
  const OrderGeo geo = order_geo(o0 + blockIdx.x, nmin, step);
  const int n = geo.n;
  const double *X = xbuf + geo.sq;
  double *H = hbuf + geo.sq;
  double *vr = vref + geo.sq;
  double *tv = taus + geo.vec;
  const int t = threadIdx.x;
  // H(i, j) = X(i, j) by columns
  for (int idx = t; idx < n * n; idx += kHG) {
    const int j = idx / n, i = idx - j * n;
    H[idx] = X[(int64_t)i * n + j];
  }
  __syncthreads();
  if (n < 3) return;
  // step 0: its reflector from column 0, then its z and p by a read pass
  {
    double x = t < n ? H[t] : 0.0;
    x = hg_reflector(x, 0, n, sv[0], &stau[0], vr, tv, red);
    if (t < n) H[t] = x;
    __syncthreads();
    double pacc[kHU];
    hg_pass<false, true>(H, n, 1, 0.0, sv[0], sz[0], sw, sv[0], sz[0], pacc);
    hg_finish(n, 1, pacc, pp, stau[0], sv[0], sz[0], sw, red);
  }
  int cur = 0;
  for (int k = 0; k <= n - 3; ++k) {
    const int nx = cur ^ 1;
    const double tau = stau[cur];
    const bool more = k + 1 <= n - 3;
    // column k + 1 under step k, then the reflector of step k + 1 from it
    const int64_t ck = (int64_t)(k + 1) * n;
    double x = 0.0;
    if (t < n) {
      x = H[ck + t];
      x -= tau * sv[cur][t] * sz[cur][k + 1] + sw[t] * sv[cur][k + 1];
    }
    if (more) x = hg_reflector(x, k + 1, n, sv[nx], &stau[nx], vr, tv, red);
    if (t < n) H[ck + t] = x;
    __syncthreads();
    // columns k + 2 .. n - 1 under step k, accumulating step k + 1's z and p
    double pacc[kHU];
    if (more) {
      if (tau != 0.0)
        hg_pass<true, true>(H, n, k + 2, tau, sv[cur], sz[cur], sw, sv[nx], sz[nx], pacc);
      else
        hg_pass<false, true>(H, n, k + 2, tau, sv[cur], sz[cur], sw, sv[nx], sz[nx], pacc);
      hg_finish(n, k + 2, pacc, pp, stau[nx], sv[nx], sz[nx], sw, red);
    } else if (tau != 0.0) {
      hg_pass<true, false>(H, n, k + 2, tau, sv[cur], sz[cur], sw, sv[nx], sz[nx], pacc);
      __syncthreads();
    }
    cur = nx;
  }
}

// ------------------------------------------------------------------ francis
namespace {

constexpr int kNB = 5;                   // bulges (shift pairs) per multishift sweep
constexpr int kFT = 64 * kNB;            // one wave per bulge
constexpr int kSM = 2 * kNB;             // order of the trailing block that supplies shifts
constexpr int kRing = 16;                // bulge-slot ring rows, >= 3 kNB + 1, power of two
constexpr int kMsMin = 24;               // active windows from this size use multishift sweeps
// Deflation tolerance of the trailing block's QR when it only supplies
// shifts: shifts accurate to about 1e-10 keep the convergence of the sweeps,
// and the block's last iterations toward machine precision are saved.
constexpr double kShiftTol = 1e-10;
// LDS after the packed H: bulge slots (2 kRing), shift pairs (2 kNB), the
// shift block's eigenvalues (2 kSM) and the shift block (kSM^2); the last two
// hold a window's reflectors during a multishift sweep.
constexpr int kExtra = 2 * kRing + 2 * kSM + 2 * kNB + kSM * kSM;
constexpr int kLdsMaxN = 200;
constexpr int kLdsDoubles = 20299 + kExtra;   // 20299 = packed size at n = 200

// Upper Hessenberg H in packed rows (row 0: columns 0..n-1; row i >= 1:
// columns i-1..n-1), followed by slots for the entries (i, i-2) and (i, i-3)
// that bulges create below the subdiagonal.  Those exist only inside the
// chain of bulges (at most 3 kNB consecutive rows), so a ring of kRing rows
// indexed by i mod kRing suffices.  Index selection is branch-free.
struct HIdx {
  int n, b2, b3;
  // packed index of (i, j), j >= i - 1, is base(i) + j
  SSI_DEV int base(int i) const { return __mul24(i, n) - (__mul24(i, i - 1) >> 1); }
  SSI_DEV int row_start(int i) const { return base(i) + (i > 0 ? i - 1 : 0); }
  SSI_DEV int operator()(int i, int j) const {
    const int bulge = (j == i - 2 ? b2 : b3) + (i & (kRing - 1));
    return j >= i - 1 ? base(i) + j : bulge;
  }
  static constexpr __host__ __device__ int packed_size(int n) {
    return n + ((n - 1) * (n + 2)) / 2;
  }
};
static_assert(HIdx::packed_size(kLdsMaxN) == 20299, "packed size at the LDS limit");
static_assert(kLdsDoubles * 8 + 64 <= 160 * 1024, "Francis LDS budget");
static_assert(kRing >= 3 * kNB + 1, "bulge ring too short for the chain");

SSI_DEV void two_by_two_eigs(double a, double b, double c, double d, double *wr, double *wi) {
  const double p = 0.5 * (a - d);
  const double disc = p * p + b * c;
  const double mid = 0.5 * (a + d);
  if (disc >= 0.0) {
    const double r = sqrt(disc);
    const double l1 = mid + copysign(r, mid == 0.0 ? 1.0 : mid);
    const double det = a * d - b * c;
    const double l2 = (l1 != 0.0) ? det / l1 : mid - copysign(r, mid == 0.0 ? 1.0 : mid);
    wr[0] = l1; wi[0] = 0.0;
    wr[1] = l2; wi[1] = 0.0;
  } else {
    const double im = sqrt(-disc);
    wr[0] = mid; wi[0] = im;
    wr[1] = mid; wi[1] = -im;
  }
}

SSI_DEV int wave_max_int(int v) { return wave_max_i(v); }

// Maximum over the workgroup; every thread gets the result.
SSI_DEV int block_max_int(int v, int *red) {
  v = wave_max_int(v);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  int r = red[0];
#pragma unroll
  for (int w = 1; w < kFT / 64; ++w) r = max(r, red[w]);
  __syncthreads();
  return __builtin_amdgcn_readfirstlane(r);        // uniform: scalar branches on it
}

// Orders LDS accesses of one wave (the lanes run in lockstep, so a fence
// against compiler reordering is all the ordering needed).
SSI_DEV void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// 3-element Householder reflector (1, v1, v2) with scalar beta that maps
// (x, y, z) to (alpha, 0, 0); beta = 0 when there is nothing to annihilate.
// 1/||.|| and 1/u0 come from the hardware estimates refined by two Newton
// steps each (r <- r (3 - s r^2) / 2 and q <- q (2 - u q)).
SSI_DEV void householder3(double x, double y, double z, double &v1, double &v2, double &beta,
                          double &alpha) {
  const double s = x * x + y * y + z * z;
  v1 = v2 = beta = alpha = 0.0;
  if (!(s > 0.0) || (y == 0.0 && z == 0.0)) return;
  double r = __builtin_amdgcn_rsq(s);
  r = r * (1.5 - 0.5 * s * r * r);
  r = r * (1.5 - 0.5 * s * r * r);
  const double nrm = s * r;
  alpha = -copysign(nrm, x);
  const double u0 = x - alpha;                 // |u0| = |x| + ||.||
  double q = __builtin_amdgcn_rcp(u0);
  q = q * (2.0 - u0 * q);
  q = q * (2.0 - u0 * q);
  v1 = y * q;
  v2 = z * q;
  beta = 1.0 + fabs(x) * r;                    // -u0 / alpha
}

// Eigenvalues of the m x m upper Hessenberg matrix a (row-major, ld kSM, m <=
// kSM; entries below the subdiagonal are zero and stay in place) by the
// double-shift QR iteration, run by one wave.  Returns false if the
// iteration limit is hit.
SSI_DEV bool small_eig(double *a, int m, double *er, double *ei, int lane, double tol) {
  int hi = m - 1, iter = 0, total = 0;
  while (hi >= 0) {
    int cand = 0;
    for (int i = hi - lane; i >= 1; i -= 64) {
      const double sub = fabs(a[i * kSM + i - 1]);
      double ref = fabs(a[(i - 1) * kSM + i - 1]) + fabs(a[i * kSM + i]);
      if (ref == 0.0) {
        if (i >= 2) ref += fabs(a[(i - 1) * kSM + i - 2]);
        if (i + 1 <= hi) ref += fabs(a[(i + 1) * kSM + i]);
      }
      if (sub <= tol * ref) {
        cand = i;
        break;
      }
    }
    const int l = wave_max_int(cand);
    wave_sync();
    if (l > 0 && lane == 0) a[l * kSM + l - 1] = 0.0;
    if (l == hi) {
      er[hi] = a[hi * kSM + hi];
      ei[hi] = 0.0;
      hi -= 1;
      iter = 0;
      wave_sync();
      continue;
    }
    if (l == hi - 1) {
      double r2[2], i2[2];
      two_by_two_eigs(a[(hi - 1) * kSM + hi - 1], a[(hi - 1) * kSM + hi], a[hi * kSM + hi - 1],
                      a[hi * kSM + hi], r2, i2);
      er[hi - 1] = r2[0]; ei[hi - 1] = i2[0];
      er[hi] = r2[1]; ei[hi] = i2[1];
      hi -= 2;
      iter = 0;
      wave_sync();
      continue;
    }
    if (++total > 30 * kSM) return false;
    ++iter;
    double sh, tt;
    if (iter % 11 == 10) {
      // exceptional shift after ten sweeps without deflation, with the
      // constants 3/4 and -0.4375 of LAPACK's DLAHQR
      const double e = fabs(a[hi * kSM + hi - 1]) + fabs(a[(hi - 1) * kSM + hi - 2]);
      const double h11 = 0.75 * e + a[hi * kSM + hi], h12 = -0.4375 * e;
      sh = 2.0 * h11;
      tt = h11 * h11 - h12 * e;
    } else {
      const double p = a[(hi - 1) * kSM + hi - 1], q = a[(hi - 1) * kSM + hi];
      const double r = a[hi * kSM + hi - 1], d = a[hi * kSM + hi];
      sh = p + d;
      tt = p * d - q * r;
    }
    const double h00 = a[l * kSM + l], h01 = a[l * kSM + l + 1], h10 = a[(l + 1) * kSM + l];
    const double h11 = a[(l + 1) * kSM + l + 1], h21 = a[(l + 2) * kSM + l + 1];
    double x = h00 * h00 + h01 * h10 - sh * h00 + tt;
    double y = h10 * (h00 + h11 - sh);
    double z = h10 * h21;
    wave_sync();
    for (int k = l; k <= hi - 1; ++k) {
      const bool three = k < hi - 1;
      const double zz = three ? z : 0.0;
      double v1, v2, beta, alpha;
      householder3(x, y, zz, v1, v2, beta, alpha);
      if (beta != 0.0) {
        const int q0 = max(l, k - 1);
        for (int j = q0 + lane; j <= hi; j += 64) {
          const double a0 = a[k * kSM + j], a1 = a[(k + 1) * kSM + j];
          const double a2 = three ? a[(k + 2) * kSM + j] : 0.0;
          const double d = beta * (a0 + v1 * a1 + v2 * a2);
          a[k * kSM + j] = a0 - d;
          a[(k + 1) * kSM + j] = a1 - d * v1;
          if (three) a[(k + 2) * kSM + j] = a2 - d * v2;
        }
        wave_sync();
        if (k > l && lane == 0) {
          a[(k + 1) * kSM + k - 1] = 0.0;
          if (three) a[(k + 2) * kSM + k - 1] = 0.0;
        }
        const int r = min(k + 3, hi);
        for (int i = l + lane; i <= r; i += 64) {
          const double a0 = a[i * kSM + k], a1 = a[i * kSM + k + 1];
          const double a2 = three ? a[i * kSM + k + 2] : 0.0;
          const double d = beta * (a0 + v1 * a1 + v2 * a2);
          a[i * kSM + k] = a0 - d;
          a[i * kSM + k + 1] = a1 - d * v1;
          if (three) a[i * kSM + k + 2] = a2 - d * v2;
        }
        wave_sync();
      }
      if (k < hi - 1) {
        x = a[(k + 1) * kSM + k];
        y = a[(k + 2) * kSM + k];
        z = (k < hi - 2) ? a[(k + 3) * kSM + k] : 0.0;
      }
      wave_sync();
    }
  }
  return true;
}

}  // namespace


SSI_DEV double readlane_d(double v, int src) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), src);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), src);
  return __hiloint2double(hi, lo);
}

// Value of element e (wave-uniform) of a row spread over the wave as
// v[e / 64] in lane e % 64.  Every register of v is read with its constant
// index and the choice is made on the wave-uniform results, so v never needs
// to be addressable memory.
template <int N>
SSI_DEV double lane_value(const double (&v)[N], int e) {
  const int u = e >> 6, ln = e & 63;
  double r = 0.0;
#pragma unroll
  for (int q = 0; q < N; ++q) {
    const double c = readlane_d(v[q], ln);
    r = (q == u) ? c : r;
  }
  return r;
}

// One double-shift sweep over the active window [l, hi] by one wave (the
// shift pair (s, t) in shp[0..1]); wave-level ordering only.  RI: row or
// column elements per lane (64 RI >= n).
template <int RI>
SSI_DEV void chase1(double *A, const HIdx &ix, int l, int hi, const double *shp, int lane) {
  constexpr int nb = 1, wave = 0;
  const int psz = ix.b2;
  const int stages = (hi - l) + 3 * (nb - 1);
  // The column a bulge needs at its next step is the one its own right-hand
  // update produced in this step (no other update touches it before the next
  // reflector), so it is forwarded from the lanes that computed it.
  bool have = false;
  double nx = 0.0, ny = 0.0, nz = 0.0;
  for (int st = 0; st < stages; ++st) {
    const int k = l + st - 3 * wave;
    const bool on = wave < nb && k >= l && k <= hi - 1;
    const bool three = k < hi - 1;
    double v1 = 0.0, v2 = 0.0, beta = 0.0, alpha = 0.0;
    if (on) {
      double x, y, z;
      if (have) {
        x = nx;
        y = ny;
        z = nz;
      } else if (k == l) {
        const double sh = shp[2 * wave], tt = shp[2 * wave + 1];
        const double h00 = A[ix(l, l)], h01 = A[ix(l, l + 1)], h10 = A[ix(l + 1, l)];
        const double h11 = A[ix(l + 1, l + 1)], h21 = A[ix(l + 2, l + 1)];
        x = h00 * h00 + h01 * h10 - sh * h00 + tt;
        y = h10 * (h00 + h11 - sh);
        z = h10 * h21;
      } else {
        x = A[ix(k, k - 1)];
        y = A[ix(k + 1, k - 1)];
        z = three ? A[ix(k + 2, k - 1)] : 0.0;
      }
      householder3(x, y, three ? z : 0.0, v1, v2, beta, alpha);
    }
    const bool act = on && beta != 0.0;
    have = false;
    if (act) {
      // rows k..k+2 over columns k..hi; entry (k+2, k) is a bulge slot
      const int r0 = ix.base(k), r1 = ix.base(k + 1);
      const int r2 = three ? ix.base(k + 2) : r1;
      const int s2 = psz + ((k + 2) & (kRing - 1));
      const int len = hi - k + 1;
      int i0[RI], i1[RI], i2[RI];
      double a0[RI], a1[RI], a2[RI];
#pragma unroll
      for (int u = 0; u < RI; ++u) {
        if (64 * u >= len) break;
        const int j = k + min(lane + 64 * u, len - 1);
        i0[u] = r0 + j;
        i1[u] = r1 + j;
        i2[u] = three ? (j == k ? s2 : r2 + j) : i1[u];
        a0[u] = A[i0[u]];
        a1[u] = A[i1[u]];
        a2[u] = three ? A[i2[u]] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < RI; ++u) {
        if (64 * u >= len) break;
        if (lane + 64 * u >= len) continue;
        const double d = beta * (a0[u] + v1 * a1[u] + v2 * a2[u]);
        A[i0[u]] = a0[u] - d;
        A[i1[u]] = a1[u] - d * v1;
        if (three) A[i2[u]] = a2[u] - d * v2;
      }
      if (k > l && lane == 0) {          // the reflected column k - 1
        A[r0 + k - 1] = alpha;
        A[psz + ((k + 1) & (kRing - 1))] = 0.0;
        if (three) A[psz + kRing + ((k + 2) & (kRing - 1))] = 0.0;
      }
    }
    wave_sync();
    if (act) {
      // columns k..k+2 over rows l..min(k+3, hi); entries (k+2, k),
      // (k+3, k) and (k+3, k+1) are bulge slots
      const int len = min(k + 3, hi) - l + 1;
      const int sk2 = psz + ((k + 2) & (kRing - 1));
      const int sk3 = psz + ((k + 3) & (kRing - 1));
      int i0[RI], i1[RI], i2[RI];
      double a0[RI], a1[RI], a2[RI], nv[RI];
#pragma unroll
      for (int u = 0; u < RI; ++u) {
        nv[u] = 0.0;
        if (64 * u >= len) break;
        const int i = l + min(lane + 64 * u, len - 1);
        const int bi = ix.base(i) + k;
        i0[u] = i < k + 2 ? bi : (i == k + 2 ? sk2 : sk3 + kRing);
        i1[u] = i < k + 3 ? bi + 1 : sk3;
        i2[u] = three ? bi + 2 : i1[u];
        a0[u] = A[i0[u]];
        a1[u] = A[i1[u]];
        a2[u] = three ? A[i2[u]] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < RI; ++u) {
        if (64 * u >= len) break;
        if (lane + 64 * u >= len) continue;
        const double d = beta * (a0[u] + v1 * a1[u] + v2 * a2[u]);
        nv[u] = a0[u] - d;
        A[i0[u]] = nv[u];
        A[i1[u]] = a1[u] - d * v1;
        if (three) A[i2[u]] = a2[u] - d * v2;
      }
      // next reflector input: column k, rows k+1, k+2 and (when the next
      // step has three rows, i.e. k + 3 <= hi) k+3
      const int e1 = k + 1 - l, e2 = k + 2 - l, e3 = k + 3 - l;
      nx = lane_value(nv, e1);
      ny = lane_value(nv, e2);
      nz = (k + 3 <= hi) ? lane_value(nv, e3) : 0.0;
      have = true;
    }
    wave_sync();
  }
}

// One sweep of kNB bulges over the active window [l, hi] in windows of
// kAdv stages (stage st puts bulge b, carried by wave b, at row k = l + st -
// 3 b).  The rows and columns [w0, w1) of a window, w0 = l + st0 - 3 (kNB -
// 1) and w1 = l + st0 + kAdv + 3 for its first stage st0, hold everything the
// chain reads in those kAdv stages.  Inside the window each reflector is
// applied from the left over columns k..w1-1 and from the right over rows
// w0..k+3, so every phase is one element per lane.  The rest of its rows
// (columns w1..hi) and of its columns (rows l..w0-1) is brought up to date
// after the window: each thread takes one such column or row segment of kWin
// entries into registers and applies the window's reflectors, recorded in
// refl, in stage order.  Reflector (s, b) of a window touches local rows s +
// 3 (kNB - 1 - b) .. + 2 whatever the window, so the registers are addressed
// at compile time.  Reflectors of one stage touch disjoint rows and commute.
// Nothing outside the window is read before it is brought up to date: a
// window's left updates stay in its rows, its right updates in its columns,
// and the next window starts after the deferred updates.
constexpr int kAdv = 8;                  // stages per window
constexpr int kWin = kAdv + 3 * kNB;     // rows and columns of a window
static_assert(kWin <= 64, "a window row or column fits one wave");
static_assert(3 * kNB * kAdv <= 2 * kSM + kSM * kSM, "a window's reflectors fit the shift area");

// x <- P_r x for the window's reflectors r in stage order (from the left on a
// column segment; from the right on a row segment, P_r being symmetric).
SSI_DEV void win_apply(double (&x)[kWin], const double *refl) {
  int off = 0;
#pragma unroll
  for (int s = 0; s < kAdv; ++s) {
    const double *rs = refl + off;
#pragma unroll
    for (int b = 0; b < kNB; ++b) {
      const int lr = s + 3 * (kNB - 1 - b);
      const double v1 = rs[3 * b], v2 = rs[3 * b + 1], beta = rs[3 * b + 2];
      const double d = beta * (x[lr] + v1 * x[lr + 1] + v2 * x[lr + 2]);
      x[lr] -= d;
      x[lr + 1] -= d * v1;
      x[lr + 2] -= d * v2;
    }
    // The next stage's reflector loads take their address through this
    // empty asm, which depends on the row this stage finished: the compiler
    // can neither hoist them nor merge them with this stage's, so one stage
    // of reflectors at a time is held in registers.
    off += 3 * kNB;
    __asm__ volatile("" : "+v"(off) : "v"(x[s]));
  }
}

// Reflector of bulge `wave` for its step at row k of a sweep: from the
// column its previous step left (forwarded in nx, ny, nz when `have`, else read
// from A), or from its shift pair when it enters at k = l.  beta = 0 when the
// bulge is outside the active window or there is nothing to annihilate.
struct Refl { double v1, v2, beta, alpha; };
SSI_DEV Refl bulge_reflector(const double *A, const HIdx &ix, int l, int hi, int k, int wave,
                             const double *shp, bool have, double nx, double ny, double nz) {
  Refl r{0.0, 0.0, 0.0, 0.0};
  if (wave >= kNB || k < l || k > hi - 1) return r;
  const bool three = k < hi - 1;
  double x, y, z;
  if (have) {
    x = nx;
    y = ny;
    z = nz;
  } else if (k == l) {
    const double sh = shp[2 * wave], tt = shp[2 * wave + 1];
    const double h00 = A[ix(l, l)], h01 = A[ix(l, l + 1)], h10 = A[ix(l + 1, l)];
    const double h11 = A[ix(l + 1, l + 1)], h21 = A[ix(l + 2, l + 1)];
    x = h00 * h00 + h01 * h10 - sh * h00 + tt;
    y = h10 * (h00 + h11 - sh);
    z = h10 * h21;
  } else {
    x = A[ix(k, k - 1)];
    y = A[ix(k + 1, k - 1)];
    z = three ? A[ix(k + 2, k - 1)] : 0.0;
  }
  householder3(x, y, three ? z : 0.0, r.v1, r.v2, r.beta, r.alpha);
  return r;
}

SSI_DEV void chase_win(double *A, const HIdx &ix, int l, int hi, const double *shp,
                       double *refl, int wave, int lane) {
  const int t = threadIdx.x;
  const int psz = ix.b2;
  const int stages = (hi - l) + 3 * (kNB - 1);
  // The reflector of a stage is computed at the end of the previous one,
  // before its closing barrier: the column it reads is the one this bulge's
  // own right-hand update just produced (forwarded), or entries that no
  // update of the previous stage's column phase touches.
  Refl rf = bulge_reflector(A, ix, l, hi, l - 3 * wave, wave, shp, false, 0.0, 0.0, 0.0);
  for (int st0 = 0; st0 < stages; st0 += kAdv) {
    const int w0 = l + st0 - 3 * (kNB - 1);
    const int w1 = l + st0 + kAdv + 3;
    const int r_beg = max(w0, l);          // first row (and column) of the window
    const int c_end = min(w1, hi + 1);     // one past its last
    for (int s = 0; s < kAdv; ++s) {
      const int k = l + st0 + s - 3 * wave;
      const bool three = k < hi - 1;
      const double v1 = rf.v1, v2 = rf.v2, beta = rf.beta;   // v2 = 0 when !three
      const bool act = beta != 0.0;
      if (wave < kNB && lane == 0) {
        double *rs = refl + 3 * (s * kNB + wave);
        rs[0] = v1;
        rs[1] = v2;
        rs[2] = beta;
      }
      if (act) {
        // rows k..k+2 over columns k..c_end-1; entry (k+2, k) is a bulge slot.
        // Without a third row the third load repeats the second (v2 = 0).
        const int r0 = ix.base(k), r1 = ix.base(k + 1);
        const int r2 = three ? ix.base(k + 2) : r1;
        const int s2 = psz + ((k + 2) & (kRing - 1));
        if (lane < c_end - k) {
          const int j = k + lane;
          const int i0 = r0 + j, i1 = r1 + j;
          const int i2 = three ? (j == k ? s2 : r2 + j) : i1;
          const double a0 = A[i0], a1 = A[i1], a2 = A[i2];
          const double d = beta * (a0 + v1 * a1 + v2 * a2);
          A[i0] = a0 - d;
          A[i1] = a1 - d * v1;
          if (three) A[i2] = a2 - d * v2;
        }
        if (k > l && lane == 0) {          // the reflected column k - 1
          A[r0 + k - 1] = rf.alpha;
          A[psz + ((k + 1) & (kRing - 1))] = 0.0;
          if (three) A[psz + kRing + ((k + 2) & (kRing - 1))] = 0.0;
        }
      }
      __syncthreads();
      bool have = false;
      double nx = 0.0, ny = 0.0, nz = 0.0;
      if (act) {
        // columns k..k+2 over rows r_beg..min(k+3, hi); entries (k+2, k),
        // (k+3, k) and (k+3, k+1) are bulge slots
        const int rend = min(k + 3, hi);
        const int sk2 = psz + ((k + 2) & (kRing - 1));
        const int sk3 = psz + ((k + 3) & (kRing - 1));
        double nv = 0.0;
        if (lane <= rend - r_beg) {
          const int i = r_beg + lane;
          const int bi = ix.base(i) + k;
          const int i0 = i < k + 2 ? bi : (i == k + 2 ? sk2 : sk3 + kRing);
          const int i1 = i < k + 3 ? bi + 1 : sk3;
          const int i2 = three ? bi + 2 : i1;
          const double a0 = A[i0], a1 = A[i1], a2 = A[i2];
          const double d = beta * (a0 + v1 * a1 + v2 * a2);
          nv = a0 - d;
          A[i0] = nv;
          A[i1] = a1 - d * v1;
          if (three) A[i2] = a2 - d * v2;
        }
        // next reflector input: column k, rows k+1, k+2 and (when the next
        // step has three rows) k+3
        nx = readlane_d(nv, k + 1 - r_beg);
        ny = readlane_d(nv, k + 2 - r_beg);
        nz = (k + 3 <= hi) ? readlane_d(nv, k + 3 - r_beg) : 0.0;
        have = true;
      }
      rf = bulge_reflector(A, ix, l, hi, k + 1, wave, shp, have, nx, ny, nz);
      __syncthreads();
    }
    // deferred updates: columns w1..hi of the window rows (from the left),
    // rows l..r_beg-1 of the window columns (from the right)
    const int n_right = max(0, hi - w1 + 1);
    const int n_top = r_beg - l;
    const int r_lo = r_beg - w0, r_hi = c_end - w0;   // local entries inside [l, hi]
    for (int sg = t; sg < n_right + n_top; sg += kFT) {
      // Entry r of this thread's segment sits at s0 + r d - (right ? r (r - 1) / 2 : 0):
      // a column of rows w0 + r (packed row starts base(w0 + r) = base(w0) + r (n - w0)
      // - r (r - 1) / 2) or a row over columns w0 + r.  Every entry is loaded, at an
      // index clamped into the matrix, so the loads carry no branches and issue back to
      // back.  Entries outside [r_lo, r_hi) are never stored: the reflectors that touch
      // them have beta = 0 (bulges not yet in, or past, the active window) or v2 = 0
      // (the last, two-row step), so they only multiply finite values by zero.
      const bool right = sg < n_right;
      const int s0 = right ? ix.base(w0) + w1 + sg : ix.base(l + sg - n_right) + w0;
      const int d = right ? ix.n - w0 : 1;
      const int rmask = right ? -1 : 0;
      const unsigned valid = ((1u << r_hi) - 1u) & ~((1u << r_lo) - 1u);
      double x[kWin];
      int at = s0;
#pragma unroll
      for (int r = 0; r < kWin; ++r) {
        x[r] = A[min(max(at, 0), psz - 1)];
        at += d - (r & rmask);
      }
      win_apply(x, refl);
      at = s0;
#pragma unroll
      for (int r = 0; r < kWin; ++r) {
        if ((valid >> r) & 1u) A[at] = x[r];
        at += d - (r & rmask);
      }
    }
    __syncthreads();
  }
}

// Eigenvalues of H_n by the QR iteration (eigenvalues only, so updates stay
// inside the active window [l, hi]).  ev: (re[n], im[n]) per order at
// 2 vec(o).  Writes the number of eigenvalues with Im > 0 to npole[o] and
// their indices to pidx at vec(o); flags[o] = 1 if the iteration limit hit.
//
// One workgroup of kNB waves per order.  Active windows of kMsMin rows or
// more take small-bulge multishift sweeps: the kSM eigenvalues of the
// trailing kSM x kSM block (computed by one wave) give kNB shift pairs, one
// per bulge; the bulges enter at the top three rows apart and are chased down
// together, kAdv rows per window of the sweep (chase_win).  Smaller active
// windows, and every eleventh sweep without deflation (ad hoc shifts), use
// one double-shift bulge chased by one wave (chase1).  Wave b carries bulge
// b.  Each stage advances every bulge by one row in two phases separated by
// barriers; bulges are three rows apart, so their reflectors touch disjoint
// rows and columns and commute:
//   rows      each wave computes its bulge's 3-element reflector (all lanes,
//             redundantly) from the column its previous step left, or from
//             its shift pair when it enters, then applies it from the left to
//             rows k..k+2, and sets the reflected column k-1 to (alpha, 0, 0);
//   columns   each wave applies its reflector from the right to columns
//             k..k+2.
// The column k-1 a wave reads at the start of a stage is changed in that
// stage only by its own row phase and by the right-hand update of the bulge
// behind it, which runs after the barrier.
// A: the matrix storage of this order (LDS = true: the workgroup's LDS).
template <bool LDS>
SSI_DEV void francis_order(int o, double *A, const double *__restrict__ hbuf, int nmin, int step,
                           double *__restrict__ evbuf, int *__restrict__ npole,
                           int *__restrict__ pidx, int *__restrict__ flags, int *red,
                           int &small_ok, int sweeps_per_row, int *__restrict__ status) {
  const OrderGeo geo = order_geo(o, nmin, step);
  const int n = geo.n;
  const double *Hin = hbuf + geo.sq;
  double *wr = evbuf + 2 * geo.vec, *wi = wr + n;
  const int t = threadIdx.x, lane = t & 63;
  const int wave = __builtin_amdgcn_readfirstlane(t >> 6);
  const int psz = HIdx::packed_size(n);
  const HIdx ix{n, psz, psz + kRing};
  double *shp = A + psz + 2 * kRing;         // [kNB][2]: s, t of each shift pair
  double *sev = shp + 2 * kNB;               // [2][kSM]
  double *sblk = sev + 2 * kSM;              // [kSM][kSM]
  double *refl = sev;                        // during a sweep: [kAdv][kNB][3] reflectors
  // Thread t copies columns t, t + kFT, ... 16 rows per round: the 16
  // loads are unconditional (clamped) and in flight together; row by row,
  // each load would wait for the previous row's store.
  for (int c = t; c < n; c += kFT) {
    for (int i0 = 0; i0 < n; i0 += 16) {
      double v[16];
#pragma unroll
      for (int r = 0; r < 16; ++r) v[r] = Hin[(int64_t)c * n + min(i0 + r, n - 1)];
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int i = i0 + r;
        const int j0 = i == 0 ? 0 : i - 1;
        if (i < n && c >= j0) A[ix.row_start(i) + c - j0] = v[r];
      }
    }
  }
  for (int i = t; i < 2 * kRing; i += kFT) A[psz + i] = 0.0;
  __syncthreads();
  // a non-finite entry would never deflate: fail the order at once instead
  // of running to the iteration limit (read after the barrier: the copy
  // above is spread over all threads)
  int nonfinite = 0;
  for (int i = t; i < psz; i += kFT) nonfinite |= !isfinite(A[i]);
  nonfinite = block_max_int(nonfinite, red);

  const double eps = 2.220446049250313e-16;
  int hi = n - 1, iter = 0, total = 0;
  // sweeps_per_row * max(10, n) QR sweeps in all (LAPACK's xLAHQR allows 30)
  const int itmax = sweeps_per_row * max(10, n);
  bool failed = nonfinite != 0;
  while (hi >= 0 && !failed) {
    // deflation: largest l in (0, hi] with a negligible subdiagonal entry
    int cand = 0;
    for (int i = hi - t; i >= 1; i -= kFT) {
      const double sub = fabs(A[ix(i, i - 1)]);
      double ref = fabs(A[ix(i - 1, i - 1)]) + fabs(A[ix(i, i)]);
      if (ref == 0.0) {
        if (i >= 2) ref += fabs(A[ix(i - 1, i - 2)]);
        if (i + 1 <= hi) ref += fabs(A[ix(i + 1, i)]);
      }
      if (sub <= eps * ref) {
        cand = i;
        break;
      }
    }
    const int l = block_max_int(cand, red);
    if (l > 0 && t == 0) A[ix(l, l - 1)] = 0.0;
    if (l == hi) {
      if (t == 0) { wr[hi] = A[ix(hi, hi)]; wi[hi] = 0.0; }
      hi -= 1;
      iter = 0;
      __syncthreads();
      continue;
    }
    if (l == hi - 1) {
      if (t == 0) {
        double r2[2], i2[2];
        two_by_two_eigs(A[ix(hi - 1, hi - 1)], A[ix(hi - 1, hi)], A[ix(hi, hi - 1)],
                        A[ix(hi, hi)], r2, i2);
        wr[hi - 1] = r2[0]; wi[hi - 1] = i2[0];
        wr[hi] = r2[1]; wi[hi] = i2[1];
      }
      hi -= 2;
      iter = 0;
      __syncthreads();
      continue;
    }
    if (++total > itmax) {
      failed = true;
      break;
    }
    // A trailing block of at most kSM rows is finished by one wave on its own
    // copy: its eigenvalues do not depend on the rows above it, and the
    // single-wave iteration needs no workgroup barriers.
    if (hi - l + 1 <= kSM) {
      const int mb = hi - l + 1;
      for (int idx = t; idx < kSM * kSM; idx += kFT) {
        const int i = idx / kSM, j = idx - i * kSM;
        sblk[idx] = (i < mb && j < mb && j >= i - 1) ? A[ix(l + i, l + j)] : 0.0;
      }
      __syncthreads();
      if (wave == 0) {
        const bool ok = small_eig(sblk, mb, sev, sev + kSM, lane, eps);
        if (lane == 0) {
          small_ok = ok ? 1 : 0;
          if (ok)
            for (int i = 0; i < mb; ++i) {
              wr[l + i] = sev[i];
              wi[l + i] = sev[kSM + i];
            }
        }
      }
      __syncthreads();
      if (__builtin_amdgcn_readfirstlane(small_ok)) {
        hi = l - 1;
        iter = 0;
        continue;
      }
    }
    ++iter;
    // ---- shifts
    int nb = 1;
    if (hi - l + 1 >= kMsMin && iter % 11 != 10) {
      const int m0 = hi - kSM + 1;
      for (int idx = t; idx < kSM * kSM; idx += kFT) {
        const int i = idx / kSM, j = idx - i * kSM;
        sblk[idx] = (j >= i - 1) ? A[ix(m0 + i, m0 + j)] : 0.0;
      }
      __syncthreads();
      if (wave == 0) {
        const bool ok = small_eig(sblk, kSM, sev, sev + kSM, lane, kShiftTol);
        if (lane == 0) {
          small_ok = ok ? 1 : 0;
          if (ok) {
            // complex conjugate pairs as they come, real shifts two by two
            int b = 0, pend = -1;
            for (int i = 0; i < kSM; ++i) {
              const double re = sev[i], im = sev[kSM + i];
              if (im > 0.0) {
                shp[2 * b] = 2.0 * re;
                shp[2 * b + 1] = re * re + im * im;
                ++b;
              } else if (im == 0.0) {
                if (pend < 0) {
                  pend = i;
                } else {
                  const double r0 = sev[pend];
                  shp[2 * b] = r0 + re;
                  shp[2 * b + 1] = r0 * re;
                  ++b;
                  pend = -1;
                }
              }
            }
            if (pend >= 0 && b < kNB) {      // cannot happen for an even kSM
              shp[2 * b] = 2.0 * sev[pend];
              shp[2 * b + 1] = sev[pend] * sev[pend];
              ++b;
            }
            small_ok = (b == kNB) ? 1 : 0;
          }
        }
      }
      __syncthreads();
      if (__builtin_amdgcn_readfirstlane(small_ok)) nb = kNB;
    }
    if (nb == 1 && t == 0) {
      double sh, tt;
      if (iter % 11 == 10) {
        // exceptional shift (constants 3/4 and -0.4375 of LAPACK's DLAHQR)
        const double e = fabs(A[ix(hi, hi - 1)]) + fabs(A[ix(hi - 1, hi - 2)]);
        const double h11 = 0.75 * e + A[ix(hi, hi)], h12 = -0.4375 * e;
        sh = 2.0 * h11;
        tt = h11 * h11 - h12 * e;
      } else {
        const double a = A[ix(hi - 1, hi - 1)], b = A[ix(hi - 1, hi)];
        const double c = A[ix(hi, hi - 1)], d = A[ix(hi, hi)];
        sh = a + d;
        tt = a * d - b * c;
      }
      shp[0] = sh;
      shp[1] = tt;
    }
    __syncthreads();

    // ---- sweep: nb bulges, bulge b (wave b) enters at stage 3 b; a single
    // bulge needs no block barriers
    if (nb > 1) {
      chase_win(A, ix, l, hi, shp, refl, wave, lane);
    } else {
      if (wave == 0) chase1<LDS ? 4 : kNMax / 64>(A, ix, l, hi, shp, lane);
      __syncthreads();
    }
  }
  __syncthreads();
  if (t == 0) {
    int cnt = 0;
    if (!failed) {
      for (int i = 0; i < n; ++i)
        if (wi[i] > 0.0) pidx[geo.vec + cnt++] = i;
    }
    npole[o] = cnt;
    flags[o] = failed ? 1 : 0;
    if (failed) atomicOr(status, ssi::kStatusEigLimit);
  }
}


// ------------------------------------------------------------------ vec
namespace {

struct cplx { double re, im; };
SSI_DEV cplx cmul(cplx a, cplx b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
SSI_DEV cplx csub(cplx a, cplx b) { return {a.re - b.re, a.im - b.im}; }
SSI_DEV double cabs1(cplx a) { return fabs(a.re) + fabs(a.im); }
SSI_DEV cplx cdiv(cplx a, cplx b) {
  // Smith's algorithm
  if (fabs(b.re) >= fabs(b.im)) {
    const double r = b.im / b.re, den = b.re + r * b.im;
    return {(a.re + a.im * r) / den, (a.im - a.re * r) / den};
  }
  const double r = b.re / b.im, den = b.im + r * b.re;
  return {(a.re * r + a.im) / den, (a.im * r - a.re) / den};
}
// Component-wise choice: a conditional on the structs themselves selects
// between their addresses, which keeps both in scratch memory.
SSI_DEV cplx csel(bool c, cplx a, cplx b) { return {c ? a.re : b.re, c ? a.im : b.im}; }
SSI_DEV double wsum(double v) { return wave_sum(v); }
SSI_DEV double wmax(double v) { return wave_max(v); }

}  // namespace

// Element e (wave-uniform) of a column spread over the wave as v[e / 64] in
// lane e % 64: the register is chosen by a uniform select, then read once.
// The empty asm hides the elements' origin: a select chain over the elements
// of a register array would otherwise be turned into a dynamically indexed
// array, which lives in scratch memory.
template <int N>
SSI_DEV double lane_pick(const double (&v)[N], int e) {
  const int u = e >> 6;
  double s = v[0];
#pragma unroll
  for (int q = 1; q < N; ++q) {
    double t = v[q];
    __asm__("" : "+v"(t));
    s = (q == u) ? t : s;
  }
  return readlane_d(s, e & 63);
}

// A pole item of order n <= 64 KU keeps rows lane + 64 u (u < KU) of a
// column in registers: KU = 4 up to order 256, 7 up to kNMax.
// columns of H in flight in the shifted solve (fewer for the wider columns,
// whose registers the persistent launch cannot spare)
template <int KU> constexpr int ring_v() { return KU <= 4 ? 4 : 2; }

// x = (H - mu I)^{-1} b for an upper Hessenberg H (column-major, column c at
// Hc + c n) by one wave, b given in registers (row i = lane + 64 u in br/bi[u]).
// Gaussian elimination by columns from the right: step j (from n - 2 down to
// 0) clears entry (j + 1, j) with column j + 1, swapping the two columns first
// when |h(j + 1, j)| exceeds the pivot (adjacent pivoting), which makes
// (H - mu I) E_{n-2} ... E_0 = R upper triangular.  Column j + 1 of R is final
// after step j, so the column-oriented back substitution R y = b runs in the
// same loop and R is never stored; then x = E_{n-2} ... E_0 y, applying E_0
// first (the multipliers and swaps wait in LDS).  A pivot below tiny is
// replaced by tiny, as in LAPACK's Hessenberg inverse iteration.  Columns of H
// arrive through a register ring ring_v<KU>() steps ahead.  Writes x to x_re/x_im.
template <int KU>
SSI_DEV void shifted_solve(const double *__restrict__ Hc, int n, cplx mu, double tiny,
                           double (&br)[KU], double (&bi)[KU], double *x_re, double *x_im,
                           double *mult_re, double *mult_im, int *swp) {
  const int lane = threadIdx.x & 63;
  auto col = [&](int c, int u) {            // clamped load of H(lane + 64 u, c)
    const int i = lane + 64 * u;
    return Hc[(int64_t)max(min(c, n - 1), 0) * n + min(i, n - 1)];
  };
  constexpr int kRingV = ring_v<KU>();
  double hq[kRingV][KU];
#pragma unroll
  for (int d = 0; d < kRingV; ++d)
#pragma unroll
    for (int u = 0; u < KU; ++u) hq[d][u] = col(n - 2 - d, u);
  // working column: column n - 1 of H - mu I
  double wr_[KU], wi_[KU];
#pragma unroll
  for (int u = 0; u < KU; ++u) {
    const int i = lane + 64 * u;
    const double h = col(n - 1, u);
    wr_[u] = i < n ? h - (i == n - 1 ? mu.re : 0.0) : 0.0;
    wi_[u] = i == n - 1 ? -mu.im : 0.0;
  }
  for (int j0 = n - 2; j0 >= 0; j0 -= kRingV) {
#pragma unroll
    for (int d = 0; d < kRingV; ++d) {
      const int j = j0 - d;                  // slot d holds column j
      if (j < 0) break;
      // column j of H - mu I: rows 0..j+1
      double ar[KU], ai[KU];
#pragma unroll
      for (int u = 0; u < KU; ++u) {
        const int i = lane + 64 * u;
        ar[u] = i <= j + 1 ? hq[d][u] - (i == j ? mu.re : 0.0) : 0.0;
        ai[u] = i == j ? -mu.im : 0.0;
        hq[d][u] = col(j - kRingV, u);       // refill with column j - kRingV
      }
      const cplx wp{lane_pick(wr_, j + 1), lane_pick(wi_, j + 1)};
      const double ap = lane_pick(ar, j + 1);      // h(j + 1, j), real
      const bool swap = fabs(ap) > cabs1(wp);
      // after the swap: pivot column pv (finalized as column j + 1 of R) and
      // the column ov being cleared at row j + 1
      cplx piv = csel(swap, cplx{ap, 0.0}, wp);
      const cplx oth = csel(swap, wp, cplx{ap, 0.0});
      piv = csel(cabs1(piv) < tiny, cplx{tiny, 0.0}, piv);
      const cplx m = cdiv(oth, piv);
      const cplx cj = {lane_pick(br, j + 1), lane_pick(bi, j + 1)};
      const cplx y = cdiv(cj, piv);
#pragma unroll
      for (int u = 0; u < KU; ++u) {
        const int i = lane + 64 * u;
        const cplx pv = csel(swap, cplx{ar[u], ai[u]}, cplx{wr_[u], wi_[u]});
        const cplx ov = csel(swap, cplx{wr_[u], wi_[u]}, cplx{ar[u], ai[u]});
        const bool above = i <= j;
        const cplx na = csub(ov, cmul(m, pv));
        const cplx nb = csub(cplx{br[u], bi[u]}, cmul(y, pv));
        wr_[u] = above ? na.re : 0.0;        // the next working column (column j)
        wi_[u] = above ? na.im : 0.0;
        br[u] = above ? nb.re : br[u];
        bi[u] = above ? nb.im : bi[u];
      }
      if (lane == 0) {
        mult_re[j] = m.re;
        mult_im[j] = m.im;
        swp[j] = swap;
        x_re[j + 1] = y.re;
        x_im[j + 1] = y.im;
      }
    }
  }
  {
    cplx piv{lane_pick(wr_, 0), lane_pick(wi_, 0)};
    piv = csel(cabs1(piv) < tiny, cplx{tiny, 0.0}, piv);
    const cplx y = cdiv(cplx{lane_pick(br, 0), lane_pick(bi, 0)}, piv);
    wave_sync();                           // x[1..n-1], mult and swp are in LDS
    // x = E_{n-2} ... E_0 y.  E_j y: y_{j+1} -= m_j y_j, then y_j and y_{j+1}
    // swap if the columns did.  cur is the current y_j (y_{j+1} is still
    // untouched in x).  Every lane runs the recurrence (the same values: LDS
    // broadcasts); lane 0 stores.
    cplx cur = y;
    for (int j = 0; j + 1 < n; ++j) {
      const cplx m{mult_re[j], mult_im[j]};
      const cplx nb = csub(cplx{x_re[j + 1], x_im[j + 1]}, cmul(m, cur));
      const bool sw = swp[j] != 0;
      const cplx fin = csel(sw, nb, cur);  // swapped: cur carries on as y_{j+1}
      cur = csel(sw, cur, nb);
      if (lane == 0) {
        x_re[j] = fin.re;
        x_im[j] = fin.im;
      }
    }
    if (lane == 0) {
      x_re[n - 1] = cur.re;
      x_im[n - 1] = cur.im;
    }
  }
  wave_sync();
}

// Vector, mode shape and continuous pole of pole j of order o, by one wave.
// x_re, x_im, mult_re, mult_im (64 KU doubles each) and swp (64 KU ints) are this
// wave's LDS.  H is stored by columns; ut is U[0:l, :k] transposed (row c
// holds column c of U, l entries).  Writes the unsorted pole f, xi, mu, phi
// (l complex) at slot pole(o) + j of the temporary arrays.
//
// Every global load in the loops below is issued by all lanes: out-of-range
// loads read a clamped address (a finite entry of the same matrix), the ring
// registers hold the raw loaded values, and the masking select happens when a
// value is used, ring_v<KU>() (or kRingQ) steps later.  A load under a branch, or a
// select right after it, makes the compiler wait for the load at once, which
// defeats the rings that keep columns and reflectors several steps ahead.
template <int KU>
SSI_DEV void vec_pole(int o, int j, const double *__restrict__ hbuf,
                      const double *__restrict__ vref, const double *__restrict__ taus,
                      const double *__restrict__ ut, const double *__restrict__ evbuf,
                      const int *__restrict__ pidx, int nmin, int step, int l, double fs,
                      double *x_re, double *x_im, double *mult_re, double *mult_im, int *swp,
                      double *__restrict__ tf, double *__restrict__ txi,
                      double *__restrict__ tmu, double *__restrict__ tphi) {
  const int lane = threadIdx.x & 63;
  const OrderGeo geo = order_geo(o, nmin, step);
  const int n = geo.n;
  const double *Hc = hbuf + geo.sq;
  const double *wr = evbuf + 2 * geo.vec, *wi = wr + n;
  const int e = pidx[geo.vec + j];
  const cplx mu{wr[e], wi[e]};
  // scale of H: max over columns c of |h(0, c)| + |h(n - 1, c)|, and |mu|
  double hnorm = 0.0;
  for (int c = lane; c < n; c += 64)
    hnorm = fmax(hnorm, fabs(Hc[(int64_t)c * n]) + fabs(Hc[(int64_t)c * n + n - 1]));
  hnorm = fmax(wmax(hnorm), cabs1(mu));
  const double tiny = 2.220446049250313e-16 * fmax(hnorm, 1e-300);
  // ---- inverse iteration: x = (H - mu I)^{-1} 1, accepted when x has grown
  // enough, max|x| tiny >= 0.1 / sqrt(n) (the acceptance test of LAPACK's
  // Hessenberg inverse iteration); otherwise a second solve with the
  // normalized x as right-hand side.
  double br[KU], bi[KU];
#pragma unroll
  for (int u = 0; u < KU; ++u) {
    br[u] = (lane + 64 * u) < n ? 1.0 : 0.0;
    bi[u] = 0.0;
  }
  for (int pass = 0; pass < 2; ++pass) {
    shifted_solve<KU>(Hc, n, mu, tiny, br, bi, x_re, x_im, mult_re, mult_im, swp);
    double mx = 0.0;
    for (int c = lane; c < n; c += 64) mx = fmax(mx, cabs1(cplx{x_re[c], x_im[c]}));
    mx = wmax(mx);
    const double inv = mx > 0.0 ? 1.0 / mx : 1.0;
#pragma unroll
    for (int u = 0; u < KU; ++u) {
      const int c = lane + 64 * u;
      const int cc = min(c, n - 1);
      br[u] = c < n ? x_re[cc] * inv : 0.0;
      bi[u] = c < n ? x_im[cc] * inv : 0.0;
    }
    wave_sync();                            // every lane has read x
#pragma unroll
    for (int u = 0; u < KU; ++u) {
      const int c = lane + 64 * u;
      if (c < n) { x_re[c] = br[u]; x_im[c] = bi[u]; }
    }
    wave_sync();
    if (mx * tiny >= 0.1 / sqrt((double)n)) break;    // grown enough: accepted
  }
  // ---- psi_X = Q psi_H, Q = H_0 H_1 ... H_{n-3} the reflectors of the
  // Hessenberg reduction (H_k = I - tau_k v_k v_k^T, v_k zero at and above
  // row k): applied from H_{n-3} down to H_0, psi in registers (lane c % 64,
  // slot c / 64), the reflector rows arriving through a register ring.
  {
    const double *vr = vref + geo.sq;
    const double *tv = taus + geo.vec;
    constexpr int kRingQ = KU <= 4 ? 8 : 4;
    double pr_[KU], pi_[KU], vq[kRingQ][KU];
#pragma unroll
    for (int u2 = 0; u2 < KU; ++u2) {
      pr_[u2] = br[u2];
      pi_[u2] = bi[u2];
    }
#pragma unroll
    for (int d = 0; d < kRingQ; ++d)
#pragma unroll
      for (int u2 = 0; u2 < KU; ++u2) {
        const int c = lane + 64 * u2, k = n - 3 - d;
        vq[d][u2] = vr[(size_t)max(k, 0) * n + min(c, n - 1)];
      }
    for (int k0 = n - 3; k0 >= 0; k0 -= kRingQ) {
#pragma unroll
      for (int d = 0; d < kRingQ; ++d) {
        const int k = k0 - d;
        if (k < 0) break;
        const double tau = tv[k];
        double vk[KU];                      // row k of the reflectors, rows < n
        double sre = 0.0, sim = 0.0;
#pragma unroll
        for (int u2 = 0; u2 < KU; ++u2) {
          vk[u2] = (lane + 64 * u2 < n) ? vq[d][u2] : 0.0;
          sre += vk[u2] * pr_[u2];
          sim += vk[u2] * pi_[u2];
        }
        sre = tau * wsum(sre);
        sim = tau * wsum(sim);
#pragma unroll
        for (int u2 = 0; u2 < KU; ++u2) {
          pr_[u2] -= sre * vk[u2];
          pi_[u2] -= sim * vk[u2];
          // refill with reflector k - kRingQ (raw: masked when it is used)
          const int c = lane + 64 * u2, kn = k - kRingQ;
          vq[d][u2] = vr[(size_t)max(kn, 0) * n + min(c, n - 1)];
        }
      }
    }
#pragma unroll
    for (int u2 = 0; u2 < KU; ++u2) {
      const int c = lane + 64 * u2;
      if (c < n) { x_re[c] = pr_[u2]; x_im[c] = pi_[u2]; }
    }
    wave_sync();
  }
  // ---- phi = U[0:l, :n] psi_X (Eq. (12) via C = first l rows of the
  // observability matrix), unit 2-norm, largest-modulus entry real positive.
  // Lane a holds rows a + 64 r of phi (r < kSR, a pass of 64 kSR rows): row
  // c of ut is read by consecutive lanes (coalesced), psi_X[c] is an LDS
  // broadcast, and the loads of kSC columns of every row block are in flight
  // together.  Columns past n read column n - 1 and are weighted by zero.
  constexpr int kSR = 4, kSC = 8;
  const int slot = geo.pole + j;
  double *ph = tphi + (size_t)slot * l * 2;
  double nrm2 = 0.0, best = -1.0, bre = 1.0, bim = 0.0;
  for (int a0 = 0; a0 < l; a0 += 64 * kSR) {
    int ac[kSR];
#pragma unroll
    for (int r = 0; r < kSR; ++r) ac[r] = min(a0 + 64 * r + lane, l - 1);
    double sre[kSR], sim[kSR];
#pragma unroll
    for (int r = 0; r < kSR; ++r) { sre[r] = 0.0; sim[r] = 0.0; }
    for (int c0 = 0; c0 < n; c0 += kSC) {
      double cv[kSC][kSR];
#pragma unroll
      for (int q = 0; q < kSC; ++q)
#pragma unroll
        for (int r = 0; r < kSR; ++r) cv[q][r] = ut[(int64_t)min(c0 + q, n - 1) * l + ac[r]];
#pragma unroll
      for (int q = 0; q < kSC; ++q) {
        const int cq = min(c0 + q, n - 1);
        const double w = (c0 + q < n) ? 1.0 : 0.0;
        const double xr = x_re[cq] * w, xi = x_im[cq] * w;
#pragma unroll
        for (int r = 0; r < kSR; ++r) {
          sre[r] += cv[q][r] * xr;
          sim[r] += cv[q][r] * xi;
        }
      }
    }
#pragma unroll
    for (int r = 0; r < kSR; ++r) {
      const int a = a0 + 64 * r + lane;
      if (a < l) {
        ph[2 * a] = sre[r];
        ph[2 * a + 1] = sim[r];
        const double m2 = sre[r] * sre[r] + sim[r] * sim[r];
        nrm2 += m2;
        if (m2 > best) { best = m2; bre = sre[r]; bim = sim[r]; }
      }
    }
  }
  nrm2 = wsum(nrm2);
  // lane holding the largest-modulus entry (ties: lowest lane)
  const double bmax = wmax(best);
  const unsigned long long ball = __ballot(best == bmax);
  const int src = __ffsll((long long)ball) - 1;
  bre = __shfl(bre, src, 64);
  bim = __shfl(bim, src, 64);
  const double bm = sqrt(bre * bre + bim * bim);
  const double inv = (nrm2 > 0.0 && bm > 0.0) ? 1.0 / (sqrt(nrm2) * bm) : 1.0;
  // multiply by conj(b) / (|b| |phi|)
  const double cre = bre * inv, cim = -bim * inv;
  for (int a = lane; a < l; a += 64) {
    const double pr = ph[2 * a], pi = ph[2 * a + 1];
    ph[2 * a] = pr * cre - pi * cim;
    ph[2 * a + 1] = pr * cim + pi * cre;
  }
  if (lane == 0) {
    const double lr = 0.5 * log(mu.re * mu.re + mu.im * mu.im) * fs;
    const double li = atan2(mu.im, mu.re) * fs;
    const double al = sqrt(lr * lr + li * li);
    tf[slot] = al / (2.0 * M_PI);
    txi[slot] = -lr / al;
    tmu[2 * slot] = mu.re;
    tmu[2 * slot + 1] = mu.im;
  }
  wave_sync();
}

// ------------------------------------------------------------------ eig
// Eigenvalues and pole vectors of every order in one persistent launch of
// one workgroup per CU, followed by a short launch for the poles left over.
// Phase 1: each workgroup takes whole orders from a counter, largest first,
// and runs the QR iteration on them; finishing an order publishes its
// eigenvalues with a release store of done[o] and then lowers the count of
// orders still running.  Phase 2: while some order is still running, each
// wave takes poles from a second counter, smallest orders first; a pole whose
// order has not finished is not waited for: the wave appends it to a deferred
// list and leaves.  Poles of small orders thus run beside the QR iterations
// of the large ones, workgroups with nothing ready leave the chip at once
// (work on other streams can use the CUs while the largest orders finish),
// and the deferred poles and those never claimed are left to the tail launch
// (pole_tail_kernel), whose waves all find their orders finished.  Every
// claim is one fetch-and-add: a compare-and-swap claim that first checks the
// order serializes thousands of waves on one counter.
namespace {
constexpr int kEigGrid = 256;                       // workgroups (one per CU)
// per-wave LDS of a pole item (doubles): x_re, x_im, mult_re, mult_im, swp
template <int KU> constexpr int vec_lds() { return 5 * 64 * KU; }
// queue: [0] next order item, [1] next pole item, [2] order items still
// running, [3] deferred poles, [4] next tail item, [5..] the deferred poles
// (at most one per wave of the persistent launch)
constexpr int kQDeferred = 5;
constexpr int kMaxDeferred = kEigGrid * (kFT / 64);
static_assert(kFT / 64 * vec_lds<kNMax / 64>() <= kLdsDoubles, "pole items fit the workgroup's LDS");

// Pole items, smallest orders first; within an order, lag by lag and pole by pole.
SSI_DEV int pole_items_total(int n_orders, int n_lags, int nmin, int step) {
  int total = 0;
  for (int o = 0; o < n_orders; ++o) total += n_lags * ((nmin + o * step) / 2);
  return total;
}
struct PoleItem { int o, g, j; };
SSI_DEV PoleItem pole_item(int it, int n_lags, int nmin, int step) {
  int o = 0, rem = it;
  while (rem >= n_lags * ((nmin + o * step) / 2)) {
    rem -= n_lags * ((nmin + o * step) / 2);
    ++o;
  }
  const int half = (nmin + o * step) / 2;
  const int g = rem / half;
  return {o, g, rem - g * half};
}

// Claims the next pole item for lane 0's wave, or returns -1 (the wave
// leaves).  Persistent launch: none once every order has finished (the rest
// is the tail's); a claimed pole of an unfinished order is deferred.  Tail
// launch: the deferred poles, then the poles never claimed.
SSI_DEV int claim_pole(int *queue, const int *done, int total, int n_orders, int n_lags,
                       int nmin, int step, bool tail, int *status) {
  if (!tail) {
    if (__hip_atomic_load(&queue[2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) <= 0) return -1;
    const int c = atomicAdd(&queue[1], 1);
    if (c >= total) return -1;
    const PoleItem pi = pole_item(c, n_lags, nmin, step);
    if (__hip_atomic_load(&done[pi.g * n_orders + pi.o], __ATOMIC_ACQUIRE,
                          __HIP_MEMORY_SCOPE_AGENT))
      return c;
    const int d = atomicAdd(&queue[3], 1);
    if (d < kMaxDeferred) queue[kQDeferred + d] = c;
    else atomicOr(status, ssi::kStatusClaimCap);    // cannot happen: one per wave
    return -1;
  }
  const int ndef = min(__hip_atomic_load(&queue[3], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT),
                       kMaxDeferred);
  const int first = min(__hip_atomic_load(&queue[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT),
                        total);
  const int t = atomicAdd(&queue[4], 1);
  if (t < ndef) return queue[kQDeferred + t];
  const int it = first + (t - ndef);
  return it < total ? it : -1;
}

// Pole items for one wave until claim_pole gives none.  x: this wave's LDS
// (vec_lds<KU>() doubles).
template <int KU>
SSI_DEV void pole_phase(bool tail, double *x, const double *__restrict__ hbuf,
                        const double *__restrict__ vref, const double *__restrict__ taus,
                        const double *__restrict__ u, int nmin, int step, int n_orders,
                        int l, double fs, const double *__restrict__ evbuf,
                        const int *__restrict__ npole, const int *__restrict__ pidx,
                        double *__restrict__ tf,
                        double *__restrict__ txi, double *__restrict__ tmu,
                        double *__restrict__ tphi, int *__restrict__ queue,
                        const int *__restrict__ done, int *__restrict__ status, int n_lags,
                        const ssi::ModalStrides &ls) {
  const int lane = threadIdx.x & 63;
  double *x_re = x, *x_im = x_re + 64 * KU, *mult_re = x_im + 64 * KU,
         *mult_im = mult_re + 64 * KU;
  int *swp = reinterpret_cast<int *>(mult_im + 64 * KU);
  const int total = pole_items_total(n_orders, n_lags, nmin, step);
  for (;;) {
    int it = -1;
    if (lane == 0)
      it = claim_pole(queue, done, total, n_orders, n_lags, nmin, step, tail, status);
    it = __builtin_amdgcn_readfirstlane(__shfl(it, 0, 64));
    if (it < 0) break;
    const PoleItem pi = pole_item(it, n_lags, nmin, step);
    const int *dn = done + pi.g * n_orders + pi.o;
    // every lane acquires the order's eigenvalues; an order that never ran
    // (the phase-1 pass cap, reported through the status word) has no poles
    if (!__hip_atomic_load(dn, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT)) continue;
    if (pi.j >= npole[pi.g * n_orders + pi.o]) continue;
    const int g = pi.g;
    vec_pole<KU>(pi.o, pi.j, hbuf + g * ls.sq, vref + g * ls.vref, taus + g * ls.taus, u + g * ls.u,
             evbuf + g * 2 * ls.vec, pidx + g * ls.vec, nmin, step, l, fs, x_re, x_im,
             mult_re, mult_im, swp, tf + g * ls.poles, txi + g * ls.poles,
             tmu + g * 2 * ls.poles, tphi + g * 2 * ls.poles * l);
  }
}
}  // namespace

__global__ void __launch_bounds__(kFT)
eig_init_kernel(int *__restrict__ queue, int *__restrict__ done, int n_items) {
  // the counters of queue (the deferred list needs no clearing)
  for (int i = threadIdx.x; i < n_items + kQDeferred; i += blockDim.x) {
    if (i < kQDeferred) queue[i] = i == 2 ? n_items : 0;
    else done[i - kQDeferred] = 0;
  }
}

template <int KU>
__global__ void __launch_bounds__(kFT)
eig_persistent_kernel(const double *__restrict__ hbuf, const double *__restrict__ vref,
                      const double *__restrict__ taus, const double *__restrict__ u,
                      int nmin, int step, int n_orders, int l, double fs,
                      double *__restrict__ gscr, int64_t gstride, double *__restrict__ evbuf,
                      int *__restrict__ npole, int *__restrict__ pidx, int *__restrict__ flags,
                      double *__restrict__ tf,
                      double *__restrict__ txi, double *__restrict__ tmu,
                      double *__restrict__ tphi, int *__restrict__ queue, int *__restrict__ done,
                      int *__restrict__ status, int sweeps_per_row, int n_lags,
                      ssi::ModalStrides ls) {
  extern __shared__ double lds_h[];
  __shared__ int red[kFT / 64];
  __shared__ int small_ok, item;
  const int t = threadIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(t >> 6);
  // Work items are (lag, order) pairs of every lag of the launch; lag g's
  // buffers sit at g times the per-lag stride of each buffer (ls).
  const int n_items = n_lags * n_orders;
  // ---- phase 1: orders, largest first across lags.  The loop exit is a wave-uniform
  // (scalar) branch, and thread 0's publish-and-claim is a single region
  // between two barriers: with the item read as a per-lane value, or the
  // claim and the publish as two separate thread-0 regions around the back
  // edge, the compiler may let lanes 1..63 of wave 0 re-enter the body
  // without thread 0 and re-read the old item.
  // Every pass claims a fresh counter value, so a workgroup makes at most
  // n_items + 1 claims; the pass count is capped at that all the same, and
  // a workgroup that reaches the cap sets status bit kStatusClaimCap and stops.
  if (t == 0) item = atomicAdd(&queue[0], 1);
  __syncthreads();
  for (int pass = 0;; ++pass) {
    const int it = __builtin_amdgcn_readfirstlane(item);
    __syncthreads();                                // every wave has read item
    if (it >= n_items) break;
    if (pass > n_items) {
      if (t == 0) atomicOr(status, ssi::kStatusClaimCap);
      break;
    }
    const int o = n_orders - 1 - it / n_lags, g = it - (it / n_lags) * n_lags;
    const double *hb = hbuf + g * ls.sq;
    double *ev = evbuf + g * 2 * ls.vec;
    int *np = npole + g * n_orders, *pi = pidx + g * ls.vec, *fl = flags + g * n_orders;
    if (nmin + o * step <= kLdsMaxN)
      francis_order<true>(o, lds_h, hb, nmin, step, ev, np, pi, fl, red, small_ok,
                          sweeps_per_row, status);
    else
      francis_order<false>(o, gscr + ((size_t)g * n_orders + o) * gstride, hb, nmin, step, ev,
                           np, pi, fl, red, small_ok, sweeps_per_row, status);
    __threadfence();
    __syncthreads();
    if (t == 0) {
      __hip_atomic_store(&done[g * n_orders + o], 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_fetch_add(&queue[2], -1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      item = atomicAdd(&queue[0], 1);
    }
    __syncthreads();
  }
  // ---- phase 2: poles of finished orders, smallest orders first
  __syncthreads();                                  // LDS of the QR iteration is free
  pole_phase<KU>(false, lds_h + wave * vec_lds<KU>(), hbuf, vref, taus, u,
             nmin, step, n_orders, l, fs, evbuf, npole, pidx, tf, txi, tmu,
             tphi, queue, done, status, n_lags, ls);
}

// The poles phase 2 left: every order has finished when this launch starts.
// kTailWaves waves per workgroup, one per SIMD.
constexpr int kTailWaves = 4;
template <int KU>
__global__ void __launch_bounds__(64 * kTailWaves)
pole_tail_kernel(const double *__restrict__ hbuf, const double *__restrict__ vref,
                 const double *__restrict__ taus, const double *__restrict__ u,
                 int nmin, int step, int n_orders, int l, double fs,
                 const double *__restrict__ evbuf, const int *__restrict__ npole,
                 const int *__restrict__ pidx,
                 double *__restrict__ tf, double *__restrict__ txi, double *__restrict__ tmu,
                 double *__restrict__ tphi, int *__restrict__ queue,
                 const int *__restrict__ done, int *__restrict__ status, int n_lags,
                 ssi::ModalStrides ls) {
  extern __shared__ double lds_v[];
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  pole_phase<KU>(true, lds_v + wave * vec_lds<KU>(), hbuf, vref, taus, u,
             nmin, step, n_orders, l, fs, evbuf, npole, pidx, tf, txi, tmu,
             tphi, queue, done, status, n_lags, ls);
}

// dst[c l + a] = U[a, c] for a < l, c < k: thread i takes entry i of dst.
__global__ void __launch_bounds__(256)
mode_head_kernel(const double *__restrict__ u, int k, int l, double *__restrict__ dst) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= (int64_t)k * l) return;
  const int64_t c = i / l, a = i - c * l;
  dst[i] = u[a * k + c];
}

// ------------------------------------------------------------------ sort
// Poles of order o sorted by (f, xi), index as the final tie-break.  The keys
// pass through LDS 256 at a time, and every thread counts the keys below its
// own (its rank); the mode shapes of 256 poles are then moved by the whole
// block, consecutive threads on consecutive floats of a row.  With one
// workgroup per order the copy is bound by load latency, not bandwidth.
__global__ void __launch_bounds__(256)
sort_kernel(int nmin, int step, int l, const int *__restrict__ npole,
            const int *__restrict__ flags_in, const double *__restrict__ tf,
            const double *__restrict__ txi, const double *__restrict__ tmu,
            const double *__restrict__ tphi, int32_t *__restrict__ count,
            int32_t *__restrict__ flags_out, double *__restrict__ f, double *__restrict__ xi,
            double *__restrict__ mu, float *__restrict__ phi, int n_orders, int64_t poles) {
  __shared__ double sf[256], sx[256];
  __shared__ int srank[256];
  const int o = blockIdx.x, t = threadIdx.x;
  // lag blockIdx.y: its inputs and its output slots at lag times the
  // per-lag sizes (n_orders counts, poles pole slots)
  {
    const int g = blockIdx.y;
    npole += g * n_orders;
    flags_in += g * n_orders;
    count += g * n_orders;
    flags_out += g * n_orders;
    tf += g * poles;
    txi += g * poles;
    f += g * poles;
    xi += g * poles;
    tmu += 2 * g * poles;
    mu += 2 * g * poles;
    tphi += 2 * g * poles * l;
    phi += 2 * g * poles * l;
  }
  const OrderGeo geo = order_geo(o, nmin, step);
  const int cnt = npole[o];
  const int base = geo.pole;
  const int row = 2 * l;                     // floats of one mode shape
  if (t == 0) {
    count[o] = cnt;
    flags_out[o] = flags_in[o];
  }
  for (int i0 = 0; i0 < cnt; i0 += 256) {
    const int i = i0 + t;
    const bool own = i < cnt;
    const double fi = own ? tf[base + i] : 0.0, xi_i = own ? txi[base + i] : 0.0;
    int rank = 0;
    for (int j0 = 0; j0 < cnt; j0 += 256) {
      __syncthreads();                       // the previous keys and ranks are read
      if (j0 + t < cnt) {
        sf[t] = tf[base + j0 + t];
        sx[t] = txi[base + j0 + t];
      }
      __syncthreads();
      const int jn = min(256, cnt - j0);
      for (int jj = 0; jj < jn; ++jj) {
        const int j = j0 + jj;
        const double fj = sf[jj], xj = sx[jj];
        rank += (fj < fi) || (fj == fi && (xj < xi_i || (xj == xi_i && j < i)));
      }
    }
    if (own) {
      const int dst = base + rank;
      srank[t] = rank;
      f[dst] = fi;
      xi[dst] = xi_i;
      mu[2 * dst] = tmu[2 * (base + i)];
      mu[2 * dst + 1] = tmu[2 * (base + i) + 1];
    }
    __syncthreads();
    // eight loads in flight per thread: indices clamped to the last entry,
    // whose repeats are not stored
    const int tot = min(256, cnt - i0) * row;
    const double *src = tphi + (size_t)(base + i0) * row;
    for (int idx0 = t; idx0 < tot; idx0 += 8 * 256) {
      double v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = src[min(idx0 + u * 256, tot - 1)];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int idx = idx0 + u * 256;
        if (idx < tot) {
          const int q = idx / row, a = idx - q * row;
          phi[(size_t)(base + srank[q]) * row + a] = (float)v[u];
        }
      }
    }
  }
  // slots past the count are zero, so the outputs never depend on what the
  // buffers held before; they are one contiguous run of rows
  const int nz = geo.n / 2 - cnt;
  for (int q = t; q < nz; q += 256) {
    const int dst = base + cnt + q;
    f[dst] = 0.0;
    xi[dst] = 0.0;
    mu[2 * dst] = 0.0;
    mu[2 * dst + 1] = 0.0;
  }
  float *pz = phi + (size_t)(base + cnt) * row;
  for (int idx = t; idx < nz * row; idx += 256) pz[idx] = 0.f;
}

// ------------------------------------------------------------------ launch
namespace ssi {

int modal_max_order() { return kNMax; }


ModalSizes modal_sizes(int nmin, int nmax, int step, int l) {
  ModalSizes s{};
  s.n_orders = (nmax - nmin) / step + 1;
  for (int o = 0; o < s.n_orders; ++o) {
    const int64_t n = nmin + (int64_t)o * step;
    s.sq += n * n;
    s.vec += n;
    s.poles += n / 2;
  }
  s.vref = s.sq;                 // reflector v_k of order n: row k of an n x n block
  s.taus = s.vec;
  // packed matrix of each order above the LDS limit in global scratch
  s.francis_glb = nmax > kLdsMaxN ? (int64_t)HIdx::packed_size(nmax) + kExtra : 0;
  s.queue_ints = kQDeferred + kMaxDeferred;
  return s;
}

ModalStrides modal_strides(const ModalSizes &s, int l, int ldu) {
  ModalStrides m{};
  m.sq = s.sq;
  m.vec = s.vec;
  m.poles = s.poles;
  m.vref = s.vref;
  m.taus = s.taus;
  m.u = (int64_t)l * ldu;
  return m;
}

hipError_t launch_modal_prep(const ModalArgs &a, int lag, hipStream_t st) {
  const ModalSizes &s = a.sizes;
  const int no = s.n_orders;
  const int nmax = a.nmin + (no - 1) * a.step;
  const ModalStrides ls = modal_strides(s, a.l, a.ldu);
  hipLaunchKernelGGL(form_x_kernel, dim3(ceil_div(nmax * nmax, 256)), dim3(256), 0, st, a.rinv,
                     a.w, a.ldw, a.nmin, a.step, no, a.xbuf);
  double *hb = a.hbuf + lag * ls.sq, *vr = a.vref + lag * ls.vref, *ta = a.taus + lag * ls.taus;
  // orders up to kNR in the register tile, the rest (orders ascend) in global memory
  const int no_reg = a.nmin > kNR ? 0 : std::min(no, (kNR - a.nmin) / a.step + 1);
  const int nmax_reg = a.nmin + (no_reg - 1) * a.step;
  if (no_reg > 0 && nmax_reg <= 16 * 13)
    hipLaunchKernelGGL(hess_kernel<13>, dim3(no_reg), dim3(kT), 0, st, a.xbuf, a.nmin, a.step,
                       hb, vr, ta);
  else if (no_reg > 0)
    hipLaunchKernelGGL(hess_kernel<kTP>, dim3(no_reg), dim3(kT), 0, st, a.xbuf, a.nmin, a.step,
                       hb, vr, ta);
  if (no > no_reg)
    hipLaunchKernelGGL(hess_glb_kernel, dim3(no - no_reg), dim3(kHG), 0, st, a.xbuf, a.nmin,
                       a.step, no_reg, hb, vr, ta);
  return hipGetLastError();
}

hipError_t launch_mode_head(const double *u, int k, int l, double *dst, hipStream_t st) {
  const int64_t total = (int64_t)k * l;
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(mode_head_kernel, dim3((unsigned)ceil_div<int64_t>(total, 256)), dim3(256), 0, st,
                     u, k, l, dst);
  return hipGetLastError();
}

namespace {
// Launches of the eigen-analysis for orders up to 64 KU.
template <int KU>
hipError_t launch_eig_ku(const ModalArgs &a, const ModalStrides &ls, int grid, hipStream_t st) {
  const ModalSizes &s = a.sizes;
  const int no = s.n_orders;
  hipError_t e = hipFuncSetAttribute((const void *)eig_persistent_kernel<KU>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)(sizeof(double) * kLdsDoubles));
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(eig_persistent_kernel<KU>, dim3(grid), dim3(kFT),
                     sizeof(double) * kLdsDoubles, st, a.hbuf, a.vref, a.taus, a.u,
                     a.nmin, a.step, no, a.l,
                     a.fs, a.gscr, s.francis_glb, a.evbuf, a.npole, a.pidx, a.flags_tmp,
                     a.tf, a.txi, a.tmu, a.tphi, a.queue, a.done, a.status,
                     a.sweeps_per_row, a.n_lags, ls);
  hipLaunchKernelGGL(pole_tail_kernel<KU>, dim3(2 * kEigGrid), dim3(64 * kTailWaves),
                     sizeof(double) * vec_lds<KU>() * kTailWaves, st, a.hbuf, a.vref, a.taus,
                     a.u, a.nmin, a.step, no, a.l, a.fs, a.evbuf, a.npole, a.pidx,
                     a.tf, a.txi, a.tmu, a.tphi, a.queue, a.done, a.status, a.n_lags, ls);
  return hipGetLastError();
}
}  // namespace

hipError_t launch_modal_eig(const ModalArgs &a, hipStream_t st) {
  const ModalSizes &s = a.sizes;
  const int no = s.n_orders;
  const int items = a.n_lags * no;
  const int nmax = a.nmin + (no - 1) * a.step;
  const ModalStrides ls = modal_strides(s, a.l, a.ldu);
  // QR iterations and pole vectors of every (lag, order) in one persistent launch
  hipLaunchKernelGGL(eig_init_kernel, dim3(1), dim3(kFT), 0, st, a.queue, a.done, items);
  // one workgroup per CU by default; a smaller grid (at least one workgroup
  // per item) leaves CUs to work on other streams
  const int grid = a.eig_grid > 0
                       ? std::min(std::max(a.eig_grid, std::min(items, kEigGrid)), kEigGrid)
                       : kEigGrid;
  const hipError_t e = nmax <= 256 ? launch_eig_ku<4>(a, ls, grid, st)
                                   : launch_eig_ku<kNMax / 64>(a, ls, grid, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(sort_kernel, dim3(no, a.n_lags), dim3(256), 0, st, a.nmin, a.step, a.l,
                     a.npole, a.flags_tmp, a.tf, a.txi, a.tmu, a.tphi, a.count, a.flags, a.f,
                     a.xi, a.mu, a.phi, no, (int64_t)s.poles);
  return hipGetLastError();
}

}  // namespace ssi
