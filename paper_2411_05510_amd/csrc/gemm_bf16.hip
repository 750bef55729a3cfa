// Reduced-precision range-finder products: C = op(T) X with both operands
// rounded to BF16 and FP32 accumulation on v_mfma_f32_16x16x32_bf16.
//
// T is the FP32 block-Toeplitz matrix as stored; each 64 x 64 tile is read
// once from HBM (16-byte loads, 256 contiguous bytes per row segment), rounded
// to BF16 (round to nearest even) and written to LDS, transposed on the way
// for op(T) = T^T.  X arrives pre-rounded and transposed (xt[j][k], BF16,
// rows padded to a multiple of 224 and columns to a multiple of 64 with
// zeros), so its tile loads need no bounds checks.  A workgroup owns 64 rows
// of the output and all 224 columns of one column block, over one K slice;
// FP32 partial sums of the K slices are added in FP64 by
// reduce_splits_f32.  The flat grid is decoded split-fastest, so the
// workgroups of one K slice share an XCD and its L2 holds their slice of X.
//
// BF16 keeps the FP32 exponent range, so no scaling is needed for these
// operands (T entries are correlations, X entries are O(1/sqrt(m))).
#include "common.h"
#include "kernels.h"

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

namespace {

constexpr int bBM = 64, bBN = 224;

// FP32 -> BF16, round to nearest even (NaN kept quiet).
SSI_DEV uint16_t bf16_rne(float f) {
  const uint32_t u = __float_as_uint(f);
  const uint32_t r = (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;
  return (uint16_t)(((u & 0x7fffffffu) > 0x7f800000u) ? ((u >> 16) | 0x40u) : r);
}

// FP64 -> BF16, round to nearest even in one rounding: truncate to FP32 and
// set the last FP32 bit when the truncation was inexact (round to odd), which
// keeps the sticky information for the final rounding to 8 significant bits.
SSI_DEV uint16_t bf16_rne(double d) {
  float f = __double2float_rz(d);
  if ((double)f != d && d == d) f = __uint_as_float(__float_as_uint(f) | 1u);
  return bf16_rne(f);
}

SSI_DEV uint32_t pack2(uint16_t lo, uint16_t hi) { return (uint32_t)lo | ((uint32_t)hi << 16); }

// Global -> registers for the tile at k0.  A: 64 x KT FP32; every load is
// issued from an index clamped into its row and the entries beyond the
// matrix or the slice are flagged in amsk (bit 4 h + c) and zeroed at store
// time, so the loads stay in flight across the MFMAs.  B: 224 x KT BF16 per
// plane, always in range (chunks past the tile, for KT = 32, reload the last
// one and are not stored).
template <bool TA, bool VEC, int KT, int NP, int AV, int BC>
SSI_DEV void bf16_tile_load(const float *__restrict__ A, int64_t lda,
                            const uint16_t *__restrict__ xt, int64_t ldx, int64_t plane, int M,
                            int K, int m0, int n0, int k0, int ke, int tid, float4 (&ra)[AV],
                            u32x4 (&rb)[NP][BC], unsigned &amsk) {
  unsigned m = 0u;
#pragma unroll
  for (int h = 0; h < AV; ++h) {
    const int idx = tid + 256 * h;
    float4 v;
    if (!TA) {
      const int r = idx / (KT / 4), c4 = idx % (KT / 4);
      const int gi = m0 + r, gk = k0 + 4 * c4;
      const float *p = A + (int64_t)min(gi, M - 1) * lda;
      if (VEC) {
        v = *reinterpret_cast<const float4 *>(p + min((int64_t)gk, lda - 4));
      } else {
        v.x = p[min(gk, K - 1)];
        v.y = p[min(gk + 1, K - 1)];
        v.z = p[min(gk + 2, K - 1)];
        v.w = p[min(gk + 3, K - 1)];
      }
#pragma unroll
      for (int c = 0; c < 4; ++c) m |= (gi < M && gk + c < ke ? 1u : 0u) << (4 * h + c);
    } else {
      const int r = idx >> 4, c4 = idx & 15;    // k row, 4-column group of i
      const int gk = k0 + r, gi = m0 + 4 * c4;
      const float *p = A + (int64_t)min(gk, K - 1) * lda;
      if (VEC) {
        v = *reinterpret_cast<const float4 *>(p + min((int64_t)gi, lda - 4));
      } else {
        v.x = p[min(gi, M - 1)];
        v.y = p[min(gi + 1, M - 1)];
        v.z = p[min(gi + 2, M - 1)];
        v.w = p[min(gi + 3, M - 1)];
      }
#pragma unroll
      for (int c = 0; c < 4; ++c) m |= (gk < ke && gi + c < M ? 1u : 0u) << (4 * h + c);
    }
    ra[h] = v;
  }
  amsk = m;
#pragma unroll
  for (int q = 0; q < NP; ++q)
#pragma unroll
    for (int h = 0; h < BC; ++h) {
      const int idx = min(tid + 256 * h, bBN * KT / 8 - 1);
      const int j = idx / (KT / 8), c8 = idx % (KT / 8);
      rb[q][h] = *reinterpret_cast<const u32x4 *>(xt + q * plane + (int64_t)(n0 + j) * ldx + k0 +
                                                  8 * c8);
    }
}

SSI_DEV uint16_t bf16_lo(float v, uint16_t h) {
  return bf16_rne(v - __uint_as_float((uint32_t)h << 16));
}

// Exact three-way split of an FP32 value into BF16 parts by truncation: hi
// keeps the top 8 significant bits, mid the next 8 and lo the last 8, and
// hi + mid + lo = v with no rounding (each remainder is exact in FP32).
SSI_DEV void bf16_split3(float v, uint16_t &h, uint16_t &m, uint16_t &l) {
  const uint32_t u = __float_as_uint(v);
  h = (uint16_t)(u >> 16);
  const float r1 = v - __uint_as_float(u & 0xffff0000u);
  const uint32_t u1 = __float_as_uint(r1);
  m = (uint16_t)(u1 >> 16);
  const float r2 = r1 - __uint_as_float(u1 & 0xffff0000u);
  l = (uint16_t)(__float_as_uint(r2) >> 16);
}

// Registers -> LDS (BF16 planes), A as As[i][k], B as Bs[j][k].
template <bool TA, int KT, int LS, int NP, int AV, int BC, int NT>
SSI_DEV void bf16_tile_store(uint16_t (&As)[NP][bBM * LS], uint16_t (&Bs)[NP][bBN * LS], int tid,
                             const float4 (&ra_in)[AV], const u32x4 (&rb)[NP][BC],
                             unsigned amsk) {
  float4 ra[AV];
#pragma unroll
  for (int h = 0; h < AV; ++h) {
    ra[h].x = (amsk >> (4 * h)) & 1u ? ra_in[h].x : 0.f;
    ra[h].y = (amsk >> (4 * h + 1)) & 1u ? ra_in[h].y : 0.f;
    ra[h].z = (amsk >> (4 * h + 2)) & 1u ? ra_in[h].z : 0.f;
    ra[h].w = (amsk >> (4 * h + 3)) & 1u ? ra_in[h].w : 0.f;
  }
#pragma unroll
  for (int q = 0; q < NP; ++q)
#pragma unroll
    for (int h = 0; h < BC; ++h) {
      const int idx = tid + 256 * h;
      if ((bBN * KT / 8) % 256 == 0 || idx < bBN * KT / 8) {
        const int j = idx / (KT / 8), c8 = idx % (KT / 8);
        *reinterpret_cast<u32x4 *>(&Bs[q][j * LS + 8 * c8]) = rb[q][h];
      }
    }
  if (NT == 6) {
#pragma unroll
    for (int h = 0; h < AV; ++h) {
      const int idx = tid + 256 * h;
      uint16_t p[3][4];
      bf16_split3(ra[h].x, p[0][0], p[1][0], p[2][0]);
      bf16_split3(ra[h].y, p[0][1], p[1][1], p[2][1]);
      bf16_split3(ra[h].z, p[0][2], p[1][2], p[2][2]);
      bf16_split3(ra[h].w, p[0][3], p[1][3], p[2][3]);
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        if (!TA) {
          const int r = idx / (KT / 4), c4 = idx % (KT / 4);
          *reinterpret_cast<uint2 *>(&As[q][r * LS + 4 * c4]) =
              make_uint2(pack2(p[q][0], p[q][1]), pack2(p[q][2], p[q][3]));
        } else {
          const int r = idx >> 4, c4 = idx & 15;
#pragma unroll
          for (int c = 0; c < 4; ++c) As[q][(4 * c4 + c) * LS + r] = p[q][c];
        }
      }
    }
    return;
  }
#pragma unroll
  for (int h = 0; h < AV; ++h) {
    const int idx = tid + 256 * h;
    const uint16_t h0 = bf16_rne(ra[h].x), h1 = bf16_rne(ra[h].y);
    const uint16_t h2 = bf16_rne(ra[h].z), h3 = bf16_rne(ra[h].w);
    if (!TA) {
      const int r = idx / (KT / 4), c4 = idx % (KT / 4);
      *reinterpret_cast<uint2 *>(&As[0][r * LS + 4 * c4]) = make_uint2(pack2(h0, h1), pack2(h2, h3));
      if (NT == 3)
        *reinterpret_cast<uint2 *>(&As[NP - 1][r * LS + 4 * c4]) =
            make_uint2(pack2(bf16_lo(ra[h].x, h0), bf16_lo(ra[h].y, h1)),
                       pack2(bf16_lo(ra[h].z, h2), bf16_lo(ra[h].w, h3)));
    } else {
      const int r = idx >> 4, c4 = idx & 15;
      As[0][(4 * c4 + 0) * LS + r] = h0;
      As[0][(4 * c4 + 1) * LS + r] = h1;
      As[0][(4 * c4 + 2) * LS + r] = h2;
      As[0][(4 * c4 + 3) * LS + r] = h3;
      if (NT == 3) {
        As[NP - 1][(4 * c4 + 0) * LS + r] = bf16_lo(ra[h].x, h0);
        As[NP - 1][(4 * c4 + 1) * LS + r] = bf16_lo(ra[h].y, h1);
        As[NP - 1][(4 * c4 + 2) * LS + r] = bf16_lo(ra[h].z, h2);
        As[NP - 1][(4 * c4 + 3) * LS + r] = bf16_lo(ra[h].w, h3);
      }
    }
  }
}

}  // namespace

// C_part[split][i][j] = sum_{k in split} op(A)[i][k] X[k][j]
//   TA = false: A is M x K (lda);  TA = true: A is K x M (lda), op(A) = A^T.
//   xt: BF16 planes of X^T, each N_pad x ldx (ldx >= K rounded up to the
//   tile, zero-padded); plane 1 (NT = 3) holds the rounding remainders.
//   VEC: lda % 4 == 0 and A 16-byte aligned.
//   NT = 1: one BF16 product.  NT = 3: split operands a = a_hi + a_lo,
//   x = x_hi + x_lo (each part BF16) and three products a_hi x_hi + a_hi x_lo
//   + a_lo x_hi, which carry about 16 significant bits of each operand.
//   NT = 6: exact three-way splits a = a_h + a_m + a_l (FP32 T as stored) and
//   x = x_h + x_m + x_l (X rounded to FP32), and the six products of weight
//   >= 2^-16 (h h, h m, m h, h l, l h, m m), each exact in FP32: the products
//   of FP32 operands up to a relative 2^-23, accumulated in FP32.
template <bool TA, bool VEC, int NT>
__global__ void __launch_bounds__(256, 2)
gemm_tbf16_mfma(const float *__restrict__ A, int64_t lda, const uint16_t *__restrict__ xt,
                int64_t ldx, int64_t plane, float *__restrict__ C, int64_t ldc,
                int64_t split_stride, int M, int N, int K, int k_per_split, int gm, int splits) {
  constexpr int KT = NT == 1 ? 64 : 32;          // K tile
  constexpr int LS = KT + 8;                     // LDS row stride (bf16)
  constexpr int NP = NT == 1 ? 1 : (NT == 3 ? 2 : 3);   // operand planes
  constexpr int AV = KT / 16;                    // float4 of A per thread
  constexpr int BC = (bBN * KT / 8 + 255) / 256; // 16-byte chunks of B per thread and plane
  __shared__ __attribute__((aligned(16))) uint16_t As[NP][bBM * LS];
  __shared__ __attribute__((aligned(16))) uint16_t Bs[NP][bBN * LS];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wr = wave & 1, wc = wave >> 1;
  const int split = blockIdx.x % splits;
  const int rest = blockIdx.x / splits;
  const int m0 = (rest % gm) * bBM, n0 = (rest / gm) * bBN;
  const int kb = split * k_per_split;
  const int ke = min(K, kb + k_per_split);

  f32x4 acc[2][7];
#pragma unroll
  for (int rt = 0; rt < 2; ++rt)
#pragma unroll
    for (int ct = 0; ct < 7; ++ct) acc[rt][ct] = f32x4{0.f, 0.f, 0.f, 0.f};

  float4 ra[AV];
  u32x4 rb[NP][BC];
  unsigned amsk = 0u;
  if (kb < ke)
    bf16_tile_load<TA, VEC, KT, NP, AV, BC>(A, lda, xt, ldx, plane, M, K, m0, n0, kb, ke, tid, ra,
                                            rb, amsk);
  for (int k0 = kb; k0 < ke; k0 += KT) {
    __syncthreads();                       // previous tile's LDS reads are done
    bf16_tile_store<TA, KT, LS, NP, AV, BC, NT>(As, Bs, tid, ra, rb, amsk);
    __syncthreads();
    if (k0 + KT < ke)                      // next tile in flight during the MFMAs
      bf16_tile_load<TA, VEC, KT, NP, AV, BC>(A, lda, xt, ldx, plane, M, K, m0, n0, k0 + KT, ke,
                                              tid, ra, rb, amsk);
#pragma unroll
    for (int kk = 0; kk < KT; kk += 32) {
      const int ko = kk + 8 * (lane >> 4);
      bf16x8 af[NP][2];
#pragma unroll
      for (int q = 0; q < NP; ++q)
#pragma unroll
        for (int rt = 0; rt < 2; ++rt)
          af[q][rt] = *reinterpret_cast<const bf16x8 *>(
              &As[q][(wr * 32 + rt * 16 + (lane & 15)) * LS + ko]);
#pragma unroll
      for (int ct = 0; ct < 7; ++ct) {
        const int brow = (wc * 112 + ct * 16 + (lane & 15)) * LS + ko;
        const bf16x8 bhi = *reinterpret_cast<const bf16x8 *>(&Bs[0][brow]);
        if (NT == 6) {
          // smallest terms first: l h, h l, m m, m h, h m (then h h below)
          const bf16x8 bmid = *reinterpret_cast<const bf16x8 *>(&Bs[1][brow]);
          const bf16x8 blow = *reinterpret_cast<const bf16x8 *>(&Bs[2][brow]);
#pragma unroll
          for (int rt = 0; rt < 2; ++rt) {
            acc[rt][ct] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[2][rt], bhi, acc[rt][ct], 0, 0, 0);
            acc[rt][ct] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[0][rt], blow, acc[rt][ct], 0, 0, 0);
            acc[rt][ct] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[1][rt], bmid, acc[rt][ct], 0, 0, 0);
            acc[rt][ct] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[1][rt], bhi, acc[rt][ct], 0, 0, 0);
            acc[rt][ct] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[0][rt], bmid, acc[rt][ct], 0, 0, 0);
          }
        }
        if (NT == 3) {
          const bf16x8 blo = *reinterpret_cast<const bf16x8 *>(&Bs[NP - 1][brow]);
#pragma unroll
          for (int rt = 0; rt < 2; ++rt) {
            acc[rt][ct] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[NP - 1][rt], bhi, acc[rt][ct], 0, 0, 0);
            acc[rt][ct] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[0][rt], blo, acc[rt][ct], 0, 0, 0);
          }
        }
#pragma unroll
        for (int rt = 0; rt < 2; ++rt)
          acc[rt][ct] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[0][rt], bhi, acc[rt][ct], 0, 0, 0);
      }
    }
  }

  // D layout of 16x16 MFMA: lane holds rows 4 (lane/16) + q, column lane%16.
  float *dst = C + (int64_t)split * split_stride;
#pragma unroll
  for (int rt = 0; rt < 2; ++rt)
#pragma unroll
    for (int ct = 0; ct < 7; ++ct) {
      const int col = n0 + wc * 112 + ct * 16 + (lane & 15);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int row = m0 + wr * 32 + rt * 16 + 4 * (lane >> 4) + q;
        if (row < M && col < N) dst[(int64_t)row * ldc + col] = acc[rt][ct][q];
      }
    }
}

// out[i][j] = sum_s part[s][i][j] (FP32 partials summed in FP64, fixed order;
// loaded eight splits at a time with the split index clamped, so that the loads
// are in flight together)
__global__ void __launch_bounds__(256)
reduce_splits_f32(const float *__restrict__ part, int splits, int64_t split_stride, int64_t ldp,
                  int M, int N, double *__restrict__ out, int64_t ldo) {
  const int64_t total = (int64_t)M * N;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = idx / N, j = idx - i * N;
    const float *pp = part + i * ldp + j;
    double s = 0.0;
    for (int sp0 = 0; sp0 < splits; sp0 += 8) {
      float v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = pp[(int64_t)min(sp0 + u, splits - 1) * split_stride];
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (sp0 + u < splits) s += (double)v[u];
    }
    out[i * ldo + j] = s;
  }
}

// xt[j][k] = bf16(x[k][j]) for j < N, k < K; zero in the padding
// (j < n_pad, k < k_pad), planes `planes` apart.  nt = 1: one plane, x
// rounded to BF16.  nt = 3: a second plane with the remainder x - hi rounded
// to BF16.  nt = 6: x rounded to FP32, then split exactly into three BF16
// parts by truncation (bf16_split3), one per plane.  64 x 64 tiles through
// LDS.
__global__ void __launch_bounds__(256)
pack_bf16_t(const double *__restrict__ x, int64_t ldx, int K, int N, uint16_t *__restrict__ xt,
            int64_t planes, int nt, int64_t ldt, int n_pad, int k_pad) {
  __shared__ uint16_t tile[3][64][66];
  const int k0 = blockIdx.x * 64, j0 = blockIdx.y * 64;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  for (int r = ty; r < 64; r += 4) {          // read rows k of x, columns j
    const int k = k0 + r, j = j0 + tx;
    const double v = (k < K && j < N) ? x[(int64_t)k * ldx + j] : 0.0;
    if (nt == 6) {
      uint16_t h, m, l;
      bf16_split3((float)v, h, m, l);
      tile[0][r][tx] = h;
      tile[1][r][tx] = m;
      tile[2][r][tx] = l;
    } else {
      const uint16_t h = bf16_rne(v);
      tile[0][r][tx] = h;
      tile[1][r][tx] = bf16_rne(v - (double)__uint_as_float((uint32_t)h << 16));
    }
  }
  __syncthreads();
  const int np = nt == 1 ? 1 : (nt == 3 ? 2 : 3);
  for (int r = ty; r < 64; r += 4) {          // write rows j of xt, columns k
    const int j = j0 + r, k = k0 + tx;
    if (j < n_pad && k < k_pad)
      for (int q = 0; q < np; ++q) xt[q * planes + (int64_t)j * ldt + k] = tile[q][tx][r];
  }
}

namespace ssi {

namespace {
int grid_cap_b(int64_t work) {
  int64_t b = ceil_div<int64_t>(work, 256);
  return (int)std::max<int64_t>(1, std::min<int64_t>(b, 16384));
}
}  // namespace

BfPlan plan_gemm_tbf16(int M, int N, int K, int num_cus, int force_splits, int nt) {
  BfPlan p{};
  const int bKT = nt == 1 ? 64 : 32;
  p.nt = nt;
  p.gm = ceil_div(M, bBM);
  p.gn = ceil_div(N, bBN);
  const int64_t tiles = (int64_t)p.gm * p.gn;
  int64_t splits = ceil_div<int64_t>((int64_t)num_cus * 2, tiles);
  splits = std::max<int64_t>(1, std::min<int64_t>(std::min<int64_t>(splits, 8),
                                                  ceil_div<int64_t>(K, 512)));
  if (force_splits > 0) splits = std::min<int64_t>(force_splits, ceil_div<int64_t>(K, bKT));
  int64_t kps = ceil_div<int64_t>(ceil_div<int64_t>(K, splits), bKT) * bKT;
  p.k_per_split = (int)kps;
  p.splits = (int)ceil_div<int64_t>(K, kps);
  p.ldc = N;
  p.split_stride = (int64_t)M * N;
  p.n_pad = p.gn * bBN;
  p.k_pad = (int)(ceil_div<int64_t>(K, 64) * 64);
  p.ldx = p.k_pad;
  return p;
}

hipError_t launch_pack_bf16(const BfPlan &p, const double *x, int64_t ldx, int K, int N,
                            uint16_t *xt, hipStream_t st) {
  dim3 grid(ceil_div(p.k_pad, 64), ceil_div(p.n_pad, 64));
  hipLaunchKernelGGL(pack_bf16_t, grid, dim3(256), 0, st, x, ldx, K, N, xt, (int64_t)p.plane(),
                     p.nt, p.ldx, p.n_pad, p.k_pad);
  return hipGetLastError();
}

hipError_t launch_gemm_tbf16(const BfPlan &p, bool trans_a, const float *A, int64_t lda,
                             const uint16_t *xt, int M, int N, int K, float *part,
                             hipStream_t st) {
  const bool vec = (lda % 4 == 0) && ((uintptr_t)A % 16 == 0);
  const dim3 grid((unsigned)((int64_t)p.gm * p.gn * p.splits));
#define SSI_BF(TA, V, NT)                                                                   \
  hipLaunchKernelGGL((gemm_tbf16_mfma<TA, V, NT>), grid, dim3(256), 0, st, A, lda, xt, p.ldx, \
                     (int64_t)p.plane(), part, p.ldc, p.split_stride, M, N, K, p.k_per_split,  \
                     p.gm, p.splits)
#define SSI_BF_NT(TA, V)                                                  \
  do {                                                                    \
    if (p.nt == 6) SSI_BF(TA, V, 6);                                      \
    else if (p.nt == 3) SSI_BF(TA, V, 3);                                 \
    else SSI_BF(TA, V, 1);                                                \
  } while (0)
  if (trans_a) {
    if (vec) SSI_BF_NT(true, true); else SSI_BF_NT(true, false);
  } else {
    if (vec) SSI_BF_NT(false, true); else SSI_BF_NT(false, false);
  }
#undef SSI_BF_NT
#undef SSI_BF
  return hipGetLastError();
}

hipError_t launch_reduce_f32(const BfPlan &p, const float *part, int M, int N, double *out,
                             int64_t ldo, hipStream_t st) {
  hipLaunchKernelGGL(reduce_splits_f32, dim3(grid_cap_b((int64_t)M * N)), dim3(256), 0, st,
                     part, p.splits, p.split_stride, p.ldc, M, N, out, ldo);
  return hipGetLastError();
}

}  // namespace ssi
