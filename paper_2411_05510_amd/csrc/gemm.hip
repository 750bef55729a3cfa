// Dense products of the randomized SVD and the modal stage.
//
// gemm_tf64w: C = op(T) X with T in FP32 (the Toeplitz matrix as stored) and
//   X in FP64, on v_mfma_f64_16x16x4f64 with FP64 accumulation: the sketch,
//   power-iteration and projection products Y = T X, Z = T^T X.  T is
//   converted exactly to FP64 in registers, so the only rounding is FP64
//   accumulation.  Tile 128 x 224 x 32 on 8 waves, double-buffered LDS with
//   the next K tile prefetched into registers during the MFMAs, one
//   workgroup per CU.  The thin side (ell = k + p columns) fits one column
//   block; the long side is split across workgroups and along K, with the
//   number of K slices chosen to fill whole rounds of the CUs.  The flat grid
//   is decoded split-fastest.  Partial sums (FP64) are added by
//   reduce_splits in a fixed order.
// gemm_f64: FP64 operands on v_mfma_f64_16x16x4f64 (Gram matrices, basis
//   updates, small triangular products).  Tile 64 x 64 x 16.
#include "common.h"
#include "kernels.h"

namespace {

constexpr int dBM = 64, dBN = 64, dKT = 16, dLS = dKT + 2;    // fp64 tiles

}  // namespace

// C_part[split][i][j] = sum_{k in split} op(A)[i][k] B[k][j]
//   TA = false: A is M x K (lda);  TA = true: A is K x M (lda), op(A) = A^T.
//   A FP32, B FP64 K x N (ldb).  VEC: lda % 4 == 0 and A 16-byte aligned;
//   BVEC: ldb even and B 16-byte aligned.
// BM x 224 output tile (BM = 128 or 64), 32-deep K tiles and 8 waves (4 x 2,
// each BM/4 x 112): the LDS tiles are double-buffered and the next K tile is
// loaded into registers while the MFMAs of the current one run, so a
// workgroup streams T with one barrier per K tile.  One workgroup per CU
// (150 / 135 KB of LDS); the FP64 operand is read from L2 once per BM rows.
// The autotuner picks BM with the K-slice count: 128 halves the re-reads of
// the FP64 operand, 64 gives twice the row tiles on short sides.
namespace {
constexpr int wBN = 224, wKT = 32;
constexpr int wLA = wKT + 4;          // FP32 A row stride (floats), A stored [i][k]
constexpr int wLB = wBN + 4;          // FP64 B row stride (doubles), B stored [k][j]
constexpr int wBS = wKT * wLB;        // one B buffer, elements
template <int BM> constexpr int wAS = BM * wLA;   // one A buffer, elements
typedef double f64x2v __attribute__((ext_vector_type(2)));
typedef float f32x4v __attribute__((ext_vector_type(4)));

// Every load is issued unconditionally, from an index clamped into its row;
// the entries outside the tile's range are flagged in msk (bit 4 h + c of the
// A part, bit 8 + 2 h + c of the B part) and zeroed when the tile is stored.
// The loads then stay in flight across the MFMAs of the current tile: with a
// bounds branch around each load the compiler waits for every load before
// issuing the next.
template <int BM, bool TA, bool VEC, bool BVEC>
SSI_DEV void tf64w_load(const float *__restrict__ A, int64_t lda, const double *__restrict__ B,
                        int64_t ldb, int M, int N, int m0, int n0, int k0, int ke, int tid,
                        f32x4v (&ra)[BM / 64], f64x2v (&rb)[7], unsigned &msk) {
  constexpr int kI4 = BM / 4;                              // 4-row groups of i (TA)
  unsigned m = 0u;
#pragma unroll
  for (int h = 0; h < BM / 64; ++h) {
    const int idx = tid + 512 * h;
    f32x4v v;
    if (!TA) {
      const int r = idx >> 3, c4 = idx & 7;               // row, 4-column group of k
      const int gi = m0 + r, gk = k0 + 4 * c4;
      const float *p = A + (int64_t)min(gi, M - 1) * lda;
      if (VEC) {
        v = *reinterpret_cast<const f32x4v *>(p + min((int64_t)gk, lda - 4));
      } else {
        v.x = p[min(gk, ke - 1)];
        v.y = p[min(gk + 1, ke - 1)];
        v.z = p[min(gk + 2, ke - 1)];
        v.w = p[min(gk + 3, ke - 1)];
      }
#pragma unroll
      for (int c = 0; c < 4; ++c) m |= (gi < M && gk + c < ke ? 1u : 0u) << (4 * h + c);
    } else {
      const int kr = idx / kI4, c4 = idx % kI4;           // k row, 4-column group of i
      const int gk = k0 + kr, gi = m0 + 4 * c4;
      const float *p = A + (int64_t)min(gk, ke - 1) * lda;
      if (VEC) {
        v = *reinterpret_cast<const f32x4v *>(p + min((int64_t)gi, lda - 4));
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
#pragma unroll
  for (int h = 0; h < 7; ++h) {
    const int idx = tid + 512 * h;                       // 32 k rows x 112 double pairs
    const int kr = idx / 112, c2 = idx - kr * 112;
    const int gk = k0 + kr, gj = n0 + 2 * c2;
    const double *q = B + (int64_t)min(gk, ke - 1) * ldb;
    f64x2v v;
    if (BVEC) {
      v = *reinterpret_cast<const f64x2v *>(q + min((int64_t)gj, ldb - 2));
    } else {
      v.x = q[min(gj, N - 1)];
      v.y = q[min(gj + 1, N - 1)];
    }
    m |= (gk < ke && gj < N ? 1u : 0u) << (8 + 2 * h);
    m |= (gk < ke && gj + 1 < N ? 1u : 0u) << (9 + 2 * h);
    rb[h] = v;
  }
  msk = m;
}

template <int BM, bool TA>
SSI_DEV void tf64w_store(float *__restrict__ As, double *__restrict__ Bs, int tid,
                         const f32x4v (&ra)[BM / 64], const f64x2v (&rb)[7], unsigned msk) {
  constexpr int kI4 = BM / 4;
#pragma unroll
  for (int h = 0; h < BM / 64; ++h) {
    const int idx = tid + 512 * h;
    f32x4v v = ra[h];
    v.x = (msk >> (4 * h)) & 1u ? v.x : 0.f;
    v.y = (msk >> (4 * h + 1)) & 1u ? v.y : 0.f;
    v.z = (msk >> (4 * h + 2)) & 1u ? v.z : 0.f;
    v.w = (msk >> (4 * h + 3)) & 1u ? v.w : 0.f;
    if (!TA) {
      const int r = idx >> 3, c4 = idx & 7;
      *reinterpret_cast<f32x4v *>(&As[r * wLA + 4 * c4]) = v;
    } else {
      const int kr = idx / kI4, c4 = idx % kI4;
      As[(4 * c4 + 0) * wLA + kr] = v.x;
      As[(4 * c4 + 1) * wLA + kr] = v.y;
      As[(4 * c4 + 2) * wLA + kr] = v.z;
      As[(4 * c4 + 3) * wLA + kr] = v.w;
    }
  }
#pragma unroll
  for (int h = 0; h < 7; ++h) {
    const int idx = tid + 512 * h;
    const int kr = idx / 112, c2 = idx - kr * 112;
    f64x2v v = rb[h];
    v.x = (msk >> (8 + 2 * h)) & 1u ? v.x : 0.0;
    v.y = (msk >> (9 + 2 * h)) & 1u ? v.y : 0.0;
    *reinterpret_cast<f64x2v *>(&Bs[kr * wLB + 2 * c2]) = v;
  }
}
}  // namespace

template <int BM, bool TA, bool VEC, bool BVEC>
__global__ void __launch_bounds__(512, 1)
gemm_tf64w_mfma(const float *__restrict__ A, int64_t lda, const double *__restrict__ B,
                int64_t ldb, double *__restrict__ C, int64_t ldc, int64_t split_stride, int M,
                int N, int K, int k_per_split, int gm, int splits) {
  constexpr int RT = BM / 64;                                    // row tiles of 16 per wave
  constexpr int AS = wAS<BM>;
  extern __shared__ __attribute__((aligned(16))) double smem[];
  float *Asb = reinterpret_cast<float *>(smem);                  // [2][AS] floats
  double *Bsb = smem + AS;                                        // [2][wBS] doubles (AS even)
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);   // uniform: the column
                                                               // checks stay scalar
  const int wr = wave & 3, wc = wave >> 2;
  const int split = blockIdx.x % splits;
  const int rest = blockIdx.x / splits;
  const int m0 = (rest % gm) * BM, n0 = (rest / gm) * wBN;
  const int kb = split * k_per_split;
  const int ke = min(K, kb + k_per_split);

  f64x4 acc[RT][7];
#pragma unroll
  for (int rt = 0; rt < RT; ++rt)
#pragma unroll
    for (int ct = 0; ct < 7; ++ct) acc[rt][ct] = f64x4{0.0, 0.0, 0.0, 0.0};
  // A wave whose 112 columns all lie past N skips its products; otherwise
  // all seven column tiles run (columns past N hold zeros in the B tile and
  // are not stored): a branch per tile would split the MFMA sequence into
  // blocks, with a wait for every LDS read at each block boundary.
  const bool wave_cols = n0 + wc * 112 < N;

  f32x4v ra[RT];
  f64x2v rb[7];
  unsigned msk = 0u;
  int buf = 0;
  if (kb < ke) {
    tf64w_load<BM, TA, VEC, BVEC>(A, lda, B, ldb, M, N, m0, n0, kb, ke, tid, ra, rb, msk);
    tf64w_store<BM, TA>(Asb, Bsb, tid, ra, rb, msk);
  }
  __syncthreads();
  for (int k0 = kb; k0 < ke; k0 += wKT) {
    const bool more = k0 + wKT < ke;
    if (more)
      tf64w_load<BM, TA, VEC, BVEC>(A, lda, B, ldb, M, N, m0, n0, k0 + wKT, ke, tid, ra, rb, msk);
    const float *As = Asb + buf * AS;
    const double *Bs = Bsb + buf * wBS;
#pragma unroll
    for (int hk = 0; hk < wKT / 16; ++hk) {
      if (!wave_cols) break;
      const int ko = 16 * hk + 4 * (lane >> 4);
      f32x4v a4[RT];
#pragma unroll
      for (int rt = 0; rt < RT; ++rt)
        a4[rt] = *reinterpret_cast<const f32x4v *>(
            &As[(wr * 16 * RT + rt * 16 + (lane & 15)) * wLA + ko]);
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        double bv[7];
#pragma unroll
        for (int ct = 0; ct < 7; ++ct) bv[ct] = Bs[(ko + s) * wLB + wc * 112 + ct * 16 + (lane & 15)];
#pragma unroll
        for (int ct = 0; ct < 7; ++ct) {
#pragma unroll
          for (int rt = 0; rt < RT; ++rt)
            acc[rt][ct] = __builtin_amdgcn_mfma_f64_16x16x4f64((double)a4[rt][s], bv[ct],
                                                               acc[rt][ct], 0, 0, 0);
        }
      }
    }
    if (more) {
      // the other buffer was last read before the previous barrier
      tf64w_store<BM, TA>(Asb + (buf ^ 1) * AS, Bsb + (buf ^ 1) * wBS, tid, ra, rb, msk);
    }
    __syncthreads();
    buf ^= 1;
  }

  // D layout of 16x16x4f64: lane holds rows (lane/16) + 4 q, column lane%16.
  double *dst = C + (int64_t)split * split_stride;
#pragma unroll
  for (int rt = 0; rt < RT; ++rt)
#pragma unroll
    for (int ct = 0; ct < 7; ++ct) {
      const int col = n0 + wc * 112 + ct * 16 + (lane & 15);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int row = m0 + wr * 16 * RT + rt * 16 + (lane >> 4) + 4 * q;
        if (row < M && col < N) dst[(int64_t)row * ldc + col] = acc[rt][ct][q];
      }
    }
}

// C_part[split][i][j] = sum_{k in split} op(A)[i][k] B[k][j], FP64 operands.
template <bool TA>
__global__ void __launch_bounds__(256)
gemm_f64_mfma(const double *__restrict__ A, int64_t lda, const double *__restrict__ B,
              int64_t ldb, double *__restrict__ C, int64_t ldc, int64_t split_stride, int M,
              int N, int K, int k_per_split) {
  __shared__ double As[dBM * dLS];
  __shared__ double Bs[dBN * dLS];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wr = wave & 1, wc = wave >> 1;
  const int m0 = blockIdx.x * dBM, n0 = blockIdx.y * dBN;
  const int kb = blockIdx.z * k_per_split;
  const int ke = min(K, kb + k_per_split);

  f64x4 acc[2][2];
#pragma unroll
  for (int rt = 0; rt < 2; ++rt)
#pragma unroll
    for (int ct = 0; ct < 2; ++ct) acc[rt][ct] = f64x4{0.0, 0.0, 0.0, 0.0};

  // The next K tile is loaded into registers (from indices clamped into the
  // matrices, entries outside the tile flagged in msk) while the MFMAs of the
  // current one run; it is masked and stored after the next barrier.
  double ra[4], rb[4];
  unsigned msk = 0u;
  auto load = [&](int k0) {
    unsigned m = 0u;
#pragma unroll
    for (int h = 0; h < 4; ++h) {
      const int idx = tid + 256 * h;          // 1024 elements per tile
      if (!TA) {
        const int r = idx >> 4, kr = idx & 15;
        const int gi = m0 + r, gk = k0 + kr;
        ra[h] = A[(int64_t)min(gi, M - 1) * lda + min(gk, ke - 1)];
        m |= (gi < M && gk < ke ? 1u : 0u) << h;
      } else {
        const int kr = idx >> 6, c = idx & 63;
        const int gi = m0 + c, gk = k0 + kr;
        ra[h] = A[(int64_t)min(gk, ke - 1) * lda + min(gi, M - 1)];
        m |= (gi < M && gk < ke ? 1u : 0u) << h;
      }
      const int kr = idx >> 6, c = idx & 63;
      const int gj = n0 + c, gk = k0 + kr;
      rb[h] = B[(int64_t)min(gk, ke - 1) * ldb + min(gj, N - 1)];
      m |= (gj < N && gk < ke ? 1u : 0u) << (4 + h);
    }
    msk = m;
  };
  if (kb < ke) load(kb);
  for (int k0 = kb; k0 < ke; k0 += dKT) {
    __syncthreads();
#pragma unroll
    for (int h = 0; h < 4; ++h) {
      const int idx = tid + 256 * h;
      const double a = (msk >> h) & 1u ? ra[h] : 0.0;
      const double b = (msk >> (4 + h)) & 1u ? rb[h] : 0.0;
      if (!TA) {
        As[(idx >> 4) * dLS + (idx & 15)] = a;
      } else {
        As[(idx & 63) * dLS + (idx >> 6)] = a;
      }
      Bs[(idx & 63) * dLS + (idx >> 6)] = b;
    }
    __syncthreads();
    if (k0 + dKT < ke) load(k0 + dKT);
#pragma unroll
    for (int s = 0; s < dKT / 4; ++s) {
      const int ko = 4 * s + (lane >> 4);
      double av[2], bv[2];
#pragma unroll
      for (int rt = 0; rt < 2; ++rt) av[rt] = As[(wr * 32 + rt * 16 + (lane & 15)) * dLS + ko];
#pragma unroll
      for (int ct = 0; ct < 2; ++ct) bv[ct] = Bs[(wc * 32 + ct * 16 + (lane & 15)) * dLS + ko];
#pragma unroll
      for (int rt = 0; rt < 2; ++rt)
#pragma unroll
        for (int ct = 0; ct < 2; ++ct)
          acc[rt][ct] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[rt], bv[ct], acc[rt][ct], 0, 0, 0);
    }
  }

  // D layout of 16x16x4f64: lane holds rows (lane/16) + 4 q, column lane%16.
  double *dst = C + (int64_t)blockIdx.z * split_stride;
#pragma unroll
  for (int rt = 0; rt < 2; ++rt)
#pragma unroll
    for (int ct = 0; ct < 2; ++ct) {
      const int col = n0 + wc * 32 + ct * 16 + (lane & 15);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int row = m0 + wr * 32 + rt * 16 + (lane >> 4) + 4 * q;
        if (row < M && col < N) dst[(int64_t)row * ldc + col] = acc[rt][ct][q];
      }
    }
}

// out[i][j] = scale * sum_s part[s][i][j]; optional FP32 copy.  One thread
// per output element over the flattened M x N range (grid-stride), so every
// lane of every workgroup works also when N is not a multiple of the
// workgroup width (N = 220 with a workgroup per row used 86 % of its lanes and
// ran at 1.6 TB/s); splits summed in order.  The partials are loaded eight at
// a time, unconditionally (split index clamped to the last one, whose repeats
// are not added), so the eight loads are in flight together; a load per split
// inside the summing loop waited for the previous.
__global__ void __launch_bounds__(256)
reduce_splits(const double *__restrict__ part, int splits, int64_t split_stride, int64_t ldp,
              int M, int N, double scale, double *__restrict__ out, int64_t ldo,
              float *__restrict__ out32, int64_t ld32) {
  const int64_t total = (int64_t)M * N;
  for (int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * 256) {
    const int64_t i = idx / N;
    const int j = (int)(idx - i * N);
    const double *pp = part + i * ldp + j;
    double s = 0.0;
    for (int sp0 = 0; sp0 < splits; sp0 += 8) {
      double v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = pp[(int64_t)min(sp0 + u, splits - 1) * split_stride];
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (sp0 + u < splits) s += v[u];
    }
    s *= scale;
    if (out) out[i * ldo + j] = s;
    if (out32) out32[i * ld32 + j] = (float)s;
  }
}

// out32[i][j] = (float) in[i][j]
__global__ void __launch_bounds__(256)
convert_f64_f32(const double *__restrict__ in, int64_t ldi, int M, int N,
                float *__restrict__ out, int64_t ldo) {
  const int64_t total = (int64_t)M * N;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = idx / N, j = idx - i * N;
    out[i * ldo + j] = (float)in[i * ldi + j];
  }
}

// out[i][j] = (double) in[i][j]
__global__ void __launch_bounds__(256)
convert_f32_f64(const float *__restrict__ in, int64_t ldi, int M, int N,
                double *__restrict__ out, int64_t ldo) {
  const int64_t total = (int64_t)M * N;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = idx / N, j = idx - i * N;
    out[i * ldo + j] = (double)in[i * ldi + j];
  }
}

// sigma[i] = sqrt(max(evals[i], 0)), i < k
__global__ void sqrt_clamp_kernel(const double *__restrict__ ev, int k, double *__restrict__ sigma) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < k) sigma[i] = sqrt(fmax(ev[i], 0.0));
}

// out[j][i] = (double) in[i][j]  (FP32 -> FP64 transpose, m x n -> n x m)
__global__ void __launch_bounds__(256)
transpose_f32_f64(const float *__restrict__ in, int64_t ldi, int M, int N,
                  double *__restrict__ out, int64_t ldo) {
  const int64_t total = (int64_t)M * N;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t j = idx / M, i = idx - j * M;
    out[j * ldo + i] = (double)in[i * ldi + j];
  }
}

namespace ssi {

namespace {
int grid_cap(int64_t work) {
  int64_t b = ceil_div<int64_t>(work, 256);
  if (b > 16384) b = 16384;
  if (b < 1) b = 1;
  return (int)b;
}
}  // namespace

GemmPlan plan_gemm_tf64(int M, int N, int K, int num_cus, int force_splits, int bm) {
  GemmPlan p{};
  p.bm = bm == 64 ? 64 : 128;
  p.gm = ceil_div(M, p.bm);
  p.gn = ceil_div(N, wBN);
  // One workgroup per CU: pick the K-slice count whose workgroup count fills
  // whole rounds of the CUs best (fewest idle CU slots), at most 16 slices
  // and at least 512 rows of K per slice.
  const int64_t tiles = (int64_t)p.gm * p.gn;
  const int64_t max_splits = std::max<int64_t>(1, std::min<int64_t>(16, ceil_div<int64_t>(K, 512)));
  int64_t splits = 1;
  double best = -1.0;
  for (int64_t sp = 1; sp <= max_splits; ++sp) {
    const int64_t wgs = tiles * sp;
    const int64_t rounds = ceil_div<int64_t>(wgs, num_cus);
    const double fill = (double)wgs / (double)(rounds * num_cus);
    // prefer full rounds; among equal fill, fewer slices (less partial traffic)
    if (fill > best + 1e-9) {
      best = fill;
      splits = sp;
    }
  }
  if (force_splits > 0) splits = std::min<int64_t>(force_splits, ceil_div<int64_t>(K, wKT));
  int64_t kps = ceil_div<int64_t>(K, splits);
  kps = ceil_div<int64_t>(kps, wKT) * wKT;
  p.k_per_split = (int)kps;
  p.splits = (int)ceil_div<int64_t>(K, kps);
  p.ldc = N;
  p.split_stride = (int64_t)M * N;
  return p;
}

GemmPlan plan_gemm_f64(int M, int N, int K, int num_cus) {
  GemmPlan p{};
  p.gm = ceil_div(M, dBM);
  p.gn = ceil_div(N, dBN);
  const int64_t tiles = (int64_t)p.gm * p.gn;
  int64_t splits = ceil_div<int64_t>((int64_t)num_cus * 2, tiles);
  const int64_t max_splits = ceil_div<int64_t>(K, 128);
  splits = std::max<int64_t>(1, std::min(splits, max_splits));
  int64_t kps = ceil_div<int64_t>(K, splits);
  kps = ceil_div<int64_t>(kps, dKT) * dKT;
  p.k_per_split = (int)kps;
  p.splits = (int)ceil_div<int64_t>(K, kps);
  p.ldc = N;
  p.split_stride = (int64_t)M * N;
  return p;
}

template <int BM, bool TA>
static hipError_t launch_tf64_variant(const GemmPlan &p, bool vec, bool bvec, const float *A,
                                      int64_t lda, const double *B, int64_t ldb, int M, int N,
                                      int K, double *part, hipStream_t st) {
  const dim3 grid((unsigned)((int64_t)p.gm * p.gn * p.splits));
  // two FP32 A buffers (AS floats each = AS doubles in all) and two FP64 B buffers
  const size_t lds = sizeof(double) * (size_t)(wAS<BM> + 2 * wBS);
#define SSI_TF64(V, BV)                                                                        \
  do {                                                                                         \
    hipError_t e = hipFuncSetAttribute((const void *)gemm_tf64w_mfma<BM, TA, V, BV>,           \
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);  \
    if (e != hipSuccess) return e;                                                             \
    hipLaunchKernelGGL((gemm_tf64w_mfma<BM, TA, V, BV>), grid, dim3(512), lds, st, A, lda, B,  \
                       ldb, part, p.ldc, p.split_stride, M, N, K, p.k_per_split, p.gm,         \
                       p.splits);                                                              \
  } while (0)
  if (vec && bvec) SSI_TF64(true, true);
  else if (vec) SSI_TF64(true, false);
  else if (bvec) SSI_TF64(false, true);
  else SSI_TF64(false, false);
#undef SSI_TF64
  return hipSuccess;
}

hipError_t launch_gemm_tf64(const GemmPlan &p, bool trans_a, const float *A, int64_t lda,
                            const double *B, int64_t ldb, int M, int N, int K, double *part,
                            hipStream_t st) {
  const bool vec = (lda % 4 == 0) && ((uintptr_t)A % 16 == 0);
  const bool bvec = (ldb % 2 == 0) && ((uintptr_t)B % 16 == 0);
  hipError_t e;
  if (p.bm == 64)
    e = trans_a ? launch_tf64_variant<64, true>(p, vec, bvec, A, lda, B, ldb, M, N, K, part, st)
                : launch_tf64_variant<64, false>(p, vec, bvec, A, lda, B, ldb, M, N, K, part, st);
  else
    e = trans_a ? launch_tf64_variant<128, true>(p, vec, bvec, A, lda, B, ldb, M, N, K, part, st)
                : launch_tf64_variant<128, false>(p, vec, bvec, A, lda, B, ldb, M, N, K, part,
                                                  st);
  if (e != hipSuccess) return e;
  return hipGetLastError();
}

hipError_t launch_gemm_f64(const GemmPlan &p, bool trans_a, const double *A, int64_t lda,
                           const double *B, int64_t ldb, int M, int N, int K, double *part,
                           hipStream_t st) {
  dim3 grid(p.gm, p.gn, p.splits);
  if (trans_a)
    hipLaunchKernelGGL((gemm_f64_mfma<true>), grid, dim3(256), 0, st, A, lda, B, ldb, part,
                       p.ldc, p.split_stride, M, N, K, p.k_per_split);
  else
    hipLaunchKernelGGL((gemm_f64_mfma<false>), grid, dim3(256), 0, st, A, lda, B, ldb, part,
                       p.ldc, p.split_stride, M, N, K, p.k_per_split);
  return hipGetLastError();
}

hipError_t launch_reduce(const GemmPlan &p, const double *part, int M, int N, double scale,
                         double *out, int64_t ldo, float *out32, int64_t ld32, hipStream_t st) {
  if (M <= 0 || N <= 0) return hipSuccess;
  hipLaunchKernelGGL(reduce_splits, dim3(grid_cap((int64_t)M * N)), dim3(256), 0, st, part,
                     p.splits, p.split_stride, p.ldc, M, N, scale, out, ldo, out32, ld32);
  return hipGetLastError();
}

hipError_t launch_convert(const double *in, int64_t ldi, int M, int N, float *out, int64_t ldo,
                          hipStream_t st) {
  hipLaunchKernelGGL(convert_f64_f32, dim3(grid_cap((int64_t)M * N)), dim3(256), 0, st, in,
                     ldi, M, N, out, ldo);
  return hipGetLastError();
}

hipError_t launch_convert_f32_f64(const float *in, int64_t ldi, int M, int N, double *out,
                                  int64_t ldo, hipStream_t st) {
  hipLaunchKernelGGL(convert_f32_f64, dim3(grid_cap((int64_t)M * N)), dim3(256), 0, st, in,
                     ldi, M, N, out, ldo);
  return hipGetLastError();
}

hipError_t launch_sqrt_clamp(const double *ev, int k, double *sigma, hipStream_t st) {
  hipLaunchKernelGGL(sqrt_clamp_kernel, dim3(ceil_div(k, 256)), dim3(256), 0, st, ev, k, sigma);
  return hipGetLastError();
}

hipError_t launch_transpose_f32_f64(const float *in, int64_t ldi, int M, int N, double *out,
                                    int64_t ldo, hipStream_t st) {
  hipLaunchKernelGGL(transpose_f32_f64, dim3(grid_cap((int64_t)M * N)), dim3(256), 0, st, in,
                     ldi, M, N, out, ldo);
  return hipGetLastError();
}

}  // namespace ssi
