// Dense kernels around the filter for gfx950: Gram and tall-skinny products
// on the FP64 matrix cores (v_mfma_f64_16x16x4f64), CholQR's small Cholesky
// factor and its inverse, the Rayleigh-Ritz eigensolve of the projected
// matrix (parallel cyclic Jacobi), residual and column norms, casts, a
// counter-based Gaussian generator and small Lanczos helpers.  All
// reductions are two-pass and in a fixed order (no floating-point atomics),
// so repeated runs are bitwise identical.
#include "internal.h"

namespace pfe {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

inline unsigned nblocks(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

// D(16x16) += A(16x4) B(4x16).  Lane l supplies A[l%16][l/16] and
// B[l/16][l%16]; accumulator element r of lane l is D[l/16 + 4r][l%16].
__device__ __forceinline__ d4 mfma16x16x4(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// ------------------------------------------------------------------ Gram
// Each work-group owns a 64x64 tile of G and a contiguous range of rows;
// rows are staged 16 at a time through LDS.  Partial tiles go to
// work[split][q1][q2] and are summed in split order by k_gram_reduce.
constexpr int kGramRows = 16;

__global__ __launch_bounds__(256) void k_gram_partial(int64_t n, int q1, int q2,
                                                      const double* __restrict__ A, int64_t lda,
                                                      const double* __restrict__ B, int64_t ldb,
                                                      int64_t rows_per_split,
                                                      double* __restrict__ work) {
  __shared__ double sA[kGramRows][64 + 1];
  __shared__ double sB[kGramRows][64 + 1];
  const int tiles_n = (q2 + 63) / 64;
  const int tm = blockIdx.y / tiles_n, tn = blockIdx.y % tiles_n;
  const int m0 = tm * 64, n0 = tn * 64;
  const int split = blockIdx.x;
  const int64_t r_begin = (int64_t)split * rows_per_split;
  int64_t r_end = r_begin + rows_per_split;
  if (r_end > n) r_end = n;
  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  d4 acc[2][2];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) acc[i][j] = d4(0.0);

  for (int64_t r0 = r_begin; r0 < r_end; r0 += kGramRows) {
    // stage: 16 rows x 64 cols of A and of B; thread -> (row tid/16, 4 cols)
    {
      const int rr = tid >> 4, cc = (tid & 15) * 4;
      const int64_t r = r0 + rr;
      for (int t = 0; t < 4; ++t) {
        const int ca = m0 + cc + t, cb = n0 + cc + t;
        sA[rr][cc + t] = (r < r_end && ca < q1) ? A[r * lda + ca] : 0.0;
        sB[rr][cc + t] = (r < r_end && cb < q2) ? B[r * ldb + cb] : 0.0;
      }
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < kGramRows; kk += 4) {
      const int k = kk + (lane >> 4);
      const double a0 = sA[k][wm + (lane & 15)];
      const double a1 = sA[k][wm + 16 + (lane & 15)];
      const double b0 = sB[k][wn + (lane & 15)];
      const double b1 = sB[k][wn + 16 + (lane & 15)];
      acc[0][0] = mfma16x16x4(a0, b0, acc[0][0]);
      acc[0][1] = mfma16x16x4(a0, b1, acc[0][1]);
      acc[1][0] = mfma16x16x4(a1, b0, acc[1][0]);
      acc[1][1] = mfma16x16x4(a1, b1, acc[1][1]);
    }
    __syncthreads();
  }
  double* out = work + (int64_t)split * q1 * q2;
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j)
      for (int r = 0; r < 4; ++r) {
        const int row = m0 + wm + i * 16 + (lane >> 4) + 4 * r;
        const int col = n0 + wn + j * 16 + (lane & 15);
        if (row < q1 && col < q2) out[(int64_t)row * q2 + col] = acc[i][j][r];
      }
}

// G = sum over splits of the partial tiles, in a fixed order: 16 outputs per
// work-group, 16 threads per output each summing every sixteenth split, then
// the sixteen sums in thread order.
__global__ __launch_bounds__(256) void k_gram_reduce(int nsplit, int64_t count,
                                                     const double* __restrict__ work,
                                                     double* __restrict__ G) {
  __shared__ double part[16][17];
  const int o = threadIdx.x & 15, grp = threadIdx.x >> 4;
  const int64_t i = (int64_t)blockIdx.x * 16 + o;
  double s = 0.0;
  if (i < count)
    for (int p = grp; p < nsplit; p += 16) s += work[(int64_t)p * count + i];
  part[grp][o] = s;
  __syncthreads();
  if (grp == 0 && i < count) {
    double t = part[0][o];
    for (int g = 1; g < 16; ++g) t += part[g][o];
    G[i] = t;
  }
}

// Small Gram (q1, q2 <= 128): one work-group forms the whole q1 x q2 product
// of its row range, so nothing is padded beyond a multiple of 32.  Waves are
// 2 x 2, each owning MT x NT MFMA tiles of 16 x 16; rows are staged 16 at a
// time through LDS and the next 16 are loaded into registers while the
// current ones multiply.
constexpr int kGramSmallRows = 16;

template <int MT, int NT>
__global__ __launch_bounds__(256) void k_gram_small(int64_t n, int q1, int q2,
                                                    const double* __restrict__ A, int64_t lda,
                                                    const double* __restrict__ B, int64_t ldb,
                                                    int64_t rows_per_split,
                                                    double* __restrict__ work) {
  constexpr int Q1 = 32 * MT, Q2 = 32 * NT;
  constexpr int LA = (kGramSmallRows * Q1) / 256, LB = (kGramSmallRows * Q2) / 256;
  __shared__ double sA[kGramSmallRows][Q1 + 1];
  __shared__ double sB[kGramSmallRows][Q2 + 1];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int wm = (wave >> 1) * 16 * MT, wn = (wave & 1) * 16 * NT;
  const int64_t r_begin = (int64_t)blockIdx.x * rows_per_split;
  const int64_t r_end = min(n, r_begin + rows_per_split);
  d4 acc[MT][NT];
#pragma unroll
  for (int i = 0; i < MT; ++i)
#pragma unroll
    for (int j = 0; j < NT; ++j) acc[i][j] = d4(0.0);
  double ra[LA], rb[LB];
  auto fetch = [&](int64_t r0) {
#pragma unroll
    for (int t = 0; t < LA; ++t) {
      const int idx = tid + 256 * t, rr = idx / Q1, c = idx % Q1;
      const int64_t r = r0 + rr;
      ra[t] = (r < r_end && c < q1) ? A[r * lda + c] : 0.0;
    }
#pragma unroll
    for (int t = 0; t < LB; ++t) {
      const int idx = tid + 256 * t, rr = idx / Q2, c = idx % Q2;
      const int64_t r = r0 + rr;
      rb[t] = (r < r_end && c < q2) ? B[r * ldb + c] : 0.0;
    }
  };
  if (r_begin < r_end) fetch(r_begin);
  for (int64_t r0 = r_begin; r0 < r_end; r0 += kGramSmallRows) {
#pragma unroll
    for (int t = 0; t < LA; ++t) {
      const int idx = tid + 256 * t;
      sA[idx / Q1][idx % Q1] = ra[t];
    }
#pragma unroll
    for (int t = 0; t < LB; ++t) {
      const int idx = tid + 256 * t;
      sB[idx / Q2][idx % Q2] = rb[t];
    }
    __syncthreads();
    if (r0 + kGramSmallRows < r_end) fetch(r0 + kGramSmallRows);
#pragma unroll
    for (int kk = 0; kk < kGramSmallRows; kk += 4) {
      const int k = kk + (lane >> 4);
      double a[MT], b[NT];
#pragma unroll
      for (int i = 0; i < MT; ++i) a[i] = sA[k][wm + 16 * i + (lane & 15)];
#pragma unroll
      for (int j = 0; j < NT; ++j) b[j] = sB[k][wn + 16 * j + (lane & 15)];
#pragma unroll
      for (int i = 0; i < MT; ++i)
#pragma unroll
        for (int j = 0; j < NT; ++j) acc[i][j] = mfma16x16x4(a[i], b[j], acc[i][j]);
    }
    __syncthreads();
  }
  double* out = work + (int64_t)blockIdx.x * q1 * q2;
#pragma unroll
  for (int i = 0; i < MT; ++i)
#pragma unroll
    for (int j = 0; j < NT; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = wm + 16 * i + (lane >> 4) + 4 * r;
        const int col = wn + 16 * j + (lane & 15);
        if (row < q1 && col < q2) out[(int64_t)row * q2 + col] = acc[i][j][r];
      }
}

// Gram for 128 < max(q1, q2) <= 256: a work-group forms one 128 x 128 tile
// (tm, tn) of G over a contiguous row range, wave w its 64 x 64 quarter as
// 4 x 4 MFMA tiles; rows are staged 16 at a time through LDS, the next 16
// loaded into registers meanwhile.  Work-group b runs on XCD b % 8; the T
// tiles of one row range take consecutive ids on the same XCD (b, b + 8, ...),
// so they stream the same rows together and share them through that XCD's
// L2.  With A = B (sym) only tiles tm <= tn are formed, and an off-diagonal
// tile is also written transposed.  Partial tiles go to work[split][q1][q2].
constexpr int kGramRtTile = 128, kGramRtRows = 16;

__global__ __launch_bounds__(256, 2) void k_gram_rt(int64_t n, int q1, int q2,
                                                    const double* __restrict__ A, int64_t lda,
                                                    const double* __restrict__ B, int64_t ldb,
                                                    int64_t rows_per_split, int nsplit, int tiles_n,
                                                    int ntiles, int sym, double* __restrict__ work) {
  constexpr int TT = kGramRtTile, KR = kGramRtRows;
  constexpr int L = KR * TT / 256;   // 8 per thread and operand
  __shared__ double sA[KR][TT + 2];
  __shared__ double sB[KR][TT + 2];
  const int b = blockIdx.x, xcd = b & 7, s8 = b >> 3;
  const int split = (s8 / ntiles) * 8 + xcd, tile = s8 % ntiles;
  if (split >= nsplit) return;
  int tm, tn;
  if (sym) {   // upper-triangle tiles in row order
    tm = 0;
    int t = tile;
    while (t >= tiles_n - tm) {
      t -= tiles_n - tm;
      ++tm;
    }
    tn = tm + t;
  } else {
    tm = tile / tiles_n;
    tn = tile % tiles_n;
  }
  const int m0 = tm * TT, n0 = tn * TT;
  const int64_t r_begin = (int64_t)split * rows_per_split;
  const int64_t r_end = min(n, r_begin + rows_per_split);
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int wm = (wave >> 1) * 64, wn = (wave & 1) * 64;
  d4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = d4(0.0);
  double ra[L], rb[L];
  auto fetch = [&](int64_t rr0) {
#pragma unroll
    for (int t = 0; t < L; ++t) {
      const int idx = tid + 256 * t, rr = idx / TT, c = idx % TT;
      const int64_t r = rr0 + rr;
      ra[t] = (r < r_end && m0 + c < q1) ? A[r * lda + m0 + c] : 0.0;
      rb[t] = (r < r_end && n0 + c < q2) ? B[r * ldb + n0 + c] : 0.0;
    }
  };
  if (r_begin < r_end) fetch(r_begin);
  for (int64_t rr0 = r_begin; rr0 < r_end; rr0 += KR) {
#pragma unroll
    for (int t = 0; t < L; ++t) {
      const int idx = tid + 256 * t;
      sA[idx / TT][idx % TT] = ra[t];
      sB[idx / TT][idx % TT] = rb[t];
    }
    __syncthreads();
    if (rr0 + KR < r_end) fetch(rr0 + KR);
#pragma unroll
    for (int kk = 0; kk < KR; kk += 4) {
      const int k = kk + (lane >> 4);
      double a[4], bb[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = sA[k][wm + 16 * i + (lane & 15)];
#pragma unroll
      for (int j = 0; j < 4; ++j) bb[j] = sB[k][wn + 16 * j + (lane & 15)];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = mfma16x16x4(a[i], bb[j], acc[i][j]);
    }
    __syncthreads();
  }
  double* out = work + (int64_t)split * q1 * q2;
  const bool mirror = sym && tm != tn;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = m0 + wm + 16 * i + (lane >> 4) + 4 * r;
        const int col = n0 + wn + 16 * j + (lane & 15);
        if (row < q1 && col < q2) {
          out[(int64_t)row * q2 + col] = acc[i][j][r];
          if (mirror) out[(int64_t)col * q2 + row] = acc[i][j][r];
        }
      }
}

// Splits of the tiled Gram: about 512 work-groups, a multiple of 8 row
// ranges (one round per XCD), at least 256 rows each.
int gram_rt_splits(int64_t n, int ntiles) {
  int64_t want = (512 + ntiles - 1) / ntiles;
  want = ((want + 7) / 8) * 8;
  const int64_t maxs = std::max<int64_t>(1, (n + 255) / 256);
  return (int)std::max<int64_t>(1, std::min(want, maxs));
}

bool gram_rt_applies(int q1, int q2) {
  return std::max(q1, q2) > 128 && q1 <= 256 && q2 <= 256;
}

int gram_rt_tiles(int q1, int q2, bool sym) {
  const int tm = (q1 + kGramRtTile - 1) / kGramRtTile, tn = (q2 + kGramRtTile - 1) / kGramRtTile;
  return sym ? tn * (tn + 1) / 2 : tm * tn;
}

constexpr int kGramSmallMax = 128;

int gram_splits(int64_t n, int q1, int q2) {
  if (q1 <= kGramSmallMax && q2 <= kGramSmallMax) {
    int64_t want = std::min<int64_t>(512, (n + 255) / 256);   // two work-groups per CU
    return (int)std::max<int64_t>(want, 1);
  }
  const int tiles = ((q1 + 63) / 64) * ((q2 + 63) / 64);
  int64_t want = 1024 / tiles;                     // ~1024 work-groups in total
  if (want < 8) want = 8;
  const int64_t maxs = (n + 255) / 256;            // at least 256 rows per split
  if (want > maxs) want = maxs;
  if (want < 1) want = 1;
  return (int)want;
}

// ------------------------------------------------------------ tall GEMM
// C[r][:q2] = A[r][:q1] Bm.  A work-group stages RB full rows of A in LDS
// (so C may overwrite A), then produces 64-column output tiles.  RB = 32:
// waves are 2 (16 rows) x 2 (32 columns); RB = 16 (wide q1, LDS <= 64 KB):
// waves are 1 x 4 (16 columns each).  B fragments come from global memory
// (q1 x q2 is small and L2-resident).
template <int RB>
__global__ __launch_bounds__(256) void k_gemm_tall(int64_t n, int q1, int q2,
                                                   const double* A, int64_t lda,
                                                   const double* __restrict__ Bm, double* C,
                                                   int64_t ldc) {
  extern __shared__ double sA[];   // [RB][q1p]
  const int q1p = ((q1 + 3) / 4) * 4 + 1;
  const int64_t r0 = (int64_t)blockIdx.x * RB;
  const int tid = threadIdx.x;
  for (int idx = tid; idx < RB * q1p; idx += 256) {
    const int rr = idx / q1p, c = idx % q1p;
    const int64_t r = r0 + rr;
    sA[idx] = (r < n && c < q1) ? A[r * lda + c] : 0.0;
  }
  __syncthreads();
  const int wave = tid >> 6, lane = tid & 63;
  constexpr int kTiles = (RB == 32) ? 2 : 1;            // 16-column MFMA tiles per wave
  const int wr = (RB == 32) ? (wave >> 1) * 16 : 0;
  const int wc = (RB == 32) ? (wave & 1) * 32 : wave * 16;
  const int kq = (q1 + 3) / 4;
  for (int n0 = 0; n0 < q2; n0 += 64) {
    d4 acc[kTiles];
    int cc[kTiles];
#pragma unroll
    for (int t = 0; t < kTiles; ++t) {
      acc[t] = d4(0.0);
      cc[t] = n0 + wc + 16 * t + (lane & 15);
    }
    for (int kb = 0; kb < kq; ++kb) {
      const int k = kb * 4 + (lane >> 4);
      const double a = sA[(wr + (lane & 15)) * q1p + k];
#pragma unroll
      for (int t = 0; t < kTiles; ++t) {
        const double b = (k < q1 && cc[t] < q2) ? Bm[(int64_t)k * q2 + cc[t]] : 0.0;
        acc[t] = mfma16x16x4(a, b, acc[t]);
      }
    }
    for (int r = 0; r < 4; ++r) {
      const int64_t row = r0 + wr + (lane >> 4) + 4 * r;
      if (row < n) {
#pragma unroll
        for (int t = 0; t < kTiles; ++t)
          if (cc[t] < q2) C[row * ldc + cc[t]] = acc[t][r];
      }
    }
  }
}

// Tall GEMM for 128 < max(q1, q2) <= 256: a work-group owns 64 rows of C
// and every output column; wave w forms columns [64 w, 64 w + 64) of them as
// 4 x 4 MFMA tiles (64 accumulators per lane), so each element of Bm is read
// from L2 once per 64 rows (not once per 16-row MFMA tile).  K advances 16 at
// a time: the 64 x 16 slice of A (k-major) and the 16 x 256 slice of Bm are
// staged in LDS while the next slices are loaded into registers.  Every A row
// of the work-group is read before any C row is written, so C may overwrite A.
constexpr int kGemmRtRows = 64, kGemmRtK = 16, kGemmRtCols = 256;

__global__ __launch_bounds__(256, 2) void k_gemm_rt(int64_t n, int q1, int q2, const double* A,
                                                 int64_t lda, const double* __restrict__ Bm,
                                                 double* C, int64_t ldc) {
  constexpr int RB = kGemmRtRows, KC = kGemmRtK, QC = kGemmRtCols;
  constexpr int LA = RB * KC / 256, LB = KC * QC / 256;   // 4 and 16 per thread
  __shared__ double sA[KC][RB + 1];
  __shared__ double sB[KC][QC + 2];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int64_t r0 = (int64_t)blockIdx.x * RB;
  const bool active = 64 * wave < q2;   // waves past q2 only help with the loads
  d4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = d4(0.0);
  double ra[LA], rb[LB];
  // A: thread -> (row tid / 4, k (tid % 4) * 4 .. + 3); Bm: idx -> (k idx / 256, column idx % 256)
  auto fetch = [&](int k0) {
    const int rr = tid >> 2, kb = (tid & 3) * 4;
    const int64_t r = r0 + rr;
#pragma unroll
    for (int t = 0; t < LA; ++t) {
      const int k = k0 + kb + t;
      ra[t] = (r < n && k < q1) ? A[r * lda + k] : 0.0;
    }
#pragma unroll
    for (int t = 0; t < LB; ++t) {
      const int idx = tid + 256 * t, k = k0 + idx / QC, c = idx % QC;
      rb[t] = (k < q1 && c < q2) ? Bm[(int64_t)k * q2 + c] : 0.0;
    }
  };
  fetch(0);
  for (int k0 = 0; k0 < q1; k0 += KC) {
    {
      const int rr = tid >> 2, kb = (tid & 3) * 4;
#pragma unroll
      for (int t = 0; t < LA; ++t) sA[kb + t][rr] = ra[t];
#pragma unroll
      for (int t = 0; t < LB; ++t) {
        const int idx = tid + 256 * t;
        sB[idx / QC][idx % QC] = rb[t];
      }
    }
    __syncthreads();
    if (k0 + KC < q1) fetch(k0 + KC);
    if (active) {
#pragma unroll
      for (int kk = 0; kk < KC; kk += 4) {
        const int k = kk + (lane >> 4);
        double a[4], b[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) a[i] = sA[k][16 * i + (lane & 15)];
#pragma unroll
        for (int j = 0; j < 4; ++j) b[j] = sB[k][64 * wave + 16 * j + (lane & 15)];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int j = 0; j < 4; ++j) acc[i][j] = mfma16x16x4(a[i], b[j], acc[i][j]);
      }
    }
    __syncthreads();
  }
  if (!active) return;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t row = r0 + 16 * i + (lane >> 4) + 4 * r;
      if (row < n) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int col = 64 * wave + 16 * j + (lane & 15);
          if (col < q2) C[row * ldc + col] = acc[i][j][r];
        }
      }
    }
}

// Tall GEMM for q1, q2 <= 128: Bm (padded to KM x 16 NT) is staged once per
// work-group in LDS; each wave then walks 16-row tiles of A with NT
// independent 16 x 16 accumulators, its A fragments loaded straight from
// memory one tile ahead.  A wave reads all of a tile's rows before writing
// them, so C may overwrite A.
template <int KM, int NT>
__global__ __launch_bounds__(256) void k_gemm_bres(int64_t n, int q1, int q2, const double* A,
                                                   int64_t lda, const double* __restrict__ Bm,
                                                   double* C, int64_t ldc) {
  constexpr int Q2 = 16 * NT, LDB = Q2 + 1;
  __shared__ double sB[KM * LDB];
  const int tid = threadIdx.x;
  for (int idx = tid; idx < KM * Q2; idx += 256) {
    const int k = idx / Q2, c = idx % Q2;
    sB[k * LDB + c] = (k < q1 && c < q2) ? Bm[(int64_t)k * q2 + c] : 0.0;
  }
  __syncthreads();
  const int wave = tid >> 6, lane = tid & 63;
  const int64_t ntile = (n + 15) / 16;
  const int64_t stride = (int64_t)gridDim.x * 4;
  constexpr int KT = KM / 4;
  // A fragments of one tile: lane l holds A[r0 + l % 16][4 kb + l / 16]
  auto load = [&](double (&f)[KT], int64_t t) {
    const int64_t r0 = t * 16, r = r0 + (lane & 15);
    const bool rok = r < n;
    const double* arow = A + (rok ? r : r0) * lda;
#pragma unroll
    for (int kb = 0; kb < KT; ++kb) {
      const int k = 4 * kb + (lane >> 4);
      f[kb] = (rok && k < q1) ? arow[k] : 0.0;
    }
  };
  double fn[KT];
  int64_t t = (int64_t)blockIdx.x * 4 + wave;
  if (t < ntile) load(fn, t);
  for (; t < ntile; t += stride) {
    double fc[KT];
#pragma unroll
    for (int kb = 0; kb < KT; ++kb) fc[kb] = fn[kb];
    // the next tile's fragments are in flight during this tile's products;
    // its rows differ from this tile's, so C overwriting A stays safe
    if (t + stride < ntile) load(fn, t + stride);
    d4 acc[NT];
#pragma unroll
    for (int j = 0; j < NT; ++j) acc[j] = d4(0.0);
#pragma unroll
    for (int kb = 0; kb < KT; ++kb) {
      const int k = 4 * kb + (lane >> 4);
#pragma unroll
      for (int j = 0; j < NT; ++j)
        acc[j] = mfma16x16x4(fc[kb], sB[k * LDB + 16 * j + (lane & 15)], acc[j]);
      // one k-step's B reads at a time (the MFMAs in flight cover their
      // latency); hoisting them all would cost KT x NT registers
      __builtin_amdgcn_sched_barrier(0);
    }
    const int64_t r0 = t * 16;
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) {
      const int64_t row = r0 + (lane >> 4) + 4 * rr;
      if (row < n) {
#pragma unroll
        for (int j = 0; j < NT; ++j) {
          const int col = 16 * j + (lane & 15);
          if (col < q2) C[row * ldc + col] = acc[j][rr];
        }
      }
    }
  }
}

// ------------------------------------------------ Cholesky and inverse
// Single work-group.  R (upper) is formed in place in Rinv's buffer by a
// right-looking factorisation, then inverted column by column into work
// that is copied back.  info[0] = 0 or the failing pivot + 1.
__global__ __launch_bounds__(1024) void k_chol_inv(int q, const double* __restrict__ G,
                                                   double shift, double* R, double* Z,
                                                   int* info, double* diag_max) {
  __shared__ int bad;
  const int tid = threadIdx.x, nt = blockDim.x;
  if (tid == 0) {
    bad = 0;
    double mx = 0.0;
    for (int i = 0; i < q; ++i) mx = fmax(mx, G[i * q + i]);
    if (diag_max) diag_max[0] = mx;
  }
  for (int idx = tid; idx < q * q; idx += nt) {
    const int i = idx / q, j = idx % q;
    R[idx] = (j >= i) ? G[idx] + (i == j ? shift : 0.0) : 0.0;
  }
  __syncthreads();
  for (int k = 0; k < q; ++k) {
    if (tid == 0) {
      const double d = R[k * q + k];
      if (!(d > 0.0) || !isfinite(d)) {
        bad = k + 1;
      } else {
        R[k * q + k] = sqrt(d);
      }
    }
    __syncthreads();
    if (bad) break;
    const double rkk = R[k * q + k];
    for (int j = k + 1 + tid; j < q; j += nt) R[k * q + j] /= rkk;
    __syncthreads();
    const int m = q - k - 1;   // trailing upper triangle of size m
    for (int idx = tid; idx < m * m; idx += nt) {
      const int i = k + 1 + idx / m, j = k + 1 + idx % m;
      if (j >= i) R[i * q + j] -= R[k * q + i] * R[k * q + j];
    }
    __syncthreads();
  }
  if (bad) {
    if (tid == 0) info[0] = bad;
    return;
  }
  // Z = R^{-1} (upper) column by column from Z R = I: column j needs only
  // the columns before it, and its entries above the diagonal,
  //   Z[i][j] = -(sum_{i <= k < j} Z[i][k] R[k][j]) / R[j][j],
  // are independent dot products, four threads each (a group of four lanes
  // shares its row, so the shuffles stay inside active groups)
  for (int idx = tid; idx < q * q; idx += nt) Z[idx] = 0.0;
  __syncthreads();
  for (int j = 0; j < q; ++j) {
    const double rjj = R[j * q + j];
    const int sub = tid & 3;
    for (int i = tid >> 2; i < j; i += nt >> 2) {
      double acc = 0.0;
      for (int k = i + sub; k < j; k += 4) acc += Z[i * q + k] * R[k * q + j];
      acc += __shfl_xor(acc, 1, 64);
      acc += __shfl_xor(acc, 2, 64);
      if (sub == 0) Z[i * q + j] = -acc / rjj;
    }
    if (tid == 0) Z[j * q + j] = 1.0 / rjj;
    __syncthreads();
  }
  for (int idx = tid; idx < q * q; idx += nt) R[idx] = Z[idx];
  if (tid == 0) info[0] = 0;
}

// LDS-resident variant for q <= kCholLdsMax: the factor is built in place
// in LDS (two barriers per column: scale row k, then the trailing update),
// then inverted in place column by column from Z R = I:
// Z[0:j, j] = -Z[0:j, 0:j] R[0:j, j] / R[j][j], whose j dot products run on
// 8 threads each, so no step waits on a serial substitution chain.
constexpr int kCholLdsMax = 128;

__global__ __launch_bounds__(1024) void k_chol_inv_lds(int q, const double* __restrict__ G,
                                                       double shift, double* __restrict__ Rout,
                                                       int* info, double* diag_max) {
  __shared__ double R[kCholLdsMax * kCholLdsMax];
  __shared__ double col[kCholLdsMax];
  const int tid = threadIdx.x, nt = blockDim.x;
  if (tid == 0 && diag_max) {
    double mx = 0.0;
    for (int i = 0; i < q; ++i) mx = fmax(mx, G[i * q + i]);
    diag_max[0] = mx;
  }
  for (int idx = tid; idx < q * q; idx += nt) {
    const int i = idx / q, j = idx - i * q;
    R[idx] = (j >= i) ? G[idx] + (i == j ? shift : 0.0) : 0.0;
  }
  __syncthreads();
  for (int k = 0; k < q; ++k) {
    const double d = R[k * q + k];   // the same value in every thread
    if (!(d > 0.0) || !isfinite(d)) {
      if (tid == 0) info[0] = k + 1;
      return;
    }
    const double rkk = sqrt(d);
    for (int j = k + 1 + tid; j < q; j += nt) R[k * q + j] /= rkk;
    __syncthreads();
    if (tid == 0) R[k * q + k] = rkk;
    for (int i = k + 1 + (tid >> 5); i < q; i += (nt >> 5)) {
      const double rki = R[k * q + i];
      for (int j = i + (tid & 31); j < q; j += 32) R[i * q + j] -= rki * R[k * q + j];
    }
    __syncthreads();
  }
  const int ri = tid >> 3, rl = tid & 7;   // 8 threads per row of Z
  for (int j = 0; j < q; ++j) {
    if (tid < j) col[tid] = R[tid * q + j];
    __syncthreads();
    const double zjj = 1.0 / R[j * q + j];
    double sum = 0.0;
    if (ri < j)
      for (int k = ri + rl; k < j; k += 8) sum += R[ri * q + k] * col[k];
    sum += __shfl_xor(sum, 1);
    sum += __shfl_xor(sum, 2);
    sum += __shfl_xor(sum, 4);
    __syncthreads();
    if (rl == 0 && ri < j) R[ri * q + j] = -zjj * sum;
    if (tid == 0) R[j * q + j] = zjj;
  }
  __syncthreads();
  for (int idx = tid; idx < q * q; idx += nt) Rout[idx] = R[idx];
  if (tid == 0) info[0] = 0;
}

// ------------------------------------------------------- Jacobi eigensolve
// One work-group, A and V in global scratch.  Round-robin (circle method)
// ordering: m/2 disjoint rotations per step, m-1 steps per sweep.  A
// rotation is skipped when |a_pq| <= eps sqrt(|a_pp a_qq|) or below an
// absolute floor 1e-18 ||A||_F; sweeps stop when none is applied.
__device__ __forceinline__ void rr_pair(int m, int step, int k, int* p, int* q) {
  if (k == 0) {
    *p = m - 1;
    *q = step;
  } else {
    *p = (step + k) % (m - 1);
    *q = (step - k + (m - 1)) % (m - 1);
  }
}

constexpr int kJb = 4;   // 2 x 2 blocks per batch in k_jacobi

__global__ __launch_bounds__(1024) void k_jacobi(int q, const double* __restrict__ S,
                                                 double* A, double* V, double* evals, double* Q,
                                                 int* info) {
  __shared__ double cs[512], sn[512];
  __shared__ int pp[512], qq[512];
  __shared__ int rotated;
  __shared__ double red[1024];
  const int tid = threadIdx.x, nt = blockDim.x;
  const int m = q + (q & 1);
  const int half = m / 2;
  double loc = 0.0;
  for (int idx = tid; idx < q * q; idx += nt) {
    const int i = idx / q, j = idx % q;
    const double a = 0.5 * (S[i * q + j] + S[j * q + i]);
    A[idx] = a;
    V[idx] = (i == j) ? 1.0 : 0.0;
    loc += a * a;
  }
  red[tid] = loc;
  __syncthreads();
  for (int s = nt / 2; s > 0; s >>= 1) {
    if (tid < s) red[tid] += red[tid + s];
    __syncthreads();
  }
  const double floor_abs = 1e-18 * sqrt(red[0]) + 1e-300;
  const double eps = 2.220446049250313e-16;
  int sweep = 0;
  const int max_sweeps = 60;
  bool converged = (q < 2);
  // threads per row pair in the fused update (a power of two)
  int tpp = 1;
  while (tpp * 2 * half <= nt && tpp < 32) tpp *= 2;
  for (; sweep < max_sweeps && !converged; ++sweep) {
    if (tid == 0) rotated = 0;
    __syncthreads();
    for (int step = 0; step < m - 1; ++step) {
      if (tid < half) {
        int p, r;
        rr_pair(m, step, tid, &p, &r);
        double c = 1.0, s = 0.0;
        if (p < q && r < q) {
          const double apq = A[p * q + r];
          const double app = A[p * q + p], arr = A[r * q + r];
          if (fabs(apq) > floor_abs && fabs(apq) > eps * sqrt(fabs(app * arr))) {
            const double theta = (arr - app) / (2.0 * apq);
            const double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
            c = 1.0 / sqrt(t * t + 1.0);
            s = t * c;
            rotated = 1;
          }
        }
        cs[tid] = c;
        sn[tid] = s;
        pp[tid] = p;
        qq[tid] = r;
      }
      __syncthreads();
      // One pass per step: rows p, r of the pair k meet columns p', r' of
      // every pair k' in a 2 x 2 block, which takes the row rotation of k and
      // then the column rotation of k' (the same products, in the same order,
      // as rotating all rows first and all columns after; a pair without a
      // rotation changes nothing).  The rotated pair's own off-diagonal
      // entries get their exact zero.  V is kept transposed: its rows p, r
      // take the row rotation only.
      for (int w = tid; w < half * tpp; w += nt) {
        const int k = w / tpp, sub = w % tpp;
        const double c = cs[k], s = sn[k];
        const int p = pp[k], r = qq[k];
        const bool rp = p < q, rr = r < q;
        // blocks in batches of kJb: all loads of a batch are issued before
        // its stores (they touch distinct entries, which the compiler cannot
        // see through one pointer)
        for (int k0 = sub; k0 < half; k0 += kJb * tpp) {
          double a[kJb][4];
#pragma unroll
          for (int b = 0; b < kJb; ++b) {
            const int k2 = k0 + b * tpp;
            const bool in = k2 < half;
            const int p2 = in ? pp[k2] : q, r2 = in ? qq[k2] : q;
            a[b][0] = (rp && p2 < q) ? A[p * q + p2] : 0.0;
            a[b][1] = (rp && r2 < q) ? A[p * q + r2] : 0.0;
            a[b][2] = (rr && p2 < q) ? A[r * q + p2] : 0.0;
            a[b][3] = (rr && r2 < q) ? A[r * q + r2] : 0.0;
          }
#pragma unroll
          for (int b = 0; b < kJb; ++b) {
            const int k2 = k0 + b * tpp;
            if (k2 >= half) continue;
            double a11 = a[b][0], a12 = a[b][1], a21 = a[b][2], a22 = a[b][3];
            if (s != 0.0) {
              const double b11 = c * a11 - s * a21, b21 = s * a11 + c * a21;
              const double b12 = c * a12 - s * a22, b22 = s * a12 + c * a22;
              a11 = b11;
              a21 = b21;
              a12 = b12;
              a22 = b22;
            }
            const double c2 = cs[k2], s2 = sn[k2];
            if (s2 != 0.0) {
              const double b11 = c2 * a11 - s2 * a12, b12 = s2 * a11 + c2 * a12;
              const double b21 = c2 * a21 - s2 * a22, b22 = s2 * a21 + c2 * a22;
              a11 = b11;
              a12 = b12;
              a21 = b21;
              a22 = b22;
              if (k2 == k) {
                a12 = 0.0;
                a21 = 0.0;
              }
            }
            const int p2 = pp[k2], r2 = qq[k2];
            if (rp && p2 < q) A[p * q + p2] = a11;
            if (rp && r2 < q) A[p * q + r2] = a12;
            if (rr && p2 < q) A[r * q + p2] = a21;
            if (rr && r2 < q) A[r * q + r2] = a22;
          }
        }
        if (s != 0.0) {
          for (int j0 = sub; j0 < q; j0 += 2 * kJb * tpp) {
            double va[2 * kJb], vb[2 * kJb];
#pragma unroll
            for (int b = 0; b < 2 * kJb; ++b) {
              const int j2 = j0 + b * tpp;
              va[b] = j2 < q ? V[p * q + j2] : 0.0;
              vb[b] = j2 < q ? V[r * q + j2] : 0.0;
            }
#pragma unroll
            for (int b = 0; b < 2 * kJb; ++b) {
              const int j2 = j0 + b * tpp;
              if (j2 < q) {
                V[p * q + j2] = c * va[b] - s * vb[b];
                V[r * q + j2] = s * va[b] + c * vb[b];
              }
            }
          }
        }
      }
      __syncthreads();
    }
    converged = (rotated == 0);
    __syncthreads();
  }
  // sort ascending (rank with index tie-break)
  for (int i = tid; i < q; i += nt) {
    const double di = A[i * q + i];
    int rank = 0;
    for (int j = 0; j < q; ++j) {
      const double dj = A[j * q + j];
      if (dj < di || (dj == di && j < i)) ++rank;
    }
    evals[rank] = di;
    for (int r = 0; r < q; ++r) Q[r * q + rank] = V[i * q + r];   // V holds V^T
  }
  if (tid == 0) info[0] = converged ? sweep : -sweep;
}

// The same Jacobi over several work-groups, one kernel per round-robin step
// (q above kJacobiOneGroupMax, where one work-group's path to L2 limits the
// single-kernel form).  A is double-buffered: every work-group forms all of
// the step's rotations from the previous step's matrix (which no work-group
// of this step writes), then work-group k applies them to row pair k (its
// 2 x 2 blocks with every column pair, into the other buffer, then its rows
// of V^T in place), with the products of k_jacobi; the host reads one flag
// per sweep.  Work: A0, A1, V [q][q], floor, one flag per sweep.
constexpr int kJacobiOneGroupMax = 128;
constexpr int kJacobiMaxSweeps = 60;

__global__ __launch_bounds__(1024) void k_jac_init(int q, const double* __restrict__ S, double* A,
                                                   double* V, double* floor_abs, int* flags) {
  __shared__ double red[1024];
  const int tid = threadIdx.x, nt = blockDim.x;
  double loc = 0.0;
  for (int idx = tid; idx < q * q; idx += nt) {
    const int i = idx / q, j = idx % q;
    const double a = 0.5 * (S[i * q + j] + S[j * q + i]);
    A[idx] = a;
    V[idx] = (i == j) ? 1.0 : 0.0;
    loc += a * a;
  }
  red[tid] = loc;
  if (tid < kJacobiMaxSweeps) flags[tid] = 0;
  __syncthreads();
  for (int s = nt / 2; s > 0; s >>= 1) {
    if (tid < s) red[tid] += red[tid + s];
    __syncthreads();
  }
  if (tid == 0) floor_abs[0] = 1e-18 * sqrt(red[0]) + 1e-300;
}

__global__ __launch_bounds__(512) void k_jac_step(int q, int step, const double* __restrict__ Ain,
                                                  double* __restrict__ Aout, double* V,
                                                  const double* __restrict__ floor_abs,
                                                  int* rotated) {
  __shared__ double cs[512], sn[512];
  __shared__ int pp[512], qq[512];
  const int m = q + (q & 1), half = m / 2;
  const double eps = 2.220446049250313e-16;
  for (int k = threadIdx.x; k < half; k += blockDim.x) {
    int p, r;
    rr_pair(m, step, k, &p, &r);
    double c = 1.0, s = 0.0;
    if (p < q && r < q) {
      const double apq = Ain[p * q + r];
      const double app = Ain[p * q + p], arr = Ain[r * q + r];
      if (fabs(apq) > floor_abs[0] && fabs(apq) > eps * sqrt(fabs(app * arr))) {
        const double theta = (arr - app) / (2.0 * apq);
        const double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
        c = 1.0 / sqrt(t * t + 1.0);
        s = t * c;
        if (blockIdx.x == 0) rotated[0] = 1;
      }
    }
    cs[k] = c;
    sn[k] = s;
    pp[k] = p;
    qq[k] = r;
  }
  __syncthreads();
  const int k = blockIdx.x;
  const double c = cs[k], s = sn[k];
  const int p = pp[k], r = qq[k];
  const bool rp = p < q, rr = r < q;
  for (int k2 = threadIdx.x; k2 < half; k2 += blockDim.x) {
    const double c2 = cs[k2], s2 = sn[k2];
    const int p2 = pp[k2], r2 = qq[k2];
    const bool cp = p2 < q, cr = r2 < q;
    double a11 = (rp && cp) ? Ain[p * q + p2] : 0.0, a12 = (rp && cr) ? Ain[p * q + r2] : 0.0;
    double a21 = (rr && cp) ? Ain[r * q + p2] : 0.0, a22 = (rr && cr) ? Ain[r * q + r2] : 0.0;
    if (s != 0.0) {
      const double b11 = c * a11 - s * a21, b21 = s * a11 + c * a21;
      const double b12 = c * a12 - s * a22, b22 = s * a12 + c * a22;
      a11 = b11;
      a21 = b21;
      a12 = b12;
      a22 = b22;
    }
    if (s2 != 0.0) {
      const double b11 = c2 * a11 - s2 * a12, b12 = s2 * a11 + c2 * a12;
      const double b21 = c2 * a21 - s2 * a22, b22 = s2 * a21 + c2 * a22;
      a11 = b11;
      a12 = b12;
      a21 = b21;
      a22 = b22;
      if (k2 == k) {
        a12 = 0.0;
        a21 = 0.0;
      }
    }
    if (rp && cp) Aout[p * q + p2] = a11;
    if (rp && cr) Aout[p * q + r2] = a12;
    if (rr && cp) Aout[r * q + p2] = a21;
    if (rr && cr) Aout[r * q + r2] = a22;
  }
  if (s != 0.0) {
    for (int j = threadIdx.x; j < q; j += blockDim.x) {
      const double va = V[p * q + j], vb = V[r * q + j];
      V[p * q + j] = c * va - s * vb;
      V[r * q + j] = s * va + c * vb;
    }
  }
}

__global__ __launch_bounds__(1024) void k_jac_final(int q, const double* __restrict__ A,
                                                    const double* __restrict__ V, double* evals,
                                                    double* Q, int* info, int sweeps) {
  for (int i = threadIdx.x; i < q; i += blockDim.x) {
    const double di = A[i * q + i];
    int rank = 0;
    for (int j = 0; j < q; ++j) {
      const double dj = A[j * q + j];
      if (dj < di || (dj == di && j < i)) ++rank;
    }
    evals[rank] = di;
    for (int r = 0; r < q; ++r) Q[r * q + rank] = V[i * q + r];   // V holds V^T
  }
  if (threadIdx.x == 0) info[0] = sweeps;
}

// LDS-resident variant for q <= kJacobiLdsMax: A and V^T live in LDS with
// row stride q+1 (column sweeps hit distinct banks); same ordering, skip
// rule and stopping rule as k_jacobi.
constexpr int kJacobiLdsMax = 96;

__global__ __launch_bounds__(1024) void k_jacobi_lds(int q, const double* __restrict__ S,
                                                     double* __restrict__ evals,
                                                     double* __restrict__ Q, int* info) {
  __shared__ double A[kJacobiLdsMax * (kJacobiLdsMax + 1)];
  __shared__ double VT[kJacobiLdsMax * (kJacobiLdsMax + 1)];
  __shared__ double cs[kJacobiLdsMax / 2 + 1], sn[kJacobiLdsMax / 2 + 1];
  __shared__ int pp[kJacobiLdsMax / 2 + 1], qq[kJacobiLdsMax / 2 + 1];
  __shared__ int rotated;
  __shared__ double red[1024];
  const int tid = threadIdx.x, nt = blockDim.x;
  const int ldq = q + 1;
  const int m = q + (q & 1);
  const int half = m / 2;
  double loc = 0.0;
  for (int idx = tid; idx < q * q; idx += nt) {
    const int i = idx / q, j = idx % q;
    const double a = 0.5 * (S[i * q + j] + S[j * q + i]);
    A[i * ldq + j] = a;
    VT[i * ldq + j] = (i == j) ? 1.0 : 0.0;
    loc += a * a;
  }
  red[tid] = loc;
  __syncthreads();
  for (int s = nt / 2; s > 0; s >>= 1) {
    if (tid < s) red[tid] += red[tid + s];
    __syncthreads();
  }
  const double floor_abs = 1e-18 * sqrt(red[0]) + 1e-300;
  const double eps = 2.220446049250313e-16;
  int sweep = 0;
  bool converged = (q < 2);
  for (; sweep < 60 && !converged; ++sweep) {
    if (tid == 0) rotated = 0;
    __syncthreads();
    for (int step = 0; step < m - 1; ++step) {
      if (tid < half) {
        int p, r;
        rr_pair(m, step, tid, &p, &r);
        double c = 1.0, s = 0.0;
        if (p < q && r < q) {
          const double apq = A[p * ldq + r];
          const double app = A[p * ldq + p], arr = A[r * ldq + r];
          if (fabs(apq) > floor_abs && fabs(apq) > eps * sqrt(fabs(app * arr))) {
            const double theta = (arr - app) / (2.0 * apq);
            const double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
            c = 1.0 / sqrt(t * t + 1.0);
            s = t * c;
            rotated = 1;
          }
        }
        cs[tid] = c;
        sn[tid] = s;
        pp[tid] = p;
        qq[tid] = r;
      }
      __syncthreads();
      // rows p, r of A and of V^T: rotation k on thread rows k = tid/32 (+32),
      // element j on the 32 lanes of that row group
      for (int k = tid >> 5; k < half; k += nt >> 5) {
        const double s = sn[k];
        if (s == 0.0) continue;
        const double c = cs[k];
        const int p = pp[k], r = qq[k];
        for (int j = tid & 31; j < q; j += 32) {
          const double a = A[p * ldq + j], b = A[r * ldq + j];
          A[p * ldq + j] = c * a - s * b;
          A[r * ldq + j] = s * a + c * b;
          const double va = VT[p * ldq + j], vb = VT[r * ldq + j];
          VT[p * ldq + j] = c * va - s * vb;
          VT[r * ldq + j] = s * va + c * vb;
        }
      }
      __syncthreads();
      // columns p, r of A; the pivot pair (p, r) is set to its exact zero here
      for (int k = tid >> 5; k < half; k += nt >> 5) {
        const double s = sn[k];
        if (s == 0.0) continue;
        const double c = cs[k];
        const int p = pp[k], r = qq[k];
        for (int i = tid & 31; i < q; i += 32) {
          const double a = A[i * ldq + p], b = A[i * ldq + r];
          A[i * ldq + p] = (i == r) ? 0.0 : c * a - s * b;
          A[i * ldq + r] = (i == p) ? 0.0 : s * a + c * b;
        }
      }
      __syncthreads();
    }
    converged = (rotated == 0);
    __syncthreads();
  }
  for (int i = tid; i < q; i += nt) {
    const double di = A[i * ldq + i];
    int rank = 0;
    for (int j = 0; j < q; ++j) {
      const double dj = A[j * ldq + j];
      if (dj < di || (dj == di && j < i)) ++rank;
    }
    evals[rank] = di;
    for (int r = 0; r < q; ++r) Q[r * q + rank] = VT[i * ldq + r];
  }
  if (tid == 0) info[0] = converged ? sweep : -sweep;
}

// ------------------------------------------------------- column reductions
constexpr int kColRows = 128;   // rows per partial block

// Column partials over kColRows rows: lanes take columns (64 per pass), the
// four waves every fourth row, summed across waves in wave order.  MODE 0:
// sum (W - theta X)^2 (X may be null); MODE 1: sum X * Y (W holds X).
template <int MODE>
__global__ __launch_bounds__(256) void k_col_partial(int64_t n, int q, const double* __restrict__ W,
                                                     const double* __restrict__ X, int64_t ld,
                                                     const double* __restrict__ theta,
                                                     double* __restrict__ part) {
  __shared__ double red[4][64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t r0 = (int64_t)blockIdx.x * kColRows;
  const int64_t r1 = min(n, r0 + kColRows);
  for (int j0 = 0; j0 < q; j0 += 64) {
    const int j = j0 + lane;
    double s = 0.0;
    if (j < q) {
      const double th = (MODE == 0 && theta) ? theta[j] : 0.0;
#pragma unroll 4
      for (int64_t r = r0 + wave; r < r1; r += 4) {
        if (MODE == 0) {
          double v = W[r * ld + j];
          if (X) v -= th * X[r * ld + j];
          s += v * v;
        } else {
          s += W[r * ld + j] * X[r * ld + j];
        }
      }
    }
    red[wave][lane] = s;
    __syncthreads();
    if (wave == 0 && j < q)
      part[(int64_t)blockIdx.x * q + j] = ((red[0][lane] + red[1][lane]) + red[2][lane]) + red[3][lane];
    __syncthreads();
  }
}

// res[j] = f(sum over blocks of part[b][j]): 16 columns per work-group, 16
// threads per column summing every sixteenth block, then in thread order.
// f = scale * sqrt (norms) or the identity (dots).
template <bool SQRT>
__global__ __launch_bounds__(256) void k_col_final(int nblk, int q, const double* __restrict__ part,
                                                   double scale, double* __restrict__ res) {
  __shared__ double acc[16][17];
  const int o = threadIdx.x & 15, grp = threadIdx.x >> 4;
  const int j = blockIdx.x * 16 + o;
  double s = 0.0;
  if (j < q)
    for (int b = grp; b < nblk; b += 16) s += part[(int64_t)b * q + j];
  acc[grp][o] = s;
  __syncthreads();
  if (grp == 0 && j < q) {
    double t = acc[0][o];
    for (int g = 1; g < 16; ++g) t += acc[g][o];
    res[j] = SQRT ? sqrt(t) * scale : t;
  }
}

__global__ void k_col_scale_inv(int64_t n, int q, double* __restrict__ X, int64_t ld,
                                const double* __restrict__ nrm) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n * q) return;
  const int64_t r = i / q, c = i % q;
  X[r * ld + c] /= nrm[c];
}

// ------------------------------------------------------------ elementwise
__global__ void k_cast_d2f(int64_t n, int q, const double* __restrict__ X, int64_t ldx,
                           float* __restrict__ Y, int64_t ldy) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n * q) return;
  const int64_t r = i / q, c = i % q;
  Y[r * ldy + c] = (float)X[r * ldx + c];
}
__global__ void k_cast_f2d(int64_t n, int q, const float* __restrict__ X, int64_t ldx,
                           double* __restrict__ Y, int64_t ldy) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n * q) return;
  const int64_t r = i / q, c = i % q;
  Y[r * ldy + c] = (double)X[r * ldx + c];
}
__global__ void k_copy_cols(int64_t n, int q, const double* __restrict__ X, int64_t ldx,
                            double* __restrict__ Y, int64_t ldy) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n * q) return;
  const int64_t r = i / q, c = i % q;
  Y[r * ldy + c] = X[r * ldx + c];
}
// Y[:, :q] -= X[:, :q]
__global__ void k_sub_cols(int64_t n, int q, const double* __restrict__ X, int64_t ldx,
                           double* __restrict__ Y, int64_t ldy) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n * q) return;
  const int64_t r = i / q, c = i % q;
  Y[r * ldy + c] -= X[r * ldx + c];
}
// Y[:, c] = X[:, perm[c]] for c < q (column permutation of a row-major block).
__global__ void k_permute_cols(int64_t n, int q, const double* __restrict__ X, int64_t ld,
                               const int* __restrict__ perm, double* __restrict__ Y) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n * q) return;
  const int64_t r = i / q, c = i % q;
  Y[r * ld + c] = X[r * ld + perm[c]];
}
template <typename T>
__global__ void k_zero(T* p, int64_t count) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = T(0);
}
__global__ void k_scale(int64_t count, double a, double* p) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] *= a;
}

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as
// easy as 1, 2, 3", SC 2011): 10 rounds of the Philox S-box on a 128-bit
// counter with a 64-bit key bumped by the Weyl constants.
__device__ __forceinline__ void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u, W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = (uint64_t)M0 * c[0];
    const uint64_t p1 = (uint64_t)M1 * c[2];
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    const uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
    k0 += W0;
    k1 += W1;
  }
}

__global__ void k_gauss(int64_t n, int q, double* __restrict__ X, int64_t ld, uint64_t seed) {
  const int64_t pair = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t total = n * q;
  if (2 * pair >= total) return;
  uint32_t c[4] = {(uint32_t)pair, (uint32_t)((uint64_t)pair >> 32), 0u, 0u};
  philox4x32_10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
  const double two53 = 1.0 / 9007199254740992.0;
  const uint64_t a = (((uint64_t)c[0] << 32) | c[1]) >> 11;
  const uint64_t b = (((uint64_t)c[2] << 32) | c[3]) >> 11;
  const double u1 = ((double)a + 0.5) * two53, u2 = ((double)b + 0.5) * two53;
  const double rad = sqrt(-2.0 * log(u1));
  const double ang = 6.283185307179586 * u2;
  const double z[2] = {rad * cos(ang), rad * sin(ang)};
  for (int t = 0; t < 2; ++t) {
    const int64_t e = 2 * pair + t;
    if (e < total) X[(e / q) * ld + (e % q)] = z[t];
  }
}

// sign fix: partial argmax of |X[:, sel[s]]| per block, then per column
__global__ __launch_bounds__(256) void k_absmax_partial(int64_t n, const double* __restrict__ X,
                                                        int64_t ld, const int* __restrict__ sel,
                                                        double* __restrict__ pval,
                                                        int64_t* __restrict__ pidx) {
  __shared__ double sv[256];
  __shared__ int64_t si[256];
  const int s = blockIdx.y;
  const int col = sel[s];
  const int64_t chunk = (n + gridDim.x - 1) / gridDim.x;
  const int64_t r0 = (int64_t)blockIdx.x * chunk;
  int64_t r1 = r0 + chunk;
  if (r1 > n) r1 = n;
  double bv = -1.0;
  int64_t bi = -1;
  for (int64_t r = r0 + threadIdx.x; r < r1; r += 256) {
    const double v = fabs(X[r * ld + col]);
    if (v > bv) {
      bv = v;
      bi = r;
    }
  }
  sv[threadIdx.x] = bv;
  si[threadIdx.x] = bi;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (threadIdx.x < st) {
      const double ov = sv[threadIdx.x + st];
      const int64_t oi = si[threadIdx.x + st];
      if (ov > sv[threadIdx.x] || (ov == sv[threadIdx.x] && oi >= 0 && (si[threadIdx.x] < 0 || oi < si[threadIdx.x]))) {
        sv[threadIdx.x] = ov;
        si[threadIdx.x] = oi;
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    pval[(int64_t)s * gridDim.x + blockIdx.x] = sv[0];
    pidx[(int64_t)s * gridDim.x + blockIdx.x] = si[0];
  }
}

__global__ void k_sign_final(int nsel, int nblk, const double* __restrict__ X, int64_t ld,
                             const int* __restrict__ sel, const double* __restrict__ pval,
                             const int64_t* __restrict__ pidx, double* __restrict__ sign) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nsel) return;
  double bv = -1.0;
  int64_t bi = -1;
  for (int b = 0; b < nblk; ++b) {
    const double v = pval[(int64_t)s * nblk + b];
    const int64_t i = pidx[(int64_t)s * nblk + b];
    if (i >= 0 && (v > bv || (v == bv && i < bi))) {
      bv = v;
      bi = i;
    }
  }
  sign[s] = (bi >= 0 && X[bi * ld + sel[s]] < 0.0) ? -1.0 : 1.0;
}

__global__ void k_gather_t(int64_t n, int nsel, const double* __restrict__ X, int64_t ld,
                           const int* __restrict__ sel, const double* __restrict__ sign,
                           double* __restrict__ out) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int s = blockIdx.y;
  if (r >= n) return;
  out[(int64_t)s * n + r] = X[r * ld + sel[s]] * sign[s];
}

__global__ void k_transpose_rows(int64_t m, int64_t n, const double* __restrict__ in,
                                 double* __restrict__ out, int64_t ld) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t c = blockIdx.y;
  if (r >= n) return;
  out[r * ld + c] = in[c * n + r];
}

// ------------------------------------------------------------- Lanczos
constexpr int kDotBlocks = 256;
__global__ __launch_bounds__(256) void k_multidot_partial(int64_t n, int m,
                                                          const double* __restrict__ V,
                                                          const double* __restrict__ w,
                                                          double* __restrict__ part) {
  __shared__ double red[256];
  const int64_t chunk = (n + gridDim.x - 1) / gridDim.x;
  const int64_t r0 = (int64_t)blockIdx.x * chunk;
  int64_t r1 = r0 + chunk;
  if (r1 > n) r1 = n;
  for (int j = 0; j < m; ++j) {
    double s = 0.0;
    for (int64_t r = r0 + threadIdx.x; r < r1; r += 256) s += V[(int64_t)j * n + r] * w[r];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
      if (threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
      __syncthreads();
    }
    if (threadIdx.x == 0) part[(int64_t)blockIdx.x * m + j] = red[0];
    __syncthreads();
  }
}
__global__ void k_multidot_final(int nblk, int m, const double* __restrict__ part,
                                 double* __restrict__ h) {
  const int j = threadIdx.x;
  if (j >= m) return;
  double s = 0.0;
  for (int b = 0; b < nblk; ++b) s += part[(int64_t)b * m + j];
  h[j] = s;
}
__global__ void k_multi_axpy(int64_t n, int m, const double* __restrict__ V,
                             const double* __restrict__ h, double* __restrict__ w) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  double s = w[r];
  for (int j = 0; j < m; ++j) s -= h[j] * V[(int64_t)j * n + r];
  w[r] = s;
}
__global__ void k_axpby(int64_t n, double a, const double* __restrict__ x, double b,
                        double* __restrict__ y) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r < n) y[r] = a * x[r] + b * y[r];
}
__global__ void k_scale_by_inv(int64_t n, const double* __restrict__ x,
                               const double* __restrict__ nrm, double* __restrict__ y) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r < n) y[r] = x[r] / nrm[0];
}

}  // namespace

// ================================================================ launchers
size_t gram_work_bytes(int64_t n, int q1, int q2) {
  int ns = gram_splits(n, q1, q2);
  // the tiled Gram takes at most 256 splits (two or more tiles); callers size
  // the workspace for their widest product, and a narrower one of the same
  // call site may use more splits than that product's own count
  if (std::max(q1, q2) > 128) ns = std::max(ns, 256);
  return (size_t)ns * q1 * q2 * sizeof(double);
}

hipError_t gram_f64(int64_t n, int q1, int q2, const double* A, int64_t lda, const double* B,
                    int64_t ldb, double* G, void* work, hipStream_t s) {
  if (q1 == 0 || q2 == 0) return hipSuccess;
  if (gram_rt_applies(q1, q2)) {
    const bool sym = A == B && lda == ldb && q1 == q2;
    const int ntiles = gram_rt_tiles(q1, q2, sym);
    const int tiles_n = (q2 + kGramRtTile - 1) / kGramRtTile;
    const int nsplit = gram_rt_splits(n, ntiles);
    int64_t rows = (n + nsplit - 1) / nsplit;
    rows = ((rows + kGramRtRows - 1) / kGramRtRows) * kGramRtRows;
    const int rounds = (nsplit + 7) / 8;
    double* w = static_cast<double*>(work);
    hipLaunchKernelGGL(k_gram_rt, dim3((unsigned)(rounds * 8 * ntiles)), dim3(256), 0, s, n, q1,
                       q2, A, lda, B, ldb, rows, nsplit, tiles_n, ntiles, sym ? 1 : 0, w);
    const int64_t count = (int64_t)q1 * q2;
    hipLaunchKernelGGL(k_gram_reduce, dim3(nblocks(count, 16)), dim3(256), 0, s, nsplit, count, w,
                       G);
    return hipGetLastError();
  }
  const int nsplit = gram_splits(n, q1, q2);
  int64_t rows = (n + nsplit - 1) / nsplit;
  rows = ((rows + kGramSmallRows - 1) / kGramSmallRows) * kGramSmallRows;
  double* w = static_cast<double*>(work);
  if (q1 <= kGramSmallMax && q2 <= kGramSmallMax) {
    const int mt = (q1 + 31) / 32, nt = (q2 + 31) / 32;
#define PFE_GRAM_CASE(M_, N_)                                                                  \
    if (mt == M_ && nt == N_)                                                                  \
      hipLaunchKernelGGL((k_gram_small<M_, N_>), dim3(nsplit), dim3(256), 0, s, n, q1, q2, A,   \
                         lda, B, ldb, rows, w);
    PFE_GRAM_CASE(1, 1) PFE_GRAM_CASE(1, 2) PFE_GRAM_CASE(1, 3) PFE_GRAM_CASE(1, 4)
    PFE_GRAM_CASE(2, 1) PFE_GRAM_CASE(2, 2) PFE_GRAM_CASE(2, 3) PFE_GRAM_CASE(2, 4)
    PFE_GRAM_CASE(3, 1) PFE_GRAM_CASE(3, 2) PFE_GRAM_CASE(3, 3) PFE_GRAM_CASE(3, 4)
    PFE_GRAM_CASE(4, 1) PFE_GRAM_CASE(4, 2) PFE_GRAM_CASE(4, 3) PFE_GRAM_CASE(4, 4)
#undef PFE_GRAM_CASE
  } else {
    const int tiles = ((q1 + 63) / 64) * ((q2 + 63) / 64);
    hipLaunchKernelGGL(k_gram_partial, dim3(nsplit, tiles), dim3(256), 0, s, n, q1, q2, A, lda,
                       B, ldb, rows, w);
  }
  const int64_t count = (int64_t)q1 * q2;
  hipLaunchKernelGGL(k_gram_reduce, dim3(nblocks(count, 16)), dim3(256), 0, s, nsplit, count, w,
                     G);
  return hipGetLastError();
}

hipError_t gemm_tall_f64(int64_t n, int q1, int q2, const double* A, int64_t lda,
                         const double* Bm, double* C, int64_t ldc, hipStream_t s) {
  if (n == 0 || q2 == 0) return hipSuccess;
  if (q1 <= 128 && q2 <= 128) {
    const int km = (q1 + 31) / 32, nt = (q2 + 15) / 16;
    const int64_t tiles = (n + 15) / 16;
    // two work-groups per CU when Bm fits twice in the 160 KB of LDS
    const int per_cu = (km * 32 * (16 * nt + 1) * 8 <= 80 * 1024) ? 2 : 1;
    const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>((tiles + 3) / 4, 256 * per_cu));
#define PFE_GEMM_CASE(K_, N_)                                                                \
    if (km == K_ && nt == N_) {                                                              \
      hipLaunchKernelGGL((k_gemm_bres<32 * K_, N_>), dim3(grid), dim3(256), 0, s, n, q1, q2, \
                         A, lda, Bm, C, ldc);                                                \
      return hipGetLastError();                                                              \
    }
#define PFE_GEMM_ROW(K_) PFE_GEMM_CASE(K_, 1) PFE_GEMM_CASE(K_, 2) PFE_GEMM_CASE(K_, 3) \
    PFE_GEMM_CASE(K_, 4) PFE_GEMM_CASE(K_, 5) PFE_GEMM_CASE(K_, 6) PFE_GEMM_CASE(K_, 7) PFE_GEMM_CASE(K_, 8)
    PFE_GEMM_ROW(1) PFE_GEMM_ROW(2) PFE_GEMM_ROW(3) PFE_GEMM_ROW(4)
#undef PFE_GEMM_ROW
#undef PFE_GEMM_CASE
  }
  if (q1 <= kGemmRtCols && q2 <= kGemmRtCols) {
    hipLaunchKernelGGL(k_gemm_rt, dim3(nblocks(n, kGemmRtRows)), dim3(256), 0, s, n, q1, q2, A,
                       lda, Bm, C, ldc);
    return hipGetLastError();
  }
  const int q1p = ((q1 + 3) / 4) * 4 + 1;
  if ((size_t)32 * q1p * sizeof(double) <= 65536) {
    hipLaunchKernelGGL(k_gemm_tall<32>, dim3(nblocks(n, 32)), dim3(256),
                       (size_t)32 * q1p * sizeof(double), s, n, q1, q2, A, lda, Bm, C, ldc);
  } else if ((size_t)16 * q1p * sizeof(double) <= 65536) {
    hipLaunchKernelGGL(k_gemm_tall<16>, dim3(nblocks(n, 16)), dim3(256),
                       (size_t)16 * q1p * sizeof(double), s, n, q1, q2, A, lda, Bm, C, ldc);
  } else {
    return hipErrorInvalidValue;   // q1 > 511
  }
  return hipGetLastError();
}

hipError_t chol_inv_f64(int q, const double* G, double shift, double* Rinv, int* info,
                        double* diag_max, hipStream_t s) {
  // Rinv doubles as R during the factorisation; the inverse is built in the
  // second half of the same allocation (caller provides 2 q^2 doubles).
  if (q <= kCholLdsMax) {
    hipLaunchKernelGGL(k_chol_inv_lds, dim3(1), dim3(1024), 0, s, q, G, shift, Rinv, info,
                       diag_max);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_chol_inv, dim3(1), dim3(1024), 0, s, q, G, shift, Rinv, Rinv + (int64_t)q * q,
                     info, diag_max);
  return hipGetLastError();
}

size_t jacobi_work_bytes(int q) {
  return ((size_t)3 * q * q + 16) * sizeof(double) + kJacobiMaxSweeps * sizeof(int);
}

hipError_t sym_eig_f64(int q, const double* S, double* evals, double* Q, void* work, int* info,
                       hipStream_t s) {
  if (q > 1024) return hipErrorInvalidValue;
  if (q <= kJacobiLdsMax) {
    hipLaunchKernelGGL(k_jacobi_lds, dim3(1), dim3(1024), 0, s, q, S, evals, Q, info);
    return hipGetLastError();
  }
  double* A = static_cast<double*>(work);
  double* V = A + (int64_t)q * q;
  if (q <= kJacobiOneGroupMax) {
    hipLaunchKernelGGL(k_jacobi, dim3(1), dim3(1024), 0, s, q, S, A, V, evals, Q, info);
    return hipGetLastError();
  }
  const int m = q + (q & 1), half = m / 2;
  double* A1 = V + (int64_t)q * q;
  double* floor_abs = A1 + (int64_t)q * q;
  int* flags = reinterpret_cast<int*>(floor_abs + 2);
  hipLaunchKernelGGL(k_jac_init, dim3(1), dim3(1024), 0, s, q, S, A, V, floor_abs, flags);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const unsigned bt = (unsigned)std::min(512, ((half + 63) / 64) * 64);
  double* Ab[2] = {A, A1};
  int cur = 0;
  int sweep = 0;
  bool converged = false;
  for (; sweep < kJacobiMaxSweeps && !converged; ++sweep) {
    for (int step = 0; step < m - 1; ++step) {
      hipLaunchKernelGGL(k_jac_step, dim3((unsigned)half), dim3(bt), 0, s, q, step, Ab[cur],
                         Ab[cur ^ 1], V, floor_abs, flags + sweep);
      cur ^= 1;
    }
    if ((e = hipGetLastError()) != hipSuccess) return e;
    int rot = 0;
    if ((e = hipMemcpyAsync(&rot, flags + sweep, sizeof(int), hipMemcpyDeviceToHost, s)) != hipSuccess)
      return e;
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
    converged = rot == 0;
  }
  A = Ab[cur];
  hipLaunchKernelGGL(k_jac_final, dim3(1), dim3(1024), 0, s, q, A, V, evals, Q, info,
                     converged ? sweep : -sweep);
  return hipGetLastError();
}

size_t colnorm_work_bytes(int64_t n, int q) {
  return (size_t)std::max(1u, nblocks(n, kColRows)) * q * sizeof(double);
}

hipError_t resid_norms_f64(int64_t n, int q, const double* W, const double* X, int64_t ld,
                           const double* theta, double inv_scale, double* res, void* work,
                           hipStream_t s) {
  const unsigned nb = std::max(1u, nblocks(n, kColRows));   // n = 0: one zero partial
  double* part = static_cast<double*>(work);
  if (q == 0) return hipSuccess;
  hipLaunchKernelGGL(k_col_partial<0>, dim3(nb), dim3(256), 0, s, n, q, W, X, ld, theta, part);
  hipLaunchKernelGGL(k_col_final<true>, dim3(nblocks(q, 16)), dim3(256), 0, s, (int)nb, q, part,
                     inv_scale, res);
  return hipGetLastError();
}

hipError_t col_norms_f64(int64_t n, int q, const double* X, int64_t ld, double* res, void* work,
                         hipStream_t s) {
  return resid_norms_f64(n, q, X, nullptr, ld, nullptr, 1.0, res, work, s);
}

hipError_t col_dots_f64(int64_t n, int q, const double* X, const double* Y, int64_t ld,
                        double* res, void* work, hipStream_t s) {
  const unsigned nb = std::max(1u, nblocks(n, kColRows));   // n = 0: one zero partial
  double* part = static_cast<double*>(work);
  if (q == 0) return hipSuccess;
  hipLaunchKernelGGL(k_col_partial<1>, dim3(nb), dim3(256), 0, s, n, q, X, Y, ld, nullptr, part);
  hipLaunchKernelGGL(k_col_final<false>, dim3(nblocks(q, 16)), dim3(256), 0, s, (int)nb, q, part,
                     1.0, res);
  return hipGetLastError();
}
hipError_t col_scale_inv_f64(int64_t n, int q, double* X, int64_t ld, const double* nrm,
                             hipStream_t s) {
  if (n * q == 0) return hipSuccess;
  hipLaunchKernelGGL(k_col_scale_inv, dim3(nblocks(n * q, 256)), dim3(256), 0, s, n, q, X, ld,
                     nrm);
  return hipGetLastError();
}
hipError_t cast_f64_to_f32(int64_t n, int q, const double* X, int64_t ldx, float* Y, int64_t ldy,
                           hipStream_t s) {
  if (n * q == 0) return hipSuccess;
  hipLaunchKernelGGL(k_cast_d2f, dim3(nblocks(n * q, 256)), dim3(256), 0, s, n, q, X, ldx, Y, ldy);
  return hipGetLastError();
}
hipError_t cast_f32_to_f64(int64_t n, int q, const float* X, int64_t ldx, double* Y, int64_t ldy,
                           hipStream_t s) {
  if (n * q == 0) return hipSuccess;
  hipLaunchKernelGGL(k_cast_f2d, dim3(nblocks(n * q, 256)), dim3(256), 0, s, n, q, X, ldx, Y, ldy);
  return hipGetLastError();
}
hipError_t copy_cols_f64(int64_t n, int q, const double* X, int64_t ldx, double* Y, int64_t ldy,
                         hipStream_t s) {
  if (n * q == 0) return hipSuccess;
  hipLaunchKernelGGL(k_copy_cols, dim3(nblocks(n * q, 256)), dim3(256), 0, s, n, q, X, ldx, Y, ldy);
  return hipGetLastError();
}
hipError_t sub_cols_f64(int64_t n, int q, const double* X, int64_t ldx, double* Y, int64_t ldy,
                        hipStream_t s) {
  if (n * q == 0) return hipSuccess;
  hipLaunchKernelGGL(k_sub_cols, dim3(nblocks(n * q, 256)), dim3(256), 0, s, n, q, X, ldx, Y, ldy);
  return hipGetLastError();
}
hipError_t permute_cols_f64(int64_t n, int q, const double* X, int64_t ld, const int* perm,
                            double* Y, hipStream_t s) {
  if (n * q == 0) return hipSuccess;
  hipLaunchKernelGGL(k_permute_cols, dim3(nblocks(n * q, 256)), dim3(256), 0, s, n, q, X, ld, perm, Y);
  return hipGetLastError();
}
hipError_t zero_f64(double* p, int64_t count, hipStream_t s) {
  if (count == 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero<double>, dim3(nblocks(count, 256)), dim3(256), 0, s, p, count);
  return hipGetLastError();
}
hipError_t zero_f32(float* p, int64_t count, hipStream_t s) {
  if (count == 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero<float>, dim3(nblocks(count, 256)), dim3(256), 0, s, p, count);
  return hipGetLastError();
}
hipError_t scale_f64(int64_t count, double a, double* p, hipStream_t s) {
  if (count == 0) return hipSuccess;
  hipLaunchKernelGGL(k_scale, dim3(nblocks(count, 256)), dim3(256), 0, s, count, a, p);
  return hipGetLastError();
}
hipError_t gaussian_fill_f64(int64_t n, int q, double* X, int64_t ld, uint64_t seed, hipStream_t s) {
  const int64_t pairs = (n * q + 1) / 2;
  if (pairs == 0) return hipSuccess;
  hipLaunchKernelGGL(k_gauss, dim3(nblocks(pairs, 256)), dim3(256), 0, s, n, q, X, ld, seed);
  return hipGetLastError();
}

hipError_t gather_transpose_signfix(int64_t n, int nsel, const double* X, int64_t ld,
                                    const int* sel, double* out, void* work, hipStream_t s) {
  if (nsel == 0 || n == 0) return hipSuccess;
  const int nblk = 64;
  double* pval = static_cast<double*>(work);
  int64_t* pidx = reinterpret_cast<int64_t*>(pval + (int64_t)nsel * nblk);
  double* sign = reinterpret_cast<double*>(pidx + (int64_t)nsel * nblk);
  hipLaunchKernelGGL(k_absmax_partial, dim3(nblk, nsel), dim3(256), 0, s, n, X, ld, sel, pval,
                     pidx);
  hipLaunchKernelGGL(k_sign_final, dim3(nblocks(nsel, 64)), dim3(64), 0, s, nsel, nblk, X, ld, sel,
                     pval, pidx, sign);
  hipLaunchKernelGGL(k_gather_t, dim3(nblocks(n, 256), nsel), dim3(256), 0, s, n, nsel, X, ld, sel,
                     sign, out);
  return hipGetLastError();
}

hipError_t transpose_to_rows(int64_t m, int64_t n, const double* in, double* out, int64_t ld,
                             hipStream_t s) {
  if (m == 0 || n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_transpose_rows, dim3(nblocks(n, 256), (unsigned)m), dim3(256), 0, s, m, n,
                     in, out, ld);
  return hipGetLastError();
}

size_t multidot_work_bytes(int64_t n, int m) { return (size_t)kDotBlocks * m * sizeof(double); }

hipError_t multi_dot_f64(int64_t n, int m, const double* V, const double* w, double* h,
                         void* work, hipStream_t s) {
  if (m == 0) return hipSuccess;
  double* part = static_cast<double*>(work);
  hipLaunchKernelGGL(k_multidot_partial, dim3(kDotBlocks), dim3(256), 0, s, n, m, V, w, part);
  hipLaunchKernelGGL(k_multidot_final, dim3(1), dim3(1024), 0, s, kDotBlocks, m, part, h);
  return hipGetLastError();
}
hipError_t multi_axpy_f64(int64_t n, int m, const double* V, const double* h, double* w,
                          hipStream_t s) {
  if (m == 0 || n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_multi_axpy, dim3(nblocks(n, 256)), dim3(256), 0, s, n, m, V, h, w);
  return hipGetLastError();
}
hipError_t axpby_f64(int64_t n, double a, const double* x, double b, double* y, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_axpby, dim3(nblocks(n, 256)), dim3(256), 0, s, n, a, x, b, y);
  return hipGetLastError();
}
hipError_t scale_by_inv_f64(int64_t n, const double* x, const double* nrm, double* y,
                            hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_scale_by_inv, dim3(nblocks(n, 256)), dim3(256), 0, s, n, x, nrm, y);
  return hipGetLastError();
}

}  // namespace pfe
