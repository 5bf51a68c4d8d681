// Reverse mode of the Chebyshev filter (no counterpart in the paper; it is
// the chain rule applied to Algorithm 2) and the gradient kernels.
//
// The reverse recurrence itself runs on the fused filter step (H_hat is
// symmetric).  The block gradient G_b = sum_k w_k a_{k+1}[i] t_k[j]^T over
// the stored blocks b = (i, j) is an SDDMM: one wavefront per atom row i, the
// three rows of the wave's own atom against the three rows of each
// neighbour, a 3x3 matrix of dot products over the q columns reduced across
// the wave.  Every block is written only by the wave of its row, so the
// accumulation needs no atomics and is deterministic.
#include <algorithm>
#include <cstdlib>

#include "internal.h"

namespace pfe {
namespace {

__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// G[b] (+)= sum_c w_c a[3i+p][c] t[3j+q][c] for stored b = (i, j): rows of a
// are the wave's own, rows of t are gathered.
template <int NP>
__global__ __launch_bounds__(256) void k_sddmm(int n_atoms, const int64_t* __restrict__ row_ptr,
                                               const int32_t* __restrict__ col_idx, int q,
                                               const double* __restrict__ a,
                                               const double* __restrict__ t, int64_t ld,
                                               const double* __restrict__ colw, double* G,
                                               int accumulate) {
  const int wave = uniform(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int row = uniform(blockIdx.x * 4 + wave);
  if (row >= n_atoms) return;
  double ar[3][NP];
  bool act[NP];
#pragma unroll
  for (int p = 0; p < NP; ++p) {
    const int c = lane + 64 * p;
    act[p] = c < q;
    const double w = (act[p] && colw) ? colw[c] : 1.0;
    for (int r = 0; r < 3; ++r) ar[r][p] = act[p] ? w * a[(int64_t)(3 * row + r) * ld + c] : 0.0;
  }
  for (int64_t k = row_ptr[row]; k < row_ptr[row + 1]; ++k) {
    const int j = col_idx[k];
    double x[3][NP];
#pragma unroll
    for (int p = 0; p < NP; ++p)
      for (int r = 0; r < 3; ++r)
        x[r][p] = act[p] ? t[(int64_t)(3 * j + r) * ld + lane + 64 * p] : 0.0;
    double g[9];
#pragma unroll
    for (int pa = 0; pa < 3; ++pa)
#pragma unroll
      for (int qb = 0; qb < 3; ++qb) {
        double s = 0.0;
#pragma unroll
        for (int p = 0; p < NP; ++p) s += ar[pa][p] * x[qb][p];
        g[pa * 3 + qb] = wave_sum(s);
      }
    if (lane < 9) {
      double v = 0.0;
#pragma unroll
      for (int s = 0; s < 9; ++s)
        if (lane == s) v = g[s];
      if (accumulate)
        G[k * 9 + lane] += v;
      else
        G[k * 9 + lane] = v;
    }
  }
}

// Block gradient of a whole checkpoint segment in one pass:
//   G[b] (+)= sum_m w_m sum_c a_m[3i+p][c] t_m[3j+q][c]   for stored b = (i, j),
// with a_m = A + m * a_stride (rows of the wave's own atom i) and
// t_m = T + m * t_stride (rows of the neighbour j).  Every lane keeps its
// nine partial sums over all m pairs, so each block is reduced across the
// wave once per segment instead of once per recurrence step.
template <int NP>
__global__ __launch_bounds__(256) void k_sddmm_seg(int n_atoms, const int64_t* __restrict__ row_ptr,
                                                   const int32_t* __restrict__ col_idx, int q, int m,
                                                   const double* __restrict__ A, int64_t a_stride,
                                                   const double* __restrict__ T, int64_t t_stride,
                                                   int64_t ld, const double* __restrict__ w,
                                                   double* G) {
  const int wave = uniform(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int row = uniform(blockIdx.x * 4 + wave);
  if (row >= n_atoms) return;
  bool act[NP];
#pragma unroll
  for (int p = 0; p < NP; ++p) act[p] = lane + 64 * p < q;
  for (int64_t k = row_ptr[row]; k < row_ptr[row + 1]; ++k) {
    const int j = col_idx[k];
    double g[9];
#pragma unroll
    for (int e = 0; e < 9; ++e) g[e] = 0.0;
    // several pairs' loads in flight at once (the pair loop is latency-bound)
#pragma unroll 4
    for (int mm = 0; mm < m; ++mm) {
      const double wm = w[mm];
      const double* am = A + mm * a_stride;
      const double* tm = T + mm * t_stride;
#pragma unroll
      for (int p = 0; p < NP; ++p) {
        if (!act[p]) continue;
        const int c = lane + 64 * p;
        double ar[3], tr[3];
#pragma unroll
        for (int r = 0; r < 3; ++r) {
          ar[r] = wm * am[(int64_t)(3 * row + r) * ld + c];
          tr[r] = tm[(int64_t)(3 * j + r) * ld + c];
        }
#pragma unroll
        for (int pa = 0; pa < 3; ++pa)
#pragma unroll
          for (int qb = 0; qb < 3; ++qb) g[pa * 3 + qb] += ar[pa] * tr[qb];
      }
    }
    double v = 0.0;
#pragma unroll
    for (int e = 0; e < 9; ++e) {
      const double tot = wave_sum(g[e]);
      if (lane == e) v = tot;
    }
    if (lane < 9) G[k * 9 + lane] += v;
  }
}

// q <= 64 and m <= MM: the wave's own three rows of every a_m (with w_m
// folded in) stay in registers across the row's blocks, so a block loads
// only its neighbour's rows; same products and order as k_sddmm_seg.
//
// Work-groups are dealt to the XCDs in chunks of `chunk` (work-group b runs on
// XCD b % 8; chunk c of consecutive rows goes to XCD c % 8), as in the fused
// filter step: with eight chunks spanning the pattern's typical neighbour
// offset, a row and its neighbours one lattice plane away share an L2, so
// their gathered rows of T are fetched from memory once per XCD.
__device__ __forceinline__ int xcd_chunk_row_group(int b, int chunk) {
  const int xcd = b & 7, s = b >> 3;
  return ((s / chunk) * 8 + xcd) * chunk + (s % chunk);
}

template <int MM>
__global__ __launch_bounds__(256) void k_sddmm_seg_reg(int n_atoms, const int64_t* __restrict__ row_ptr,
                                                       const int32_t* __restrict__ col_idx, int q,
                                                       int m, const double* __restrict__ A,
                                                       int64_t a_stride,
                                                       const double* __restrict__ T,
                                                       int64_t t_stride, int64_t ld,
                                                       const double* __restrict__ w, double* G,
                                                       int chunk) {
  const int wave = uniform(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int row = uniform(xcd_chunk_row_group(blockIdx.x, chunk) * 4 + wave);
  if (row >= n_atoms) return;
  const bool act = lane < q;
  const int c = act ? lane : 0;
  double ar[MM][3];
#pragma unroll
  for (int mm = 0; mm < MM; ++mm) {
    const double wm = (mm < m) ? w[mm] : 0.0;
#pragma unroll
    for (int r = 0; r < 3; ++r)
      ar[mm][r] = (mm < m && act) ? wm * A[mm * a_stride + (int64_t)(3 * row + r) * ld + c] : 0.0;
  }
  // Software-pipelined over the row's blocks: the next block's rows of t_m
  // and its current value in G are requested before this block's sums are
  // reduced and stored, so the reductions overlap those loads and a store
  // is never older than the loads the next wait is for.
  const int64_t k0 = row_ptr[row], k1 = row_ptr[row + 1];
  double tr[MM][3];
  double gnext = 0.0;
  auto fetch = [&](int64_t kk) {
    const int j = col_idx[kk];
#pragma unroll
    for (int mm = 0; mm < MM; ++mm) {
      const double* tm = T + mm * t_stride + (int64_t)(3 * j) * ld + c;
#pragma unroll
      for (int r = 0; r < 3; ++r) tr[mm][r] = (mm < m && act) ? tm[(int64_t)r * ld] : 0.0;
    }
    gnext = lane < 9 ? G[kk * 9 + lane] : 0.0;
  };
  if (k0 < k1) fetch(k0);
  for (int64_t k = k0; k < k1; ++k) {
    double g[9];
#pragma unroll
    for (int e = 0; e < 9; ++e) g[e] = 0.0;
#pragma unroll
    for (int mm = 0; mm < MM; ++mm) {
      if (mm < m) {
#pragma unroll
        for (int pa = 0; pa < 3; ++pa)
#pragma unroll
          for (int qb = 0; qb < 3; ++qb) g[pa * 3 + qb] += ar[mm][pa] * tr[mm][qb];
      }
    }
    const double gk = gnext;
    if (k + 1 < k1) fetch(k + 1);
    __builtin_amdgcn_sched_barrier(0);   // the next block's loads go out before the reductions
    double v = 0.0;
#pragma unroll
    for (int e = 0; e < 9; ++e) {
      const double tot = wave_sum(g[e]);
      if (lane == e) v = tot;
    }
    if (lane < 9) G[k * 9 + lane] = gk + v;
  }
}

__device__ int64_t find_block(const int64_t* row_ptr, const int32_t* col_idx, int i, int j) {
  int64_t lo = row_ptr[i], hi = row_ptr[i + 1] - 1;
  while (lo <= hi) {
    const int64_t mid = (lo + hi) >> 1;
    const int c = col_idx[mid];
    if (c == j) return mid;
    if (c < j)
      lo = mid + 1;
    else
      hi = mid - 1;
  }
  return -1;
}

__global__ void k_spring_dk(int64_t P, int n_atoms, const int64_t* __restrict__ row_ptr,
                            const int32_t* __restrict__ col_idx, const double* __restrict__ m,
                            const double* __restrict__ G, const int64_t* __restrict__ pairs,
                            const double* __restrict__ unit, double* __restrict__ dk, int* err) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= P) return;
  const int64_t pi = pairs[2 * p], pj = pairs[2 * p + 1];
  if (pi < 0 || pi >= n_atoms || pj < 0 || pj >= n_atoms || pi == pj) {
    atomicOr(err, 2);
    dk[p] = 0.0;
    return;
  }
  const int i = (int)pi, j = (int)pj;
  const int64_t bii = find_block(row_ptr, col_idx, i, i);
  const int64_t bjj = find_block(row_ptr, col_idx, j, j);
  const int64_t bij = find_block(row_ptr, col_idx, i, j);
  const int64_t bji = find_block(row_ptr, col_idx, j, i);
  if (bii < 0 || bjj < 0 || bij < 0 || bji < 0) {
    atomicOr(err, 1);
    dk[p] = 0.0;
    return;
  }
  const double u[3] = {unit[3 * p], unit[3 * p + 1], unit[3 * p + 2]};
  const double wi = 1.0 / m[i], wj = 1.0 / m[j], wij = 1.0 / sqrt(m[i] * m[j]);
  double s = 0.0;
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) {
      const int e = a * 3 + b;
      s += u[a] * u[b] *
           (G[bii * 9 + e] * wi + G[bjj * 9 + e] * wj - (G[bij * 9 + e] + G[bji * 9 + e]) * wij);
    }
  dk[p] = s;
}

__global__ void k_spring_dm(int n_atoms, const int64_t* __restrict__ row_ptr,
                            const int32_t* __restrict__ transpose, const double* __restrict__ H,
                            const double* __restrict__ m, const double* __restrict__ G,
                            double* __restrict__ dm) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_atoms) return;
  double s = 0.0;
  for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) {
    const int64_t t = transpose[k];
    for (int e = 0; e < 9; ++e) s += G[k * 9 + e] * H[k * 9 + e] + G[t * 9 + e] * H[t * 9 + e];
  }
  dm[i] = -0.5 * s / m[i];
}

// Spring list checks: 0 <= i < j < n_atoms and strictly increasing (i, j)
// order, so the assembly can binary-search it.  err bit 5.
__global__ void k_check_pairs(int64_t P, int n_atoms, const int64_t* __restrict__ pairs, int* err) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= P) return;
  const int64_t i = pairs[2 * p], j = pairs[2 * p + 1];
  bool bad = i < 0 || j >= n_atoms || i >= j;
  if (p + 1 < P) {
    const int64_t i2 = pairs[2 * p + 2], j2 = pairs[2 * p + 3];
    bad = bad || !(i < i2 || (i == i2 && j < j2));
  }
  if (bad) atomicOr(err, 32);
}

__device__ int64_t find_pair(const int64_t* pairs, int64_t P, int64_t i, int64_t j) {
  int64_t lo = 0, hi = P - 1;
  while (lo <= hi) {
    const int64_t mid = (lo + hi) >> 1;
    const int64_t pi = pairs[2 * mid], pj = pairs[2 * mid + 1];
    if (pi == i && pj == j) return mid;
    if (pi < i || (pi == i && pj < j))
      lo = mid + 1;
    else
      hi = mid - 1;
  }
  return -1;
}

// K of a harmonic spring network on a given BSR pattern, one thread per block
// row: K_ij = -k_p u_p u_p^T for the spring p joining i and j, and
// K_ii = -sum_{j != i} K_ij.  err bit 6: an off-diagonal block has no spring;
// bit 0: the row has no diagonal block.
__global__ void k_assemble_springs(int n_atoms, const int64_t* __restrict__ row_ptr,
                                   const int32_t* __restrict__ col_idx, int64_t P,
                                   const int64_t* __restrict__ pairs,
                                   const double* __restrict__ unit, const double* __restrict__ kv,
                                   double* __restrict__ K, int* err) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_atoms) return;
  double dg[9];
  for (int e = 0; e < 9; ++e) dg[e] = 0.0;
  int64_t bd = -1;
  for (int64_t b = row_ptr[i]; b < row_ptr[i + 1]; ++b) {
    const int j = col_idx[b];
    if (j == i) {
      bd = b;
      continue;
    }
    const int64_t p = find_pair(pairs, P, i < j ? i : j, i < j ? j : i);
    if (p < 0) {
      atomicOr(err, 64);
      for (int e = 0; e < 9; ++e) K[b * 9 + e] = 0.0;
      continue;
    }
    const double u[3] = {unit[3 * p], unit[3 * p + 1], unit[3 * p + 2]};
    const double kp = kv[p];
    for (int a = 0; a < 3; ++a)
      for (int c = 0; c < 3; ++c) {
        // u_a u_c first: the product commutes exactly, so K_ji = K_ij^T bit for bit
        const double v = -kp * (u[a] * u[c]);
        K[b * 9 + 3 * a + c] = v;
        dg[3 * a + c] -= v;
      }
  }
  if (bd < 0) {
    atomicOr(err, 1);
    return;
  }
  for (int e = 0; e < 9; ++e) K[bd * 9 + e] = dg[e];
}

inline unsigned nb(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

}  // namespace

hipError_t sddmm_f64(const Bsr& A, int q, const double* a, const double* t, int64_t ld,
                     const double* colw, double* G, bool accumulate, hipStream_t s) {
  if (A.n_atoms == 0) return hipSuccess;
  const unsigned grid = nb(A.n_atoms, 4);
  if (q <= 64)
    hipLaunchKernelGGL(k_sddmm<1>, dim3(grid), dim3(256), 0, s, (int)A.n_atoms, A.row_ptr,
                       A.col_idx, q, a, t, ld, colw, G, accumulate ? 1 : 0);
  else if (q <= 128)
    hipLaunchKernelGGL(k_sddmm<2>, dim3(grid), dim3(256), 0, s, (int)A.n_atoms, A.row_ptr,
                       A.col_idx, q, a, t, ld, colw, G, accumulate ? 1 : 0);
  else if (q <= 256)
    hipLaunchKernelGGL(k_sddmm<4>, dim3(grid), dim3(256), 0, s, (int)A.n_atoms, A.row_ptr,
                       A.col_idx, q, a, t, ld, colw, G, accumulate ? 1 : 0);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t spring_chain(const Bsr& A, const int32_t* transpose, const double* H,
                        const double* masses, const double* G, int64_t P, const int64_t* pairs,
                        const double* unit, double* dk, double* dm, int* err, hipStream_t s) {
  if (P > 0)
    hipLaunchKernelGGL(k_spring_dk, dim3(nb(P, 256)), dim3(256), 0, s, P, (int)A.n_atoms, A.row_ptr, A.col_idx,
                       masses, G, pairs, unit, dk, err);
  if (A.n_atoms > 0)
    hipLaunchKernelGGL(k_spring_dm, dim3(nb(A.n_atoms, 256)), dim3(256), 0, s, (int)A.n_atoms,
                       A.row_ptr, transpose, H, masses, G, dm);
  return hipGetLastError();
}

hipError_t assemble_springs(int64_t n_atoms, const int64_t* row_ptr, const int32_t* col_idx,
                            int64_t P, const int64_t* pairs, const double* unit, const double* k,
                            double* K, int* err, hipStream_t s) {
  if (P > 0)
    hipLaunchKernelGGL(k_check_pairs, dim3(nb(P, 256)), dim3(256), 0, s, P, (int)n_atoms, pairs, err);
  if (n_atoms > 0)
    hipLaunchKernelGGL(k_assemble_springs, dim3(nb(n_atoms, 256)), dim3(256), 0, s, (int)n_atoms,
                       row_ptr, col_idx, P, pairs, unit, k, K, err);
  return hipGetLastError();
}

// Register-resident segment kernels for segments of up to 8, 13 and 16
// steps (the default stride ceil(sqrt(d)) for d <= 64, 169, 256): the rows
// of a_m and the next block's rows of t_m take 12 VGPRs per step, so the
// smallest fit keeps the most waves (148, 209 and 245 VGPRs: 3, 2 and 2
// waves per SIMD).  1e5-atom glass, q = 64, d = 150: adjoint 142.6 ->
// 134.7 ms against the kernel that loaded each block's rows after storing
// the previous block (4 waves per SIMD), same bits.
constexpr int kSegRegMax = 16;

hipError_t sddmm_seg_f64(const Bsr& A, int q, int m, const double* a, int64_t a_stride,
                         const double* t, int64_t t_stride, int64_t ld, const double* w,
                         double* G, hipStream_t s) {
  if (A.n_atoms == 0 || m == 0) return hipSuccess;
  const unsigned grid = nb(A.n_atoms, 4);
  if (q <= 64 && m <= kSegRegMax) {
    // chunks of work-groups (4 rows each), eight of them spanning the
    // pattern's neighbour span; the grid is padded to whole rounds of 8 chunks
    const int64_t per_xcd = ((int64_t)grid + 7) / 8;
    int64_t chunk = A.span > 0 ? std::max<int64_t>(1, (A.span + 16) / 32) : 1;
    const char* e = std::getenv("PFEIG_SDDMM_CHUNK");
    if (e) chunk = std::max(1, std::atoi(e));
    chunk = std::min<int64_t>(chunk, std::max<int64_t>(per_xcd, 1));
    const int64_t gridp = (((int64_t)grid + 8 * chunk - 1) / (8 * chunk)) * 8 * chunk;
#define PFE_SEG_REG(MM_)                                                                       \
  hipLaunchKernelGGL(k_sddmm_seg_reg<MM_>, dim3((unsigned)gridp), dim3(256), 0, s,               \
                     (int)A.n_atoms, A.row_ptr, A.col_idx, q, m, a, a_stride, t, t_stride, ld, w, \
                     G, (int)chunk)
    if (m <= 8)
      PFE_SEG_REG(8);
    else if (m <= 13)
      PFE_SEG_REG(13);
    else
      PFE_SEG_REG(kSegRegMax);
#undef PFE_SEG_REG
  } else if (q <= 64)
    hipLaunchKernelGGL(k_sddmm_seg<1>, dim3(grid), dim3(256), 0, s, (int)A.n_atoms, A.row_ptr,
                       A.col_idx, q, m, a, a_stride, t, t_stride, ld, w, G);
  else if (q <= 128)
    hipLaunchKernelGGL(k_sddmm_seg<2>, dim3(grid), dim3(256), 0, s, (int)A.n_atoms, A.row_ptr,
                       A.col_idx, q, m, a, a_stride, t, t_stride, ld, w, G);
  else if (q <= 256)
    hipLaunchKernelGGL(k_sddmm_seg<4>, dim3(grid), dim3(256), 0, s, (int)A.n_atoms, A.row_ptr,
                       A.col_idx, q, m, a, a_stride, t, t_stride, ld, w, G);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

}  // namespace pfe
