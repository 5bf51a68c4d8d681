// Block-sparse (3x3 BSR) kernels for gfx950: the fused Chebyshev step of
// Algorithm 2 (three-term recurrence, eq. 3-term-recurrence, with the
// spectral map of eq. transf.1 folded into scalars), the single-vector SpMV
// used by the Lanczos bounds, mass weighting (eq. intro.2) and validation.
//
// Mapping of the fused step: one wavefront per row tile (two atom rows, six
// matrix rows, for FP64, three for FP64 blocks wider than 192 columns; three
// atom rows for the FP32 filter, four above 192 columns; one atom row when
// tiles are off).  Lane l owns NP column
// chunks of VW contiguous elements, chunk = l + 64 p, so a neighbour's three
// rows of T_in (3 q contiguous elements) are read by coalesced 8-32 byte
// vector loads.  A tile's records (column, row mask) arrive with one vector
// load, a record per lane, and are taken with readlane; the block values are
// wave-uniform and go through scalar loads, a batch's all at once, so each
// batch of U records costs one memory round trip.  Work-groups are dealt to the
// XCDs in chunks sized to the pattern's neighbour span (or one range per XCD
// for the locality order), so rows that share T_in rows share an L2.
#include <algorithm>
#include <cstdlib>
#include <vector>

#include "internal.h"

namespace pfe {
namespace {

template <typename T, int N>
struct VT {
  typedef T type __attribute__((ext_vector_type(N)));
};
template <typename T>
struct VT<T, 1> {
  typedef T type;
};

#ifndef PFE_CHEB_NT_OUT
#define PFE_CHEB_NT_OUT 1       // T_out written with the nontemporal hint
#endif
constexpr int kWavesPerBlock = 4;
#ifndef PFE_CHEB_UNROLL
#define PFE_CHEB_UNROLL 4
#endif
constexpr int kUnroll = PFE_CHEB_UNROLL;
#ifndef PFE_TILE_UNROLL
#define PFE_TILE_UNROLL 2
#endif
constexpr int kTileUnroll = PFE_TILE_UNROLL;   // union columns gathered per batch (tiles)

__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

template <typename V>
__device__ __forceinline__ V ld_nt(const V* p) {
  return __builtin_nontemporal_load(p);
}
template <typename V>
__device__ __forceinline__ void st_nt(V v, V* p) {
  __builtin_nontemporal_store(v, p);
}

// One fused step computes, for every atom row i and every column,
//   out_i = alpha (H tin)_i + beta tin_i + delta prev_i + zeta add_i,
// which covers every recurrence the library runs: Clenshaw's backward
// recurrence for p(H_hat) X (b_k = g_k X + 2 H_hat b_{k+1} - b_{k+2}),
// the forward three-term recurrence of Algorithm 2 (adjoint checkpoints),
// and W = H X.  Four multivector streams at most: tin gathered, prev and add
// read, out written (out may alias prev or add).
//
// Row-to-work-group mapping: work-groups are dispatched round-robin over the
// 8 XCDs (work-group b runs on XCD b % 8).  Rows are cut into chunks of
// `chunk` work-groups; chunk c is placed on XCD c % 8, so consecutive rows
// of a chunk share one XCD's L2 while all XCDs advance through the same
// region of the matrix together (shared Infinity Cache window).
__device__ __forceinline__ int map_block(int b, int chunk) {
  const int xcd = b & 7, s = b >> 3;
  return ((s / chunk) * 8 + xcd) * chunk + (s % chunk);
}

template <typename T, int VW, int NP>
__device__ __forceinline__ void step_epilogue(typename VT<T, VW>::type (&acc)[3][NP],
                                              const bool (&act)[NP], int row, int lane, int col0,
                                              const T* __restrict__ tin, const T* prev,
                                              const T* add, T* out, int64_t ld, T alpha, T beta,
                                              T delta, T zeta) {
  using vt = typename VT<T, VW>::type;
  // All loads of the row are issued before its first store: out may alias
  // prev or add (element by element), so no load may follow a store, and
  // issuing them together costs one memory round trip instead of three.
  vt b[3][NP], d[3][NP], z[3][NP];
#pragma unroll
  for (int p = 0; p < NP; ++p) {
    if (!act[p]) continue;
    const int c = (lane + 64 * p) * VW;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const int64_t off = (int64_t)(3 * row + a) * ld + col0 + c;
      b[a][p] = beta != T(0) ? *reinterpret_cast<const vt*>(tin + off) : vt(0);
      d[a][p] = delta != T(0) ? ld_nt(reinterpret_cast<const vt*>(prev + off)) : vt(0);
      z[a][p] = zeta != T(0) ? ld_nt(reinterpret_cast<const vt*>(add + off)) : vt(0);
    }
  }
#pragma unroll
  for (int p = 0; p < NP; ++p) {
    if (!act[p]) continue;
    const int c = (lane + 64 * p) * VW;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const int64_t off = (int64_t)(3 * row + a) * ld + col0 + c;
      vt o = alpha * acc[a][p];
      o += beta * b[a][p];
      o += delta * d[a][p];
      o += zeta * z[a][p];
      if (PFE_CHEB_NT_OUT)
        st_nt(o, reinterpret_cast<vt*>(out + off));
      else
        *reinterpret_cast<vt*>(out + off) = o;
    }
  }
}

// Variant S: indices and block values through the scalar unit.
template <typename T, int VW, int NP, int U>
__global__ __launch_bounds__(256) void k_cheb_step(
    int n_atoms, const int64_t* __restrict__ row_ptr, const int32_t* __restrict__ col_idx,
    const T* __restrict__ vals, const T* __restrict__ tin, const T* prev, const T* add, T* out,
    int q, int pass_w, int64_t ld, T alpha, T beta, T delta, T zeta, int chunk) {
  using vt = typename VT<T, VW>::type;
  const int lb = map_block(blockIdx.x, chunk);
  const int wave = uniform(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int row = uniform(lb * kWavesPerBlock + wave);
  if (row >= n_atoms) return;
  const int col0 = blockIdx.y * pass_w;
  const int cend = min(q, col0 + pass_w);

  vt acc[3][NP];
  bool act[NP];
#pragma unroll
  for (int p = 0; p < NP; ++p) {
    acc[0][p] = vt(0);
    acc[1][p] = vt(0);
    acc[2][p] = vt(0);
    act[p] = col0 + (lane + 64 * p) * VW < cend;
  }
  const int64_t b0 = row_ptr[row];
  const int64_t b1 = (alpha != T(0)) ? row_ptr[row + 1] : b0;
  // col_idx and vals are padded by kBsrPad entries on the device, so the U
  // index and value loads of a group are unconditional; lanes of neighbours
  // past the row end read zeros instead of T_in.
  for (int64_t k = b0; k < b1; k += U) {
    vt x[U][3][NP];
    int j[U];
#pragma unroll
    for (int u = 0; u < U; ++u) j[u] = col_idx[k + u];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const bool valid = (u == 0) || (k + u < b1);
      const T* src = tin + (int64_t)(3 * (valid ? j[u] : row)) * ld + col0;
#pragma unroll
      for (int p = 0; p < NP; ++p) {
        const int c = (lane + 64 * p) * VW;
        if (act[p] && valid) {
          x[u][0][p] = *reinterpret_cast<const vt*>(src + c);
          x[u][1][p] = *reinterpret_cast<const vt*>(src + ld + c);
          x[u][2][p] = *reinterpret_cast<const vt*>(src + 2 * ld + c);
        } else {
          x[u][0][p] = vt(0);
          x[u][1][p] = vt(0);
          x[u][2][p] = vt(0);
        }
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const T* hv = vals + (k + u) * 9;
      T h[9];
#pragma unroll
      for (int t = 0; t < 9; ++t) h[t] = hv[t];
#pragma unroll
      for (int p = 0; p < NP; ++p) {
        acc[0][p] += h[0] * x[u][0][p] + h[1] * x[u][1][p] + h[2] * x[u][2][p];
        acc[1][p] += h[3] * x[u][0][p] + h[4] * x[u][1][p] + h[5] * x[u][2][p];
        acc[2][p] += h[6] * x[u][0][p] + h[7] * x[u][1][p] + h[8] * x[u][2][p];
      }
    }
  }
  step_epilogue<T, VW, NP>(acc, act, row, lane, col0, tin, prev, add, out, ld, alpha, beta, delta,
                           zeta);
}

// Variant T (row tiles): one wave per tile of R block rows (consecutive in
// the processing order, tile_row).  Each union column j of the tile is
// gathered once (three rows of T_in) and applied to every row of the tile
// that stores block (row, j), so a T_in row shared by neighbouring output
// rows costs one set of vector loads instead of up to R.  Block values are
// read in tile order from a running offset, so their scalar loads depend
// only on the (column, mask) records, which sit in the lanes of one vector
// register (64 per window) and cost no load inside the record loop.
//
// The step is evaluated as out_i = alpha acc_i with
//   acc_i = (delta/alpha) prev_i + (zeta/alpha) add_i        (at tile start)
//         + sum_j H_ij tin_j + (beta/alpha) tin_i            (record loop)
// (coefficients cb, cd, cz from the host).  prev and add are read with the
// tile's records, before the first gather, and the diagonal term uses the
// T_in row the loop gathers anyway (record flag bit R + r marks row r's own
// column), so the tile ends with stores only instead of two more serial
// memory round trips.  alpha == 0 (no matrix term): acc = cb tin + cd prev
// + cz add at tile start, no record loop, out = acc.
template <typename T, int VW, int NP, int U, int R>
__global__ __launch_bounds__(256) void k_cheb_tile(
    int n_atoms, int n_tiles, const int64_t* __restrict__ tile_ptr,
    const int64_t* __restrict__ tile_vptr, const int2* __restrict__ tile_cm,
    const int32_t* __restrict__ tile_row, const T* __restrict__ vals,
    const T* __restrict__ tin, const T* prev, const T* add, T* out, int q, int pass_w,
    int64_t ld, T alpha, T cb, T cd, T cz, int chunk) {
  static_assert(64 % U == 0, "a record batch must not straddle two 64-record windows");
  using vt = typename VT<T, VW>::type;
  const int lb = map_block(blockIdx.x, chunk);
  const int wave = uniform(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int tile = uniform(lb * kWavesPerBlock + wave);
  if (tile >= n_tiles) return;
  const int col0 = blockIdx.y * pass_w;   // this pass: columns [col0, min(q, col0 + pass_w))
  const int cend = min(q, col0 + pass_w);
  const bool mat = alpha != T(0);
  vt acc[R][3][NP];
  bool act[NP];
  // byte offsets of this lane's columns in the three rows of an atom, so a
  // row access is one uniform row address plus these (lanes past q read
  // column col0 of the same rows; their sums are never stored)
  uint32_t boff[3][NP];
#pragma unroll
  for (int p = 0; p < NP; ++p) {
    const int c = col0 + (lane + 64 * p) * VW;
    act[p] = c < cend;
    const int64_t e = act[p] ? c : col0;
#pragma unroll
    for (int a = 0; a < 3; ++a) boff[a][p] = (uint32_t)((a * ld + e) * (int64_t)sizeof(T));
  }
  const int64_t ld3 = 3 * ld;
  const int64_t ubase = tile_ptr[tile];
  const int nrec = mat ? (int)(tile_ptr[tile + 1] - ubase) : 0;
  const int2* rec = tile_cm + ubase;
  const T* hv = vals + tile_vptr[tile] * 9;
  int rows[R];
#pragma unroll
  for (int r = 0; r < R; ++r) rows[r] = tile_row[tile * R + r];   // -1: no row
  // the tile's records, lane i holding record w + i of the current 64-record
  // window w (requested with the accumulator start values); the loop takes
  // them with readlane, so no record load sits in the batch chain
  int rx = 0, ry = 0;
  if (lane < nrec) {
    const int2 v = rec[lane];
    rx = v.x;
    ry = v.y;
  }
  // One branch-free block per set of streams, so every start value is
  // requested before the first wait (rows past the last read row 0 and are
  // never stored).
  int64_t rb[R];   // byte offset of each row's three matrix rows
#pragma unroll
  for (int r = 0; r < R; ++r) rb[r] = (int64_t)(rows[r] >= 0 ? rows[r] : 0) * ld3 * (int64_t)sizeof(T);
  auto start2 = [&](const T* s1, T c1, const T* s2, T c2) {
    vt v1[R][3][NP], v2[R][3][NP];
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int p = 0; p < NP; ++p)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          const int64_t o = rb[r] + boff[a][p];
          v1[r][a][p] = ld_nt(reinterpret_cast<const vt*>(reinterpret_cast<const char*>(s1) + o));
          v2[r][a][p] = ld_nt(reinterpret_cast<const vt*>(reinterpret_cast<const char*>(s2) + o));
        }
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int p = 0; p < NP; ++p)
#pragma unroll
        for (int a = 0; a < 3; ++a) acc[r][a][p] = c1 * v1[r][a][p] + c2 * v2[r][a][p];
  };
  auto start1 = [&](const T* s1, T c1) {
    vt v1[R][3][NP];
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int p = 0; p < NP; ++p)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          const int64_t o = rb[r] + boff[a][p];
          v1[r][a][p] = ld_nt(reinterpret_cast<const vt*>(reinterpret_cast<const char*>(s1) + o));
        }
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int p = 0; p < NP; ++p)
#pragma unroll
        for (int a = 0; a < 3; ++a) acc[r][a][p] = c1 * v1[r][a][p];
  };
  if (!mat && cb != T(0)) {   // no matrix term: tin enters here, not through the loop
    if (cd != T(0)) {
      start2(tin, cb, prev, cd);
      if (cz != T(0)) {
        vt t[R][3][NP];
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
          for (int p = 0; p < NP; ++p)
#pragma unroll
            for (int a = 0; a < 3; ++a)
              t[r][a][p] = acc[r][a][p];
        start1(add, cz);
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
          for (int p = 0; p < NP; ++p)
#pragma unroll
            for (int a = 0; a < 3; ++a) acc[r][a][p] += t[r][a][p];
      }
    } else if (cz != T(0)) {
      start2(tin, cb, add, cz);
    } else {
      start1(tin, cb);
    }
  } else if (cd != T(0) && cz != T(0)) {
    start2(prev, cd, add, cz);
  } else if (cd != T(0)) {
    start1(prev, cd);
  } else if (cz != T(0)) {
    start1(add, cz);
  } else {
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int p = 0; p < NP; ++p)
#pragma unroll
        for (int a = 0; a < 3; ++a) acc[r][a][p] = vt(0);
  }
  __builtin_amdgcn_sched_barrier(0);   // start values in registers before the first gathers
  for (int k = 0; k < nrec; k += U) {
    if (k > 0 && (k & 63) == 0) {   // next window of 64 records
      rx = ry = 0;
      if (k + lane < nrec) {
        const int2 v = rec[k + lane];
        rx = v.x;
        ry = v.y;
      }
    }
    int2 cm[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int l = (k + u) & 63;   // U divides 64: a batch never straddles two windows
      cm[u] = make_int2(__builtin_amdgcn_readlane(rx, l), __builtin_amdgcn_readlane(ry, l));
    }
    vt x[U][3][NP];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (u == 0 || k + u < nrec) {
        const char* rowp = reinterpret_cast<const char*>(tin + (int64_t)(uint32_t)cm[u].x * ld3);
#pragma unroll
        for (int p = 0; p < NP; ++p)
#pragma unroll
          for (int a = 0; a < 3; ++a) x[u][a][p] = *reinterpret_cast<const vt*>(rowp + boff[a][p]);
      }
    }
    // Every block of the batch is requested with its gathers, before the
    // first product: block addresses are branch-free (a row without a block
    // in a record reads the next block, or the zero padding past the last
    // tile, and never uses it).
    T hb[U][R][9];
    {
      int o = 0;
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int m = (u == 0 || k + u < nrec) ? cm[u].y : 0;
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const int idx = o + __builtin_popcount(m & ((1 << r) - 1));
#pragma unroll
          for (int t = 0; t < 9; ++t) hb[u][r][t] = hv[9 * idx + t];
        }
        o += __builtin_popcount(m & ((1 << R) - 1));
      }
      hv += 9 * o;
    }
    // The empty asm reads every value in a scalar register here, so the
    // compiler cannot sink a block's load into the branch that uses it (which
    // would cost one more memory round trip per record).
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int r = 0; r < R; ++r)
#pragma unroll
        for (int t = 0; t < 9; ++t) asm volatile("" ::"s"(hb[u][r][t]));
    __builtin_amdgcn_sched_barrier(0);   // keep the request here, ahead of the products
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (u == 0 || k + u < nrec) {
        const int m = cm[u].y;
        const T (&h)[R][9] = hb[u];
#pragma unroll
        for (int r = 0; r < R; ++r) {
          if ((m >> r) & 1) {
#pragma unroll
            for (int p = 0; p < NP; ++p)
#pragma unroll
              for (int a = 0; a < 3; ++a) {
                acc[r][a][p] += h[r][3 * a] * x[u][0][p];
                acc[r][a][p] += h[r][3 * a + 1] * x[u][1][p];
                acc[r][a][p] += h[r][3 * a + 2] * x[u][2][p];
              }
          }
          if (((m >> (R + r)) & 1) && cb != T(0)) {   // row r's own column: the diagonal shift
#pragma unroll
            for (int p = 0; p < NP; ++p)
#pragma unroll
              for (int a = 0; a < 3; ++a) acc[r][a][p] += cb * x[u][a][p];
          }
        }
      }
    }
  }
  const T so = mat ? alpha : T(1);
#pragma unroll
  for (int r = 0; r < R; ++r) {
    if (rows[r] < 0) continue;
    char* op = reinterpret_cast<char*>(out) + (int64_t)rows[r] * ld3 * (int64_t)sizeof(T);
#pragma unroll
    for (int p = 0; p < NP; ++p) {
      if (!act[p]) continue;
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const vt o = so * acc[r][a][p];
        if (PFE_CHEB_NT_OUT)
          st_nt(o, reinterpret_cast<vt*>(op + boff[a][p]));
        else
          *reinterpret_cast<vt*>(op + boff[a][p]) = o;
      }
    }
  }
}

template <typename T>
__global__ void k_permute_blocks(int64_t nnzb, const int64_t* __restrict__ perm,
                                 const T* __restrict__ src, T* __restrict__ dst) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nnzb * 9) return;
  const int64_t p = i / 9, t = i % 9;
  dst[i] = src[perm[p] * 9 + t];
}

#ifndef PFE_CHEB_CHUNK
#define PFE_CHEB_CHUNK 64    // work-groups per XCD chunk (measured best on MI355X); 0: one range per XCD
#endif

// Schedule overrides, read at every launch (they change which wave computes
// a row when, never the result): PFEIG_CHEB_PASS_COLS (columns per pass) and
// PFEIG_CHEB_CHUNK (work-groups per XCD chunk).
int env_int(const char* name, int unset) {
  const char* e = std::getenv(name);
  return e ? std::atoi(e) : unset;
}
int pass_cols_override() { return env_int("PFEIG_CHEB_PASS_COLS", 0); }
int chunk_override() { return env_int("PFEIG_CHEB_CHUNK", -1); }

template <typename T, int VW, int NP>
hipError_t launch_cheb(const Bsr& A, const T* vals, const T* tin, const T* prev, const T* add,
                       T* out, int q, int pass_w, int64_t ld, T alpha, T beta, T delta,
                       T zeta, hipStream_t s) {
  const int R = (A.tile_rows >= 2 && A.tile_ptr) ? A.tile_rows : 1;   // vals in tile order
  if (R >= 2 && (3 * ld) * (int64_t)sizeof(T) > (int64_t)UINT32_MAX) return hipErrorInvalidValue;
  const int64_t units = (R >= 2) ? A.n_tiles : A.n_atoms;   // one wave per unit
  const int64_t nblk = (units + kWavesPerBlock - 1) / kWavesPerBlock;
  const int64_t per_xcd = (nblk + 7) / 8;
  // Rows in locality order: one contiguous range (a compact region) per XCD.
  // Natural order: chunks dealt round-robin, 8 chunks spanning the pattern's
  // typical long neighbour offset, so a row and its neighbour one "plane"
  // away fall on the same XCD and the second gather hits that XCD's L2 (1e6-
  // atom lattice glass: 2870 us per step against 3265 us with fixed 256-row
  // chunks; no change at 1e5 atoms, where 8 such chunks already span one
  // plane within 7 %); PFE_CHEB_CHUNK work-groups when the pattern gives none.
  int chunk = (R >= 2 && A.tile_local) ? 0 : PFE_CHEB_CHUNK;
  if (R >= 2) chunk = std::max(chunk > 0 ? 1 : 0, chunk / R);   // keep rows per chunk comparable
  if (R >= 2 && !A.tile_local && A.span > 0) {
    const int64_t rows_per_group = (int64_t)kWavesPerBlock * R;
    chunk = (int)std::max<int64_t>(1, (A.span + 4 * rows_per_group) / (8 * rows_per_group));
  }
  if (chunk_override() >= 0) chunk = chunk_override();         // work-groups, as given
  if (chunk <= 0 || chunk > per_xcd) chunk = (int)per_xcd;
  const int64_t grid_x = ((nblk + 8LL * chunk - 1) / (8LL * chunk)) * 8LL * chunk;
  if (pass_w <= 0 || pass_w > 64 * NP * VW || pass_w % VW) return hipErrorInvalidValue;
  const int npass = (q + pass_w - 1) / pass_w;
  dim3 grid((unsigned)grid_x, (unsigned)npass);
  // tile kernels: out = alpha acc, acc started from prev and add scaled by
  // 1/alpha (quotients rounded once, from the double values)
  const double sa = alpha != T(0) ? (double)alpha : 1.0;
  const T cb = (T)((double)beta / sa), cd = (T)((double)delta / sa), cz = (T)((double)zeta / sa);
  // FP64 tiles of more than two rows take one record per batch: a batch's
  // block values (U R 9 doubles) stay within the scalar registers.
  constexpr int U34 = sizeof(T) == 8 ? 1 : kTileUnroll;
  if (R == 2) {
    hipLaunchKernelGGL((k_cheb_tile<T, VW, NP, kTileUnroll, 2>), grid, dim3(256), 0, s,
                       (int)A.n_atoms, (int)A.n_tiles, A.tile_ptr, A.tile_vptr, A.tile_cm,
                       A.tile_row, vals, tin, prev, add, out, q, pass_w, ld, alpha, cb, cd, cz,
                       chunk);
  } else if (R == 3) {
    hipLaunchKernelGGL((k_cheb_tile<T, VW, NP, U34, 3>), grid, dim3(256), 0, s,
                       (int)A.n_atoms, (int)A.n_tiles, A.tile_ptr, A.tile_vptr, A.tile_cm,
                       A.tile_row, vals, tin, prev, add, out, q, pass_w, ld, alpha, cb, cd, cz,
                       chunk);
  } else if (R == 4) {
    hipLaunchKernelGGL((k_cheb_tile<T, VW, NP, U34, 4>), grid, dim3(256), 0, s,
                       (int)A.n_atoms, (int)A.n_tiles, A.tile_ptr, A.tile_vptr, A.tile_cm,
                       A.tile_row, vals, tin, prev, add, out, q, pass_w, ld, alpha, cb, cd, cz,
                       chunk);
  } else {
    hipLaunchKernelGGL((k_cheb_step<T, VW, NP, kUnroll>), grid, dim3(256), 0, s, (int)A.n_atoms,
                       A.row_ptr, A.col_idx, vals, tin, prev, add, out, q, pass_w, ld, alpha,
                       beta, delta, zeta, chunk);
  }
  return hipGetLastError();
}

template <typename T>
bool aligned(const void* p, int bytes) {
  return p == nullptr || (reinterpret_cast<uintptr_t>(p) % bytes) == 0;
}

// Chooses the vector width (largest that divides q and ld with aligned
// pointers) and the number of column passes per lane.
template <typename T, int MAXVW>
hipError_t dispatch_cheb(const Bsr& A, const T* vals, const T* tin, const T* prev, const T* add,
                         T* out, int q, int64_t ld, T alpha, T beta, T delta, T zeta,
                         hipStream_t s) {
  if (A.n_atoms == 0 || q == 0) return hipSuccess;
  // smallest vector width that covers q with one 64-lane pass, if the
  // layout allows it; otherwise the widest that does
  int want = 1;
  while (want < MAXVW && want * 64 < q) want *= 2;
  // FP64: 16-byte loads per lane even when fewer lanes are then active
  // (measured on MI355X: 7-8% faster steps for q <= 64; FP32 keeps 8-byte
  // loads with more lanes, which measured faster than 16-byte ones)
  if (sizeof(T) == 8) want = std::max(want, std::min(MAXVW, 2));
  auto fits = [&](int v) {
    const int bytes = v * (int)sizeof(T);
    return q % v == 0 && ld % v == 0 && aligned<T>(tin, bytes) && aligned<T>(prev, bytes) &&
           aligned<T>(out, bytes) && aligned<T>(add, bytes);
  };
  int vw = want;
  while (vw > 1 && !fits(vw)) vw /= 2;
  const int chunks = (q + vw - 1) / vw;
  int np = chunks <= 64 ? 1 : (chunks <= 128 ? 2 : 4);
  // Column passes (blockIdx.y): with a limit of `lim` columns the q columns
  // are split into ceil(q / lim) passes of equal width, each on the narrowest
  // lane layout that covers it.  FP64 beyond 128 columns runs passes of at
  // most 128 columns (VW 2, 8 waves per SIMD) instead of one VW-4 pass (4
  // waves), although the matrix is read once per pass: on the 1e6-atom glass
  // q = 256 8.79 -> 7.58 ms per step (two 128-column passes) and q = 160
  // 5.12 -> 4.84 ms (two of 80); in FP32 one pass measured faster (q = 160:
  // 2.32 against 3.72 ms).  PFEIG_CHEB_PASS_COLS overrides.
  int lim = pass_cols_override();
  if (lim <= 0 && sizeof(T) == 8 && q > 128) lim = 128;
  int pass_w = 64 * np * vw;
  if (lim > 0 && lim < q) {
    const int npass = (q + lim - 1) / lim;
    const int pw = (q + npass - 1) / npass;
    while (np > 1 && 64 * (np / 2) * vw >= pw) np /= 2;
    while (vw > 1 && 64 * np * (vw / 2) >= pw && fits(vw / 2)) vw /= 2;
    pass_w = std::min(64 * np * vw, ((pw + vw - 1) / vw) * vw);
  } else {
    pass_w = std::min(pass_w, ((q + vw - 1) / vw) * vw);
  }
#define PFE_CHEB_CASE(VW_, NP_)                                                               \
  if (vw == VW_ && np == NP_)                                                                 \
    return launch_cheb<T, VW_, NP_>(A, vals, tin, prev, add, out, q, pass_w, ld, alpha, beta, \
                                    delta, zeta, s);
  PFE_CHEB_CASE(1, 1)
  PFE_CHEB_CASE(1, 2)
  PFE_CHEB_CASE(1, 4)
  PFE_CHEB_CASE(2, 1)
  PFE_CHEB_CASE(2, 2)
  PFE_CHEB_CASE(2, 4)
  PFE_CHEB_CASE(4, 1)
  PFE_CHEB_CASE(4, 2)
  PFE_CHEB_CASE(4, 4)
  if constexpr (MAXVW >= 8) {
    PFE_CHEB_CASE(8, 1)
    PFE_CHEB_CASE(8, 2)
    PFE_CHEB_CASE(8, 4)
  }
#undef PFE_CHEB_CASE
  return hipErrorInvalidValue;
}

// ------------------------------------------------------------------ SpMV
__global__ __launch_bounds__(256) void k_spmv(int n_atoms, const int64_t* __restrict__ row_ptr,
                                              const int32_t* __restrict__ col_idx,
                                              const double* __restrict__ vals,
                                              const double* __restrict__ x,
                                              double* __restrict__ y) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_atoms) return;
  double a0 = 0, a1 = 0, a2 = 0;
  for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) {
    const int j = col_idx[k];
    const double* h = vals + k * 9;
    const double x0 = x[3 * (int64_t)j], x1 = x[3 * (int64_t)j + 1], x2 = x[3 * (int64_t)j + 2];
    a0 += h[0] * x0 + h[1] * x1 + h[2] * x2;
    a1 += h[3] * x0 + h[4] * x1 + h[5] * x2;
    a2 += h[6] * x0 + h[7] * x1 + h[8] * x2;
  }
  y[3 * (int64_t)i] = a0;
  y[3 * (int64_t)i + 1] = a1;
  y[3 * (int64_t)i + 2] = a2;
}

// -------------------------------------------------------- weighting, casts
__global__ void k_mass_weight(int n_atoms, const int64_t* __restrict__ row_ptr,
                              const int32_t* __restrict__ col_idx, const double* __restrict__ K,
                              const double* __restrict__ m, double* __restrict__ H) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_atoms) return;
  const double mi = m[i];
  for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) {
    const double w = 1.0 / sqrt(mi * m[col_idx[k]]);
    for (int t = 0; t < 9; ++t) H[k * 9 + t] = K[k * 9 + t] * w;
  }
}

__global__ void k_shift_scale_f32(int n_atoms, const int64_t* __restrict__ row_ptr,
                                  const int32_t* __restrict__ col_idx,
                                  const double* __restrict__ H, double c, double inv_e,
                                  float* __restrict__ H32) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_atoms) return;
  for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) {
    const bool diag = col_idx[k] == i;
    for (int t = 0; t < 9; ++t) {
      double v = H[k * 9 + t];
      if (diag && (t == 0 || t == 4 || t == 8)) v -= c;
      H32[k * 9 + t] = (float)(v * inv_e);
    }
  }
}

__global__ void k_validate(int n_atoms, const int64_t* __restrict__ row_ptr,
                           const int32_t* __restrict__ col_idx, const double* __restrict__ v,
                           int32_t* __restrict__ transpose, int* err) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_atoms) return;
  const int64_t b0 = row_ptr[i], b1 = row_ptr[i + 1];
  int flags = 0;
  bool has_diag = false;
  if (b1 < b0) flags |= 1;
  for (int64_t k = b0; k < b1; ++k) {
    const int j = col_idx[k];
    if (j < 0 || j >= n_atoms || (k > b0 && col_idx[k - 1] >= j)) {
      flags |= 1;
      continue;
    }
    if (j == i) has_diag = true;
    for (int t = 0; t < 9; ++t)
      if (!isfinite(v[k * 9 + t])) flags |= 2;
    // transpose partner (j, i) by binary search in row j
    int64_t lo = row_ptr[j], hi = row_ptr[j + 1] - 1, found = -1;
    while (lo <= hi) {
      const int64_t mid = (lo + hi) >> 1;
      const int cm = col_idx[mid];
      if (cm == i) {
        found = mid;
        break;
      }
      if (cm < i)
        lo = mid + 1;
      else
        hi = mid - 1;
    }
    if (found < 0) {
      flags |= 4;
      transpose[k] = -1;
      continue;
    }
    transpose[k] = (int32_t)found;
    for (int p = 0; p < 3; ++p)
      for (int r = 0; r < 3; ++r)
        if (v[k * 9 + p * 3 + r] != v[found * 9 + r * 3 + p]) flags |= 8;
  }
  if (!has_diag) flags |= 1;
  if (flags) atomicOr(err, flags);
}

__global__ void k_validate_masses(int n, const double* __restrict__ m, int* err) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double v = m[i];
  if (!(v > 0.0) || !isfinite(v)) atomicOr(err, 16);
}

inline unsigned nb(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

}  // namespace

hipError_t cheb_step_f64(const Bsr& A, const double* vals, const double* tin, const double* prev,
                         const double* add, double* out, int q, int64_t ld, double alpha,
                         double beta, double delta, double zeta, hipStream_t s) {
  return dispatch_cheb<double, 4>(A, vals, tin, prev, add, out, q, ld, alpha, beta, delta, zeta,
                                  s);
}

hipError_t cheb_step_f32(const Bsr& A, const float* vals, const float* tin, const float* prev,
                         const float* add, float* out, int q, int64_t ld, float alpha, float beta,
                         float delta, float zeta, hipStream_t s) {
  return dispatch_cheb<float, 8>(A, vals, tin, prev, add, out, q, ld, alpha, beta, delta, zeta, s);
}

hipError_t spmv_f64(const Bsr& A, const double* vals, const double* x, double* y, hipStream_t s) {
  if (A.n_atoms == 0) return hipSuccess;
  hipLaunchKernelGGL(k_spmv, dim3(nb(A.n_atoms, 256)), dim3(256), 0, s, (int)A.n_atoms,
                     A.row_ptr, A.col_idx, vals, x, y);
  return hipGetLastError();
}

hipError_t mass_weight(const Bsr& A, const double* K, const double* masses, double* H,
                       hipStream_t s) {
  if (A.n_atoms == 0) return hipSuccess;
  hipLaunchKernelGGL(k_mass_weight, dim3(nb(A.n_atoms, 128)), dim3(128), 0, s, (int)A.n_atoms,
                     A.row_ptr, A.col_idx, K, masses, H);
  return hipGetLastError();
}

hipError_t shift_scale_to_f32(const Bsr& A, const double* H, double c, double e, float* H32,
                              hipStream_t s) {
  if (A.n_atoms == 0) return hipSuccess;
  hipLaunchKernelGGL(k_shift_scale_f32, dim3(nb(A.n_atoms, 128)), dim3(128), 0, s,
                     (int)A.n_atoms, A.row_ptr, A.col_idx, H, c, 1.0 / e, H32);
  return hipGetLastError();
}

hipError_t validate_bsr(const Bsr& A, const double* vals, int32_t* transpose, int* err_flags,
                        hipStream_t s) {
  if (A.n_atoms == 0) return hipSuccess;
  hipLaunchKernelGGL(k_validate, dim3(nb(A.n_atoms, 128)), dim3(128), 0, s, (int)A.n_atoms,
                     A.row_ptr, A.col_idx, vals, transpose, err_flags);
  return hipGetLastError();
}

hipError_t validate_masses(int64_t n_atoms, const double* masses, int* err_flags, hipStream_t s) {
  if (n_atoms == 0) return hipSuccess;
  hipLaunchKernelGGL(k_validate_masses, dim3(nb(n_atoms, 256)), dim3(256), 0, s, (int)n_atoms,
                     masses, err_flags);
  return hipGetLastError();
}

constexpr int64_t kDiagMark = 1LL << 62;   // marks a row's diagonal flag among its blocks

void build_row_tiles(int64_t n_atoms, const int64_t* row_ptr, const int32_t* col_idx, int R,
                     const int32_t* order, std::vector<int64_t>& tile_ptr,
                     std::vector<int64_t>& tile_vptr, std::vector<int32_t>& tile_cm,
                     std::vector<int32_t>& tile_row, std::vector<int64_t>& perm) {
  const int64_t n_tiles = (n_atoms + R - 1) / R;
  tile_ptr.assign(n_tiles + 1, 0);
  tile_vptr.assign(n_tiles + 1, 0);
  tile_row.assign(n_tiles * R, -1);
  tile_cm.clear();
  perm.clear();
  perm.reserve(row_ptr[n_atoms]);
  std::vector<std::pair<int32_t, int64_t>> ent;   // (column, r << 40 | block)
  for (int64_t t = 0; t < n_tiles; ++t) {
    ent.clear();
    for (int r = 0; r < R && t * R + r < n_atoms; ++r) {
      const int64_t row = order ? order[t * R + r] : t * R + r;
      tile_row[t * R + r] = (int32_t)row;
      for (int64_t b = row_ptr[row]; b < row_ptr[row + 1]; ++b)
        ent.emplace_back(col_idx[b], ((int64_t)r << 40) | b);
      // bit R + r on the row's own column (validated patterns store the
      // diagonal block, so this only flags that record; without one it
      // would become a record of its own, carrying no block)
      ent.emplace_back((int32_t)row, kDiagMark | ((int64_t)(R + r) << 40));
    }
    std::sort(ent.begin(), ent.end());   // by column, then tile row, flags last
    tile_vptr[t] = (int64_t)perm.size();
    int64_t nu = 0;
    for (size_t e = 0; e < ent.size();) {
      const int32_t c = ent[e].first;
      int32_t mask = 0;
      for (; e < ent.size() && ent[e].first == c; ++e) {
        mask |= 1 << (int)((ent[e].second >> 40) & 0xff);
        if (!(ent[e].second & kDiagMark)) perm.push_back(ent[e].second & ((1LL << 40) - 1));
      }
      tile_cm.push_back(c);
      tile_cm.push_back(mask);
      ++nu;
    }
    tile_ptr[t + 1] = tile_ptr[t] + nu;
  }
  tile_vptr[n_tiles] = (int64_t)perm.size();
  for (int64_t p = 0; p < kBsrPad; ++p) {
    tile_cm.push_back(0);
    tile_cm.push_back(0);
  }
}

hipError_t permute_blocks_f64(int64_t nnzb, const int64_t* perm, const double* src, double* dst,
                              hipStream_t s) {
  if (nnzb == 0) return hipSuccess;
  hipLaunchKernelGGL(k_permute_blocks<double>, dim3((unsigned)((nnzb * 9 + 255) / 256)),
                     dim3(256), 0, s, nnzb, perm, src, dst);
  return hipGetLastError();
}

hipError_t permute_blocks_f32(int64_t nnzb, const int64_t* perm, const float* src, float* dst,
                              hipStream_t s) {
  if (nnzb == 0) return hipSuccess;
  hipLaunchKernelGGL(k_permute_blocks<float>, dim3((unsigned)((nnzb * 9 + 255) / 256)),
                     dim3(256), 0, s, nnzb, perm, src, dst);
  return hipGetLastError();
}

}  // namespace pfe
