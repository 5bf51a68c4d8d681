// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/pfeig.h"
#include "reorder.h"

namespace pfe {

// ----------------------------------------------------------- device buffer
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf() { release(); }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
  // (Re)allocate to at least n bytes; contents undefined unless zeroed.
  hipError_t ensure(size_t n) {
    if (n <= bytes && p) return hipSuccess;
    release();
    if (n == 0) n = 256;
    hipError_t e = hipMalloc(&p, n);
    if (e != hipSuccess) {
      p = nullptr;
      return e;
    }
    bytes = n;
    return hipSuccess;
  }
  template <typename T>
  T* as() const { return static_cast<T*>(p); }
};

// Status carrying an error message up to the C-ABI boundary.
struct Err {
  pfe_status st = PFE_OK;
  std::string msg;
  explicit operator bool() const { return st != PFE_OK; }
};
inline Err ok() { return Err{}; }
inline Err fail(pfe_status s, std::string m) { return Err{s, std::move(m)}; }
inline Err hip_fail(hipError_t e, const char* what) {
  return fail(e == hipErrorOutOfMemory ? PFE_ENOMEM : PFE_EHIP,
              std::string(what) + ": " + hipGetErrorString(e));
}
#define PFE_HIP(call)                                  \
  do {                                                 \
    hipError_t _e = (call);                            \
    if (_e != hipSuccess) return ::pfe::hip_fail(_e, #call); \
  } while (0)
#define PFE_TRY(expr)            \
  do {                           \
    ::pfe::Err _r = (expr);      \
    if (_r) return _r;           \
  } while (0)

// ------------------------------------------------------------ BSR on device
// Device copies of col_idx and of every block-value array are allocated with
// kBsrPad extra zero-filled entries (blocks), read but never used by the
// fused step's grouped loads.
constexpr int64_t kBsrPad = 16;
struct Bsr {
  int64_t n_atoms = 0;
  int64_t nnzb = 0;
  const int64_t* row_ptr = nullptr;   // [n_atoms+1]
  const int32_t* col_idx = nullptr;   // [nnzb]
  // Row tiles (optional, tile_rows >= 2): tile t holds the R = tile_rows block
  // rows tile_row[t*R .. t*R+R-1] (-1 past the last row), consecutive in the
  // processing order of the rows.  Tile t owns union columns
  // [tile_ptr[t], tile_ptr[t+1]) of tile_cm, each a (column, row mask) pair
  // (bit r set when row tile_row[t*R + r] stores a block in that column;
  // bit R + r marks that row's own column, i.e. its diagonal block, which
  // every validated pattern stores), sorted by column.  With tiles active the fused step reads its block
  // values in tile order: the blocks of tile t are [tile_vptr[t], tile_vptr[t+1]) and
  // follow (union column, tile row) order.  tile_cm carries kBsrPad padded
  // entries.
  int tile_rows = 0;
  int64_t n_tiles = 0;
  const int64_t* tile_ptr = nullptr;
  const int64_t* tile_vptr = nullptr;
  const int2* tile_cm = nullptr;
  const int32_t* tile_row = nullptr;
  bool tile_local = false;   // tile_row follows the locality order (one row range per XCD)
  int64_t span = 0;          // typical long neighbour offset in rows (natural order)
};

// Host construction of the row tiles of a block-CSR pattern (see Bsr), the
// rows taken R at a time in `order` (nullptr: natural order); perm[p] is the
// row-order index of the block at tile-order position p.
void build_row_tiles(int64_t n_atoms, const int64_t* row_ptr, const int32_t* col_idx, int R,
                     const int32_t* order, std::vector<int64_t>& tile_ptr,
                     std::vector<int64_t>& tile_vptr, std::vector<int32_t>& tile_cm,
                     std::vector<int32_t>& tile_row, std::vector<int64_t>& perm);
// dst[p] = src[perm[p]] for 3x3 blocks (FP64 and FP32).
hipError_t permute_blocks_f64(int64_t nnzb, const int64_t* perm, const double* src, double* dst,
                              hipStream_t s);
hipError_t permute_blocks_f32(int64_t nnzb, const int64_t* perm, const float* src, float* dst,
                              hipStream_t s);

// ------------------------------------------------------------- launchers
// Fused Chebyshev step (K1), for every atom row i:
//   out_i = alpha (H tin)_i + beta tin_i + delta prev_i + zeta add_i
// (prev not read if delta == 0, add not read if zeta == 0, no neighbour loop
// if alpha == 0).  tin is gathered and must not alias out; out may alias
// prev or add.  Rows of all multivectors have stride ld; columns [0, q).
hipError_t cheb_step_f64(const Bsr& A, const double* vals, const double* tin, const double* prev,
                         const double* add, double* out, int q, int64_t ld, double alpha,
                         double beta, double delta, double zeta, hipStream_t s);
hipError_t cheb_step_f32(const Bsr& A, const float* vals, const float* tin, const float* prev,
                         const float* add, float* out, int q, int64_t ld, float alpha, float beta,
                         float delta, float zeta, hipStream_t s);

// y = H x for a single vector (q = 1), FP64.
hipError_t spmv_f64(const Bsr& A, const double* vals, const double* x, double* y, hipStream_t s);

// H_b = K_b / sqrt(m_row m_col) (K8).
hipError_t mass_weight(const Bsr& A, const double* K, const double* masses, double* H,
                       hipStream_t s);
// H32_b = round_fp32((H_b - c I [diagonal blocks]) / e).
hipError_t shift_scale_to_f32(const Bsr& A, const double* H, double c, double e, float* H32,
                              hipStream_t s);
// Structure/value validation; writes transpose[b] = index of block (col, row);
// err_flags bit 0: unsorted/missing diagonal, bit 1: non-finite, bit 2: missing
// transpose partner, bit 3: K_ji != K_ij^T.
hipError_t validate_bsr(const Bsr& A, const double* vals, int32_t* transpose, int* err_flags,
                        hipStream_t s);
hipError_t validate_masses(int64_t n_atoms, const double* masses, int* err_flags, hipStream_t s);

// ------------------------------------------------------------ dense (K2..K7)
// Partial Gram products: G = A^T B over rows [0, n) with A [n][lda], B [n][ldb];
// q1 columns of A, q2 of B; result q1 x q2 row-major into G (ldg = q2).
// work must hold gram_work_bytes(n, q1, q2) bytes.
size_t gram_work_bytes(int64_t n, int q1, int q2);
hipError_t gram_f64(int64_t n, int q1, int q2, const double* A, int64_t lda, const double* B,
                    int64_t ldb, double* G, void* work, hipStream_t s);
// C[n][q2] = A[n][q1] * Bm[q1][q2] (Bm row-major, ldb = q2); C may alias A
// (in place) if ldc == lda.
hipError_t gemm_tall_f64(int64_t n, int q1, int q2, const double* A, int64_t lda,
                         const double* Bm, double* C, int64_t ldc, hipStream_t s);
// Cholesky G = R^T R (R upper) of a q x q SPD matrix (row-major) and Rinv = R^{-1}
// (Rinv must hold 2 q^2 doubles; the inverse is left in the first q^2).
// shift added to the diagonal first.  info[0] = 0 on success, k+1 if pivot k
// failed.  diag_max (nullable) receives max_i G_ii.
hipError_t chol_inv_f64(int q, const double* G, double shift, double* Rinv, int* info,
                        double* diag_max, hipStream_t s);
// Symmetric eigendecomposition of S (q x q row-major, symmetrised on entry) by
// parallel cyclic Jacobi: evals ascending, Q (row-major, column k = eigenvector k).
// work: jacobi_work_bytes(q).  info[0] = sweeps used (negative if not converged).
size_t jacobi_work_bytes(int q);
hipError_t sym_eig_f64(int q, const double* S, double* evals, double* Q, void* work, int* info,
                       hipStream_t s);
// res[j] = ||W[:, j] - theta[j] X[:, j]||_2 * inv_scale for j < q.
size_t colnorm_work_bytes(int64_t n, int q);
hipError_t resid_norms_f64(int64_t n, int q, const double* W, const double* X, int64_t ld,
                           const double* theta, double inv_scale, double* res, void* work,
                           hipStream_t s);
// Column norms ||X[:, j]|| for j < q.
hipError_t col_norms_f64(int64_t n, int q, const double* X, int64_t ld, double* res, void* work,
                         hipStream_t s);
// res[j] = sum_r X[r][j] Y[r][j]; work as colnorm_work_bytes.
hipError_t col_dots_f64(int64_t n, int q, const double* X, const double* Y, int64_t ld,
                        double* res, void* work, hipStream_t s);
// X[:, j] /= nrm[j]
hipError_t col_scale_inv_f64(int64_t n, int q, double* X, int64_t ld, const double* nrm,
                             hipStream_t s);
hipError_t cast_f64_to_f32(int64_t n, int q, const double* X, int64_t ldx, float* Y, int64_t ldy,
                           hipStream_t s);
hipError_t cast_f32_to_f64(int64_t n, int q, const float* X, int64_t ldx, double* Y, int64_t ldy,
                           hipStream_t s);
// Y[:, :q] = X[:, :q] (any lds)
hipError_t copy_cols_f64(int64_t n, int q, const double* X, int64_t ldx, double* Y, int64_t ldy,
                         hipStream_t s);
// Y[:, :q] -= X[:, :q] (any lds; X and Y must not overlap)
hipError_t sub_cols_f64(int64_t n, int q, const double* X, int64_t ldx, double* Y, int64_t ldy,
                        hipStream_t s);
// Y[:, c] = X[:, perm[c]] (perm a device array of q column indices; X != Y).
hipError_t permute_cols_f64(int64_t n, int q, const double* X, int64_t ld, const int* perm,
                            double* Y, hipStream_t s);
hipError_t zero_f64(double* p, int64_t count, hipStream_t s);
hipError_t zero_f32(float* p, int64_t count, hipStream_t s);
// Standard normal entries for X[r][c], r < n, c < q, from Philox4x32-10
// (Salmon et al., SC'11) with Box-Muller; element (r, c) uses counter r*q + c.
hipError_t gaussian_fill_f64(int64_t n, int q, double* X, int64_t ld, uint64_t seed, hipStream_t s);
// out[s][r] = X[r][sel[s]] * sign_s, sign_s making the largest-|.| entry positive.
hipError_t gather_transpose_signfix(int64_t n, int nsel, const double* X, int64_t ld,
                                    const int* sel, double* out, void* work, hipStream_t s);
// out[r][c] = In[c][r] (transposes an [m][n] contiguous array into [n][ld])
hipError_t transpose_to_rows(int64_t m, int64_t n, const double* in, double* out, int64_t ld,
                             hipStream_t s);

// --------------------------------------------------------- Lanczos helpers
// h[j] = V_j . w for j < m, V stored as m contiguous vectors of length n (stride n).
size_t multidot_work_bytes(int64_t n, int m);
hipError_t multi_dot_f64(int64_t n, int m, const double* V, const double* w, double* h,
                         void* work, hipStream_t s);
// w -= sum_j h[j] V_j
hipError_t multi_axpy_f64(int64_t n, int m, const double* V, const double* h, double* w,
                          hipStream_t s);
// y = a*x + b*y ; and v_out = w / norm (norm read from device)
hipError_t axpby_f64(int64_t n, double a, const double* x, double b, double* y, hipStream_t s);
hipError_t scale_by_inv_f64(int64_t n, const double* x, const double* nrm, double* y,
                            hipStream_t s);

// ---------------------------------------------------------- adjoint (K9-K11)
// G[b] += sum_m w[m] sum_c a_m[3i+p][c] t_m[3j+q][c] for stored b = (i, j), with
// a_m = a + m a_stride, t_m = t + m t_stride ([n][ld] each), w on the device; q <= 256.
hipError_t sddmm_seg_f64(const Bsr& A, int q, int m, const double* a, int64_t a_stride,
                         const double* t, int64_t t_stride, int64_t ld, const double* w,
                         double* G, hipStream_t s);
// G[b] (+)= sum_c colw_c a[3i+p][c] t[3j+q][c] for stored b = (i, j); q <= 256.
hipError_t sddmm_f64(const Bsr& A, int q, const double* a, const double* t, int64_t ld,
                     const double* colw, double* G, bool accumulate, hipStream_t s);
// K blocks of a spring network on a BSR pattern (K_ij = -k u u^T, K_ii = -sum
// of the row's off-diagonal blocks).  err bit 5: pairs out of range or not in
// strictly increasing (i < j) order; bit 6: a block without a spring; bit 0: no
// diagonal block in a row.
hipError_t assemble_springs(int64_t n_atoms, const int64_t* row_ptr, const int32_t* col_idx,
                            int64_t P, const int64_t* pairs, const double* unit, const double* k,
                            double* K, int* err, hipStream_t s);
// dk[p] and dm[i] from block gradients G; err bit 0: a spring's block missing.
hipError_t spring_chain(const Bsr& A, const int32_t* transpose, const double* H,
                        const double* masses, const double* G, int64_t P, const int64_t* pairs,
                        const double* unit, double* dk, double* dm, int* err, hipStream_t s);
hipError_t scale_f64(int64_t count, double a, double* p, hipStream_t s);

// ------------------------------------------------------------- host design
struct FilterDesign {
  int degree = 0;
  int smoothing = 0;
  double c = 0, e = 0, xi = 0, eta = 0, eps = 0, r = 0;
  std::vector<double> coef;
};
Err design_filter(double lam_lo, double lam_hi, double lam_lb, double lam_ub, int degree,
                  double eps, double r, int smoothing, FilterDesign* out);
// Coefficients of the damped Chebyshev series of the characteristic function
// of [a, b] (Sec. 2.4, with the integral of Appendix A eq. app.3).
std::vector<double> chi_coefficients(double a, double b, int degree, int smoothing);
// value of sum_j coef_j T_j(x) for |x| <= 1
double cheb_value(const std::vector<double>& coef, double x);
// Dirac-delta filter of Sec. 2.5 (eq. cheby-delta.1): coefficients, the
// balanced centre gamma, tau = rho(xi) = rho(eta) and the peak rho(gamma).
// degree 0: smallest degree with tau / peak <= phi.
struct DiracDesign {
  int degree = 0;
  int smoothing = 0;
  double c = 0, e = 0, xi = 0, eta = 0, gamma = 0, tau = 0, peak = 0, phi = 0;
  std::vector<double> coef;
};
Err design_dirac(double lam_lo, double lam_hi, double lam_lb, double lam_ub, int degree,
                 double phi, int smoothing, DiracDesign* out);

}  // namespace pfe
