// Host-side bookkeeping of the thick-restart block Lanczos solver on the
// Dirac-delta filter (Sec. 2.5 and Sec. 3): the projected matrix
// T = V^T rho(H_hat) V of the basis V, its Ritz residuals and its form after a
// thick restart.  Plain C++ (no HIP), so the same code is checked by a CPU
// build with bounds-checked containers and address sanitising.
//
// Every routine checks the indices it is about to touch against the sizes
// it was given and returns a nonzero code instead of reading or writing
// outside them: 1 for a shape outside the documented range, 2 for an input
// shorter than the shape requires.
#pragma once

#include <vector>

namespace pfe {

// A basis of m columns followed by one residual block of b: T is [M1][M1],
// M1 = m + b, row-major.
struct LanczosShape {
  int m = 0, b = 0, M1 = 0;
};

// 0 when 1 <= b <= 64, m is a multiple of b, 3b <= m and m + b <= 511.
int lanczos_shape(int m, int b, LanczosShape* s);

// Stores columns [p - b, p) of T, and the same rows by symmetry, from the
// Gram block C[r][c] = v_r . rho(H_hat) v_{p-b+c} for r < p + b (row-major,
// b columns).  p is a multiple of b in [b, m].
int lanczos_store_block(const LanczosShape& s, int p, const std::vector<double>& C,
                        std::vector<double>& T);

// Tm [m][m] = leading m x m part of T.
int lanczos_leading(const LanczosShape& s, const std::vector<double>& T, std::vector<double>& Tm);

// rA[i] = || B Q[m-b:m, i] ||, B = T[m:m+b, m-b:m]: with the eigenvectors Q
// ([m][m], row-major, column i for Ritz value i) of the leading m x m part,
// the norm of rho(H_hat) y_i - theta_i y_i for y_i = V[:, 0:m] Q[:, i].
int lanczos_ritz_residuals(const LanczosShape& s, const std::vector<double>& T,
                           const std::vector<double>& Q, std::vector<double>& rA);

// Ritz vectors kept at a restart when nw are wanted: a multiple of b, at
// least nw + b and 2b, at most m - b.  Returns -1 when nw > m - 2b (the
// basis cannot hold the wanted vectors and a residual block).
int lanczos_keep(const LanczosShape& s, int nw);

// M [m][cols.size()] with M[r][c] = Q[r][cols[c]].
int lanczos_select_columns(const LanczosShape& s, const std::vector<double>& Q,
                           const std::vector<int>& cols, std::vector<double>& M);

// T after a thick restart that keeps the k largest Ritz pairs (theta
// ascending in th[m], eigenvectors in the columns of Q) as the new columns
// 0..k-1, largest first, and moves the residual block to columns k..k+b-1:
// diag(th[m-1], ..., th[m-k]) in the leading k x k block, the coupling
// B Q[m-b:m, m-1-c] in rows and columns k..k+b-1, zero elsewhere.
int lanczos_restart(const LanczosShape& s, int k, const std::vector<double>& th,
                    const std::vector<double>& Q, std::vector<double>& T);

}  // namespace pfe
