/* Plain block-CSR (3x3) times dense block product for the CPU oracle.
 *
 * TEST INFRASTRUCTURE ONLY.  Y[3i+a][c] = sum_{b in row i} sum_k V[b][a][k] X[3 col[b] + k][c]
 * for row-major X, Y of width q: the textbook definition, one OpenMP thread
 * per range of block rows, no blocking or reordering of the sums within a row.
 */
#include <stdint.h>

void oracle_bsr3_matmul(int64_t n_atoms, const int64_t* row_ptr, const int64_t* col_idx,
                        const double* vals, const double* X, double* Y, int64_t q) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n_atoms; ++i) {
    for (int a = 0; a < 3; ++a)
      for (int64_t c = 0; c < q; ++c) Y[(3 * i + a) * q + c] = 0.0;
    for (int64_t b = row_ptr[i]; b < row_ptr[i + 1]; ++b) {
      const int64_t j = col_idx[b];
      const double* v = vals + 9 * b;
      for (int a = 0; a < 3; ++a)
        for (int k = 0; k < 3; ++k) {
          const double h = v[3 * a + k];
          const double* x = X + (3 * j + k) * q;
          double* y = Y + (3 * i + a) * q;
          for (int64_t c = 0; c < q; ++c) y[c] += h * x[c];
        }
    }
  }
}
