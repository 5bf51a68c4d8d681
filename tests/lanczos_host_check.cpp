// CPU check of the thick-restart block Lanczos solver's host bookkeeping
// (paper_1902_07041_amd/csrc/lanczos_host.cpp): the projected matrix
// T = V^T A V built block by block, the Ritz residual norms read from T, the
// number of kept vectors and T after a thick restart (Sec. 2.5 and Sec. 3).
//
// A dense random symmetric A stands in for rho(H_hat); the basis, the
// products and the small eigenproblems are done here in plain loops, and only
// the bookkeeping comes from the library source.  Built with bounds-checked
// containers and the address and undefined-behaviour sanitisers, so an
// access outside any buffer ends the run.  Prints one line per case and
// "ALL OK" at the end; exit status 1 on the first mismatch.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <vector>

#include "lanczos_host.h"

namespace {

using Vec = std::vector<double>;

struct Rng {
  uint64_t s;
  uint64_t next() {  // splitmix64
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  }
  double uni() { return ((next() >> 11) + 0.5) * (1.0 / 9007199254740992.0); }
  double gauss() { return std::sqrt(-2.0 * std::log(uni())) * std::cos(6.283185307179586 * uni()); }
};

int g_fail = 0;

void expect(bool ok, const char* what, int b, int m, double got = 0, double lim = 0) {
  if (!ok && !g_fail) {
    std::printf("FAIL b=%d m=%d: %s (%.3e > %.3e)\n", b, m, what, got, lim);
    g_fail = 1;
  }
}

// column c of a row-major [n][ld] array
double dot_cols(const Vec& X, int ldx, int cx, const Vec& Y, int ldy, int cy, int n) {
  double s = 0;
  for (int r = 0; r < n; ++r) s += X[(size_t)r * ldx + cx] * Y[(size_t)r * ldy + cy];
  return s;
}

// y[:, cy] = A x[:, cx] for the dense row-major A [n][n]
void matvec(const Vec& A, int n, const Vec& X, int ldx, int cx, Vec& Y, int ldy, int cy) {
  for (int r = 0; r < n; ++r) {
    double s = 0;
    for (int j = 0; j < n; ++j) s += A[(size_t)r * n + j] * X[(size_t)j * ldx + cx];
    Y[(size_t)r * ldy + cy] = s;
  }
}

// Columns [p, p + b) of V: projected twice against columns [0, p), then
// orthonormalised among themselves by modified Gram-Schmidt, twice.
void orth_block(Vec& V, int ld, int n, int p, int b) {
  for (int pass = 0; pass < 2; ++pass)
    for (int c = p; c < p + b; ++c)
      for (int j = 0; j < p; ++j) {
        const double h = dot_cols(V, ld, j, V, ld, c, n);
        for (int r = 0; r < n; ++r) V[(size_t)r * ld + c] -= h * V[(size_t)r * ld + j];
      }
  for (int pass = 0; pass < 2; ++pass)
    for (int c = p; c < p + b; ++c) {
      for (int j = p; j < c; ++j) {
        const double h = dot_cols(V, ld, j, V, ld, c, n);
        for (int r = 0; r < n; ++r) V[(size_t)r * ld + c] -= h * V[(size_t)r * ld + j];
      }
      const double nr = std::sqrt(dot_cols(V, ld, c, V, ld, c, n));
      for (int r = 0; r < n; ++r) V[(size_t)r * ld + c] /= nr;
    }
}

// Cyclic Jacobi: S [m][m] symmetric -> eigenvalues ascending in th, the
// eigenvectors in the columns of Q (row-major).
void jacobi(const Vec& S0, int m, Vec& th, Vec& Q) {
  Vec S = S0, U((size_t)m * m, 0.0);
  for (int i = 0; i < m; ++i) U[(size_t)i * m + i] = 1.0;
  for (int sweep = 0; sweep < 60; ++sweep) {
    double off = 0, tot = 0;
    for (int i = 0; i < m; ++i)
      for (int j = 0; j < m; ++j) {
        const double v = S[(size_t)i * m + j] * S[(size_t)i * m + j];
        tot += v;
        if (i != j) off += v;
      }
    if (off <= 1e-30 * tot) break;
    for (int p = 0; p < m; ++p)
      for (int q = p + 1; q < m; ++q) {
        const double apq = S[(size_t)p * m + q];
        if (apq == 0.0) continue;
        const double tau = (S[(size_t)q * m + q] - S[(size_t)p * m + p]) / (2 * apq);
        const double t = (tau >= 0 ? 1.0 : -1.0) / (std::fabs(tau) + std::sqrt(1 + tau * tau));
        const double c = 1 / std::sqrt(1 + t * t), s = t * c;
        for (int k = 0; k < m; ++k) {  // S <- S J
          const double a = S[(size_t)k * m + p], bq = S[(size_t)k * m + q];
          S[(size_t)k * m + p] = c * a - s * bq;
          S[(size_t)k * m + q] = s * a + c * bq;
        }
        for (int k = 0; k < m; ++k) {  // S <- J^T S
          const double a = S[(size_t)p * m + k], bq = S[(size_t)q * m + k];
          S[(size_t)p * m + k] = c * a - s * bq;
          S[(size_t)q * m + k] = s * a + c * bq;
        }
        for (int k = 0; k < m; ++k) {  // U <- U J
          const double a = U[(size_t)k * m + p], bq = U[(size_t)k * m + q];
          U[(size_t)k * m + p] = c * a - s * bq;
          U[(size_t)k * m + q] = s * a + c * bq;
        }
      }
  }
  std::vector<int> idx(m);
  for (int i = 0; i < m; ++i) idx[i] = i;
  std::sort(idx.begin(), idx.end(),
            [&](int a, int b) { return S[(size_t)a * m + a] < S[(size_t)b * m + b]; });
  th.assign(m, 0.0);
  Q.assign((size_t)m * m, 0.0);
  for (int i = 0; i < m; ++i) {
    th[i] = S[(size_t)idx[i] * m + idx[i]];
    for (int r = 0; r < m; ++r) Q[(size_t)r * m + i] = U[(size_t)r * m + idx[i]];
  }
}

// Three restart cycles of the solver's host sequence on a dense A.
void run_case(int b, int m, uint64_t seed) {
  pfe::LanczosShape s;
  expect(pfe::lanczos_shape(m, b, &s) == 0, "valid shape rejected", b, m);
  if (g_fail) return;
  const int M1 = s.M1;
  const int n = std::max(3 * M1 + 17, 64);
  const int ld = M1;
  Rng rng{seed};
  Vec A((size_t)n * n);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j <= i; ++j) A[(size_t)i * n + j] = A[(size_t)j * n + i] = rng.gauss() / std::sqrt(n);
  double anorm = 0;
  for (double v : A) anorm += v * v;
  anorm = std::sqrt(anorm);
  const double tol = 1e-11 * anorm;

  Vec V((size_t)n * ld, 0.0), W((size_t)n * b), T((size_t)M1 * M1, 0.0), Cf((size_t)M1 * b);
  Vec Tm((size_t)m * m), th, Q, rA(m), Mk;
  for (int r = 0; r < n; ++r)
    for (int c = 0; c < b; ++c) V[(size_t)r * ld + c] = rng.gauss();
  orth_block(V, ld, n, 0, b);
  int p = b;
  double worst_T = 0, worst_r = 0, worst_R = 0;
  for (int cycle = 0; cycle < 3 && !g_fail; ++cycle) {
    while (p < m + b) {
      for (int c = 0; c < b; ++c) matvec(A, n, V, ld, p - b + c, W, b, c);
      for (int r = 0; r < n; ++r)
        for (int c = 0; c < b; ++c) V[(size_t)r * ld + p + c] = W[(size_t)r * b + c];
      orth_block(V, ld, n, p, b);
      for (int r = 0; r < p + b; ++r)
        for (int c = 0; c < b; ++c) Cf[(size_t)r * b + c] = dot_cols(V, ld, r, W, b, c, n);
      expect(pfe::lanczos_store_block(s, p, Cf, T) == 0, "store_block", b, m);
      p += b;
    }
    // T[:, 0:m] against V^T A V
    Vec AV((size_t)n * m);
    for (int c = 0; c < m; ++c) matvec(A, n, V, ld, c, AV, m, c);
    for (int r = 0; r < M1; ++r)
      for (int c = 0; c < m; ++c)
        worst_T = std::max(worst_T, std::fabs(T[(size_t)r * M1 + c] - dot_cols(V, ld, r, AV, m, c, n)));
    expect(worst_T <= tol, "T != V^T A V", b, m, worst_T, tol);
    expect(pfe::lanczos_leading(s, T, Tm) == 0, "leading", b, m);
    jacobi(Tm, m, th, Q);
    expect(pfe::lanczos_ritz_residuals(s, T, Q, rA) == 0, "ritz_residuals", b, m);
    // rA[i] against || A y_i - theta_i y_i ||, y_i = V[:, 0:m] Q[:, i]
    for (int i = 0; i < m; ++i) {
      double s2 = 0;
      for (int r = 0; r < n; ++r) {
        double y = 0, ay = 0;
        for (int j = 0; j < m; ++j) {
          y += V[(size_t)r * ld + j] * Q[(size_t)j * m + i];
          ay += AV[(size_t)r * m + j] * Q[(size_t)j * m + i];
        }
        s2 += (ay - th[i] * y) * (ay - th[i] * y);
      }
      worst_r = std::max(worst_r, std::fabs(std::sqrt(s2) - rA[i]));
    }
    expect(worst_r <= 1e2 * tol, "Ritz residual from T", b, m, worst_r, 1e2 * tol);
    // kept vectors for a wanted count that changes with the cycle
    const int nw = (cycle * 7 + b + 1) % (m - 2 * b + 1);
    const int k = pfe::lanczos_keep(s, nw);
    expect(k % b == 0 && k >= nw + b && k >= 2 * b && k <= m - b, "keep", b, m, k, m - b);
    expect(pfe::lanczos_keep(s, m - 2 * b + 1) == -1, "keep beyond capacity", b, m);
    if (g_fail) return;
    std::vector<int> cols(k);
    for (int c = 0; c < k; ++c) cols[c] = m - 1 - c;
    expect(pfe::lanczos_select_columns(s, Q, cols, Mk) == 0, "select_columns", b, m);
    Vec Vn((size_t)n * ld, 0.0);
    for (int r = 0; r < n; ++r) {
      for (int c = 0; c < k; ++c) {
        double v = 0;
        for (int j = 0; j < m; ++j) v += V[(size_t)r * ld + j] * Mk[(size_t)j * k + c];
        Vn[(size_t)r * ld + c] = v;
      }
      for (int a = 0; a < b; ++a) Vn[(size_t)r * ld + k + a] = V[(size_t)r * ld + m + a];
    }
    V.swap(Vn);
    expect(pfe::lanczos_restart(s, k, th, Q, T) == 0, "restart", b, m);
    // the arrow matrix against Vn^T A Vn: leading k x k and the coupling rows
    Vec AVk((size_t)n * k);
    for (int c = 0; c < k; ++c) matvec(A, n, V, ld, c, AVk, k, c);
    for (int r = 0; r < k + b; ++r)
      for (int c = 0; c < k; ++c)
        worst_R = std::max(worst_R, std::fabs(T[(size_t)r * M1 + c] - dot_cols(V, ld, r, AVk, k, c, n)));
    expect(worst_R <= 1e2 * tol, "restarted T != V^T A V", b, m, worst_R, 1e2 * tol);
    p = k + b;
  }
  if (!g_fail)
    std::printf("b=%d m=%d n=%d: T %.1e, Ritz residuals %.1e, restart %.1e (|A|_F %.2f)\n", b, m, n,
                worst_T, worst_r, worst_R, anorm);
}

// Out-of-range shapes and short inputs come back as codes, touching nothing.
void rejections() {
  pfe::LanczosShape s;
  const int bad[][2] = {{8, 0}, {8, 65}, {20, 8}, {16, 8}, {504, 8}, {0, 1}, {2, 1}};
  for (auto& mb : bad) expect(pfe::lanczos_shape(mb[0], mb[1], &s) != 0, "bad shape accepted", mb[1], mb[0]);
  expect(pfe::lanczos_shape(48, 8, nullptr) != 0, "null shape", 8, 48);
  expect(pfe::lanczos_shape(48, 8, &s) == 0, "shape 8/48", 8, 48);
  Vec T((size_t)s.M1 * s.M1), C((size_t)s.M1 * s.b), Q((size_t)s.m * s.m), th(s.m), rA(s.m), M;
  expect(pfe::lanczos_store_block(s, 0, C, T) == 1, "store p = 0", 8, 48);
  expect(pfe::lanczos_store_block(s, 52, C, T) == 1, "store p not a multiple", 8, 48);
  expect(pfe::lanczos_store_block(s, 56, C, T) == 1, "store p > m", 8, 48);
  Vec Cs((size_t)(48 + 8) * 8 - 1), Ts(T.size() - 1);
  expect(pfe::lanczos_store_block(s, 48, Cs, T) == 2, "store short C", 8, 48);
  expect(pfe::lanczos_store_block(s, 48, C, Ts) == 2, "store short T", 8, 48);
  Vec Qs(Q.size() - 1), rAs(s.m - 1), ths(s.m - 1);
  expect(pfe::lanczos_ritz_residuals(s, T, Qs, rA) == 2, "residuals short Q", 8, 48);
  expect(pfe::lanczos_ritz_residuals(s, T, Q, rAs) == 2, "residuals short rA", 8, 48);
  expect(pfe::lanczos_select_columns(s, Q, {0, 48}, M) == 1, "column index m", 8, 48);
  expect(pfe::lanczos_select_columns(s, Q, {-1}, M) == 1, "column index -1", 8, 48);
  expect(pfe::lanczos_restart(s, 0, th, Q, T) == 1, "restart k = 0", 8, 48);
  expect(pfe::lanczos_restart(s, 41, th, Q, T) == 1, "restart k > m - b", 8, 48);
  expect(pfe::lanczos_restart(s, 16, ths, Q, T) == 2, "restart short th", 8, 48);
  expect(pfe::lanczos_keep(s, -1) == -1, "keep -1", 8, 48);
  if (!g_fail) std::printf("rejections: ok\n");
}

}  // namespace

int main() {
  rejections();
  const int cases[][2] = {{1, 3}, {1, 8}, {2, 12}, {4, 16}, {4, 40}, {8, 24}, {8, 48},
                          {16, 48}, {16, 64}, {24, 144}, {32, 96}, {64, 192}};
  uint64_t seed = 1;
  for (auto& c : cases) {
    if (g_fail) break;
    run_case(c[0], c[1], seed++);
  }
  if (g_fail) return 1;
  std::printf("ALL OK\n");
  return 0;
}
