// Host-side bookkeeping of the thick-restart block Lanczos solver (Sec. 2.5
// and Sec. 3); see lanczos_host.h.
#include "lanczos_host.h"

#include <algorithm>
#include <cmath>
#include <cstddef>

namespace pfe {

namespace {

constexpr int kBadShape = 1;
constexpr int kShort = 2;

bool valid(const LanczosShape& s) {
  return s.b >= 1 && s.b <= 64 && s.m % s.b == 0 && s.m >= 3 * s.b && s.M1 == s.m + s.b &&
         s.M1 <= 511;
}

size_t sq(int a) { return (size_t)a * (size_t)a; }

}  // namespace

int lanczos_shape(int m, int b, LanczosShape* s) {
  if (!s) return kBadShape;
  LanczosShape t;
  t.m = m;
  t.b = b;
  t.M1 = m + b;
  if (!valid(t)) return kBadShape;
  *s = t;
  return 0;
}

int lanczos_store_block(const LanczosShape& s, int p, const std::vector<double>& C,
                        std::vector<double>& T) {
  if (!valid(s) || p < s.b || p > s.m || p % s.b != 0) return kBadShape;
  const int rows = p + s.b;
  if (C.size() < (size_t)rows * s.b || T.size() < sq(s.M1)) return kShort;
  for (int r = 0; r < rows; ++r)
    for (int c = 0; c < s.b; ++c) {
      const double v = C[(size_t)r * s.b + c];
      T[(size_t)r * s.M1 + (p - s.b + c)] = v;
      T[(size_t)(p - s.b + c) * s.M1 + r] = v;
    }
  return 0;
}

int lanczos_leading(const LanczosShape& s, const std::vector<double>& T, std::vector<double>& Tm) {
  if (!valid(s)) return kBadShape;
  if (T.size() < sq(s.M1) || Tm.size() < sq(s.m)) return kShort;
  for (int r = 0; r < s.m; ++r)
    for (int c = 0; c < s.m; ++c) Tm[(size_t)r * s.m + c] = T[(size_t)r * s.M1 + c];
  return 0;
}

int lanczos_ritz_residuals(const LanczosShape& s, const std::vector<double>& T,
                           const std::vector<double>& Q, std::vector<double>& rA) {
  if (!valid(s)) return kBadShape;
  const int m = s.m, b = s.b;
  if (T.size() < sq(s.M1) || Q.size() < sq(m) || rA.size() < (size_t)m) return kShort;
  for (int i = 0; i < m; ++i) {
    double s2 = 0;
    for (int a = 0; a < b; ++a) {
      double v = 0;
      for (int r = 0; r < b; ++r)
        v += T[(size_t)(m + a) * s.M1 + (m - b + r)] * Q[(size_t)(m - b + r) * m + i];
      s2 += v * v;
    }
    rA[i] = std::sqrt(s2);
  }
  return 0;
}

int lanczos_keep(const LanczosShape& s, int nw) {
  if (!valid(s) || nw < 0 || nw > s.m - 2 * s.b) return -1;
  const int want = std::max(nw + s.b, 2 * s.b);
  const int k = (want + s.b - 1) / s.b * s.b;
  return std::min(s.m - s.b, k);
}

int lanczos_select_columns(const LanczosShape& s, const std::vector<double>& Q,
                           const std::vector<int>& cols, std::vector<double>& M) {
  if (!valid(s)) return kBadShape;
  const int m = s.m;
  const size_t nc = cols.size();
  if (Q.size() < sq(m)) return kShort;
  for (int c : cols)
    if (c < 0 || c >= m) return kBadShape;
  M.assign((size_t)m * nc, 0.0);
  for (int r = 0; r < m; ++r)
    for (size_t c = 0; c < nc; ++c) M[(size_t)r * nc + c] = Q[(size_t)r * m + cols[c]];
  return 0;
}

int lanczos_restart(const LanczosShape& s, int k, const std::vector<double>& th,
                    const std::vector<double>& Q, std::vector<double>& T) {
  if (!valid(s) || k < 1 || k > s.m - s.b) return kBadShape;
  const int m = s.m, b = s.b, M1 = s.M1;
  if (th.size() < (size_t)m || Q.size() < sq(m) || T.size() < sq(M1)) return kShort;
  std::vector<double> Tn(sq(M1), 0.0);
  for (int c = 0; c < k; ++c) Tn[(size_t)c * M1 + c] = th[m - 1 - c];
  for (int a = 0; a < b; ++a)
    for (int c = 0; c < k; ++c) {
      double v = 0;
      for (int r = 0; r < b; ++r)
        v += T[(size_t)(m + a) * M1 + (m - b + r)] * Q[(size_t)(m - b + r) * m + (m - 1 - c)];
      Tn[(size_t)(k + a) * M1 + c] = v;
      Tn[(size_t)c * M1 + (k + a)] = v;
    }
  T.swap(Tn);
  return 0;
}

}  // namespace pfe
