// CPU check of the row orders the fused filter step's tiles are built in
// (paper_1902_07041_amd/csrc/reorder.cpp): the windowed regrouping of the
// natural order, the locality order, and the two pattern statistics that
// choose between them.
//
// Patterns are periodic cubic lattices with every site within distance sqrt(2)
// as a neighbour (18 neighbours plus the diagonal), optionally with vacancies
// removed and the remaining sites renumbered in lattice order, and a ring.
// Built with bounds-checked containers and the address and undefined-
// behaviour sanitisers, so an access outside any buffer ends the run.  Prints
// one line per case and "ALL OK" at the end; exit status 1 if any check
// failed.
#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <set>
#include <vector>

#include "reorder.h"

namespace {

struct Pattern {
  int64_t n = 0;
  std::vector<int64_t> rp{0};
  std::vector<int32_t> ci;
};

int fails = 0;

void check(bool ok, const char* what) {
  if (!ok) {
    std::printf("FAIL: %s\n", what);
    ++fails;
  }
}

// L^3 lattice, x fastest; every `hole`-th site (hole > 0) left empty.
Pattern lattice(int L, int hole) {
  std::vector<int64_t> atom((size_t)L * L * L, -1);
  int64_t n = 0;
  for (int64_t s = 0; s < (int64_t)L * L * L; ++s)
    if (hole <= 0 || s % hole != 3) atom[s] = n++;
  Pattern p;
  p.n = n;
  for (int z = 0; z < L; ++z)
    for (int y = 0; y < L; ++y)
      for (int x = 0; x < L; ++x) {
        const int64_t a = atom[((int64_t)z * L + y) * L + x];
        if (a < 0) continue;
        std::vector<int32_t> cols;
        for (int dz = -1; dz <= 1; ++dz)
          for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
              if (dx * dx + dy * dy + dz * dz > 2) continue;
              const int64_t b = atom[(((int64_t)(z + dz + L) % L) * L + (y + dy + L) % L) * L +
                                     (x + dx + L) % L];
              if (b >= 0) cols.push_back((int32_t)b);
            }
        std::sort(cols.begin(), cols.end());
        cols.erase(std::unique(cols.begin(), cols.end()), cols.end());
        p.ci.insert(p.ci.end(), cols.begin(), cols.end());
        p.rp.push_back((int64_t)p.ci.size());
      }
  return p;
}

Pattern ring(int n) {
  Pattern p;
  p.n = n;
  for (int i = 0; i < n; ++i) {
    std::vector<int32_t> c{(i + n - 1) % n, i, (i + 1) % n};
    std::sort(c.begin(), c.end());
    c.erase(std::unique(c.begin(), c.end()), c.end());
    p.ci.insert(p.ci.end(), c.begin(), c.end());
    p.rp.push_back((int64_t)p.ci.size());
  }
  return p;
}

bool is_permutation_of_range(const std::vector<int32_t>& o, size_t from, size_t to, int64_t lo) {
  std::vector<int32_t> s(o.begin() + (long)from, o.begin() + (long)to);
  std::sort(s.begin(), s.end());
  for (size_t i = 0; i < s.size(); ++i)
    if (s[i] != lo + (int64_t)i) return false;
  return true;
}

// Distinct block columns of tiles of R consecutive rows in `order`, per row.
double union_per_row(const Pattern& p, const std::vector<int32_t>& order, int R) {
  int64_t tot = 0;
  for (size_t t = 0; t < order.size(); t += (size_t)R) {
    std::set<int32_t> u;
    for (size_t r = t; r < std::min(order.size(), t + (size_t)R); ++r)
      for (int64_t k = p.rp[order[r]]; k < p.rp[order[r] + 1]; ++k) u.insert(p.ci[k]);
    tot += (int64_t)u.size();
  }
  return p.n > 0 ? (double)tot / (double)p.n : 0.0;
}

void check_window(const Pattern& p, int64_t window, int R, const char* name) {
  std::vector<int32_t> o;
  pfe::window_group_order(p.n, p.rp.data(), p.ci.data(), window, R, o);
  const int Rc = std::max(R, 1);
  const int64_t W = std::max<int64_t>(Rc, (window + Rc - 1) / Rc * Rc);
  bool ok = (int64_t)o.size() == p.n && is_permutation_of_range(o, 0, o.size(), 0);
  bool in_window = true, seeds = true;
  for (int64_t a = 0; a < p.n && ok; a += W) {
    const int64_t b = std::min(p.n, a + W);
    in_window = in_window && is_permutation_of_range(o, (size_t)a, (size_t)b, a);
    // every group starts at the lowest row of its window not in an earlier group
    std::vector<char> used((size_t)(b - a), 0);
    for (int64_t g = a; g < b; g += Rc) {
      int64_t first = a;
      while (first < b && used[(size_t)(first - a)]) ++first;
      seeds = seeds && o[(size_t)g] == first;
      for (int64_t r = g; r < std::min(b, g + Rc); ++r)
        if (o[(size_t)r] >= a && o[(size_t)r] < b) used[(size_t)(o[(size_t)r] - a)] = 1;
    }
  }
  std::vector<int32_t> nat((size_t)p.n);
  for (int64_t i = 0; i < p.n; ++i) nat[(size_t)i] = (int32_t)i;
  const double un = union_per_row(p, nat, Rc), uw = ok ? union_per_row(p, o, Rc) : 0.0;
  std::printf("window %s n=%lld W=%lld R=%d: union per row %.3f (natural %.3f)\n", name,
              (long long)p.n, (long long)window, R, uw, un);
  check(ok, "window order is a permutation");
  check(in_window, "rows stay in their window");
  check(seeds, "groups start at the first free row of the window");
  if (R >= 3 && p.n >= 1000 && window >= 64)   // a window of R rows is the natural grouping
    check(uw < un, "regrouping shares more block columns");
  if (R <= 1) check(o == nat, "R = 1 keeps the natural order");
}

}  // namespace

int main() {
  const Pattern cube = lattice(12, 0);       // 1728 sites
  const Pattern holes = lattice(13, 29);     // 2197 sites, every 29th empty
  const Pattern small = lattice(3, 0);
  for (int R : {1, 2, 3, 4})
    for (int64_t W : {1, 64, 1000, 4096}) {
      check_window(cube, W, R, "cube");
      check_window(holes, W, R, "holes");
    }
  check_window(small, 16, 4, "small");
  Pattern empty;
  check_window(empty, 16, 4, "empty");
  const Pattern one = ring(1);
  check_window(one, 16, 4, "one");
  const Pattern r5 = ring(5);
  check_window(r5, 3, 4, "ring5");

  for (int R : {1, 2, 4}) {
    std::vector<int32_t> o;
    pfe::locality_order(holes.n, holes.rp.data(), holes.ci.data(), 64, R, o);
    const bool ok = (int64_t)o.size() == holes.n && is_permutation_of_range(o, 0, o.size(), 0);
    std::printf("locality holes R=%d: permutation %d\n", R, (int)ok);
    check(ok, "locality order is a permutation");
  }

  // a ring: every off-diagonal offset is 1, except the wrap-around (n - 1),
  // which the span leaves out
  const Pattern r40 = ring(40);
  const int64_t span = pfe::neighbour_span(r40.n, r40.rp.data(), r40.ci.data());
  const double far0 = pfe::far_block_fraction(r40.n, r40.rp.data(), r40.ci.data(), nullptr, 0);
  const double far1 = pfe::far_block_fraction(r40.n, r40.rp.data(), r40.ci.data(), nullptr, 1);
  std::printf("ring40: span %lld far(0) %.3f far(1) %.3f\n", (long long)span, far0, far1);
  check(span == 1, "ring span is 1");
  check(far0 == 1.0, "every off-diagonal block is beyond window 0");
  check(far1 == 2.0 / 80.0, "only the two wrap-around blocks are beyond window 1");

  if (fails) return 1;
  std::printf("ALL OK\n");
  return 0;
}
