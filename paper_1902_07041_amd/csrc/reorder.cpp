// Locality order of the atom graph for the fused filter step's row tiles.
//
// The filter step gathers, for every output atom row, the T_in rows of its
// neighbours.  Which XCD processes a row, and when, decides how often a T_in
// row leaves HBM: a neighbour gathered by another XCD, or long after it left
// this XCD's L2, is fetched again.  Rows are therefore taken in an order in
// which every contiguous range is a compact region of the graph, found by
// recursive bisection at breadth-first-search levels: a range is ordered by
// BFS from a pseudo-peripheral vertex (found by a first BFS), so the first
// half is a ball around that vertex and the second half the rest, and each
// half is ordered the same way until ranges reach `leaf` vertices.  Inside
// a leaf the rows are grouped R at a time (one tile each) by largest overlap
// of their block columns, so a tile's gathers are shared as much as in
// consecutive rows of a lattice-like order.  Only
// the order of work changes: atoms keep their indices, so no vector is
// permuted.  Cost O(nnzb log(n / leaf)) on the host, once per pattern.
#include <algorithm>
#include <cstdint>
#include <cstdlib>
#include <utility>
#include <vector>

#include "reorder.h"

namespace pfe {

// Common columns of two sorted column lists.
static int overlap(const int32_t* a, int64_t na, const int32_t* b, int64_t nb) {
  int c = 0;
  int64_t i = 0, j = 0;
  while (i < na && j < nb) {
    if (a[i] < b[j])
      ++i;
    else if (b[j] < a[i])
      ++j;
    else {
      ++c;
      ++i;
      ++j;
    }
  }
  return c;
}

void locality_order(int64_t n, const int64_t* row_ptr, const int32_t* col_idx, int leaf, int R,
                    std::vector<int32_t>& order) {
  order.resize((size_t)n);
  for (int64_t i = 0; i < n; ++i) order[i] = (int32_t)i;
  if (n <= 2) return;
  R = std::max(R, 1);
  leaf = std::max(leaf, 2 * R);
  std::vector<int32_t> part((size_t)n, 0);   // id of the range a vertex belongs to
  std::vector<int32_t> seen((size_t)n, -1);  // id of the last BFS that reached it
  std::vector<int32_t> queue;
  queue.reserve((size_t)n);
  int32_t next_part = 1, next_bfs = 0;
  // Breadth-first order of the vertices of range [a, b) (tagged `pid`), from
  // `start`; unreached vertices start new searches in their current order.
  // Returns the last vertex reached from `start`'s own component.
  auto bfs = [&](int64_t a, int64_t b, int32_t pid, int32_t start) -> int32_t {
    const int32_t id = next_bfs++;
    queue.clear();
    int32_t last = start;
    int64_t scan = a;
    int32_t src = start;
    for (;;) {
      size_t head = queue.size();
      seen[src] = id;
      queue.push_back(src);
      while (head < queue.size()) {
        const int32_t v = queue[head++];
        for (int64_t k = row_ptr[v]; k < row_ptr[v + 1]; ++k) {
          const int32_t w = col_idx[k];
          if (part[w] == pid && seen[w] != id) {
            seen[w] = id;
            queue.push_back(w);
          }
        }
      }
      if (src == start) last = queue.back();
      if ((int64_t)queue.size() == b - a) break;
      while (seen[order[scan]] == id) ++scan;
      src = order[scan];
    }
    return last;
  };
  // Groups of R consecutive rows become one tile: inside a leaf range, each
  // group starts at the first free row and grows by the free neighbour (in
  // the leaf) that shares the most block columns with it.
  std::vector<int32_t> grouped;
  auto group_leaf = [&](int64_t a, int64_t b, int32_t pid) {
    if (R < 2) return;
    for (int64_t i = a; i < b; ++i) part[order[i]] = pid;   // pid marks "free, in this leaf"
    grouped.clear();
    for (int64_t i = a; i < b; ++i) {
      const int32_t v0 = order[i];
      if (part[v0] != pid) continue;
      part[v0] = 0;
      grouped.push_back(v0);
      const size_t g0 = grouped.size() - 1;
      while ((int64_t)(grouped.size() - g0) < R) {
        int32_t best = -1, best_ov = -1;
        for (size_t gi = g0; gi < grouped.size(); ++gi) {
          const int32_t u = grouped[gi];
          for (int64_t k = row_ptr[u]; k < row_ptr[u + 1]; ++k) {
            const int32_t w = col_idx[k];
            if (part[w] != pid) continue;
            int ov = 0;
            for (size_t gj = g0; gj < grouped.size(); ++gj) {
              const int32_t x = grouped[gj];
              ov += overlap(col_idx + row_ptr[x], row_ptr[x + 1] - row_ptr[x], col_idx + row_ptr[w],
                            row_ptr[w + 1] - row_ptr[w]);
            }
            if (ov > best_ov || (ov == best_ov && w < best)) {
              best_ov = ov;
              best = w;
            }
          }
        }
        if (best < 0) break;   // no free neighbour: the group is completed below
        part[best] = 0;
        grouped.push_back(best);
      }
      if ((int64_t)(grouped.size() - g0) < R) {   // fill with the next free rows in order
        for (int64_t j = i + 1; j < b && (int64_t)(grouped.size() - g0) < R; ++j)
          if (part[order[j]] == pid) {
            part[order[j]] = 0;
            grouped.push_back(order[j]);
          }
      }
    }
    std::copy(grouped.begin(), grouped.end(), order.begin() + a);
  };
  std::vector<std::pair<int64_t, int64_t>> ranges{{0, n}}, next;
  while (!ranges.empty()) {
    next.clear();
    for (const auto& r : ranges) {
      const int64_t a = r.first, b = r.second;
      const int32_t pid = next_part++;
      if (b - a <= leaf) {
        group_leaf(a, b, pid);
        continue;
      }
      for (int64_t i = a; i < b; ++i) part[order[i]] = pid;
      const int32_t far = bfs(a, b, pid, order[a]);
      bfs(a, b, pid, far);
      std::copy(queue.begin(), queue.end(), order.begin() + a);
      // split at a multiple of R so that tiles never straddle two ranges
      const int64_t mid = a + std::max<int64_t>(R, ((b - a) / 2 / R) * R);
      next.emplace_back(a, mid);
      next.emplace_back(mid, b);
    }
    ranges.swap(next);
  }
}

void window_group_order(int64_t n, const int64_t* row_ptr, const int32_t* col_idx,
                        int64_t window, int R, std::vector<int32_t>& order) {
  order.clear();
  order.reserve((size_t)std::max<int64_t>(n, 0));
  R = std::max(R, 1);
  window = std::max<int64_t>(R, (window + R - 1) / R * R);
  std::vector<char> taken((size_t)std::max<int64_t>(n, 0), 0);
  std::vector<int32_t> mark((size_t)std::max<int64_t>(n, 0), -1);   // group stamp of union columns
  std::vector<int32_t> cand((size_t)std::max<int64_t>(n, 0), -1);   // step stamp of visited candidates
  std::vector<int32_t> group;
  int32_t gstamp = 0, cstamp = 0;
  for (int64_t a = 0; a < n; a += window) {
    const int64_t b = std::min(n, a + window);
    int64_t next_free = a;   // rows only ever become taken, so this only moves forward
    for (int64_t v0 = a; v0 < b; ++v0) {
      if (taken[v0]) continue;
      ++gstamp;
      group.assign(1, (int32_t)v0);
      taken[v0] = 1;
      for (int64_t k = row_ptr[v0]; k < row_ptr[v0 + 1]; ++k) mark[col_idx[k]] = gstamp;
      while ((int)group.size() < R) {
        ++cstamp;
        int32_t best = -1;
        int64_t best_new = 0, best_ov = 0;
        for (size_t gi = 0; gi < group.size(); ++gi) {
          const int32_t u = group[gi];
          for (int64_t k = row_ptr[u]; k < row_ptr[u + 1]; ++k) {
            const int32_t w = col_idx[k];
            if (w < a || w >= b || taken[w] || cand[w] == cstamp) continue;
            cand[w] = cstamp;
            int64_t ov = 0;
            for (int64_t kk = row_ptr[w]; kk < row_ptr[w + 1]; ++kk) ov += mark[col_idx[kk]] == gstamp;
            const int64_t nw = (row_ptr[w + 1] - row_ptr[w]) - ov;
            if (best < 0 || nw < best_new || (nw == best_new && (ov > best_ov ||
                                                                 (ov == best_ov && w < best)))) {
              best = w;
              best_new = nw;
              best_ov = ov;
            }
          }
        }
        if (best < 0) {   // no free neighbour in the window: the next free row
          next_free = std::max<int64_t>(next_free, v0 + 1);
          while (next_free < b && taken[next_free]) ++next_free;
          if (next_free >= b) break;
          best = (int32_t)next_free;
        }
        taken[best] = 1;
        group.push_back(best);
        for (int64_t k = row_ptr[best]; k < row_ptr[best + 1]; ++k) mark[col_idx[k]] = gstamp;
      }
      order.insert(order.end(), group.begin(), group.end());
    }
  }
}

double far_block_fraction(int64_t n, const int64_t* row_ptr, const int32_t* col_idx,
                          const int32_t* order, int64_t window) {
  std::vector<int64_t> pos;
  if (order) {
    pos.resize((size_t)n);
    for (int64_t i = 0; i < n; ++i) pos[order[i]] = i;
  }
  int64_t far = 0, off = 0;
  for (int64_t i = 0; i < n; ++i) {
    const int64_t pi = order ? pos[i] : i;
    for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) {
      const int32_t j = col_idx[k];
      if (j == i) continue;
      ++off;
      const int64_t pj = order ? pos[j] : j;
      if (std::abs(pi - pj) > window) ++far;
    }
  }
  return off > 0 ? (double)far / (double)off : 0.0;
}

int64_t neighbour_span(int64_t n, const int64_t* row_ptr, const int32_t* col_idx) {
  // every 16th block row is enough for a percentile
  std::vector<int64_t> off;
  for (int64_t i = 0; i < n; i += 16)
    for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) {
      const int64_t d = std::abs((int64_t)col_idx[k] - i);
      if (d > 0 && 2 * d <= n) off.push_back(d);
    }
  if (off.empty()) return 0;
  const size_t at = (off.size() * 9) / 10;
  std::nth_element(off.begin(), off.begin() + at, off.end());
  return off[at];
}

}  // namespace pfe
