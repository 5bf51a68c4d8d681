// Processing orders of the atom rows for the fused filter step's row tiles
// (host only, plain C++: no HIP types, so a CPU build with bounds-checked
// containers and sanitisers checks the same code).
#pragma once

#include <cstdint>
#include <vector>

namespace pfe {

// Processing order of the atom rows in which contiguous ranges are compact in
// the graph of the (symmetric) pattern: recursive BFS bisection down to
// ranges of `leaf` rows (split at multiples of R), and inside each leaf
// groups of R rows sharing many block columns.
void locality_order(int64_t n, const int64_t* row_ptr, const int32_t* col_idx, int leaf, int R,
                    std::vector<int32_t>& order);
// The natural order with its rows regrouped inside consecutive windows of
// `window` rows (rounded up to a multiple of R): each group of R starts at
// the window's first free row and grows by the free row, among its
// neighbours in the window, that adds the fewest block columns to the
// group's union (ties: most shared columns, then lowest index).  Consecutive
// groups stay in the order of their first rows, so the range of rows one
// stretch of work touches is that of the natural order.
void window_group_order(int64_t n, const int64_t* row_ptr, const int32_t* col_idx,
                        int64_t window, int R, std::vector<int32_t>& order);
// 90th percentile of the row offsets |i - j| of the off-diagonal blocks,
// leaving out offsets above n/2 (periodic wrap-around); 0 without any.
int64_t neighbour_span(int64_t n, const int64_t* row_ptr, const int32_t* col_idx);
// Fraction of the off-diagonal blocks (i, j) whose rows lie more than
// `window` positions apart in the processing order `order` (nullptr: natural).
double far_block_fraction(int64_t n, const int64_t* row_ptr, const int32_t* col_idx,
                          const int32_t* order, int64_t window);

}  // namespace pfe
