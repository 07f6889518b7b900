// Cell order of a node set (knn.hip): node ids sorted by the cell of a uniform
// grid, ascending ids inside a cell.  Used by the block-Jacobi preconditioner.
#pragma once

#include "common.hpp"

namespace rbf {
size_t cell_order_ws(int64_t N, int d);
hipError_t cell_order_enqueue(hipStream_t s, const double* X, int64_t N, int d, double per_cell, void* ws,
                              int32_t* order);
}  // namespace rbf
