// Reading a composed interchange list (the output of compose_moves, see
// common.hpp) defensively.  The trailing kernels index LDS arrays and matrix
// rows with its entries, so every count is clamped to the panel width and
// every move whose rows fall outside the block is dropped: a stale, empty or
// corrupted list (a panel that gave up at a barrier time-out leaves an empty
// one) can give wrong values but never an access outside the block.
//
// Rows are relative to the panel's first row; the block has m rows from there
// and the panel is w columns wide.  A top move writes top row dst in [0, w)
// from row src in [0, m); an extra move writes row dst in [w, m) from the top
// row src in [0, w).
#pragma once
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace lu {

__host__ __device__ inline int clamp_count(int c, int w) { return c < 0 ? 0 : (c > w ? w : c); }
__host__ __device__ inline int moves_top_count(const int* mv, int w) { return clamp_count(mv[0], w); }
__host__ __device__ inline int moves_extra_count(const int* mv, int w) { return clamp_count(mv[1], w); }

// top move s (s < moves_top_count): false if it is to be dropped
__host__ __device__ inline bool moves_top(const int* mv, int s, int w, int m, int& dst, int& src) {
    dst = mv[2 + 2 * s];
    src = mv[3 + 2 * s];
    return dst >= 0 && dst < w && src >= 0 && src < m;
}
// extra move s (s < moves_extra_count): false if it is to be dropped
__host__ __device__ inline bool moves_extra(const int* mv, int s, int w, int m, int& dst, int& src) {
    dst = mv[kMovesExtra + 2 * s];
    src = mv[kMovesExtra + 1 + 2 * s];
    return dst >= w && dst < m && src >= 0 && src < w;
}

}  // namespace lu
