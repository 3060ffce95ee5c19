// hefk_layout.hpp -- index arithmetic of the device arrays, shared by the
// kernels and by the host program that replays their loop nests with bounds
// checks (plain C++: it builds without the HIP headers).
//
//   walker state  x [6][n] (structure of arrays: coordinate plane k holds
//                 walker i at k n + i), ln w and E_L [n];
//   checkpoints   [n_ckpt][7][n]: positions 0..5, ln w 6 (the gradient's
//                 segment tape has the same layout);
//   partial rows  [grid][n_samples][8] (the per-block sample tuples).
//
// The propagate grid walks chunks of kLanes walkers: block b takes chunks
// b, b + grid, b + 2 grid, ...; lane t of chunk c holds walker c kLanes + t.
#pragma once

#include <stdint.h>

#if defined(__HIPCC__)
#define HEFK_LAYOUT_FN __host__ __device__ __forceinline__
#else
#define HEFK_LAYOUT_FN inline
#endif

namespace hefk {
namespace layout {

constexpr int kLanes = 256;  // walkers per chunk = threads per block (4 waves of 64)

HEFK_LAYOUT_FN int64_t chunks(int64_t n) { return (n + kLanes - 1) / kLanes; }

// Blocks of a persistent launch with `resident` blocks resident at once: at most one per
// chunk, and the same number of chunks per block for as many blocks as possible.
HEFK_LAYOUT_FN int64_t grid(int64_t n_chunks, int64_t resident)
{
    int64_t g = resident < 1 ? 1 : resident;
    if (g > n_chunks) g = n_chunks;
    const int64_t per_block = (n_chunks + g - 1) / g;
    return (n_chunks + per_block - 1) / per_block;
}

HEFK_LAYOUT_FN int64_t walker(int64_t chunk, uint32_t lane) { return chunk * kLanes + lane; }

// coordinate k of walker i in [6][n], and component k (0..5 position, 6 ln w) of walker i
// within a checkpoint row
HEFK_LAYOUT_FN int64_t coord(int k, int64_t n, int64_t i) { return (int64_t)k * n + i; }

// start of checkpoint row c in [n_ckpt][7][n]: its component k of walker i is
// coord(k, n, i) further on
HEFK_LAYOUT_FN size_t ckpt_row(int64_t c, int64_t n) { return (size_t)c * 7 * (size_t)n; }

// start of block b's partial rows in [grid][n_samples][8], and of its row r within them.
// block_rows is a macro: the kernels' prologue then compiles exactly as the expression
// written out (an inline function reorders it, and moves the step loop off the 32-byte
// instruction alignment it runs fastest at).
#define HEFK_BLOCK_ROWS(b, n_samples) ((size_t)(b) * (size_t)(n_samples) * 8)
HEFK_LAYOUT_FN size_t block_rows(int64_t b, int64_t n_samples) { return HEFK_BLOCK_ROWS(b, n_samples); }
HEFK_LAYOUT_FN size_t row_offset(int64_t r) { return (size_t)r * 8; }

}  // namespace layout
}  // namespace hefk
