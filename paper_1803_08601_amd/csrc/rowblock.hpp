// Row-block product (an addition to the paper's two kernels, for matrices
// whose neighbouring rows share columns, such as stencils): internal
// launchers and the blocked structure it walks.
//
// Rows are taken R at a time (R = 2, 4 or 8). For each block the plan builds
// the sorted union of the block's column indices; each union entry is one
// 32-bit word, the column in bits 0..23 and in bits 24..31 the set of the
// block's rows that hold that column. The kernel gathers every B row of the
// union once per block and adds it into the accumulators of the rows in the
// set, so a B row shared by several rows of the block is fetched once
// instead of once per entry. Row r's values are consumed in entry order
// (the union is sorted and each row's columns strictly increase), so the
// value of a union entry for row r is the next unread value of that row.
#pragma once

#include "kernels.hpp"

namespace spmmk {

constexpr int kRowBlockColBits = 24;  // columns below 2^24; row set in the top byte

// flag[0] |= 1 if some row's column indices do not strictly increase.
hipError_t launch_rowblock_check_sorted(const int* rowptr, const int* colind, int64_t m,
                                        int* flag, hipStream_t st);

// Union sizes: counts[b] for the ceil(m / R) blocks (count pass, ub_ptr null),
// or the union words into words[ub_ptr[b] ..] (fill pass).
hipError_t launch_rowblock_union(const int* rowptr, const int* colind, int64_t m, int R,
                                 const int* ub_ptr, int* out, hipStream_t st);

// In-place exclusive scan of len ints; sums holds scan_chunks(len) ints.
hipError_t exclusive_scan_i32(int* a, int64_t len, int* sums, hipStream_t st);
int64_t scan_chunks(int64_t len);

// The row-block product (ordinary semiring) for shape s (vec, g_log2, ts_log2,
// unroll, col_tiles, short_addr) over blocks of R rows; ev_after (may be null)
// is recorded after the kernel.
hipError_t launch_rowblock(int dtype, const Shape& s, int R, const ForwardArgs& a,
                           const int* ub_ptr, const int* words, hipStream_t st,
                           hipEvent_t ev_after);

}  // namespace spmmk
