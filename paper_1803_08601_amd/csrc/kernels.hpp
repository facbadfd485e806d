// Host-side launchers of the gfx950 kernels (internal to the library).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace spmmk {

constexpr int kBlock = 256;  // threads per workgroup for every SpMM kernel
constexpr int kWaveSize = 64;  // CDNA wavefront width

// Launch shape resolved for one call. Lanes of a wavefront are grouped into
// "slots" of 2^g_log2 lanes; a slot covers vec * 2^g_log2 consecutive columns
// of one B row (one column tile). Row split groups 2^ts_log2 slots into a
// team that owns one row of A.
struct Shape {
    int vec = 1;
    int g_log2 = 0;
    int ts_log2 = 0;
    int unroll = 4;
    int W = 1024;       // merge items per workgroup (nonzeros for the nonzero split)
    int col_tiles = 1;
    int nz = 0;         // merge walk over nonzero-split pieces (1-D partition)
    int short_addr = 0; // B has < 2^24 rows of < 2^24 bytes and spans < 4 GiB
    // Row split and row blocks: rows are taken in strips of strip_rows
    // through planes of plane_rows rows (0: in row order); see TileOrder.
    int64_t plane_rows = 0, strip_rows = 0;
};

// Entry offsets colind - row of A: hi = the largest |offset|; near = the
// largest |offset| below hi / 2; far_lo = the smallest |offset| at or above
// hi / 2 (two passes; out[0..2] = hi, near, far_lo, out[2] starting at
// INT_MAX and out[0], out[1] at 0).
hipError_t launch_offset_stats(const int* rowptr, const int* colind, int64_t m, int* out,
                               hipStream_t st);

// Operands of one forward product; coords, P and the carry arrays are the
// merge-based workspace (unused by row split). Row split takes row i's
// entries from rowptr[i] to rowend[i] (rowend null: rowptr + 1, the whole
// row) and, with accumulate set, adds its sums into C instead of writing
// them (one pass of a column-panel product).
struct ForwardArgs {
    const int* rowptr;
    const int* colind;
    const void* vals;
    const void* B;
    float* C;
    int64_t m, n, ld;
    const int* coords;
    int64_t P;
    float* carry_vals;
    int* carry_rows;
    const int* rowend;
    int accumulate;
};

// Column panels: starts[p * m + i] = the first entry of row i whose column
// is at least p * width (p = 0 .. P; row i's columns must not decrease), so
// panel p of row i is entries starts[p * m + i] .. starts[(p + 1) * m + i].
hipError_t launch_panel_starts(const int* rowptr, const int* colind, int64_t m, int P,
                               int64_t width, int* starts, hipStream_t st);

// The main kernel of one product and, for merge-based plans, its fix-up pass;
// ev_after (may be null) is recorded between the two.
hipError_t launch_forward_plus_times(int dtype, bool merge, const Shape& s,
                                     const ForwardArgs& a, hipStream_t st, hipEvent_t ev_after);
// The same over semiring 1 (min, +), 2 (max, +) or 3 (max, *).
hipError_t launch_forward_semiring(int semiring, int dtype, bool merge, const Shape& s,
                                   const ForwardArgs& a, hipStream_t st);

// Piece start coordinates for the merge walk: diagonals of the merge path
// (nz == 0) or the nonzero split (nz != 0).
hipError_t launch_merge_partition(const int* rowptr, int64_t m, int64_t nnz, int W, int64_t P,
                                  int nz, int* coords, hipStream_t st);

// Re-check a kept diagonal partition (P + 1 coordinates of W-item pieces for
// m rows and nnz entries) against rowptr: wrong coordinates are searched
// again; if rowptr[m] != nnz every piece is emptied, C (m x n, stride ld) is
// filled with NaN and *flag (host-visible) is set to 1.
hipError_t launch_merge_revalidate(const int* rowptr, int64_t m, int64_t nnz, int W, int64_t P,
                                   int* coords, float* C, int64_t n, int64_t ld, int* flag,
                                   hipStream_t st);

// stats[0] = longest row, stats[1] = rows with >= 1024 entries,
// stats[2] = 1 if rowptr is non-decreasing with rowptr[0] == 0 else 0.
hipError_t launch_row_stats(const int* rowptr, int64_t m, int* stats, hipStream_t st);

// flags[0] = 1 if some colind is outside [0, k).
hipError_t launch_check_cols(const int* colind, int64_t nnz, int64_t k, int* flags,
                             hipStream_t st);

size_t merge_lds_bytes(int dtype, const Shape& s);

// CSR of A^T by a stable radix sort of (column, entry) pairs that carries
// each entry's row of A along. Scratch: tmp_keys0/tmp_keys1/tmp_vals1/
// tmp_rows0 of nnz ints, scratch of transpose_scratch_len(nnz) ints.
hipError_t transpose_build(const int* rowptr, const int* colind, int64_t m, int64_t k,
                           int64_t nnz, int* at_rowptr, int* at_colind, int* perm,
                           int* tmp_keys0, int* tmp_keys1, int* tmp_vals1, int* tmp_rows0,
                           int* scratch, hipStream_t st);
int64_t transpose_scratch_len(int64_t nnz);

// out[q] = widen(vals[perm[q]]) for q < n.
hipError_t launch_gather_widen(int dtype, const void* vals, const int* perm, int64_t n,
                               float* out, hipStream_t st);

// dB = A^T dC by float atomic adds on diagonal merge pieces (dB is zeroed
// first); not bitwise repeatable.
hipError_t launch_scatter_t(int dtype, const int* rowptr, const int* colind, const void* vals,
                            const float* dC, float* dB, int64_t k, int64_t n, int64_t ld,
                            const int* coords, int64_t P, int W, hipStream_t st);

// a[0 .. count) = 0 by a kernel (no memset node when the stream is captured).
hipError_t launch_zero_f32(float* a, int64_t count, hipStream_t st);

// dvals[p] = <dC[row(p), :n], B[colind[p], :n]> over the P merge pieces of W
// items given by coords (2 * (P + 1) ints).
hipError_t launch_sddmm(int dtype, int vec, int unroll, int g_log2, int col_tiles,
                        const int* rowptr, const int* colind, const float* dC, const void* B,
                        float* dvals, int64_t n, int64_t ld, const int* coords, int64_t P, int W,
                        hipStream_t st);

// Gather calibration: threads (a multiple of kBlock) lanes read rows of
// row_bytes (32, 64, 128, 256 or 512) at pseudo-random indices of a table of rows
// rows (a power of two), steps reads each (a multiple of 8); one float per
// thread into out.
hipError_t launch_calib_gather(const void* table, int64_t rows, int row_bytes, int steps,
                               float* out, int64_t threads, hipStream_t st);

}  // namespace spmmk
