// Row-split SpMM kernel (paper Sec. 4.1); the tile function lives in tiles.hpp.

#include "tiles.hpp"

namespace spmmk {

template <class S, int VEC, int U>
__global__ __launch_bounds__(kBlock) void k_rowsplit(const int* __restrict__ rowptr,
                                                      const int* __restrict__ colind,
                                                      const typename S::T* __restrict__ vals,
                                                      const typename S::T* __restrict__ B,
                                                      float* __restrict__ C, int64_t m, int n,
                                                      int64_t ld, int g_log2, int ts_log2) {
    const int rpb_log2 = (6 - g_log2 - ts_log2) + 2;
    const int64_t nblk = (m + (int64_t(1) << rpb_log2) - 1) >> rpb_log2;
    for (int64_t blk = xcd_remap(blockIdx.x, gridDim.x); blk < nblk; blk += gridDim.x)
        rowsplit_block<S, VEC, U>(rowptr, colind, vals, B, C, m, n, ld, g_log2, ts_log2, blk,
                                  blockIdx.y);
}

template <class S, int VEC, int U>
static hipError_t go(const Shape& s, const int* rowptr, const int* colind, const void* vals,
                     const void* B, float* C, int64_t m, int64_t n, int64_t ld, hipStream_t st) {
    const int tl_log2 = s.g_log2 + s.ts_log2;
    const int64_t rows_per_block = int64_t(kWave >> tl_log2) * (kBlock / kWave);
    const int64_t need = (m + rows_per_block - 1) / rows_per_block;
    const uint32_t grid = (uint32_t)(need < (1 << 22) ? need : (1 << 22));
    hipLaunchKernelGGL((k_rowsplit<S, VEC, U>), dim3(grid, s.col_tiles), dim3(kBlock), 0, st,
                       rowptr, colind, static_cast<const typename S::T*>(vals),
                       static_cast<const typename S::T*>(B), C, m, (int)n, ld, s.g_log2,
                       s.ts_log2);
    return hipGetLastError();
}

template <class S, int VEC>
static hipError_t go_u(const Shape& s, const int* rowptr, const int* colind, const void* vals,
                       const void* B, float* C, int64_t m, int64_t n, int64_t ld,
                       hipStream_t st) {
    switch (s.unroll) {
    case 1: return go<S, VEC, 1>(s, rowptr, colind, vals, B, C, m, n, ld, st);
    case 2: return go<S, VEC, 2>(s, rowptr, colind, vals, B, C, m, n, ld, st);
    case 4: return go<S, VEC, 4>(s, rowptr, colind, vals, B, C, m, n, ld, st);
    case 8: return go<S, VEC, 8>(s, rowptr, colind, vals, B, C, m, n, ld, st);
    default: return hipErrorInvalidValue;
    }
}

template <class S>
static hipError_t go_v(const Shape& s, const int* rowptr, const int* colind, const void* vals,
                       const void* B, float* C, int64_t m, int64_t n, int64_t ld,
                       hipStream_t st) {
    if (s.vec == S::kVec16) return go_u<S, S::kVec16>(s, rowptr, colind, vals, B, C, m, n, ld, st);
    if (s.vec == 1) return go_u<S, 1>(s, rowptr, colind, vals, B, C, m, n, ld, st);
    return hipErrorInvalidValue;
}

hipError_t launch_rowsplit(int dtype, const Shape& s, const int* rowptr, const int* colind,
                           const void* vals, const void* B, float* C, int64_t m, int64_t n,
                           int64_t ld, hipStream_t st) {
    if (s.g_log2 < 0 || s.ts_log2 < 0 || s.g_log2 + s.ts_log2 > 6) return hipErrorInvalidValue;
    switch (dtype) {
    case 0: return go_v<F32>(s, rowptr, colind, vals, B, C, m, n, ld, st);
    case 1: return go_v<BF16>(s, rowptr, colind, vals, B, C, m, n, ld, st);
    case 2: return go_v<F16>(s, rowptr, colind, vals, B, C, m, n, ld, st);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace spmmk
