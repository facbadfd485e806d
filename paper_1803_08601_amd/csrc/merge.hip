// Merge-based SpMM kernels (paper Sec. 4.2, Algorithm 1): Phase 1 partition,
// Phase 2 (tile function in tiles.hpp), Phase 3 fix-up; plus CSR statistics.

#include "tiles.hpp"

namespace spmmk {

__global__ __launch_bounds__(kBlock) void k_merge_partition(const int* __restrict__ rowptr,
                                                             int64_t m, int64_t nnz, int W,
                                                             int64_t P, int* __restrict__ coords) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p > P) return;
    const int64_t total = m + nnz;
    const int64_t d = p * W < total ? p * W : total;
    int64_t lo = d - nnz > 0 ? d - nnz : 0;
    int64_t hi = d < m ? d : m;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if ((int64_t)rowptr[mid + 1] + mid < d)
            lo = mid + 1;
        else
            hi = mid;
    }
    coords[2 * p] = (int)lo;
    coords[2 * p + 1] = (int)(d - lo);
}

template <class S, int VEC, int U>
__global__ __launch_bounds__(kBlock) void k_merge(const int* __restrict__ rowptr,
                                                   const int* __restrict__ colind,
                                                   const typename S::T* __restrict__ vals,
                                                   const typename S::T* __restrict__ B,
                                                   float* __restrict__ C, int m, int n, int64_t ld,
                                                   int g_log2, const int* __restrict__ coords,
                                                   int W, float* __restrict__ carry_vals,
                                                   int* __restrict__ carry_rows) {
    extern __shared__ __align__(16) unsigned char smem[];
    merge_tile<S, VEC, U>(rowptr, colind, vals, B, C, m, n, ld, g_log2, coords, W, carry_vals,
                          carry_rows, (int)xcd_remap(blockIdx.x, gridDim.x), blockIdx.y, smem);
}

__global__ __launch_bounds__(kWave) void k_merge_fixup(float* __restrict__ C, int64_t ld, int n,
                                                        const float* __restrict__ carry_vals,
                                                        const int* __restrict__ carry_rows,
                                                        int64_t P) {
    merge_fixup_piece(C, ld, n, carry_vals, carry_rows, P, blockIdx.x);
}

size_t merge_lds_bytes(int dtype, const Shape& s) {
    (void)dtype;
    return (size_t)2 * kBlock * s.vec * sizeof(float) + (size_t)3 * s.W * sizeof(int) +
           (size_t)2 * kBlock * sizeof(int);
}

hipError_t launch_merge_partition(const int* rowptr, int64_t m, int64_t nnz, int W, int64_t P,
                                  int* coords, hipStream_t st) {
    const int64_t threads = P + 1;
    const uint32_t grid = (uint32_t)((threads + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(k_merge_partition, dim3(grid), dim3(kBlock), 0, st, rowptr, m, nnz, W, P,
                       coords);
    return hipGetLastError();
}

template <class S, int VEC, int U>
static hipError_t go(const Shape& s, const int* rowptr, const int* colind, const void* vals,
                     const void* B, float* C, int64_t m, int64_t n, int64_t ld,
                     const int* coords, int64_t P, float* carry_vals, int* carry_rows,
                     hipStream_t st) {
    const size_t lds = merge_lds_bytes(0, s);
    hipLaunchKernelGGL((k_merge<S, VEC, U>), dim3((uint32_t)P, s.col_tiles), dim3(kBlock), lds,
                       st, rowptr, colind, static_cast<const typename S::T*>(vals),
                       static_cast<const typename S::T*>(B), C, (int)m, (int)n, ld, s.g_log2,
                       coords, s.W, carry_vals, carry_rows);
    return hipGetLastError();
}

template <class S, int VEC>
static hipError_t go_u(const Shape& s, const int* rowptr, const int* colind, const void* vals,
                       const void* B, float* C, int64_t m, int64_t n, int64_t ld,
                       const int* coords, int64_t P, float* cv, int* cr, hipStream_t st) {
    switch (s.unroll) {
    case 1: return go<S, VEC, 1>(s, rowptr, colind, vals, B, C, m, n, ld, coords, P, cv, cr, st);
    case 2: return go<S, VEC, 2>(s, rowptr, colind, vals, B, C, m, n, ld, coords, P, cv, cr, st);
    case 4: return go<S, VEC, 4>(s, rowptr, colind, vals, B, C, m, n, ld, coords, P, cv, cr, st);
    case 8: return go<S, VEC, 8>(s, rowptr, colind, vals, B, C, m, n, ld, coords, P, cv, cr, st);
    default: return hipErrorInvalidValue;
    }
}

template <class S>
static hipError_t go_v(const Shape& s, const int* rowptr, const int* colind, const void* vals,
                       const void* B, float* C, int64_t m, int64_t n, int64_t ld,
                       const int* coords, int64_t P, float* cv, int* cr, hipStream_t st) {
    if (s.vec == S::kVec16)
        return go_u<S, S::kVec16>(s, rowptr, colind, vals, B, C, m, n, ld, coords, P, cv, cr, st);
    if (s.vec == 1) return go_u<S, 1>(s, rowptr, colind, vals, B, C, m, n, ld, coords, P, cv, cr, st);
    return hipErrorInvalidValue;
}

hipError_t launch_merge(int dtype, const Shape& s, const int* rowptr, const int* colind,
                        const void* vals, const void* B, float* C, int64_t m, int64_t n,
                        int64_t ld, const int* coords, int64_t P, float* carry_vals,
                        int* carry_rows, hipStream_t st) {
    if (P <= 0) return hipSuccess;
    if (s.g_log2 < 0 || s.g_log2 > 6 || s.W < 1) return hipErrorInvalidValue;
    switch (dtype) {
    case 0: return go_v<F32>(s, rowptr, colind, vals, B, C, m, n, ld, coords, P, carry_vals, carry_rows, st);
    case 1: return go_v<BF16>(s, rowptr, colind, vals, B, C, m, n, ld, coords, P, carry_vals, carry_rows, st);
    case 2: return go_v<F16>(s, rowptr, colind, vals, B, C, m, n, ld, coords, P, carry_vals, carry_rows, st);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_merge_fixup(float* C, int64_t ld, int64_t n, const float* carry_vals,
                              const int* carry_rows, int64_t P, hipStream_t st) {
    if (P <= 0 || n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_merge_fixup, dim3((uint32_t)P), dim3(kWave), 0, st, C, ld, (int)n,
                       carry_vals, carry_rows, P);
    return hipGetLastError();
}

// ------------------------------------------------------------------ statistics

__global__ __launch_bounds__(kBlock) void k_row_stats(const int* __restrict__ rowptr, int64_t m,
                                                       int* __restrict__ stats) {
    int mx = 0, nlong = 0, bad = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int len = rowptr[i + 1] - rowptr[i];
        mx = max(mx, len);
        nlong += len >= 1024;
        bad |= len < 0;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0 && rowptr[0] != 0) bad = 1;
    for (int off = kWave / 2; off > 0; off >>= 1) {
        mx = max(mx, __shfl_xor(mx, off, kWave));
        nlong += __shfl_xor(nlong, off, kWave);
        bad |= __shfl_xor(bad, off, kWave);
    }
    if ((threadIdx.x & (kWave - 1)) == 0) {
        atomicMax(&stats[0], mx);
        atomicAdd(&stats[1], nlong);
        if (bad) atomicAnd(&stats[2], 0);
    }
}

hipError_t launch_row_stats(const int* rowptr, int64_t m, int* stats, hipStream_t st) {
    int64_t blocks = (m + kBlock - 1) / kBlock;
    if (blocks > 4096) blocks = 4096;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_row_stats, dim3((uint32_t)blocks), dim3(kBlock), 0, st, rowptr, m, stats);
    return hipGetLastError();
}

__global__ __launch_bounds__(kBlock) void k_check_cols(const int* __restrict__ colind, int64_t nnz,
                                                        int64_t k, int* __restrict__ flags) {
    int bad = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nnz;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int c = colind[i];
        bad |= (c < 0) | ((int64_t)c >= k);
    }
    for (int off = kWave / 2; off > 0; off >>= 1) bad |= __shfl_xor(bad, off, kWave);
    if ((threadIdx.x & (kWave - 1)) == 0 && bad) atomicOr(&flags[0], 1);
}

hipError_t launch_check_cols(const int* colind, int64_t nnz, int64_t k, int* flags,
                             hipStream_t st) {
    int64_t blocks = (nnz + kBlock - 1) / kBlock;
    if (blocks > 4096) blocks = 4096;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_check_cols, dim3((uint32_t)blocks), dim3(kBlock), 0, st, colind, nnz, k,
                       flags);
    return hipGetLastError();
}

}  // namespace spmmk
