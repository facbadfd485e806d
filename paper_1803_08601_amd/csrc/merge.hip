// Phase 1 of the merge-based SpMM (paper Sec. 4.2, Algorithm 1): the
// merge-path partition; plus CSR statistics. Phases 2 and 3 are in tiles.hpp.

#include "tiles.hpp"

namespace spmmk {

// Rows finished on diagonal d of the merge path: the number of x in
// [max(0, d - nnz), min(d, m)) with x + rowptr[x + 1] < d (binary search).
__device__ __forceinline__ int64_t merge_path_rows(const int* __restrict__ rowptr, int64_t m,
                                                   int64_t nnz, int64_t d) {
    int64_t lo = d - nnz > 0 ? d - nnz : 0;
    int64_t hi = d < m ? d : m;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if ((int64_t)rowptr[mid + 1] + mid < d)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

__global__ __launch_bounds__(kBlock) void k_merge_partition(const int* __restrict__ rowptr,
                                                             int64_t m, int64_t nnz, int W,
                                                             int64_t P, int* __restrict__ coords) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p > P) return;
    const int64_t total = m + nnz;
    const int64_t d = p * W < total ? p * W : total;
    const int64_t i = merge_path_rows(rowptr, m, nnz, d);
    coords[2 * p] = (int)i;
    coords[2 * p + 1] = (int)(d - i);
}

// Re-check of a kept merge partition against the row offsets passed now.
// With the same m and nnz the pieces lie on the same diagonals; (i, j) is
// the state of diagonal i + j exactly when rowptr[i] <= j (the rows before i
// ended by then) and j <= rowptr[i + 1] (row i has not), so a coordinate
// that fails this is searched again. When rowptr[m] is not nnz the partition
// cannot describe the matrix: every piece is made empty (state (0, 0), so
// the merge kernels write nothing), C is filled with NaN and *flag is set
// (a host-visible word).
__global__ __launch_bounds__(kBlock) void k_merge_revalidate(const int* __restrict__ rowptr,
                                                              int64_t m, int64_t nnz, int W,
                                                              int64_t P, int* __restrict__ coords,
                                                              float* __restrict__ C, int n,
                                                              int64_t ld, int* flag) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if ((int64_t)rowptr[m] != nnz) {
        if (p <= P) {
            coords[2 * p] = 0;
            coords[2 * p + 1] = 0;
        }
        if (p == 0) __hip_atomic_store(flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        const int64_t nt = (int64_t)gridDim.x * blockDim.x;
        for (int64_t e = p; e < m * n; e += nt) C[(e / n) * ld + e % n] = __builtin_nanf("");
        return;
    }
    if (p > P) return;
    const int64_t total = m + nnz;
    const int64_t d = p * W < total ? p * W : total;
    const int64_t i = coords[2 * p], j = coords[2 * p + 1];
    const bool ok = i >= 0 && i <= m && j >= 0 && j <= nnz && i + j == d &&
                    (i == 0 || rowptr[i] <= j) && (i == m || j <= rowptr[i + 1]);
    if (!ok) {
        const int64_t r = merge_path_rows(rowptr, m, nnz, d);
        coords[2 * p] = (int)r;
        coords[2 * p + 1] = (int)(d - r);
    }
}

// Nonzero split (Sec. 4, scheme (a)): piece p starts at nonzero
// j = min(p * W, nnz) in the row found by a 1-D binary search on the row
// offsets, i.e. after the i rows whose end is <= j (ties to the row end, as
// on the merge path). Piece 0 starts at (0, 0), so it also takes the leading
// empty rows, and piece P ends at (m, nnz).
__global__ __launch_bounds__(kBlock) void k_nz_partition(const int* __restrict__ rowptr,
                                                          int64_t m, int64_t nnz, int W,
                                                          int64_t P, int* __restrict__ coords) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p > P) return;
    const int64_t j = p * W < nnz ? p * W : nnz;
    int64_t lo = 0, hi = m;
    if (p == 0) hi = 0;
    if (p == P) lo = m;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if ((int64_t)rowptr[mid + 1] <= j)
            lo = mid + 1;
        else
            hi = mid;
    }
    coords[2 * p] = (int)lo;
    coords[2 * p + 1] = (int)j;
}

size_t merge_lds_bytes(int dtype, const Shape& s) {
    (void)dtype;
    return (size_t)2 * kBlock * s.vec * sizeof(float) + (size_t)3 * s.W * sizeof(int) +
           (size_t)2 * kBlock * sizeof(int);
}

hipError_t launch_merge_partition(const int* rowptr, int64_t m, int64_t nnz, int W, int64_t P,
                                  int nz, int* coords, hipStream_t st) {
    const int64_t threads = P + 1;
    const uint32_t grid = (uint32_t)((threads + kBlock - 1) / kBlock);
    if (nz)
        hipLaunchKernelGGL(k_nz_partition, dim3(grid), dim3(kBlock), 0, st, rowptr, m, nnz, W, P,
                           coords);
    else
        hipLaunchKernelGGL(k_merge_partition, dim3(grid), dim3(kBlock), 0, st, rowptr, m, nnz, W,
                           P, coords);
    return hipGetLastError();
}

hipError_t launch_merge_revalidate(const int* rowptr, int64_t m, int64_t nnz, int W, int64_t P,
                                   int* coords, float* C, int64_t n, int64_t ld, int* flag,
                                   hipStream_t st) {
    const int64_t threads = P + 1;
    const uint32_t grid = (uint32_t)((threads + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(k_merge_revalidate, dim3(grid), dim3(kBlock), 0, st, rowptr, m, nnz, W, P,
                       coords, C, (int)n, ld, flag);
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
    // One set of atomics per workgroup: atomics from every wave on the same three
    // words serialise in L2 and cost more than the whole scan of rowptr.
    __shared__ int part[3][kBlock / kWave];
    const int wave = threadIdx.x / kWave;
    if ((threadIdx.x & (kWave - 1)) == 0) {
        part[0][wave] = mx;
        part[1][wave] = nlong;
        part[2][wave] = bad;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kBlock / kWave; ++w) {
            mx = max(mx, part[0][w]);
            nlong += part[1][w];
            bad |= part[2][w];
        }
        atomicMax(&stats[0], mx);
        if (nlong) atomicAdd(&stats[1], nlong);
        if (bad) atomicAnd(&stats[2], 0);
    }
}

hipError_t launch_row_stats(const int* rowptr, int64_t m, int* stats, hipStream_t st) {
    int64_t blocks = (m + kBlock - 1) / kBlock;
    if (blocks > 256) blocks = 256;  // one workgroup per CU: few same-word atomics
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_row_stats, dim3((uint32_t)blocks), dim3(kBlock), 0, st, rowptr, m, stats);
    return hipGetLastError();
}

// Offsets colind - row, one wavefront per row, one set of atomics per
// workgroup. PASS 0: the largest |offset|. PASS 1 (out[0] holds it): the
// largest |offset| below half of it and the smallest at or above half.
template <int PASS>
__global__ __launch_bounds__(kBlock) void k_offset_stats(const int* __restrict__ rowptr,
                                                          const int* __restrict__ colind,
                                                          int64_t m, int* __restrict__ out) {
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;
    const int64_t hi_all = PASS == 1 ? out[0] : 0;
    int64_t hi = 0, near = 0, far_lo = INT_MAX;
    const int64_t nw = (int64_t)gridDim.x * (kBlock / kWave);
    for (int64_t i = (int64_t)blockIdx.x * (kBlock / kWave) + wave; i < m; i += nw) {
        const int lo = rowptr[i], end = rowptr[i + 1];
        for (int j = lo + lane; j < end; j += kWave) {
            int64_t off = (int64_t)colind[j] - i;
            off = off < 0 ? -off : off;
            if (PASS == 0) {
                hi = off > hi ? off : hi;
            } else if (2 * off < hi_all) {
                near = off > near ? off : near;
            } else {
                far_lo = off < far_lo ? off : far_lo;
            }
        }
    }
    int h = (int)(hi < INT_MAX ? hi : INT_MAX), nr = (int)near, fl = (int)far_lo;
    for (int o = kWave / 2; o > 0; o >>= 1) {
        h = max(h, __shfl_xor(h, o, kWave));
        nr = max(nr, __shfl_xor(nr, o, kWave));
        fl = min(fl, __shfl_xor(fl, o, kWave));
    }
    __shared__ int part[3][kBlock / kWave];
    if (lane == 0) {
        part[0][wave] = h;
        part[1][wave] = nr;
        part[2][wave] = fl;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kBlock / kWave; ++w) {
            h = max(h, part[0][w]);
            nr = max(nr, part[1][w]);
            fl = min(fl, part[2][w]);
        }
        if (PASS == 0) {
            atomicMax(&out[0], h);
        } else {
            atomicMax(&out[1], nr);
            atomicMin(&out[2], fl);
        }
    }
}

hipError_t launch_offset_stats(const int* rowptr, const int* colind, int64_t m, int* out,
                               hipStream_t st) {
    if (m <= 0) return hipSuccess;
    int64_t blocks = (m + (kBlock / kWave) - 1) / (kBlock / kWave);
    if (blocks > 1024) blocks = 1024;
    hipLaunchKernelGGL(k_offset_stats<0>, dim3((uint32_t)blocks), dim3(kBlock), 0, st, rowptr,
                       colind, m, out);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_offset_stats<1>, dim3((uint32_t)blocks), dim3(kBlock), 0, st, rowptr,
                       colind, m, out);
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
