// Gather calibration: the rate at which the device reads rows of a table at
// pseudo-random row indices with 16-byte lane accesses - the access the
// products make to B, without their reads of A and writes of C. A
// measurement aid for the roofline of the gather kernels; no product uses it.

#include "common.hpp"
#include "kernels.hpp"

namespace spmmk {

__device__ __forceinline__ uint32_t calib_mix(uint32_t x) {
    x ^= x >> 16;
    x *= 0x7feb352dU;
    x ^= x >> 15;
    x *= 0x846ca68bU;
    x ^= x >> 16;
    return x;
}

// Lanes in groups of G read one row of 16 G bytes per step, eight steps in
// flight; row indices are masked into the table (rows_mask + 1 rows, a power
// of two). Each thread writes the sum of what it read.
template <int G>
__global__ __launch_bounds__(kBlock) void k_calib_gather(const f32x4* __restrict__ T,
                                                         uint32_t rows_mask, int steps,
                                                         float* __restrict__ out) {
    const uint32_t tid = blockIdx.x * kBlock + threadIdx.x;
    const uint32_t grp = tid / G, g = tid % G;
    float acc = 0.f;
    for (int it = 0; it < steps; it += 8) {
        f32x4 v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const uint32_t r = calib_mix(grp * 131u + (uint32_t)(it + u) * 0x9E3779B9u) & rows_mask;
            v[u] = T[(size_t)r * G + g];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) acc += v[u].x + v[u].y + v[u].z + v[u].w;
    }
    out[tid] = acc;
}

hipError_t launch_calib_gather(const void* table, int64_t rows, int row_bytes, int steps,
                               float* out, int64_t threads, hipStream_t st) {
    const uint32_t mask = (uint32_t)(rows - 1);
    const dim3 grid((uint32_t)(threads / kBlock));
    const f32x4* T = static_cast<const f32x4*>(table);
    switch (row_bytes) {
    case 32: hipLaunchKernelGGL(k_calib_gather<2>, grid, dim3(kBlock), 0, st, T, mask, steps, out); break;
    case 64: hipLaunchKernelGGL(k_calib_gather<4>, grid, dim3(kBlock), 0, st, T, mask, steps, out); break;
    case 128: hipLaunchKernelGGL(k_calib_gather<8>, grid, dim3(kBlock), 0, st, T, mask, steps, out); break;
    case 256: hipLaunchKernelGGL(k_calib_gather<16>, grid, dim3(kBlock), 0, st, T, mask, steps, out); break;
    case 512: hipLaunchKernelGGL(k_calib_gather<32>, grid, dim3(kBlock), 0, st, T, mask, steps, out); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace spmmk
