// Column panels of a row-split plan (the 2-D tiling of Sec. 6 with one row
// tile): the start of every panel in every row, so that pass p of the product
// takes from row i the entries starts[p m + i] .. starts[(p + 1) m + i].

#include "common.hpp"
#include "kernels.hpp"

namespace spmmk {

// One thread per (panel boundary p = 0 .. P, row i). Boundaries 0 and P are
// the row's ends; boundary p in between is the first entry of the row whose
// column is at least p * width, by binary search over the row's
// non-decreasing columns.
__global__ __launch_bounds__(kBlock) void k_panel_starts(const int* __restrict__ rowptr,
                                                         const int* __restrict__ colind,
                                                         int64_t m, int P, int64_t width,
                                                         int* __restrict__ starts) {
    const int64_t idx = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (idx >= (int64_t)(P + 1) * m) return;
    const int p = (int)(idx / m);
    const int64_t i = idx - (int64_t)p * m;
    int lo = rowptr[i], hi = rowptr[i + 1];
    if (p == 0) {
        starts[idx] = lo;
        return;
    }
    if (p == P) {
        starts[idx] = hi;
        return;
    }
    const int64_t bound = (int64_t)p * width;
    while (lo < hi) {
        const int mid = lo + ((hi - lo) >> 1);
        if ((int64_t)colind[mid] < bound)
            lo = mid + 1;
        else
            hi = mid;
    }
    starts[idx] = lo;
}

hipError_t launch_panel_starts(const int* rowptr, const int* colind, int64_t m, int P,
                               int64_t width, int* starts, hipStream_t st) {
    const int64_t threads = (int64_t)(P + 1) * m;
    if (threads <= 0) return hipSuccess;
    const int64_t grid = (threads + kBlock - 1) / kBlock;
    hipLaunchKernelGGL(k_panel_starts, dim3((uint32_t)grid), dim3(kBlock), 0, st, rowptr, colind,
                       m, P, width, starts);
    return hipGetLastError();
}

}  // namespace spmmk
