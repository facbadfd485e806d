// Batched SpMM: many independent products C_b = A_b B_b in one persistent
// kernel (not in the paper; it applies the paper's two kernels per problem).
//
// The host lays out a work list: every problem contributes work items - runs
// of row blocks (a workgroup's rows each) for row-split problems, runs of
// merge pieces for merge-based problems, about kBatchItemEntries entries per
// item - per column tile. Problems are bin-packed by cost into one
// queue per XCD (longest first onto the lightest queue), so that a problem's
// B rows are pulled into one XCD's L2 rather than all eight. A grid of exactly
// as many workgroups as fit on the GPU at once starts on the queue of its
// XCD (workgroup b runs on XCD b mod 8) and takes tiles from that queue's
// atomic counter; when the queue is exhausted it moves on to the next queue,
// so the tails of the queues are shared. Counters only grow, so every
// workgroup finds every queue exhausted after finitely many attempts and
// exits. Each tile runs the same device function as the single-product
// kernels, with that problem's shape. A second launch adds the carry-outs of
// all merge-based problems (Phase 3), and a small kernel re-arms the counters
// for the next run.

#include "batch.hpp"
#include "tiles.hpp"

namespace spmmk {

__global__ void k_batch_reset(unsigned long long* counters) {
    if (threadIdx.x < kBatchQueues) counters[threadIdx.x] = 0ull;
}

// Next work item for this workgroup (thread 0 only): from its current queue,
// moving on through the other queues as they run dry; -1 when all are.
__device__ __forceinline__ int64_t take_item(const int64_t* __restrict__ queues,
                                             unsigned long long* __restrict__ counters, int& q,
                                             int& exhausted) {
    while (exhausted < kBatchQueues) {
        const int64_t i = (int64_t)atomicAdd(&counters[q], 1ull);
        if (i < queues[kBatchQueues + q]) return queues[q] + i;
        q = (q + 1) % kBatchQueues;
        ++exhausted;
    }
    return -1;
}

template <class S, int U>
__global__ __launch_bounds__(kBlock) void k_batch(const BatchProb* __restrict__ probs,
                                                   const WorkItem* __restrict__ items,
                                                   const int64_t* __restrict__ queues,
                                                   unsigned long long* __restrict__ counters) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int64_t s_item;
    int q = blockIdx.x % kBatchQueues;  // queue of this workgroup's XCD
    int exhausted = 0;
    if (threadIdx.x == 0) s_item = take_item(queues, counters, q, exhausted);
    __syncthreads();
    int64_t it = s_item;
    while (it >= 0) {
        // Claim a slot of the current queue now and look at it only after
        // this item's work, so the atomic's latency overlaps that work.
        unsigned long long claim = 0;
        if (threadIdx.x == 0 && exhausted < kBatchQueues) claim = atomicAdd(&counters[q], 1ull);
        const WorkItem w = items[it];
        const BatchProb& p = probs[w.prob];
        const typename S::T* vals = static_cast<const typename S::T*>(p.vals);
        const typename S::T* B = static_cast<const typename S::T*>(p.B);
        for (int t = w.first; t < w.first + w.count; ++t) {
            if (p.kernel == 0) {
                if (p.vec == 1)
                    rowsplit_block<S, 1, U>(p.rowptr, p.rowptr + 1, p.colind, vals, B, p.C, p.m,
                                            p.n, p.ld, p.g_log2, p.ts_log2, t, w.coltile, false);
                else
                    rowsplit_block<S, S::kVec16, U>(p.rowptr, p.rowptr + 1, p.colind, vals, B,
                                                    p.C, p.m, p.n, p.ld, p.g_log2, p.ts_log2, t,
                                                    w.coltile, false);
            } else {
                if (p.vec == 1 && !p.nz)
                    merge_tile<S, 1, U>(p.rowptr, p.colind, vals, B, p.C, (int)p.m, p.n, p.ld,
                                        p.g_log2, p.coords, p.W, p.carry_vals, p.carry_rows, t,
                                        w.coltile, smem);
                else if (!p.nz)
                    merge_tile<S, S::kVec16, U>(p.rowptr, p.colind, vals, B, p.C, (int)p.m, p.n,
                                                p.ld, p.g_log2, p.coords, p.W, p.carry_vals,
                                                p.carry_rows, t, w.coltile, smem);
                else if (p.vec == 1)
                    merge_tile<S, 1, U, PlusTimes, true>(p.rowptr, p.colind, vals, B, p.C,
                                                         (int)p.m, p.n, p.ld, p.g_log2, p.coords,
                                                         p.W, p.carry_vals, p.carry_rows, t,
                                                         w.coltile, smem);
                else
                    merge_tile<S, S::kVec16, U, PlusTimes, true>(
                        p.rowptr, p.colind, vals, B, p.C, (int)p.m, p.n, p.ld, p.g_log2, p.coords,
                        p.W, p.carry_vals, p.carry_rows, t, w.coltile, smem);
                __syncthreads();  // LDS is reused by the next piece
            }
        }
        __syncthreads();  // every thread has read s_item for this item
        if (threadIdx.x == 0) {
            int64_t next = -1;
            if (exhausted < kBatchQueues) {
                if ((int64_t)claim < queues[kBatchQueues + q]) {
                    next = queues[q] + (int64_t)claim;
                } else {
                    q = (q + 1) % kBatchQueues;
                    ++exhausted;
                    next = take_item(queues, counters, q, exhausted);
                }
            }
            s_item = next;
        }
        __syncthreads();
        it = s_item;
    }
}

// Phase 3 of every merge-based problem: piece g of the concatenated piece
// list belongs to the last merge problem whose first piece is <= g.
__global__ __launch_bounds__(kBlock) void k_batch_fixup(const BatchProb* __restrict__ probs,
                                                         const int* __restrict__ merge_ids,
                                                         const int64_t* __restrict__ piece_off,
                                                         int nmerge, int64_t total_pieces) {
    const int64_t gp = (int64_t)blockIdx.x * kFixupWaves + threadIdx.x / kWave;
    if (gp >= total_pieces) return;
    int lo = 0, hi = nmerge - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (piece_off[mid] <= gp) lo = mid; else hi = mid - 1;
    }
    const BatchProb& p = probs[merge_ids[lo]];
    merge_fixup_piece(p.C, p.ld, p.n, p.carry_vals, p.carry_rows, p.P, gp - piece_off[lo],
                      threadIdx.x & (kWave - 1));
}

template <class S, int U>
static const void* batch_kernel_ptr() {
    return reinterpret_cast<const void*>(&k_batch<S, U>);
}

static const void* batch_fn(int dtype) {
    switch (dtype) {
    case 0: return batch_kernel_ptr<F32, kBatchUnroll>();
    case 1: return batch_kernel_ptr<BF16, kBatchUnroll>();
    case 2: return batch_kernel_ptr<F16, kBatchUnroll>();
    default: return nullptr;
    }
}

hipError_t batch_grid(int dtype, size_t lds, int* grid) {
    const void* fn = batch_fn(dtype);
    if (!fn) return hipErrorInvalidValue;
    int dev = 0, cus = 0, per_cu = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kBlock, lds);
    if (e != hipSuccess) return e;
    if (per_cu < 1) per_cu = 1;
    *grid = cus * per_cu;
    return hipSuccess;
}

hipError_t launch_batch(int dtype, int grid, size_t lds, const BatchProb* probs,
                        const WorkItem* items, int64_t total, const int64_t* queues,
                        unsigned long long* counters, const int* merge_ids,
                        const int64_t* piece_off, int nmerge, int64_t total_pieces,
                        hipStream_t st) {
    hipLaunchKernelGGL(k_batch_reset, dim3(1), dim3(kWave), 0, st, counters);
    if (total > 0) {
        switch (dtype) {
        case 0: hipLaunchKernelGGL((k_batch<F32, kBatchUnroll>), dim3(grid), dim3(kBlock), lds, st,
                                   probs, items, queues, counters); break;
        case 1: hipLaunchKernelGGL((k_batch<BF16, kBatchUnroll>), dim3(grid), dim3(kBlock), lds, st,
                                   probs, items, queues, counters); break;
        case 2: hipLaunchKernelGGL((k_batch<F16, kBatchUnroll>), dim3(grid), dim3(kBlock), lds, st,
                                   probs, items, queues, counters); break;
        default: return hipErrorInvalidValue;
        }
    }
    if (nmerge > 0 && total_pieces > 0)
        hipLaunchKernelGGL(k_batch_fixup,
                           dim3((uint32_t)((total_pieces + kFixupWaves - 1) / kFixupWaves)),
                           dim3(kBlock), 0, st, probs, merge_ids, piece_off, nmerge,
                           total_pieces);
    return hipGetLastError();
}

}  // namespace spmmk
