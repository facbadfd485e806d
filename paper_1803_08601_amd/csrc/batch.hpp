// Work description of the batched persistent kernel (internal).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace spmmk {

// Unroll of the batched kernel: one instantiation keeps its register use
// (and so its occupancy) independent of the mix of problems.
constexpr int kBatchUnroll = 4;
// One work queue per XCD.
constexpr int kBatchQueues = 8;
// Largest merge piece in a batch: the persistent kernel reserves the LDS of
// its largest piece in every workgroup, so pieces stay small enough that LDS
// does not limit occupancy below what registers allow.
constexpr int kBatchMaxW = 1024;
// Entries a work item aims at: several row blocks or merge pieces per item,
// so the per-item cost of taking work from a queue stays small.
constexpr int kBatchItemEntries = 4096;

// One unit of work: `count` consecutive row blocks (row split) or merge
// pieces of problem `prob`, column tile `coltile`.
struct WorkItem {
    int prob;
    int coltile;
    int first;
    int count;
};

struct BatchProb {
    const int* rowptr;
    const int* colind;
    const void* vals;
    const void* B;
    float* C;
    int64_t m;
    int64_t ld;
    int n;
    int kernel;   // 0 row split, otherwise the merge walk
    int vec;
    int g_log2;
    int ts_log2;
    int W;
    int col_tiles;
    int nz;       // merge walk over nonzero-split pieces
    const int* coords;
    float* carry_vals;
    int* carry_rows;
    int64_t P;
};

// Workgroups of the persistent kernel that fit on the device at once.
hipError_t batch_grid(int dtype, size_t lds, int* grid);

// queues: kBatchQueues first-item offsets followed by kBatchQueues lengths;
// counters: kBatchQueues counters (re-armed by the launch).
hipError_t launch_batch(int dtype, int grid, size_t lds, const BatchProb* probs,
                        const WorkItem* items, int64_t total, const int64_t* queues,
                        unsigned long long* counters, const int* merge_ids,
                        const int64_t* piece_off, int nmerge, int64_t total_pieces,
                        hipStream_t st);

}  // namespace spmmk
