// Plan object and host helpers shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "../../include/spmm.h"
#include "kernels.hpp"

namespace spmmh {

int fail(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
int hip_fail(hipError_t e, const char* what);

#define SPMM_HIP(call)                                      \
    do {                                                    \
        hipError_t e_ = (call);                             \
        if (e_ != hipSuccess) return spmmh::hip_fail(e_, #call); \
    } while (0)

// Merge-based workspace: P + 1 coordinates, P carry-out rows of n floats and
// P carry-out row ids.
struct MergeWs {
    int* coords = nullptr;
    float* carry_vals = nullptr;
    int* carry_rows = nullptr;
    int64_t P = 0;
    int64_t cap_P = 0;  // allocated capacity in pieces
    int64_t cap_n = 0;
};

// Row-block structure: union offsets (one per block of R rows, plus one)
// and union words (column | row set << 24).
struct RowBlocks {
    int* ub_ptr = nullptr;
    int* words = nullptr;
    int64_t mb = 0, U = 0;
    int R = 0;
};

// Column panels of a row-split plan: (P + 1) * m panel starts.
struct ColPanels {
    int* starts = nullptr;
    int P = 0;
};

struct Transpose {
    int* at_rowptr = nullptr;
    int* at_colind = nullptr;
    int* perm = nullptr;
    void* at_vals = nullptr;  // gathered values, plan dtype
};

}  // namespace spmmh

struct spmm_plan_s {
    const int32_t* rowptr = nullptr;
    const int32_t* colind = nullptr;
    int64_t m = 0, k = 0, nnz = 0, n = 0, ld = 0;
    int32_t dtype = 0, mode = 0, paper_choice = 0;
    spmm_config cfg{};
    int64_t max_row_len = 0, long_rows = 0;
    double tuned_ms = 0.0;
    int device = 0;
    spmmh::MergeWs ws;
    spmmh::MergeWs sddmm_ws;  // SDDMM's partition unless the plan's own serves (kSddmmW)
    spmmh::RowBlocks rb;      // ROWBLOCK plans
    spmmh::ColPanels cp;      // row-split plans with column panels
    int sorted = -1;          // columns strictly increase in every row: 1 / 0 / -1 unknown
    // plane structure for the tile order of row split and row blocks (plane
    // distance and strip in rows, 0 when none was found)
    int64_t found_plane = 0, found_strip = 0;
    spmmh::Transpose tr;
    spmm_plan_s* tplan = nullptr;  // plan over A^T (k rows, m columns)
    // One-call plans of the merge kernel: a host-visible word the partition
    // re-check sets when the row offsets passed no longer end at nnz
    // (pinned host memory and its device address).
    int* guard_host = nullptr;
    int* guard_dev = nullptr;
    int* aux_dev = nullptr;  // one-call plans: row statistics and nnz read back at creation
};

namespace spmmh {

// Merge items per workgroup of the SDDMM kernel (and of the atomic dB
// scatter). Timed on the GCN and power-law matrices at n = 64 and 128 in
// FP32 and BF16, pieces of 512 to 1024 items were 3-6 % faster than 2048
// (more workgroups per CU for the 8 KB of staged row ends and columns)
// and 256 slower again. A merge plan with pieces of this size shares its
// own partition; every other plan gets one at creation.
constexpr int kSddmmW = 1024;

// Whether SDDMM and the atomic dB scatter run on the plan's own partition:
// a merge plan (diagonal pieces) whose pieces hold kSddmmW items.
inline bool sddmm_shares_partition(const spmm_plan_s& p) {
    return p.cfg.kernel == SPMM_KERNEL_MERGE && p.cfg.items_per_wg == kSddmmW;
}

bool plan_alive(const spmm_plan_s* p);
bool aligned16(const void* ptr);
void slot_geometry(int64_t n, int vec, int* g_log2, int* col_tiles, int tile_cols = 0);
int elem_bytes(int dtype);
int vec16(int dtype);
spmmk::Shape resolve_shape(const spmm_plan_s& p, int vec);
int forward(const spmm_plan_s& p, const int* rowptr, const int* colind, const void* vals,
            const void* B, float* C, hipStream_t st, hipEvent_t ev_before = nullptr,
            hipEvent_t ev_after = nullptr, int semiring = SPMM_PLUS_TIMES);
// Options of plan creation used inside the library: a fixed unroll for every
// candidate, and buffers of the caller to time candidates on (else scratch).
struct TuneOpts {
    int fixed_unroll = 0;
    int max_W = 0;  // largest merge piece allowed (0: no limit)
    bool rowblock = true;  // the row-block kernel may be a candidate
    bool panels = true;    // column panels may be a candidate
    // row statistics already known (longest row, rows of >= 1024 entries):
    // no statistics pass
    bool known_stats = false;
    int64_t max_row_len = 0, long_rows = 0;
    bool no_sddmm = false;  // no SDDMM partition (a plan that never runs SDDMM)
    bool no_sync = false;   // do not synchronise the stream at the end
    bool no_planes = false; // no plane-structure pass (the tile order stays the row order)
    const void* vals = nullptr;
    const void* B = nullptr;
    float* C = nullptr;
};

int create_plan(spmm_plan_t* out, const int32_t* rowptr, const int32_t* colind, int64_t m,
                int64_t k, int64_t nnz, int64_t n, int64_t ld, int32_t dtype, int32_t mode,
                const spmm_config* forced, hipStream_t st, bool register_plan,
                const TuneOpts* opts = nullptr);
void destroy_plan(spmm_plan_s* p);
// Host checks of sizes (signs, int32 limits, the nnz cap, ld >= max(1, n)).
int check_dims(int64_t m, int64_t k, int64_t nnz, int64_t n, int64_t ld);

}  // namespace spmmh
