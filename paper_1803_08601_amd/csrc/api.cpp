// C ABI of the library: argument checks, plans (kernel choice by the Sec. 5.4
// rule or by timing), the merge-path workspace, the one-call entry point with
// its plan cache, and CSR validation. See include/spmm.h for the contract.

#include <hip/hip_runtime.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <memory>
#include <mutex>
#include <set>
#include <string>
#include <tuple>
#include <vector>

#include "plan.hpp"
#include "rowblock.hpp"

namespace spmmh {

static thread_local std::string t_err;

int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    t_err = buf;
    return code;
}

int hip_fail(hipError_t e, const char* what) {
    return fail(SPMM_ERR_HIP, "%s failed: %s", what, hipGetErrorString(e));
}

static std::mutex g_mu;
static std::set<const spmm_plan_s*> g_plans;

bool plan_alive(const spmm_plan_s* p) {
    std::lock_guard<std::mutex> lk(g_mu);
    return p && g_plans.count(p);
}

int elem_bytes(int dtype) { return dtype == SPMM_F32 ? 4 : 2; }
int vec16(int dtype) { return dtype == SPMM_F32 ? 4 : 8; }

static int ilog2_ceil(int64_t x) {
    int l = 0;
    while ((int64_t(1) << l) < x) ++l;
    return l;
}

// Lanes that cover one column tile of a B row (the whole row up to a
// wavefront, or tile_cols columns when given) and the number of column tiles.
void slot_geometry(int64_t n, int vec, int* g_log2, int* col_tiles, int tile_cols) {
    const int64_t width = tile_cols > 0 && tile_cols < n ? tile_cols : n;
    int64_t lanes = (width + vec - 1) / vec;
    if (lanes < 1) lanes = 1;
    if (lanes > spmmk::kWaveSize) lanes = spmmk::kWaveSize;
    *g_log2 = ilog2_ceil(lanes);
    const int64_t span = int64_t(vec) << *g_log2;
    *col_tiles = (int)((n + span - 1) / span);
    if (*col_tiles < 1) *col_tiles = 1;
}

// Tile order (spmm_config.tile_order): strips across planes when the plan
// found plane structure and, in the automatic choice, one plane's B rows are
// more than one XCD's L2 holds.
constexpr int64_t kL2Bytes = int64_t(4) << 20;
constexpr int64_t kStripBytes = int64_t(2) << 20;

spmmk::Shape resolve_shape(const spmm_plan_s& p, int vec) {
    spmmk::Shape s;
    s.vec = vec;
    slot_geometry(p.n, vec, &s.g_log2, &s.col_tiles, p.cfg.tile_cols);
    int lpr = std::max<int>(p.cfg.lanes_per_row, 1 << s.g_log2);
    lpr = std::min(lpr, spmmk::kWaveSize);
    s.ts_log2 = ilog2_ceil(lpr) - s.g_log2;
    s.unroll = p.cfg.unroll;
    s.W = p.cfg.items_per_wg;
    s.nz = p.cfg.kernel == SPMM_KERNEL_NZSPLIT ? 1 : 0;
    const int64_t row_bytes = p.ld * elem_bytes(p.dtype);
    s.short_addr = p.k < (int64_t(1) << 24) && row_bytes < (int64_t(1) << 24) &&
                   p.k * row_bytes <= int64_t(0xffffffff);
    const bool rows = p.cfg.kernel == SPMM_KERNEL_ROWSPLIT || p.cfg.kernel == SPMM_KERNEL_ROWBLOCK;
    const bool use = p.found_strip > 0 &&
                     (p.cfg.tile_order == 2 ||
                      (p.cfg.tile_order == 0 && p.found_plane * row_bytes > kL2Bytes));
    if (rows && use) {
        s.plane_rows = p.found_plane;
        s.strip_rows = p.found_strip;
    }
    return s;
}

bool aligned16(const void* ptr) { return (reinterpret_cast<uintptr_t>(ptr) & 15u) == 0; }

static size_t lds_limit() {
    static size_t lim = 0;
    if (!lim) {
        int dev = 0;
        hipDeviceProp_t prop;
        if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
            lim = prop.sharedMemPerBlock;
        if (!lim) lim = 65536;
    }
    return lim;
}

static bool is_merge(int kernel) {
    return kernel == SPMM_KERNEL_MERGE || kernel == SPMM_KERNEL_NZSPLIT;
}

int forward(const spmm_plan_s& p, const int* rowptr, const int* colind, const void* vals,
            const void* B, float* C, hipStream_t st, hipEvent_t ev_before, hipEvent_t ev_after,
            int semiring) {
    if (p.m == 0 || p.n == 0) return SPMM_OK;
    int vec = p.cfg.vec;
    if (vec != 1 && (!aligned16(B) || !aligned16(C))) vec = 1;
    const spmmk::Shape s = resolve_shape(p, vec);
    const bool merge = is_merge(p.cfg.kernel);
    if (merge && !p.ws.coords) return fail(SPMM_ERR_STATE, "merge plan without partition");
    const spmmk::ForwardArgs a{rowptr, colind, vals, B, C, p.m, p.n, p.ld,
                               p.ws.coords, p.ws.P, p.ws.carry_vals, p.ws.carry_rows};
    if (ev_before) SPMM_HIP(hipEventRecord(ev_before, st));
    if (p.cfg.kernel == SPMM_KERNEL_ROWBLOCK && semiring == SPMM_PLUS_TIMES) {
        if (!p.rb.ub_ptr) return fail(SPMM_ERR_STATE, "row-block plan without its structure");
        const hipError_t e = spmmk::launch_rowblock(p.dtype, s, p.rb.R, a, p.rb.ub_ptr,
                                                    p.rb.words, st, ev_after);
        if (e != hipSuccess) return hip_fail(e, "row-block launch");
        return SPMM_OK;
    }
    if (p.cfg.kernel == SPMM_KERNEL_ROWSPLIT && p.cfg.col_panels >= 2) {
        // one row-split pass per column panel, each adding into C after the first
        if (!p.cp.starts || p.cp.P != p.cfg.col_panels)
            return fail(SPMM_ERR_STATE, "column-panel plan without its panel starts");
        for (int q = 0; q < p.cp.P; ++q) {
            spmmk::ForwardArgs aq = a;
            aq.rowptr = p.cp.starts + (int64_t)q * p.m;
            aq.rowend = p.cp.starts + (int64_t)(q + 1) * p.m;
            aq.accumulate = q > 0;
            const hipError_t e =
                semiring == SPMM_PLUS_TIMES
                    ? spmmk::launch_forward_plus_times(p.dtype, false, s, aq, st,
                                                       q == p.cp.P - 1 ? ev_after : nullptr)
                    : spmmk::launch_forward_semiring(semiring, p.dtype, false, s, aq, st);
            if (e != hipSuccess) return hip_fail(e, "column-panel launch");
        }
        return SPMM_OK;
    }
    // (other semirings on a row-block plan run row split with its lane shape)
    const hipError_t e =
        semiring == SPMM_PLUS_TIMES
            ? spmmk::launch_forward_plus_times(p.dtype, merge, s, a, st, ev_after)
            : spmmk::launch_forward_semiring(semiring, p.dtype, merge, s, a, st);
    if (e != hipSuccess) return hip_fail(e, merge ? "merge-based launch" : "row-split launch");
    return SPMM_OK;
}

static void free_ws(MergeWs& ws) {
    if (ws.coords) (void)hipFree(ws.coords);
    if (ws.carry_vals) (void)hipFree(ws.carry_vals);
    if (ws.carry_rows) (void)hipFree(ws.carry_rows);
    ws = MergeWs{};
}

// Pieces of the merge walk: diagonal pieces of W merge items, or (nonzero
// split) pieces of W nonzeros, at least one when there are rows.
static int64_t num_pieces(int64_t m, int64_t nnz, int W, bool nz) {
    if (!nz) return (m + nnz + W - 1) / W;
    if (m == 0) return 0;
    return std::max<int64_t>(1, (nnz + W - 1) / W);
}

// Allocate (if needed) and fill the merge workspace for W items per piece.
static int prepare_merge(const spmm_plan_s& p, MergeWs& ws, int W, bool nz, hipStream_t st) {
    const int64_t P = num_pieces(p.m, p.nnz, W, nz);
    if (P > ws.cap_P || p.n > ws.cap_n || !ws.coords) {
        free_ws(ws);
        const int64_t capP = std::max<int64_t>(P, 1);
        const int64_t capn = std::max<int64_t>(p.n, 1);
        SPMM_HIP(hipMalloc(&ws.coords, sizeof(int) * 2 * (capP + 1)));
        SPMM_HIP(hipMalloc(&ws.carry_vals, sizeof(float) * capP * capn));
        SPMM_HIP(hipMalloc(&ws.carry_rows, sizeof(int) * capP));
        ws.cap_P = capP;
        ws.cap_n = capn;
    }
    ws.P = P;
    hipError_t e = spmmk::launch_merge_partition(p.rowptr, p.m, p.nnz, W, P, nz ? 1 : 0,
                                                 ws.coords, st);
    if (e != hipSuccess) return hip_fail(e, "merge partition launch");
    return SPMM_OK;
}

static void free_cp(ColPanels& cp) {
    if (cp.starts) (void)hipFree(cp.starts);
    cp = ColPanels{};
}

// Panel starts of P column panels of ceil(k / P) columns each.
static int prepare_panels(const spmm_plan_s& p, ColPanels& cp, int P, hipStream_t st) {
    if (cp.starts && cp.P == P) return SPMM_OK;
    free_cp(cp);
    const int64_t width = (p.k + P - 1) / P;
    SPMM_HIP(hipMalloc(&cp.starts, sizeof(int) * std::max<int64_t>(1, (int64_t)(P + 1) * p.m)));
    const hipError_t e = spmmk::launch_panel_starts(p.rowptr, p.colind, p.m, P, width, cp.starts, st);
    if (e != hipSuccess) {
        free_cp(cp);
        return hip_fail(e, "panel starts");
    }
    cp.P = P;
    return SPMM_OK;
}

static void free_rb(RowBlocks& rb) {
    if (rb.ub_ptr) (void)hipFree(rb.ub_ptr);
    if (rb.words) (void)hipFree(rb.words);
    rb = RowBlocks{};
}

// Whether every row's column indices strictly increase (once per plan).
static int ensure_sorted(spmm_plan_s& p, hipStream_t st) {
    if (p.sorted >= 0) return SPMM_OK;
    if (p.m == 0 || p.nnz == 0) {
        p.sorted = 1;
        return SPMM_OK;
    }
    int* d = nullptr;
    int h = 0;
    SPMM_HIP(hipMalloc(&d, sizeof(int)));
    hipError_t e = hipMemsetAsync(d, 0, sizeof(int), st);
    if (e == hipSuccess) e = spmmk::launch_rowblock_check_sorted(p.rowptr, p.colind, p.m, d, st);
    if (e == hipSuccess) e = hipMemcpyAsync(&h, d, sizeof(int), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    (void)hipFree(d);
    if (e != hipSuccess) return hip_fail(e, "row order check");
    p.sorted = h ? 0 : 1;
    return SPMM_OK;
}

// Build the row-block structure for blocks of R rows: union sizes, their
// scan, then the union words. One host sync (the total size).
static int prepare_rowblock(const spmm_plan_s& p, RowBlocks& rb, int R, hipStream_t st) {
    if (rb.ub_ptr && rb.R == R) return SPMM_OK;
    free_rb(rb);
    const int64_t mb = (p.m + R - 1) / R;
    int* sums = nullptr;
    hipError_t e = hipMalloc(&rb.ub_ptr, sizeof(int) * (mb + 1));
    if (e == hipSuccess)
        e = hipMalloc(&sums, sizeof(int) * std::max<int64_t>(1, spmmk::scan_chunks(mb + 1)));
    if (e == hipSuccess) e = hipMemsetAsync(rb.ub_ptr + mb, 0, sizeof(int), st);
    if (e == hipSuccess)
        e = spmmk::launch_rowblock_union(p.rowptr, p.colind, p.m, R, nullptr, rb.ub_ptr, st);
    if (e == hipSuccess) e = spmmk::exclusive_scan_i32(rb.ub_ptr, mb + 1, sums, st);
    int total = 0;
    if (e == hipSuccess)
        e = hipMemcpyAsync(&total, rb.ub_ptr + mb, sizeof(int), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (sums) (void)hipFree(sums);
    if (e == hipSuccess) e = hipMalloc(&rb.words, sizeof(int) * std::max(1, total));
    if (e == hipSuccess)
        e = spmmk::launch_rowblock_union(p.rowptr, p.colind, p.m, R, rb.ub_ptr, rb.words, st);
    if (e != hipSuccess) {
        free_rb(rb);
        return hip_fail(e, "row-block structure");
    }
    rb.mb = mb;
    rb.U = total;
    rb.R = R;
    return SPMM_OK;
}

// Plane structure of A for the tile order: the offsets colind - row form a
// near cluster (|offset| <= near) and a far one, from far_lo to hi, around
// +-D = (far_lo + hi) / 2 and no wider than the near one, with D at least 16
// times the near extent (a 3-D stencil: D = one grid plane). The strip S is
// the largest power of two dividing D whose rows' B rows for three planes
// take at most kStripBytes. Computed once per plan (two passes over colind
// and one synchronisation).
static int find_planes(spmm_plan_s& p, hipStream_t st) {
    p.found_plane = p.found_strip = 0;
    if (p.m == 0 || p.nnz == 0) return SPMM_OK;
    int* d = nullptr;
    int h[3] = {0, 0, INT32_MAX};
    SPMM_HIP(hipMalloc(&d, sizeof h));
    hipError_t e = hipMemcpyAsync(d, h, sizeof h, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = spmmk::launch_offset_stats(p.rowptr, p.colind, p.m, d, st);
    if (e == hipSuccess) e = hipMemcpyAsync(h, d, sizeof h, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    (void)hipFree(d);
    if (e != hipSuccess) return hip_fail(e, "offset statistics");
    const int64_t hi = h[0], near = std::max(h[1], 1), far_lo = h[2];
    if (far_lo == INT32_MAX || hi < 2) return SPMM_OK;
    const int64_t D = (far_lo + hi) / 2;
    if (hi - far_lo > 2 * near + 2 || D < 16 * near) return SPMM_OK;
    const int64_t row_bytes = p.ld * elem_bytes(p.dtype);
    int64_t S = 1;
    while (S * 2 * 3 * row_bytes <= kStripBytes) S *= 2;
    while (S > 1 && D % S) S /= 2;
    if (S < 64 || S >= D) return SPMM_OK;
    p.found_plane = D;
    p.found_strip = S;
    return SPMM_OK;
}

// Column panels: at most kMaxPanels; autotuner candidates when the rows hold
// kPanelMinMean entries or more on average and B is larger than an L2, with
// panels whose B slice is about kPanelBytes.
constexpr int kMaxPanels = 64;
constexpr double kPanelMinMean = 64.0;
constexpr int64_t kPanelBytes = int64_t(2) << 20;

// Distinct columns per entry of blocks of 2 rows at or below which row blocks
// are worth trying (mode RULE also needs n >= kRuleMinN).
constexpr double kRuleUnionRatio = 0.9;
constexpr int64_t kRuleMinN = 32;

static int check_config(const spmm_plan_s& p, spmm_config& c) {
    const int v16 = vec16(p.dtype);
    const bool can16 = (p.n % v16 == 0) && (p.ld % v16 == 0);
    if (c.kernel != SPMM_KERNEL_ROWSPLIT && c.kernel != SPMM_KERNEL_MERGE &&
        c.kernel != SPMM_KERNEL_NZSPLIT && c.kernel != SPMM_KERNEL_ROWBLOCK)
        return fail(SPMM_ERR_INVALID, "config.kernel %d is not a kernel", c.kernel);
    if (c.kernel == SPMM_KERNEL_ROWBLOCK) {
        if (c.rows_per_block == 0) c.rows_per_block = 2;
        if (c.rows_per_block != 2 && c.rows_per_block != 4 && c.rows_per_block != 8)
            return fail(SPMM_ERR_UNSUPPORTED, "config.rows_per_block %d: use 2, 4 or 8",
                        c.rows_per_block);
        if (p.k >= (int64_t(1) << spmmk::kRowBlockColBits))
            return fail(SPMM_ERR_UNSUPPORTED, "row-block kernel needs k < 2^24 (k = %lld)",
                        (long long)p.k);
        if (p.sorted != 1)
            return fail(SPMM_ERR_UNSUPPORTED,
                        "row-block kernel needs strictly increasing column indices in every row");
    } else {
        c.rows_per_block = 0;
    }
    if (c.tile_order < 0 || c.tile_order > 2)
        return fail(SPMM_ERR_INVALID, "config.tile_order %d: use 0, 1 or 2", c.tile_order);
    if (c.col_panels == 1) c.col_panels = 0;
    if (c.col_panels != 0) {
        if (c.kernel != SPMM_KERNEL_ROWSPLIT)
            return fail(SPMM_ERR_UNSUPPORTED, "config.col_panels needs the row-split kernel");
        if (c.col_panels < 2 || c.col_panels > kMaxPanels)
            return fail(SPMM_ERR_UNSUPPORTED, "config.col_panels %d: use 0 .. %d", c.col_panels,
                        kMaxPanels);
        if (p.sorted != 1)
            return fail(SPMM_ERR_UNSUPPORTED,
                        "column panels need strictly increasing column indices in every row");
    }
    if (c.vec == 0) c.vec = can16 ? v16 : 1;
    if (c.vec != 1 && c.vec != v16)
        return fail(SPMM_ERR_UNSUPPORTED, "config.vec %d: use 1 or %d for this dtype", c.vec, v16);
    if (c.vec == v16 && !can16)
        return fail(SPMM_ERR_UNSUPPORTED, "config.vec %d needs n and ld divisible by %d", c.vec, v16);
    if (c.tile_cols < 0 || (c.tile_cols % c.vec) != 0)
        return fail(SPMM_ERR_UNSUPPORTED, "config.tile_cols %d: a multiple of vec %d", c.tile_cols,
                    c.vec);
    int g_log2, tiles;
    slot_geometry(p.n, c.vec, &g_log2, &tiles, c.tile_cols);
    const int g = 1 << g_log2;
    if (c.unroll == 0) c.unroll = 4;
    if (c.unroll != 1 && c.unroll != 2 && c.unroll != 4 && c.unroll != 8)
        return fail(SPMM_ERR_UNSUPPORTED, "config.unroll %d: use 1, 2, 4 or 8", c.unroll);
    if (c.lanes_per_row == 0 && c.kernel == SPMM_KERNEL_ROWBLOCK) {
        // one slot per block: the fastest in the row-block sweep from n = 64 on
        c.lanes_per_row = g;
    } else if (c.lanes_per_row == 0) {
        // about four entries of an average row per slot
        const double d = p.m ? double(p.nnz) / double(p.m) : 0.0;
        int ts = 1;
        while (ts * 2 * g <= spmmk::kWaveSize && ts * 2 * 4 <= d) ts *= 2;
        c.lanes_per_row = ts * g;
    }
    if (c.lanes_per_row < 1 || c.lanes_per_row > spmmk::kWaveSize ||
        (c.lanes_per_row & (c.lanes_per_row - 1)))
        return fail(SPMM_ERR_UNSUPPORTED, "config.lanes_per_row %d: power of two up to 64",
                    c.lanes_per_row);
    if (c.lanes_per_row < g) c.lanes_per_row = g;
    if (c.items_per_wg == 0) {
        const int slots = spmmk::kBlock / g;
        c.items_per_wg = std::max(1024, slots * 8);
    }
    if (c.items_per_wg < 64 || c.items_per_wg > 8192)
        return fail(SPMM_ERR_UNSUPPORTED, "config.items_per_wg %d outside 64..8192", c.items_per_wg);
    if (is_merge(c.kernel)) {
        spmmk::Shape s;
        s.vec = c.vec;
        s.W = c.items_per_wg;
        if (spmmk::merge_lds_bytes(p.dtype, s) > lds_limit())
            return fail(SPMM_ERR_UNSUPPORTED, "items_per_wg %d needs more LDS than a workgroup has",
                        c.items_per_wg);
        if (num_pieces(p.m, p.nnz, c.items_per_wg, c.kernel == SPMM_KERNEL_NZSPLIT) >=
            (int64_t(1) << 31))
            return fail(SPMM_ERR_UNSUPPORTED, "too many merge pieces");
    }
    return SPMM_OK;
}

// ------------------------------------------------------------------ autotuner

struct TuneKey {
    int device;
    int64_t m, k, nnz, n, ld, maxrow, longrows;
    int dtype, unroll, max_W;
    bool rowblock, panels;
    bool operator<(const TuneKey& o) const {
        return std::tie(device, m, k, nnz, n, ld, maxrow, longrows, dtype, unroll, max_W,
                        rowblock, panels) <
               std::tie(o.device, o.m, o.k, o.nnz, o.n, o.ld, o.maxrow, o.longrows, o.dtype,
                        o.unroll, o.max_W, o.rowblock, o.panels);
    }
};
static std::map<TuneKey, std::pair<spmm_config, double>> g_tuned;

static std::vector<spmm_config> tune_candidates(const spmm_plan_s& p, int fixed_unroll,
                                                int max_W, bool rowblock,
                                                const std::vector<int>& panels) {
    std::vector<spmm_config> out;
    const int v16 = vec16(p.dtype);
    const int vec = (p.n % v16 == 0 && p.ld % v16 == 0) ? v16 : 1;
    std::vector<int> unrolls = {2, 4, 8};
    if (fixed_unroll) unrolls = {fixed_unroll};
    // Column tiles: the full row width, and for wide rows half of it (each
    // tile re-reads A but gathers only its half of every B row, which halves
    // the set of B lines a workgroup keeps in cache).
    std::vector<int> tiles = {0};
    if (p.n >= 64 && p.n % (2 * vec) == 0) tiles.push_back((int)(p.n / 2));
    // Merge-based first: its time does not depend on row lengths, so it sets
    // a bar that lets hopeless row-split shapes stop after one run. Row split
    // goes from whole-wavefront teams (best for long rows) down.
    for (int tc : tiles) {
        int g_log2, nt;
        slot_geometry(p.n, vec, &g_log2, &nt, tc);
        for (int W : {2048, 1024, 4096, 512})
            if (!max_W || W <= max_W)
                for (int u : unrolls) out.push_back({SPMM_KERNEL_MERGE, vec, 1 << g_log2, u, W, tc});
    }
    // The nonzero split (the paper's own merge-based partition) after the
    // diagonal one: within the tie margin the earlier candidate is kept.
    for (int tc : tiles) {
        int g_log2, nt;
        slot_geometry(p.n, vec, &g_log2, &nt, tc);
        for (int W : {2048, 1024})
            if (!max_W || W <= max_W)
                for (int u : unrolls)
                    out.push_back({SPMM_KERNEL_NZSPLIT, vec, 1 << g_log2, u, W, tc});
    }
    for (int tc : tiles) {
        int g_log2, nt;
        slot_geometry(p.n, vec, &g_log2, &nt, tc);
        for (int lpr = spmmk::kWaveSize; lpr >= (1 << g_log2); lpr /= 2)
            for (int u : unrolls) out.push_back({SPMM_KERNEL_ROWSPLIT, vec, lpr, u, 1024, tc});
    }
    // Row blocks last: chosen only when faster than every kernel of the paper
    // by more than the tie margin.
    if (rowblock)
        for (int R : {2, 4})
            for (int tc : tiles) {
                int g_log2, nt;
                slot_geometry(p.n, vec, &g_log2, &nt, tc);
                for (int lpr = spmmk::kWaveSize; lpr >= (1 << g_log2); lpr /= 2)
                    for (int u : unrolls)
                        out.push_back({SPMM_KERNEL_ROWBLOCK, vec, lpr, u, 1024, tc, R});
            }
    // Column panels (long sorted rows, B larger than an L2): row split with
    // whole or half wavefronts per row, one pass per panel.
    for (int P : panels) {
        int g_log2, nt;
        slot_geometry(p.n, vec, &g_log2, &nt, 0);
        for (int lpr : {spmmk::kWaveSize, spmmk::kWaveSize / 2})
            if (lpr >= (1 << g_log2))
                for (int u : unrolls)
                    out.push_back({SPMM_KERNEL_ROWSPLIT, vec, lpr, u, 1024, 0, 0, 0, P});
    }
    return out;
}

static int autotune(spmm_plan_s& p, hipStream_t st, const TuneOpts* opts) {
    const int fixed_unroll = opts ? opts->fixed_unroll : 0;
    const int max_W = opts ? opts->max_W : 0;
    const bool own = opts && opts->C && (p.nnz == 0 || (opts->vals && opts->B));
    const TuneKey key{p.device, p.m, p.k, p.nnz, p.n, p.ld, p.max_row_len, p.long_rows, p.dtype,
                      fixed_unroll, max_W, !opts || opts->rowblock, !opts || opts->panels};
    {
        std::pair<spmm_config, double> hit{};
        bool found = false;
        {
            std::lock_guard<std::mutex> lk(g_mu);
            auto it = g_tuned.find(key);
            if (it != g_tuned.end()) {
                hit = it->second;
                found = true;
            }
        }
        // A cached row-block choice holds only for a matrix with sorted rows
        // (the key does not see the order of columns): else tune afresh.
        if (found && (hit.first.kernel == SPMM_KERNEL_ROWBLOCK || hit.first.col_panels >= 2)) {
            const int rc0 = ensure_sorted(p, st);
            if (rc0 != SPMM_OK) return rc0;
            found = p.sorted == 1;
        }
        if (found) {
            // entries loaded from a file pass the checks of a forced shape;
            // one this matrix cannot use is tuned afresh
            spmm_config c = hit.first;
            if (check_config(p, c) == SPMM_OK) {
                p.cfg = c;
                p.tuned_ms = hit.second;
                return SPMM_OK;
            }
        }
    }
    if (p.m == 0 || p.n == 0) {
        p.cfg = spmm_config{p.paper_choice, 0, 0, fixed_unroll, 0, 0};
        return check_config(p, p.cfg);
    }
    const int eb = elem_bytes(p.dtype);
    void *vals = nullptr, *B = nullptr;
    float* C = nullptr;
    const void* use_vals = own ? opts->vals : nullptr;
    const void* use_B = own ? opts->B : nullptr;
    float* use_C = own ? opts->C : nullptr;
    MergeWs ws;
    RowBlocks rb2, rb4;  // row-block structures of the candidates
    std::map<int, ColPanels> cps;  // panel starts of the column-panel candidates
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc = SPMM_OK;
    auto cleanup = [&]() {
        if (vals) (void)hipFree(vals);
        if (B) (void)hipFree(B);
        if (C) (void)hipFree(C);
        free_ws(ws);
        free_rb(rb2);
        free_rb(rb4);
        for (auto& kv : cps) free_cp(kv.second);
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
    };
#define TUNE_HIP(call)                                  \
    do {                                                \
        hipError_t e_ = (call);                         \
        if (e_ != hipSuccess) {                         \
            rc = hip_fail(e_, #call);                   \
            cleanup();                                  \
            return rc;                                  \
        }                                               \
    } while (0)
    if (!own) {
        if (p.nnz > 0) TUNE_HIP(hipMalloc(&vals, (size_t)eb * p.nnz));
        if (p.k > 0) TUNE_HIP(hipMalloc(&B, (size_t)eb * p.k * p.ld));
        TUNE_HIP(hipMalloc(&C, sizeof(float) * p.m * p.ld));
        if (vals) TUNE_HIP(hipMemsetAsync(vals, 0x3c, (size_t)eb * p.nnz, st));
        if (B) TUNE_HIP(hipMemsetAsync(B, 0x3c, (size_t)eb * p.k * p.ld, st));
        use_vals = vals;
        use_B = B;
        use_C = C;
    }
    TUNE_HIP(hipEventCreate(&e0));
    TUNE_HIP(hipEventCreate(&e1));

    // The row-block kernel is a candidate for sorted rows of moderate length
    // whose blocks of 2 rows share enough columns to save gathers (the same
    // test as mode RULE, without its bound on n).
    bool rowblock = (!opts || opts->rowblock) && p.nnz > 0 &&
                    p.k < (int64_t(1) << spmmk::kRowBlockColBits) && p.max_row_len <= 4096;
    if (rowblock) {
        rc = ensure_sorted(p, st);
        if (rc != SPMM_OK) { cleanup(); return rc; }
        rowblock = p.sorted == 1;
    }
    if (rowblock) {
        rc = prepare_rowblock(p, rb2, 2, st);
        if (rc != SPMM_OK) { cleanup(); return rc; }
        rowblock = double(rb2.U) <= kRuleUnionRatio * double(p.nnz);
        if (!rowblock) free_rb(rb2);
    }

    // Column panels for long sorted rows when B does not fit an L2: about
    // kPanelBytes of B per panel (P0, a power of two), and half and twice that.
    std::vector<int> panels;
    const int64_t b_bytes = p.k * p.ld * elem_bytes(p.dtype);
    const double mean = p.m ? double(p.nnz) / double(p.m) : 0.0;
    if ((!opts || opts->panels) && p.nnz > 0 && mean >= kPanelMinMean && b_bytes > kL2Bytes) {
        rc = ensure_sorted(p, st);
        if (rc != SPMM_OK) { cleanup(); return rc; }
        if (p.sorted == 1) {
            int P0 = 2;
            while (P0 < kMaxPanels && int64_t(P0) * kPanelBytes < b_bytes) P0 *= 2;
            for (int P : {P0 / 2, P0, P0 * 2})
                if (P >= 2 && P <= kMaxPanels && mean >= 4.0 * P) panels.push_back(P);
        }
    }

    // Candidates within kTie (1.5 %, above the run-to-run spread of the
    // median) of the fastest count as equal; the earliest in
    // candidate order wins, so repeated tuning of one matrix picks one shape.
    constexpr double kTie = 1.015;
    double best = 1e30;
    std::vector<std::pair<spmm_config, double>> timed;
    int slow_rowsplit = 0;
    for (spmm_config c : tune_candidates(p, fixed_unroll, max_W, rowblock, panels)) {
        if (c.kernel == SPMM_KERNEL_ROWSPLIT && slow_rowsplit >= 3) continue;
        spmm_plan_s q = p;  // shallow copy: never destroyed
        q.ws = MergeWs{};
        q.rb = RowBlocks{};
        q.cp = ColPanels{};
        if (check_config(q, c) != SPMM_OK) continue;
        q.cfg = c;
        if (is_merge(c.kernel)) {
            rc = prepare_merge(q, ws, c.items_per_wg, c.kernel == SPMM_KERNEL_NZSPLIT, st);
            if (rc != SPMM_OK) { cleanup(); return rc; }
            q.ws = ws;
        }
        if (c.kernel == SPMM_KERNEL_ROWBLOCK) {
            RowBlocks& rb = c.rows_per_block == 2 ? rb2 : rb4;
            rc = prepare_rowblock(p, rb, c.rows_per_block, st);
            if (rc != SPMM_OK) { cleanup(); return rc; }
            q.rb = rb;
        }
        if (c.col_panels >= 2) {
            rc = prepare_panels(p, cps[c.col_panels], c.col_panels, st);
            if (rc != SPMM_OK) { cleanup(); return rc; }
            q.cp = cps[c.col_panels];
        }
        std::vector<float> times;
        for (int rep = 0; rep < 6; ++rep) {
            TUNE_HIP(hipEventRecord(e0, st));
            rc = forward(q, q.rowptr, q.colind, use_vals, use_B, use_C, st);
            if (rc != SPMM_OK) { cleanup(); return rc; }
            TUNE_HIP(hipEventRecord(e1, st));
            TUNE_HIP(hipEventSynchronize(e1));
            float ms = 0.f;
            TUNE_HIP(hipEventElapsedTime(&ms, e0, e1));
            if (rep > 0) times.push_back(ms);
            if (rep == 0 && ms > 2.0 * best) break;  // clearly slower: skip the timed reps
        }
        if (times.empty()) {
            if (c.kernel == SPMM_KERNEL_ROWSPLIT) ++slow_rowsplit;
            continue;
        }
        std::sort(times.begin(), times.end());
        const double med = times[times.size() / 2];
        if (c.kernel == SPMM_KERNEL_ROWSPLIT) slow_rowsplit = med > 3.0 * best ? slow_rowsplit + 1 : 0;
        best = std::min(best, med);
        timed.push_back({c, med});
    }
    spmm_config best_cfg{};
    double best_ms = 1e30;
    for (const auto& t : timed) {
        if (t.second <= best * kTie) {
            best_cfg = t.first;
            best_ms = t.second;
            break;
        }
    }
    if (best_cfg.kernel == SPMM_KERNEL_ROWBLOCK && best_ms < 1e30) {
        // hand the chosen structure to the plan
        RowBlocks& rb = best_cfg.rows_per_block == 2 ? rb2 : rb4;
        free_rb(p.rb);
        p.rb = rb;
        rb = RowBlocks{};
    }
    if (best_cfg.col_panels >= 2 && best_ms < 1e30) {
        free_cp(p.cp);
        p.cp = cps[best_cfg.col_panels];
        cps[best_cfg.col_panels] = ColPanels{};
    }
    cleanup();
#undef TUNE_HIP
    if (best_ms >= 1e30) return fail(SPMM_ERR_UNSUPPORTED, "autotune: no candidate ran");
    p.cfg = best_cfg;
    p.tuned_ms = best_ms;
    std::lock_guard<std::mutex> lk(g_mu);
    g_tuned[key] = {best_cfg, best_ms};
    return SPMM_OK;
}

// ------------------------------------------------------------------ plans

static int row_stats(spmm_plan_s& p, hipStream_t st) {
    if (p.m == 0) return SPMM_OK;
    int* d = nullptr;
    int h[3] = {0, 0, 1};
    SPMM_HIP(hipMalloc(&d, sizeof h));
    hipError_t e = hipMemcpyAsync(d, h, sizeof h, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = spmmk::launch_row_stats(p.rowptr, p.m, d, st);
    if (e == hipSuccess) e = hipMemcpyAsync(h, d, sizeof h, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    (void)hipFree(d);
    if (e != hipSuccess) return hip_fail(e, "row statistics");
    p.max_row_len = h[0];
    p.long_rows = h[1];
    return SPMM_OK;
}

// Kernel choice re-derived on MI355X (mode RULE): merge-based for very short
// rows on average (mean below 4) and whenever one row is long enough that a
// single row-split team would hold up the grid (4096 entries or more).
static int rule_choice(const spmm_plan_s& p) {
    if (p.m == 0) return SPMM_KERNEL_ROWSPLIT;
    const bool short_rows = p.nnz < 4 * p.m;
    const bool long_row = p.max_row_len >= 4096;
    return short_rows || long_row ? SPMM_KERNEL_MERGE : SPMM_KERNEL_ROWSPLIT;
}

// Row blocks in mode RULE (from the row-block sweep on MI355X): for a matrix
// row split would take, when n >= 32, the rows are sorted, k < 2^24 and blocks
// of 2 rows hold at most 0.9 distinct columns per entry. Builds the
// structure for blocks of 2 rows, kept when chosen.

static int rule_rowblock(spmm_plan_s& p, hipStream_t st, bool* chosen) {
    *chosen = false;
    if (p.n < kRuleMinN || p.nnz == 0 || p.k >= (int64_t(1) << spmmk::kRowBlockColBits) ||
        p.max_row_len > 4096)
        return SPMM_OK;
    int rc = ensure_sorted(p, st);
    if (rc != SPMM_OK || p.sorted != 1) return rc;
    rc = prepare_rowblock(p, p.rb, 2, st);
    if (rc != SPMM_OK) return rc;
    *chosen = double(p.rb.U) <= kRuleUnionRatio * double(p.nnz);
    if (!*chosen) free_rb(p.rb);
    return SPMM_OK;
}

// Largest nnz: entry indices are int32 in the kernels, and their chunk loops
// step up to 4096 entries past an index below nnz without overflowing.
constexpr int64_t kMaxNnz = (int64_t(1) << 31) - 1 - 4096;

int check_dims(int64_t m, int64_t k, int64_t nnz, int64_t n, int64_t ld) {
    const int64_t lim = (int64_t(1) << 31) - 1;
    if (m < 0 || k < 0 || nnz < 0 || n < 0)
        return fail(SPMM_ERR_INVALID, "negative size (m=%lld k=%lld nnz=%lld n=%lld)",
                    (long long)m, (long long)k, (long long)nnz, (long long)n);
    if (m > lim || k > lim || nnz > lim || n > lim)
        return fail(SPMM_ERR_UNSUPPORTED, "sizes must fit int32");
    if (nnz > kMaxNnz)
        return fail(SPMM_ERR_UNSUPPORTED, "nnz = %lld: at most 2^31 - 4097 entries",
                    (long long)nnz);
    if (ld < std::max<int64_t>(1, n))
        return fail(SPMM_ERR_INVALID, "ld=%lld must be >= max(1, n=%lld)", (long long)ld,
                    (long long)n);
    if (m > 0 && nnz > 0 && k == 0) return fail(SPMM_ERR_INVALID, "nnz > 0 with k == 0");
    return SPMM_OK;
}

void destroy_plan(spmm_plan_s* p) {
    if (!p) return;
    (void)hipDeviceSynchronize();
    free_ws(p->ws);
    free_ws(p->sddmm_ws);
    free_rb(p->rb);
    free_cp(p->cp);
    if (p->tr.at_rowptr) (void)hipFree(p->tr.at_rowptr);
    if (p->tr.at_colind) (void)hipFree(p->tr.at_colind);
    if (p->tr.perm) (void)hipFree(p->tr.perm);
    if (p->tr.at_vals) (void)hipFree(p->tr.at_vals);
    if (p->tplan) destroy_plan(p->tplan);
    if (p->guard_host) (void)hipHostFree(p->guard_host);
    if (p->aux_dev) (void)hipFree(p->aux_dev);
    delete p;
}

int create_plan(spmm_plan_t* out, const int32_t* rowptr, const int32_t* colind, int64_t m,
                int64_t k, int64_t nnz, int64_t n, int64_t ld, int32_t dtype, int32_t mode,
                const spmm_config* forced, hipStream_t st, bool register_plan,
                const TuneOpts* opts) {
    if (!out) return fail(SPMM_ERR_INVALID, "out_plan is NULL");
    *out = nullptr;
    int rc = check_dims(m, k, nnz, n, ld);
    if (rc) return rc;
    if (dtype != SPMM_F32 && dtype != SPMM_BF16 && dtype != SPMM_F16)
        return fail(SPMM_ERR_UNSUPPORTED, "dtype %d", dtype);
    if (!forced && (mode < SPMM_MODE_PAPER || mode > SPMM_MODE_ROWBLOCK))
        return fail(SPMM_ERR_INVALID, "mode %d", mode);
    if (m > 0 && !rowptr) return fail(SPMM_ERR_INVALID, "A_rowptr is NULL");
    if (nnz > 0 && !colind) return fail(SPMM_ERR_INVALID, "A_colind is NULL");

    spmm_plan_s* p = new (std::nothrow) spmm_plan_s;
    if (!p) return fail(SPMM_ERR_NOMEM, "plan");
    p->rowptr = rowptr;
    p->colind = colind;
    p->m = m; p->k = k; p->nnz = nnz; p->n = n; p->ld = ld;
    p->dtype = dtype;
    p->mode = forced ? -1 : mode;
    // Sec. 5.4: merge-based when the mean row length nnz / m is below 9.35.
    p->paper_choice = (m > 0 && 100 * nnz < 935 * m) ? SPMM_KERNEL_MERGE : SPMM_KERNEL_ROWSPLIT;
    hipError_t e = hipGetDevice(&p->device);
    if (e != hipSuccess) { delete p; return hip_fail(e, "hipGetDevice"); }

    if (opts && opts->known_stats) {
        p->max_row_len = opts->max_row_len;
        p->long_rows = opts->long_rows;
    } else {
        rc = row_stats(*p, st);
    }
    const bool want_rowblock = forced ? forced->kernel == SPMM_KERNEL_ROWBLOCK ||
                                            forced->col_panels >= 2
                                      : mode == SPMM_MODE_ROWBLOCK;
    if (rc == SPMM_OK && want_rowblock) rc = ensure_sorted(*p, st);
    // plane structure for the tile order: looked for when B is larger than
    // an L2 (the automatic order needs more than that) or the order is forced
    if (rc == SPMM_OK && p->m > 0 && p->nnz > 0 &&
        ((forced && forced->tile_order == 2) ||
         p->k * p->ld * elem_bytes(p->dtype) > kL2Bytes) &&
        !(forced && (forced->tile_order == 1 || forced->kernel == SPMM_KERNEL_MERGE ||
                     forced->kernel == SPMM_KERNEL_NZSPLIT)) &&
        !(opts && (opts->known_stats || opts->no_planes)))
        rc = find_planes(*p, st);
    if (rc == SPMM_OK) {
        if (forced) {
            p->cfg = *forced;
            rc = check_config(*p, p->cfg);
        } else if (mode == SPMM_MODE_AUTOTUNE) {
            rc = autotune(*p, st, opts);
        } else {
            int kern = mode == SPMM_MODE_PAPER     ? p->paper_choice
                       : mode == SPMM_MODE_RULE    ? rule_choice(*p)
                       : mode == SPMM_MODE_MERGE   ? SPMM_KERNEL_MERGE
                       : mode == SPMM_MODE_NZSPLIT ? SPMM_KERNEL_NZSPLIT
                       : mode == SPMM_MODE_ROWBLOCK ? SPMM_KERNEL_ROWBLOCK
                                                    : SPMM_KERNEL_ROWSPLIT;
            if (mode == SPMM_MODE_RULE && kern == SPMM_KERNEL_ROWSPLIT && (!opts || opts->rowblock)) {
                bool rb = false;
                rc = rule_rowblock(*p, st, &rb);
                if (rb) kern = SPMM_KERNEL_ROWBLOCK;
            }
            p->cfg = spmm_config{kern, 0, 0, opts ? opts->fixed_unroll : 0, 0, 0};
            if (rc == SPMM_OK) rc = check_config(*p, p->cfg);
        }
    }
    if (rc == SPMM_OK && opts && opts->max_W && p->cfg.items_per_wg > opts->max_W)
        p->cfg.items_per_wg = opts->max_W;
    if (rc == SPMM_OK && is_merge(p->cfg.kernel))
        rc = prepare_merge(*p, p->ws, p->cfg.items_per_wg, p->cfg.kernel == SPMM_KERNEL_NZSPLIT,
                           st);
    if (rc == SPMM_OK && p->cfg.kernel == SPMM_KERNEL_ROWBLOCK && p->m > 0)
        rc = prepare_rowblock(*p, p->rb, p->cfg.rows_per_block, st);
    if (rc == SPMM_OK && p->cfg.kernel == SPMM_KERNEL_ROWSPLIT && p->cfg.col_panels >= 2 &&
        p->m > 0)
        rc = prepare_panels(*p, p->cp, p->cfg.col_panels, st);
    // SDDMM walks diagonal merge pieces of kSddmmW items (their row ends fit
    // its LDS); a merge plan of that piece size shares its own partition.
    if (rc == SPMM_OK && !sddmm_shares_partition(*p) && p->m > 0 && p->nnz > 0 &&
        !(opts && opts->no_sddmm))
        rc = prepare_merge(*p, p->sddmm_ws, kSddmmW, false, st);
    if (rc == SPMM_OK && !(opts && opts->no_sync)) {
        e = hipStreamSynchronize(st);
        if (e != hipSuccess) rc = hip_fail(e, "plan synchronise");
    }
    if (rc != SPMM_OK) {
        destroy_plan(p);
        return rc;
    }
    if (register_plan) {
        std::lock_guard<std::mutex> lk(g_mu);
        g_plans.insert(p);
    }
    *out = p;
    return SPMM_OK;
}

// ------------------------------------------------------------------ plan cache

// Cached plans are shared: a call holds its own reference while it enqueues
// work, so an eviction by another thread frees the plan only after that.
using CacheKey =
    std::tuple<const void*, const void*, int64_t, int64_t, int64_t, int64_t, int, const void*>;
using PlanRef = std::shared_ptr<spmm_plan_s>;
static std::map<CacheKey, PlanRef> g_cache;
static std::vector<CacheKey> g_cache_order;  // least recently used first
static constexpr size_t kCacheCap = 64;

static void fill_info(const spmm_plan_s* plan, spmm_plan_info* info) {
    memset(info, 0, sizeof *info);
    info->m = plan->m; info->k = plan->k; info->nnz = plan->nnz; info->n = plan->n;
    info->ld = plan->ld;
    info->dtype = plan->dtype;
    info->mode = plan->mode;
    info->paper_choice = plan->paper_choice;
    info->config = plan->cfg;
    const spmmk::Shape s = resolve_shape(*plan, plan->cfg.vec);
    info->lanes_per_slot = 1 << s.g_log2;
    info->col_tiles = s.col_tiles;
    info->num_parts = is_merge(plan->cfg.kernel) ? plan->ws.P : 0;
    info->max_row_len = plan->max_row_len;
    info->mean_row_len = plan->m ? double(plan->nnz) / double(plan->m) : 0.0;
    info->tuned_ms = plan->tuned_ms;
    info->has_transpose = plan->tr.at_rowptr != nullptr || (plan->k == 0 && plan->tplan);
    info->long_rows = plan->long_rows;
    info->plane_rows = s.plane_rows;
    info->strip_rows = s.strip_rows;
}

// The one-call path plans in mode RULE over the paper's two kernels (row
// blocks are left out: their plan-time column structure would have to be
// kept in step with A_colind). A miss reads back nnz and the row statistics
// together (one stream synchronisation). A cached row-split plan depends on
// the structure only through m; a cached merge plan's partition depends on
// the row offsets, so every call re-checks it on the device first (see
// spmm.h for what happens when the structure changed).
static int csr_create(const int32_t* A_rowptr, const int32_t* A_colind, int64_t m, int64_t k,
                      int64_t n, int64_t ld, hipStream_t st, bool pointers_ok, PlanRef* out) {
    int* aux = nullptr;
    SPMM_HIP(hipMalloc(&aux, 4 * sizeof(int)));
    int h[4] = {0, 0, 1, 0};
    hipError_t e = hipMemcpyAsync(aux, h, 3 * sizeof(int), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = spmmk::launch_row_stats(A_rowptr, m, aux, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(aux + 3, A_rowptr + m, sizeof(int), hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(h, aux, sizeof h, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
        (void)hipFree(aux);
        return hip_fail(e, "one-call structure read-back");
    }
    const int64_t nnz = h[3];
    auto refuse = [&](int code, const char* msg) {
        (void)hipFree(aux);
        return fail(code, "%s", msg);
    };
    if (nnz < 0) return refuse(SPMM_ERR_INVALID, "A_rowptr[m] < 0");
    if (!h[2]) return refuse(SPMM_ERR_INVALID, "A_rowptr[0] != 0 or A_rowptr decreases");
    if (nnz > 0 && !pointers_ok)
        return refuse(SPMM_ERR_INVALID, "A_colind, A_vals or B is NULL");
    TuneOpts o;
    o.rowblock = false;
    o.known_stats = true;
    o.max_row_len = h[0];
    o.long_rows = h[1];
    o.no_sddmm = true;
    o.no_sync = true;
    spmm_plan_s* fresh = nullptr;
    int rc = create_plan(&fresh, A_rowptr, A_colind, m, k, nnz, n, ld, SPMM_F32, SPMM_MODE_RULE,
                         nullptr, st, false, &o);
    if (rc) {
        (void)hipFree(aux);
        return rc;
    }
    fresh->aux_dev = aux;
    if (is_merge(fresh->cfg.kernel)) {
        e = hipHostMalloc(reinterpret_cast<void**>(&fresh->guard_host), sizeof(int),
                          hipHostMallocMapped);
        if (e == hipSuccess) {
            *fresh->guard_host = 0;
            e = hipHostGetDevicePointer(reinterpret_cast<void**>(&fresh->guard_dev),
                                        fresh->guard_host, 0);
        }
        if (e != hipSuccess) {
            destroy_plan(fresh);
            return hip_fail(e, "one-call guard word");
        }
    }
    *out = PlanRef(fresh, destroy_plan);
    return SPMM_OK;
}

// ------------------------------------------------------------------ no allocation

// Device memory of spmm_csr_noalloc: the merge-path coordinates, carry-out
// row ids and carry-out rows of one call. Every device holds its own copy at
// its own address for the life of the process; host code never uses the
// name itself (a host-side stand-in), only the address hipGetSymbolAddress
// returns with that device current, kept per device below.
static __device__ __align__(256) unsigned char scratch[SPMM_NOALLOC_SCRATCH_BYTES];

static std::mutex g_scratch_mu;
static std::map<int, unsigned char*> g_scratch_addr;

static int scratch_address(int dev, unsigned char** out) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch_addr.find(dev);
    if (it == g_scratch_addr.end()) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!ptr) return fail(SPMM_ERR_HIP, "hipGetSymbolAddress(scratch) gave NULL");
        it = g_scratch_addr.emplace(dev, static_cast<unsigned char*>(ptr)).first;
    }
    *out = it->second;
    return SPMM_OK;
}

static int64_t round256(int64_t b) { return (b + 255) & ~int64_t(255); }

static CacheKey csr_key(const int32_t* A_rowptr, const int32_t* A_colind, int64_t m, int64_t k,
                        int64_t n, int64_t ld, int dev, void* stream) {
    // keyed by stream too: a merge-based plan's workspace must not be shared
    // by work on two streams
    return CacheKey{A_rowptr, A_colind, m, k, n, ld, dev, stream};
}

}  // namespace spmmh

using namespace spmmh;

extern "C" {

const char* spmm_status_string(int status) {
    switch (status) {
    case SPMM_OK: return "ok";
    case SPMM_ERR_INVALID: return "invalid argument";
    case SPMM_ERR_UNSUPPORTED: return "unsupported";
    case SPMM_ERR_HIP: return "HIP runtime error";
    case SPMM_ERR_NOMEM: return "out of memory";
    case SPMM_ERR_STATE: return "invalid state or handle";
    default: return "unknown status";
    }
}

const char* spmm_last_error(void) { return t_err.c_str(); }

const char* spmm_version(void) { return "0.1.0"; }

int spmm_plan_create(spmm_plan_t* out_plan, const int32_t* A_rowptr, const int32_t* A_colind,
                     int64_t m, int64_t k, int64_t nnz, int64_t n, int64_t ld, int32_t dtype,
                     int32_t mode, void* stream) {
    return create_plan(out_plan, A_rowptr, A_colind, m, k, nnz, n, ld, dtype, mode, nullptr,
                       static_cast<hipStream_t>(stream), true);
}

int spmm_plan_create_config(spmm_plan_t* out_plan, const int32_t* A_rowptr,
                            const int32_t* A_colind, int64_t m, int64_t k, int64_t nnz,
                            int64_t n, int64_t ld, int32_t dtype, const spmm_config* config_host,
                            void* stream) {
    if (!config_host) return fail(SPMM_ERR_INVALID, "config is NULL");
    return create_plan(out_plan, A_rowptr, A_colind, m, k, nnz, n, ld, dtype, 0, config_host,
                       static_cast<hipStream_t>(stream), true);
}

int spmm_execute(spmm_plan_t plan, const void* A_vals, const void* B, float* C, void* stream) {
    if (!plan_alive(plan)) return fail(SPMM_ERR_STATE, "plan is destroyed or not a plan");
    if (plan->m == 0 || plan->n == 0) return SPMM_OK;
    if (!C) return fail(SPMM_ERR_INVALID, "C is NULL");
    if (plan->nnz > 0 && (!A_vals || !B)) return fail(SPMM_ERR_INVALID, "A_vals or B is NULL");
    return forward(*plan, plan->rowptr, plan->colind, A_vals, B, C,
                   static_cast<hipStream_t>(stream));
}

int spmm_execute_events(spmm_plan_t plan, const void* A_vals, const void* B, float* C,
                        void* ev_before, void* ev_after, void* stream) {
    if (!plan_alive(plan)) return fail(SPMM_ERR_STATE, "plan is destroyed or not a plan");
    if (plan->m == 0 || plan->n == 0) return SPMM_OK;
    if (!C) return fail(SPMM_ERR_INVALID, "C is NULL");
    if (plan->nnz > 0 && (!A_vals || !B)) return fail(SPMM_ERR_INVALID, "A_vals or B is NULL");
    return forward(*plan, plan->rowptr, plan->colind, A_vals, B, C,
                   static_cast<hipStream_t>(stream), static_cast<hipEvent_t>(ev_before),
                   static_cast<hipEvent_t>(ev_after));
}

int spmm_execute_semiring(spmm_plan_t plan, int32_t semiring, const void* A_vals, const void* B,
                          float* C, void* stream) {
    if (!plan_alive(plan)) return fail(SPMM_ERR_STATE, "plan is destroyed or not a plan");
    if (semiring < SPMM_PLUS_TIMES || semiring > SPMM_MAX_TIMES)
        return fail(SPMM_ERR_INVALID, "semiring %d", semiring);
    if (plan->m == 0 || plan->n == 0) return SPMM_OK;
    if (!C) return fail(SPMM_ERR_INVALID, "C is NULL");
    if (plan->nnz > 0 && (!A_vals || !B)) return fail(SPMM_ERR_INVALID, "A_vals or B is NULL");
    return forward(*plan, plan->rowptr, plan->colind, A_vals, B, C,
                   static_cast<hipStream_t>(stream), nullptr, nullptr, semiring);
}

int spmm_plan_info_get(spmm_plan_t plan, spmm_plan_info* info) {
    if (!plan_alive(plan)) return fail(SPMM_ERR_STATE, "plan is destroyed or not a plan");
    if (!info) return fail(SPMM_ERR_INVALID, "info is NULL");
    fill_info(plan, info);
    return SPMM_OK;
}


int spmm_plan_partition(spmm_plan_t plan, int32_t* coords_host, int64_t cap) {
    if (!plan_alive(plan)) return fail(SPMM_ERR_STATE, "plan is destroyed or not a plan");
    if (!is_merge(plan->cfg.kernel))
        return fail(SPMM_ERR_STATE, "row-split or row-block plan has no merge partition");
    if (!coords_host) return fail(SPMM_ERR_INVALID, "coords_host is NULL");
    if (cap < plan->ws.P + 1)
        return fail(SPMM_ERR_INVALID, "cap %lld < P + 1 = %lld", (long long)cap,
                    (long long)(plan->ws.P + 1));
    SPMM_HIP(hipMemcpy(coords_host, plan->ws.coords, sizeof(int) * 2 * (plan->ws.P + 1),
                       hipMemcpyDeviceToHost));
    return SPMM_OK;
}

int spmm_plan_destroy(spmm_plan_t plan) {
    {
        std::lock_guard<std::mutex> lk(g_mu);
        if (!plan || !g_plans.count(plan))
            return fail(SPMM_ERR_STATE, "plan is destroyed or not a plan");
        g_plans.erase(plan);
    }
    destroy_plan(plan);
    return SPMM_OK;
}

int spmm_csr(const int32_t* A_rowptr, const int32_t* A_colind, const float* A_vals,
             const float* B, float* C, int64_t m, int64_t k, int64_t n, int64_t ld,
             void* stream) {
    int rc = check_dims(m, k, 0, n, ld);
    if (rc) return rc;
    if (m == 0 || n == 0) return SPMM_OK;
    if (!A_rowptr || !C) return fail(SPMM_ERR_INVALID, "A_rowptr or C is NULL");
    hipStream_t st = static_cast<hipStream_t>(stream);
    int dev = 0;
    SPMM_HIP(hipGetDevice(&dev));
    const CacheKey key = csr_key(A_rowptr, A_colind, m, k, n, ld, dev, stream);
    const bool pointers_ok = A_colind && A_vals && B;
    PlanRef p;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        auto it = g_cache.find(key);
        if (it != g_cache.end()) {
            p = it->second;
            auto pos = std::find(g_cache_order.begin(), g_cache_order.end(), key);
            if (pos != g_cache_order.end()) g_cache_order.erase(pos);
            g_cache_order.push_back(key);
        }
    }
    if (p && p->guard_host && __atomic_load_n(p->guard_host, __ATOMIC_ACQUIRE)) {
        // an earlier call found A_rowptr[m] != the plan's nnz: drop the plan
        const long long old_nnz = (long long)p->nnz;
        {
            std::lock_guard<std::mutex> lk(g_mu);
            auto it = g_cache.find(key);
            if (it != g_cache.end() && it->second == p) {
                g_cache.erase(it);
                auto pos = std::find(g_cache_order.begin(), g_cache_order.end(), key);
                if (pos != g_cache_order.end()) g_cache_order.erase(pos);
            }
        }
        return fail(SPMM_ERR_STATE,
                    "the CSR structure at these pointers changed: A_rowptr[m] is no longer the "
                    "nnz (%lld) its cached plan was made for, and an earlier call filled its C "
                    "with NaN; the plan is dropped and the next call plans afresh",
                    old_nnz);
    }
    if (!p) {
        rc = csr_create(A_rowptr, A_colind, m, k, n, ld, st, pointers_ok, &p);
        if (rc) return rc;
        std::vector<PlanRef> evict;  // released after the lock
        {
            std::lock_guard<std::mutex> lk(g_mu);
            auto it = g_cache.find(key);
            if (it != g_cache.end()) {
                evict.push_back(p);  // another thread cached this key meanwhile: use its plan
                p = it->second;
            } else {
                g_cache[key] = p;
                g_cache_order.push_back(key);
            }
            while (g_cache_order.size() > kCacheCap) {
                evict.push_back(g_cache[g_cache_order.front()]);
                g_cache.erase(g_cache_order.front());
                g_cache_order.erase(g_cache_order.begin());
            }
        }
    } else if (p->nnz > 0 && !pointers_ok) {
        return fail(SPMM_ERR_INVALID, "A_colind, A_vals or B is NULL");
    }
    if (p->guard_dev && is_merge(p->cfg.kernel)) {
        const hipError_t e = spmmk::launch_merge_revalidate(
            A_rowptr, m, p->nnz, p->cfg.items_per_wg, p->ws.P, p->ws.coords, C, n, ld,
            p->guard_dev, st);
        if (e != hipSuccess) return hip_fail(e, "partition re-check launch");
    }
    return forward(*p, A_rowptr, A_colind, A_vals, B, C, st);
}

int spmm_csr_noalloc(const int32_t* A_rowptr, const int32_t* A_colind, const float* A_vals,
                     const float* B, float* C, int64_t m, int64_t k, int64_t nnz, int64_t n,
                     int64_t ld, void* stream) {
    int rc = check_dims(m, k, nnz, n, ld);
    if (rc) return rc;
    if (m == 0 || n == 0) return SPMM_OK;
    if (!A_rowptr || !C) return fail(SPMM_ERR_INVALID, "A_rowptr or C is NULL");
    if (nnz > 0 && (!A_colind || !A_vals || !B))
        return fail(SPMM_ERR_INVALID, "A_colind, A_vals or B is NULL");
    hipStream_t st = static_cast<hipStream_t>(stream);
    // A plan on the stack: the Sec. 5.4 choice from m and nnz, the default
    // shape of that kernel, no row statistics and no tile order (each would
    // need a read-back), and, for the merge-based kernel, its workspace in
    // this device's static scratch.
    spmm_plan_s p;
    p.rowptr = A_rowptr;
    p.colind = A_colind;
    p.m = m; p.k = k; p.nnz = nnz; p.n = n; p.ld = ld;
    p.dtype = SPMM_F32;
    p.mode = SPMM_MODE_PAPER;
    p.paper_choice = 100 * nnz < 935 * m ? SPMM_KERNEL_MERGE : SPMM_KERNEL_ROWSPLIT;
    p.cfg = spmm_config{p.paper_choice, 0, 0, 0, 0, 0};
    rc = check_config(p, p.cfg);
    if (rc) return rc;
    if (is_merge(p.cfg.kernel)) {
        const int64_t P = num_pieces(m, nnz, p.cfg.items_per_wg, false);
        const int64_t coords_b = round256(int64_t(sizeof(int)) * 2 * (P + 1));
        const int64_t rows_b = round256(int64_t(sizeof(int)) * P);
        const int64_t vals_b = int64_t(sizeof(float)) * P * n;
        if (coords_b + rows_b + vals_b > int64_t(SPMM_NOALLOC_SCRATCH_BYTES))
            return fail(SPMM_ERR_UNSUPPORTED,
                        "spmm_csr_noalloc: %lld merge pieces of %d items at n = %lld need %lld "
                        "bytes of scratch, more than its %lld",
                        (long long)P, p.cfg.items_per_wg, (long long)n,
                        (long long)(coords_b + rows_b + vals_b),
                        (long long)SPMM_NOALLOC_SCRATCH_BYTES);
        SPMM_HIP(hipGetDevice(&p.device));
        unsigned char* base = nullptr;
        rc = scratch_address(p.device, &base);
        if (rc) return rc;
        p.ws.coords = reinterpret_cast<int*>(base);
        p.ws.carry_rows = reinterpret_cast<int*>(base + coords_b);
        p.ws.carry_vals = reinterpret_cast<float*>(base + coords_b + rows_b);
        p.ws.P = P;
        // every coordinate and carry-out row id is written before it is read
        // (an open row's carry-out values too), so nothing needs clearing
        const hipError_t e = spmmk::launch_merge_partition(A_rowptr, m, nnz, p.cfg.items_per_wg,
                                                           P, 0, p.ws.coords, st);
        if (e != hipSuccess) return hip_fail(e, "merge partition launch");
    }
    return forward(p, A_rowptr, A_colind, A_vals, B, C, st);
}

int spmm_csr_plan_info(const int32_t* A_rowptr, const int32_t* A_colind, int64_t m, int64_t k,
                       int64_t n, int64_t ld, void* stream, spmm_plan_info* info_host) {
    if (!info_host) return fail(SPMM_ERR_INVALID, "info is NULL");
    int dev = 0;
    SPMM_HIP(hipGetDevice(&dev));
    PlanRef p;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        auto it = g_cache.find(csr_key(A_rowptr, A_colind, m, k, n, ld, dev, stream));
        if (it != g_cache.end()) p = it->second;
    }
    if (!p) return fail(SPMM_ERR_STATE, "no cached spmm_csr plan for these arguments");
    fill_info(p.get(), info_host);
    return SPMM_OK;
}

int spmm_cache_clear(void) {
    std::vector<PlanRef> all;  // plans in use elsewhere are freed by their last user
    {
        std::lock_guard<std::mutex> lk(g_mu);
        for (auto& kv : g_cache) all.push_back(kv.second);
        g_cache.clear();
        g_cache_order.clear();
    }
    return SPMM_OK;
}

int spmm_tune_cache_save(const char* path_host) {
    if (!path_host) return fail(SPMM_ERR_INVALID, "path is NULL");
    std::vector<std::pair<TuneKey, std::pair<spmm_config, double>>> all;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        all.assign(g_tuned.begin(), g_tuned.end());
    }
    FILE* f = fopen(path_host, "w");
    if (!f) return fail(SPMM_ERR_INVALID, "cannot write %s", path_host);
    fprintf(f, "spmm-tune-cache 2\n");
    for (const auto& kv : all) {
        const TuneKey& k = kv.first;
        const spmm_config& c = kv.second.first;
        fprintf(f,
                "%d %lld %lld %lld %lld %lld %lld %lld %d %d %d %d %d  %d %d %d %d %d %d %d %d %d"
                "  %.9g\n",
                k.device, (long long)k.m, (long long)k.k, (long long)k.nnz, (long long)k.n,
                (long long)k.ld, (long long)k.maxrow, (long long)k.longrows, k.dtype, k.unroll,
                k.max_W, k.rowblock ? 1 : 0, k.panels ? 1 : 0, c.kernel, c.vec, c.lanes_per_row,
                c.unroll, c.items_per_wg, c.tile_cols, c.rows_per_block, c.tile_order,
                c.col_panels, kv.second.second);
    }
    const bool ok = fclose(f) == 0;
    return ok ? SPMM_OK : fail(SPMM_ERR_INVALID, "cannot write %s", path_host);
}

int spmm_tune_cache_load(const char* path_host) {
    if (!path_host) return fail(SPMM_ERR_INVALID, "path is NULL");
    FILE* f = fopen(path_host, "r");
    if (!f) return fail(SPMM_ERR_INVALID, "cannot read %s", path_host);
    int version = 0;
    if (fscanf(f, "spmm-tune-cache %d", &version) != 1 || version != 2) {
        fclose(f);
        return fail(SPMM_ERR_INVALID, "%s is not a version-2 tune cache", path_host);
    }
    std::vector<std::pair<TuneKey, std::pair<spmm_config, double>>> got;
    for (;;) {
        TuneKey k{};
        spmm_config c{};
        long long m, kk, nnz, n, ld, maxrow, longrows;
        int rowblock = 0, panels = 0;
        double ms = 0.0;
        const int r = fscanf(f,
                             "%d %lld %lld %lld %lld %lld %lld %lld %d %d %d %d %d %d %d %d %d %d "
                             "%d %d %d %d %lf",
                             &k.device, &m, &kk, &nnz, &n, &ld, &maxrow, &longrows, &k.dtype,
                             &k.unroll, &k.max_W, &rowblock, &panels, &c.kernel, &c.vec,
                             &c.lanes_per_row, &c.unroll, &c.items_per_wg, &c.tile_cols,
                             &c.rows_per_block, &c.tile_order, &c.col_panels, &ms);
        if (r == EOF) break;
        if (r != 23) {
            fclose(f);
            return fail(SPMM_ERR_INVALID, "%s: malformed entry %zu", path_host, got.size() + 1);
        }
        k.m = m; k.k = kk; k.nnz = nnz; k.n = n; k.ld = ld; k.maxrow = maxrow;
        k.longrows = longrows; k.rowblock = rowblock != 0; k.panels = panels != 0;
        got.push_back({k, {c, ms}});
    }
    fclose(f);
    // each entry passes the same shape checks as a forced config when a plan
    // uses it; here only the kernel id is checked
    for (const auto& kv : got)
        if (kv.second.first.kernel < SPMM_KERNEL_ROWSPLIT ||
            kv.second.first.kernel > SPMM_KERNEL_ROWBLOCK)
            return fail(SPMM_ERR_INVALID, "%s: kernel %d is not a kernel", path_host,
                        kv.second.first.kernel);
    std::lock_guard<std::mutex> lk(g_mu);
    for (const auto& kv : got) g_tuned[kv.first] = kv.second;
    return SPMM_OK;
}

int spmm_csr_validate(const int32_t* A_rowptr, const int32_t* A_colind, int64_t m, int64_t k,
                      int64_t nnz, void* stream) {
    int rc = check_dims(m, k, nnz, 0, 1);
    if (rc) return rc;
    if (!A_rowptr) return fail(SPMM_ERR_INVALID, "A_rowptr is NULL");
    if (nnz > 0 && !A_colind) return fail(SPMM_ERR_INVALID, "A_colind is NULL");
    hipStream_t st = static_cast<hipStream_t>(stream);
    int* d = nullptr;
    int h[4] = {0, 0, 1, 0};
    SPMM_HIP(hipMalloc(&d, sizeof h));
    hipError_t e = hipMemcpyAsync(d, h, sizeof h, hipMemcpyHostToDevice, st);
    if (e == hipSuccess && m > 0) e = spmmk::launch_row_stats(A_rowptr, m, d, st);
    if (e == hipSuccess && nnz > 0) e = spmmk::launch_check_cols(A_colind, nnz, k, d + 3, st);
    if (e == hipSuccess) e = hipMemcpyAsync(h, d, sizeof h, hipMemcpyDeviceToHost, st);
    int32_t last = 0, first = 0;
    if (e == hipSuccess)
        e = hipMemcpyAsync(&last, A_rowptr + m, sizeof last, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipMemcpyAsync(&first, A_rowptr, sizeof first, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    (void)hipFree(d);
    if (e != hipSuccess) return hip_fail(e, "validate");
    if (first != 0) return fail(SPMM_ERR_INVALID, "A_rowptr[0] = %d, expected 0", first);
    if (!h[2]) return fail(SPMM_ERR_INVALID, "A_rowptr decreases");
    if (last != nnz)
        return fail(SPMM_ERR_INVALID, "A_rowptr[m] = %d but nnz = %lld", last, (long long)nnz);
    if (h[3]) return fail(SPMM_ERR_INVALID, "a column index is outside [0, k)");
    return SPMM_OK;
}

int spmm_calibrate_gather(const void* table, int64_t table_rows, int32_t row_bytes,
                          int32_t steps, float* out, int64_t threads, void* stream) {
    if (!table || !out) return fail(SPMM_ERR_INVALID, "table or out is NULL");
    if (row_bytes != 32 && row_bytes != 64 && row_bytes != 128 && row_bytes != 256 &&
        row_bytes != 512)
        return fail(SPMM_ERR_INVALID, "row_bytes %d: use 32, 64, 128, 256 or 512", row_bytes);
    if (table_rows < 1 || table_rows > (int64_t(1) << 31) || (table_rows & (table_rows - 1)))
        return fail(SPMM_ERR_INVALID, "table_rows %lld: a power of two up to 2^31",
                    (long long)table_rows);
    if (steps < 8 || steps % 8)
        return fail(SPMM_ERR_INVALID, "steps %d: a positive multiple of 8", steps);
    if (threads < spmmk::kBlock || threads % spmmk::kBlock ||
        threads / spmmk::kBlock > (int64_t(1) << 31) - 1 || threads > (int64_t(1) << 32))
        return fail(SPMM_ERR_INVALID, "threads %lld: a multiple of %d", (long long)threads,
                    spmmk::kBlock);
    if ((reinterpret_cast<uintptr_t>(table) & 15u) != 0)
        return fail(SPMM_ERR_INVALID, "table is not 16-byte aligned");
    const hipError_t e = spmmk::launch_calib_gather(table, table_rows, row_bytes, steps, out,
                                                    threads, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "gather calibration launch");
    return SPMM_OK;
}

}  // extern "C"
