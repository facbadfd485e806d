// C ABI of batched SpMM: per-problem plans, the persistent kernel's work
// list, and its capture into a hipGraph.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <numeric>
#include <set>
#include <vector>

#include "batch.hpp"
#include "plan.hpp"

using namespace spmmh;

struct spmm_batch_s {
    int device = 0;
    int32_t dtype = 0;
    std::vector<spmm_plan_s*> plans;     // one per problem, in the caller's order
    std::vector<spmm_problem> problems;
    spmmk::BatchProb* d_probs = nullptr;  // problems with work
    spmmk::WorkItem* d_items = nullptr;
    int* d_merge_ids = nullptr;
    int64_t* d_piece_off = nullptr;
    int64_t* d_queues = nullptr;
    unsigned long long* d_counter = nullptr;
    int nprob = 0, nmerge = 0, grid = 1;
    int64_t total_items = 0, total_pieces = 0;
    size_t lds = 0;
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace {

std::mutex g_bmu;
std::set<const spmm_batch_s*> g_batches;

bool batch_alive(const spmm_batch_s* b) {
    std::lock_guard<std::mutex> lk(g_bmu);
    return b && g_batches.count(b);
}

void free_batch(spmm_batch_s* b) {
    if (!b) return;
    (void)hipDeviceSynchronize();
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
    for (void* p : {(void*)b->d_probs, (void*)b->d_items, (void*)b->d_merge_ids,
                    (void*)b->d_piece_off, (void*)b->d_queues, (void*)b->d_counter})
        if (p) (void)hipFree(p);
    for (auto* p : b->plans) destroy_plan(p);
    delete b;
}

int launch(const spmm_batch_s& b, hipStream_t st) {
    hipError_t e = spmmk::launch_batch(b.dtype, b.grid, b.lds, b.d_probs, b.d_items,
                                       b.total_items, b.d_queues, b.d_counter, b.d_merge_ids,
                                       b.d_piece_off, b.nmerge, b.total_pieces, st);
    if (e != hipSuccess) return hip_fail(e, "batched launch");
    return SPMM_OK;
}

template <class T>
int upload(T** dst, const std::vector<T>& v, hipStream_t st) {
    const size_t bytes = sizeof(T) * std::max<size_t>(v.size(), 1);
    SPMM_HIP(hipMalloc(dst, bytes));
    if (!v.empty())
        SPMM_HIP(hipMemcpyAsync(*dst, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice, st));
    return SPMM_OK;
}

}  // namespace

extern "C" {

int spmm_batch_plan(spmm_batch_t* out_batch, const spmm_problem* problems_host, int64_t count,
                    int32_t dtype, int32_t mode, void* stream) {
    if (!out_batch) return fail(SPMM_ERR_INVALID, "out_batch is NULL");
    *out_batch = nullptr;
    if (count < 0 || count > (int64_t(1) << 30)) return fail(SPMM_ERR_INVALID, "count %lld", (long long)count);
    if (count > 0 && !problems_host) return fail(SPMM_ERR_INVALID, "problems is NULL");
    if (dtype != SPMM_F32 && dtype != SPMM_BF16 && dtype != SPMM_F16)
        return fail(SPMM_ERR_UNSUPPORTED, "dtype %d", dtype);
    if (mode < SPMM_MODE_PAPER || mode > SPMM_MODE_NZSPLIT) return fail(SPMM_ERR_INVALID, "mode %d", mode);
    for (int64_t i = 0; i < count; ++i) {
        const spmm_problem& q = problems_host[i];
        const int rc = check_dims(q.m, q.k, q.nnz, q.n, q.ld);
        if (rc != SPMM_OK) return fail(rc, "problem %lld: %s", (long long)i, spmm_last_error());
    }
    hipStream_t st = static_cast<hipStream_t>(stream);

    spmm_batch_s* b = new (std::nothrow) spmm_batch_s;
    if (!b) return fail(SPMM_ERR_NOMEM, "batch");
    b->dtype = dtype;
    b->problems.assign(problems_host, problems_host + count);
    int rc = SPMM_OK;
    hipError_t e = hipGetDevice(&b->device);
    if (e != hipSuccess) { free_batch(b); return hip_fail(e, "hipGetDevice"); }

    // One plan per problem; the batched kernel has one unroll for all.
    for (int64_t i = 0; i < count && rc == SPMM_OK; ++i) {
        const spmm_problem& q = b->problems[i];
        if (q.m > 0 && q.n > 0 && !q.C) rc = fail(SPMM_ERR_INVALID, "problem %lld: C is NULL", (long long)i);
        if (rc == SPMM_OK && q.nnz > 0 && q.n > 0 && (!q.A_vals || !q.B))
            rc = fail(SPMM_ERR_INVALID, "problem %lld: A_vals or B is NULL", (long long)i);
        if (rc != SPMM_OK) break;
        TuneOpts opts;
        opts.fixed_unroll = spmmk::kBatchUnroll;
        opts.max_W = spmmk::kBatchMaxW;
        opts.rowblock = false;  // the persistent kernel runs row split and merge tiles only
        opts.panels = false;    // ... each in one pass
        opts.no_planes = true;  // ... in its own order of work items
        opts.no_sddmm = true;   // the batch runs forward products only
        opts.vals = q.A_vals;
        opts.B = q.B;
        opts.C = q.C;
        spmm_plan_s* p = nullptr;
        rc = create_plan(&p, q.A_rowptr, q.A_colind, q.m, q.k, q.nnz, q.n, q.ld, dtype, mode,
                         nullptr, st, false, &opts);
        if (rc != SPMM_OK) {
            int rc2 = fail(rc, "problem %lld: %s", (long long)i, spmm_last_error());
            rc = rc2;
            break;
        }
        b->plans.push_back(p);
    }
    if (rc != SPMM_OK) { free_batch(b); return rc; }

    // Problems with work, their tile size and cost.
    struct Entry { double tile_cost; int64_t tiles; int per_item; spmmk::BatchProb bp; };
    std::vector<Entry> work;
    for (int64_t i = 0; i < count; ++i) {
        const spmm_plan_s& p = *b->plans[i];
        if (p.m == 0 || p.n == 0) continue;
        const spmm_problem& q = b->problems[i];
        int vec = p.cfg.vec;
        if (vec != 1 && (!aligned16(q.B) || !aligned16(q.C))) vec = 1;
        const spmmk::Shape s = resolve_shape(p, vec);
        spmmk::BatchProb bp{};
        bp.rowptr = q.A_rowptr; bp.colind = q.A_colind; bp.vals = q.A_vals; bp.B = q.B; bp.C = q.C;
        bp.m = p.m; bp.ld = p.ld; bp.n = (int)p.n;
        bp.kernel = p.cfg.kernel; bp.vec = vec; bp.g_log2 = s.g_log2; bp.ts_log2 = s.ts_log2;
        bp.W = s.W; bp.col_tiles = s.col_tiles; bp.nz = s.nz;
        const double mean = double(p.nnz) / double(p.m);
        const double tile_cols = std::min<double>(double(p.n), double(vec << s.g_log2));
        Entry en{};
        double entries_per_tile;
        if (p.cfg.kernel == SPMM_KERNEL_ROWSPLIT) {
            const int64_t rows_per_block = int64_t(spmmk::kWaveSize >> (s.g_log2 + s.ts_log2)) *
                                           (spmmk::kBlock / spmmk::kWaveSize);
            en.tiles = (p.m + rows_per_block - 1) / rows_per_block;
            entries_per_tile = double(rows_per_block) * (1.0 + mean);
        } else {
            bp.coords = p.ws.coords; bp.carry_vals = p.ws.carry_vals; bp.carry_rows = p.ws.carry_rows;
            bp.P = p.ws.P;
            en.tiles = p.ws.P;
            entries_per_tile = double(s.W);
            b->lds = std::max(b->lds, spmmk::merge_lds_bytes(dtype, s));
        }
        en.tile_cost = entries_per_tile * tile_cols;
        en.per_item = (int)std::max(1.0, std::round(spmmk::kBatchItemEntries / entries_per_tile));
        en.bp = bp;
        work.push_back(en);
    }
    // Bin-pack problems into one queue per XCD: largest total first onto the
    // lightest queue; inside a queue, costliest tiles first.
    constexpr int NQ = spmmk::kBatchQueues;
    std::vector<int> order(work.size());
    std::iota(order.begin(), order.end(), 0);
    auto total_cost = [&](int i) {
        return work[i].tile_cost * double(work[i].tiles) * work[i].bp.col_tiles;
    };
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int c) { return total_cost(a) > total_cost(c); });
    std::vector<std::vector<int>> bins(NQ);
    std::vector<double> load(NQ, 0.0);
    for (int i : order) {
        const int q = int(std::min_element(load.begin(), load.end()) - load.begin());
        bins[q].push_back(i);
        load[q] += total_cost(i);
    }
    std::vector<spmmk::BatchProb> probs;
    std::vector<spmmk::WorkItem> witems;
    std::vector<int64_t> piece_off, queues(2 * NQ, 0);
    std::vector<int> merge_ids;
    int64_t pieces = 0;
    for (int q = 0; q < NQ; ++q) {
        std::stable_sort(bins[q].begin(), bins[q].end(),
                         [&](int a, int c) { return work[a].tile_cost > work[c].tile_cost; });
        queues[q] = (int64_t)witems.size();
        for (int i : bins[q]) {
            const Entry& w = work[i];
            const int pid = (int)probs.size();
            if (w.bp.kernel != SPMM_KERNEL_ROWSPLIT && w.bp.P > 0) {
                merge_ids.push_back(pid);
                piece_off.push_back(pieces);
                pieces += w.bp.P;
            }
            for (int ct = 0; ct < w.bp.col_tiles; ++ct)
                for (int64_t t = 0; t < w.tiles; t += w.per_item)
                    witems.push_back({pid, ct, (int)t, (int)std::min<int64_t>(w.per_item, w.tiles - t)});
            probs.push_back(w.bp);
        }
        queues[NQ + q] = (int64_t)witems.size() - queues[q];
    }
    const int64_t items = (int64_t)witems.size();
    b->nprob = (int)probs.size();
    b->nmerge = (int)merge_ids.size();
    b->total_items = items;
    b->total_pieces = pieces;
    if (rc == SPMM_OK) rc = upload(&b->d_probs, probs, st);
    if (rc == SPMM_OK) rc = upload(&b->d_items, witems, st);
    if (rc == SPMM_OK) rc = upload(&b->d_merge_ids, merge_ids, st);
    if (rc == SPMM_OK) rc = upload(&b->d_piece_off, piece_off, st);
    if (rc == SPMM_OK) rc = upload(&b->d_queues, queues, st);
    if (rc == SPMM_OK) {
        e = hipMalloc(&b->d_counter, sizeof(unsigned long long) * NQ);
        if (e != hipSuccess) rc = hip_fail(e, "hipMalloc counter");
    }
    if (rc == SPMM_OK) {
        e = spmmk::batch_grid(dtype, b->lds, &b->grid);
        if (e != hipSuccess) rc = hip_fail(e, "occupancy query");
        if (b->grid > items) b->grid = (int)std::max<int64_t>(items, 1);
    }
    if (rc == SPMM_OK) {
        e = hipStreamSynchronize(st);
        if (e != hipSuccess) rc = hip_fail(e, "batch upload");
    }
    // Capture reset + persistent kernel + fix-up once; runs replay it.
    if (rc == SPMM_OK) {
        e = hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            rc = launch(*b, b->cap_stream);
            hipGraph_t g = nullptr;
            hipError_t e2 = hipStreamEndCapture(b->cap_stream, &g);
            b->graph = g;
            if (rc == SPMM_OK && e2 != hipSuccess) rc = hip_fail(e2, "hipStreamEndCapture");
        }
        if (rc == SPMM_OK && e == hipSuccess) e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
        if (rc == SPMM_OK && e != hipSuccess) rc = hip_fail(e, "graph capture");
    }
    if (rc != SPMM_OK) { free_batch(b); return rc; }
    {
        std::lock_guard<std::mutex> lk(g_bmu);
        g_batches.insert(b);
    }
    *out_batch = b;
    return SPMM_OK;
}

int spmm_batch_run(spmm_batch_t batch, void* stream) {
    if (!batch_alive(batch)) return fail(SPMM_ERR_STATE, "batch is destroyed or not a batch");
    SPMM_HIP(hipGraphLaunch(batch->exec, static_cast<hipStream_t>(stream)));
    return SPMM_OK;
}

int spmm_batch_run_direct(spmm_batch_t batch, void* stream) {
    if (!batch_alive(batch)) return fail(SPMM_ERR_STATE, "batch is destroyed or not a batch");
    return launch(*batch, static_cast<hipStream_t>(stream));
}

int spmm_batch_problem_config(spmm_batch_t batch, int64_t b, spmm_config* config_host) {
    if (!batch_alive(batch)) return fail(SPMM_ERR_STATE, "batch is destroyed or not a batch");
    if (!config_host) return fail(SPMM_ERR_INVALID, "config is NULL");
    if (b < 0 || b >= (int64_t)batch->plans.size())
        return fail(SPMM_ERR_INVALID, "problem index %lld out of range", (long long)b);
    *config_host = batch->plans[b]->cfg;
    return SPMM_OK;
}

int spmm_batch_destroy(spmm_batch_t batch) {
    {
        std::lock_guard<std::mutex> lk(g_bmu);
        if (!batch || !g_batches.count(batch))
            return fail(SPMM_ERR_STATE, "batch is destroyed or not a batch");
        g_batches.erase(batch);
    }
    free_batch(batch);
    return SPMM_OK;
}

}  // extern "C"
