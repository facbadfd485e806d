// C ABI of the backward pass: transpose build, dB = A^T dC and SDDMM.

#include <hip/hip_runtime.h>

#include "plan.hpp"

using namespace spmmh;

namespace {

// SDDMM keeps 4 entries in flight per slot, 2 with 8-wide 16-bit rows (whose
// dC chunks take 8 registers each) so that occupancy stays at 8 waves/SIMD.
int sddmm_unroll(int vec) { return vec == 8 ? 2 : 4; }

}  // namespace

extern "C" {

int spmm_transpose_build(spmm_plan_t plan, void* stream) {
    if (!plan_alive(plan)) return fail(SPMM_ERR_STATE, "plan is destroyed or not a plan");
    if (plan->tplan) return SPMM_OK;  // once per structure
    hipStream_t st = static_cast<hipStream_t>(stream);
    spmm_plan_s& p = *plan;
    Transpose& tr = p.tr;
    // The sort's temporaries (two key arrays, values, row ids, histogram and scan
    // scratch) share one allocation: one hipMalloc and one hipFree instead of five.
    int *tmp = nullptr, *k0 = nullptr, *k1 = nullptr, *v1 = nullptr, *r0 = nullptr,
        *hist = nullptr;
    auto free_tmp = [&]() {
        if (tmp) (void)hipFree(tmp);
    };
    auto free_tr = [&]() {
        if (tr.at_rowptr) (void)hipFree(tr.at_rowptr);
        if (tr.at_colind) (void)hipFree(tr.at_colind);
        if (tr.perm) (void)hipFree(tr.perm);
        if (tr.at_vals) (void)hipFree(tr.at_vals);
        tr = Transpose{};
    };
    hipError_t e = hipMalloc(&tr.at_rowptr, sizeof(int) * (p.k + 1));
    if (e == hipSuccess && p.nnz > 0) e = hipMalloc(&tr.at_colind, sizeof(int) * p.nnz);
    if (e == hipSuccess && p.nnz > 0) e = hipMalloc(&tr.perm, sizeof(int) * p.nnz);
    if (e == hipSuccess && p.nnz > 0) e = hipMalloc(&tr.at_vals, sizeof(float) * p.nnz);
    if (e == hipSuccess && p.nnz > 0) {
        const size_t arr = ((size_t)p.nnz + 63) / 64 * 64;  // 256-byte aligned pieces
        const size_t total = 4 * arr + (size_t)spmmk::transpose_scratch_len(p.nnz);
        e = hipMalloc(&tmp, sizeof(int) * total);
        if (e == hipSuccess) {
            k0 = tmp;
            k1 = tmp + arr;
            v1 = tmp + 2 * arr;
            r0 = tmp + 3 * arr;
            hist = tmp + 4 * arr;
        }
    }
    if (e == hipSuccess) {
        if (p.nnz > 0)
            e = spmmk::transpose_build(p.rowptr, p.colind, p.m, p.k, p.nnz, tr.at_rowptr,
                                       tr.at_colind, tr.perm, k0, k1, v1, r0, hist, st);
        else
            e = hipMemsetAsync(tr.at_rowptr, 0, sizeof(int) * (p.k + 1), st);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    free_tmp();
    if (e != hipSuccess) {
        free_tr();
        return hip_fail(e, "transpose build");
    }
    // The product with A^T runs in float32 (values are widened at gather),
    // planned by the plan's own mode (the MI355X rule for a forced shape, and
    // for a forced row-block plan, whose conditions A^T need not meet).
    // It never runs SDDMM, so it gets no SDDMM partition.
    const int mode = p.mode >= 0 && p.mode != SPMM_MODE_ROWBLOCK ? p.mode : SPMM_MODE_RULE;
    spmm_plan_s* tp = nullptr;
    TuneOpts topts;
    topts.no_sddmm = true;
    int rc = create_plan(&tp, tr.at_rowptr, tr.at_colind, p.k, p.m, p.nnz, p.n, p.ld, SPMM_F32,
                         mode, nullptr, st, false, &topts);
    if (rc != SPMM_OK) {
        free_tr();
        return rc;
    }
    p.tplan = tp;
    return SPMM_OK;
}

int spmm_transpose_get(spmm_plan_t plan, int32_t* AT_rowptr, int32_t* AT_colind, int32_t* perm,
                       void* stream) {
    if (!plan_alive(plan)) return fail(SPMM_ERR_STATE, "plan is destroyed or not a plan");
    if (!plan->tplan) return fail(SPMM_ERR_STATE, "spmm_transpose_build has not run");
    if (!AT_rowptr || (plan->nnz > 0 && (!AT_colind || !perm)))
        return fail(SPMM_ERR_INVALID, "output pointer is NULL");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const auto d2d = hipMemcpyDeviceToDevice;
    SPMM_HIP(hipMemcpyAsync(AT_rowptr, plan->tr.at_rowptr, sizeof(int) * (plan->k + 1), d2d, st));
    if (plan->nnz > 0) {
        SPMM_HIP(hipMemcpyAsync(AT_colind, plan->tr.at_colind, sizeof(int) * plan->nnz, d2d, st));
        SPMM_HIP(hipMemcpyAsync(perm, plan->tr.perm, sizeof(int) * plan->nnz, d2d, st));
    }
    return SPMM_OK;
}

int spmm_execute_t(spmm_plan_t plan, const void* A_vals, const float* dC, float* dB,
                   void* stream) {
    if (!plan_alive(plan)) return fail(SPMM_ERR_STATE, "plan is destroyed or not a plan");
    if (!plan->tplan) return fail(SPMM_ERR_STATE, "spmm_transpose_build has not run");
    if (plan->k == 0 || plan->n == 0) return SPMM_OK;
    if (!dB) return fail(SPMM_ERR_INVALID, "dB is NULL");
    if (plan->nnz > 0 && (!A_vals || !dC)) return fail(SPMM_ERR_INVALID, "A_vals or dC is NULL");
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (plan->nnz > 0) {
        hipError_t e = spmmk::launch_gather_widen(plan->dtype, A_vals, plan->tr.perm, plan->nnz,
                                                  static_cast<float*>(plan->tr.at_vals), st);
        if (e != hipSuccess) return hip_fail(e, "value gather launch");
    }
    const spmm_plan_s& tp = *plan->tplan;
    return forward(tp, tp.rowptr, tp.colind, plan->tr.at_vals, dC, dB, st);
}

int spmm_execute_t_scatter(spmm_plan_t plan, const void* A_vals, const float* dC, float* dB,
                           void* stream) {
    if (!plan_alive(plan)) return fail(SPMM_ERR_STATE, "plan is destroyed or not a plan");
    if (plan->k == 0 || plan->n == 0) return SPMM_OK;
    if (!dB) return fail(SPMM_ERR_INVALID, "dB is NULL");
    if (plan->nnz > 0 && (!A_vals || !dC)) return fail(SPMM_ERR_INVALID, "A_vals or dC is NULL");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const MergeWs& ws = sddmm_shares_partition(*plan) ? plan->ws : plan->sddmm_ws;
    const int W = kSddmmW;
    const int64_t P = plan->nnz > 0 && plan->m > 0 ? ws.P : 0;
    if (P > 0 && !ws.coords) return fail(SPMM_ERR_STATE, "plan has no merge partition");
    hipError_t e = spmmk::launch_scatter_t(plan->dtype, plan->rowptr, plan->colind, A_vals, dC, dB,
                                           plan->k, plan->n, plan->ld, ws.coords, P, W, st);
    if (e != hipSuccess) return hip_fail(e, "scatter launch");
    return SPMM_OK;
}

int spmm_sddmm(spmm_plan_t plan, const float* dC, const void* B, float* dvals, void* stream) {
    if (!plan_alive(plan)) return fail(SPMM_ERR_STATE, "plan is destroyed or not a plan");
    if (plan->nnz == 0 || plan->m == 0) return SPMM_OK;
    if (!dvals) return fail(SPMM_ERR_INVALID, "dvals is NULL");
    if (plan->n > 0 && (!dC || !B)) return fail(SPMM_ERR_INVALID, "dC or B is NULL");
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (plan->n == 0) {  // every dot product is empty
        const hipError_t e = spmmk::launch_zero_f32(dvals, plan->nnz, st);
        return e == hipSuccess ? SPMM_OK : hip_fail(e, "SDDMM zero fill");
    }
    int vec = plan->cfg.vec;
    if (vec != 1 && (!aligned16(dC) || !aligned16(B))) vec = 1;
    int g_log2, col_tiles;
    slot_geometry(plan->n, vec, &g_log2, &col_tiles);
    const MergeWs& ws = sddmm_shares_partition(*plan) ? plan->ws : plan->sddmm_ws;
    const int W = kSddmmW;
    if (!ws.coords) return fail(SPMM_ERR_STATE, "plan has no merge partition for SDDMM");
    hipError_t e = spmmk::launch_sddmm(plan->dtype, vec, sddmm_unroll(vec), g_log2, col_tiles,
                                       plan->rowptr, plan->colind, dC, B, dvals, plan->n,
                                       plan->ld, ws.coords, ws.P, W, st);
    if (e != hipSuccess) return hip_fail(e, "SDDMM launch");
    return SPMM_OK;
}

}  // extern "C"
