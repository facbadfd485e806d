// Entry points whose kernels are not built yet: they report UNSUPPORTED.
#include "plan.hpp"

using namespace spmmh;

extern "C" {
int spmm_batch_plan(spmm_batch_t*, const spmm_problem*, int64_t, int32_t, int32_t, void*) { return fail(SPMM_ERR_UNSUPPORTED, "not built yet"); }
int spmm_batch_run(spmm_batch_t, void*) { return fail(SPMM_ERR_UNSUPPORTED, "not built yet"); }
int spmm_batch_run_direct(spmm_batch_t, void*) { return fail(SPMM_ERR_UNSUPPORTED, "not built yet"); }
int spmm_batch_problem_config(spmm_batch_t, int64_t, spmm_config*) { return fail(SPMM_ERR_UNSUPPORTED, "not built yet"); }
int spmm_batch_destroy(spmm_batch_t) { return fail(SPMM_ERR_UNSUPPORTED, "not built yet"); }
}
