// Batched small products: plans, persistent launch and HIP graph replay.
#include "sj_internal.h"

using namespace sj;

extern "C" {

sj_status sj_batch_plan(sj_handle, const int32_t *, int64_t, sj_plan *) { return fail(SJ_ERR_UNSUPPORTED, "batch plans are not built yet"); }
sj_status sj_batch_run(sj_plan, const double *, const double *, double *, void *) { return fail(SJ_ERR_UNSUPPORTED, "batch plans are not built yet"); }
sj_status sj_batch_graph_capture(sj_plan, const double *, const double *, double *, void *) { return fail(SJ_ERR_UNSUPPORTED, "batch plans are not built yet"); }
sj_status sj_batch_graph_launch(sj_plan, void *) { return fail(SJ_ERR_UNSUPPORTED, "batch plans are not built yet"); }
sj_status sj_batch_plan_arrays(sj_plan, const int32_t **, const int64_t **, int64_t *) { return fail(SJ_ERR_UNSUPPORTED, "batch plans are not built yet"); }
sj_status sj_plan_destroy(sj_plan) { return fail(SJ_ERR_UNSUPPORTED, "batch plans are not built yet"); }
sj_status sj_run_adam(sj_handle, void *const *, int, int64_t, double, double, double, double, void *) { return fail(SJ_ERR_UNSUPPORTED, "not built yet"); }

}
