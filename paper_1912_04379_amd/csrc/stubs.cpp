// Temporary: grouped plans not built yet.
#include "mgemm.h"
extern "C" {
int mgemm_grouped_plan_create(const mgemm_problem*, int64_t, int, const int*, void*, mgemm_plan**, int64_t*, int*) { return MGEMM_ERR_UNSUPPORTED; }
int mgemm_grouped_plan_launch(mgemm_plan*, void*) { return MGEMM_ERR_BAD_PLAN; }
int mgemm_grouped_plan_run(mgemm_plan*, void*) { return MGEMM_ERR_BAD_PLAN; }
int mgemm_grouped_plan_info(const mgemm_plan*, int64_t*, int64_t*) { return MGEMM_ERR_BAD_PLAN; }
int mgemm_grouped_plan_destroy(mgemm_plan*) { return MGEMM_ERR_BAD_PLAN; }
int mgemm_grouped_bucket(int64_t, int64_t, int64_t) { return 0; }
}
