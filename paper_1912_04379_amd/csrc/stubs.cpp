// Temporary: precision forms and grouped plans not built yet.
#include "mgemm.h"
#include "kernels.hpp"
#include "host_common.hpp"
namespace mgemm {
int bf16x3_config_count() { return 0; }
TileConfigInfo bf16x3_config_info(int) { return {0,0,0,0}; }
int bf16x3_default_config(int64_t, int64_t, int64_t) { return 0; }
hipError_t launch_bf16x3(int, bool, bool, const GemmDesc&, hipStream_t) { return hipErrorInvalidValue; }
int f16s_config_count() { return 0; }
TileConfigInfo f16s_config_info(int) { return {0,0,0,0}; }
int f16s_default_config(int64_t, int64_t, int64_t) { return 0; }
hipError_t launch_f16_exponents(bool, bool, const GemmDesc&, int*, int*, hipStream_t) { return hipErrorInvalidValue; }
hipError_t launch_f16s(int, bool, bool, const GemmDesc&, hipStream_t) { return hipErrorInvalidValue; }
}
extern "C" {
int mgemm_grouped_plan_create(const mgemm_problem*, int64_t, int, const int*, void*, mgemm_plan**, int64_t*, int*) { return MGEMM_ERR_UNSUPPORTED; }
int mgemm_grouped_plan_launch(mgemm_plan*, void*) { return MGEMM_ERR_BAD_PLAN; }
int mgemm_grouped_plan_run(mgemm_plan*, void*) { return MGEMM_ERR_BAD_PLAN; }
int mgemm_grouped_plan_info(const mgemm_plan*, int64_t*, int64_t*) { return MGEMM_ERR_BAD_PLAN; }
int mgemm_grouped_plan_destroy(mgemm_plan*) { return MGEMM_ERR_BAD_PLAN; }
int mgemm_grouped_bucket(int64_t, int64_t, int64_t) { return 0; }
}
