// tuner.cpp -- tile-configuration choice for single calls: a table of
// measured choices consulted before the built-in heuristic, and the tuner
// that fills it by timing every configuration on the caller's buffers.
#include <hip/hip_runtime.h>

#include <functional>
#include <map>
#include <mutex>
#include <string>
#include <tuple>

#include "host_common.hpp"
#include "mgemm.h"

namespace mgemm {

using ChoiceKey = std::tuple<int, int, int, int64_t, int64_t, int64_t>;

static std::mutex g_choice_mu;
static std::map<ChoiceKey, int> g_choices;

int recorded_choice(int precision, int ta, int tb, int64_t M, int64_t N, int64_t K) {
    std::lock_guard<std::mutex> lk(g_choice_mu);
    auto it = g_choices.find(ChoiceKey{precision, ta, tb, M, N, K});
    return it == g_choices.end() ? -1 : it->second;
}

static void record(int precision, int ta, int tb, int64_t M, int64_t N, int64_t K, int cfg) {
    std::lock_guard<std::mutex> lk(g_choice_mu);
    g_choices[ChoiceKey{precision, ta, tb, M, N, K}] = cfg;
}

void for_each_choice(
    const std::function<void(int, int, int, int64_t, int64_t, int64_t, int)>& fn) {
    std::lock_guard<std::mutex> lk(g_choice_mu);
    for (const auto& kv : g_choices) {
        const ChoiceKey& k = kv.first;
        fn(std::get<0>(k), std::get<1>(k), std::get<2>(k), std::get<3>(k), std::get<4>(k),
           std::get<5>(k), kv.second);
    }
}

}  // namespace mgemm

using namespace mgemm;

extern "C" {

int mgemm_record_choice(int precision, char transA, char transB, int64_t M, int64_t N,
                        int64_t K, int config) {
    const int ta = trans_code(transA), tb = trans_code(transB);
    if (ta < 0) return fail(-1, "transA must be N, T or C");
    if (tb < 0) return fail(-2, "transB must be N, T or C");
    if (config < 0 || config >= config_count(precision))
        return fail(MGEMM_ERR_UNSUPPORTED, "unknown precision or tile configuration");
    record(precision, ta, tb, M, N, K, config);
    return MGEMM_OK;
}

int mgemm_clear_choices(void) {
    std::lock_guard<std::mutex> lk(g_choice_mu);
    g_choices.clear();
    return MGEMM_OK;
}

int mgemm_tune_sgemm(char transA, char transB, int64_t M, int64_t N, int64_t K, float alpha,
                     const float* A, int64_t lda, const float* B, int64_t ldb, float beta,
                     float* C, int64_t ldc, void* stream, int precision, int reps,
                     int* best_config, float* best_ms) {
    std::string why;
    const int bad = validate(transA, transB, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, why);
    if (bad) return fail(bad, why);
    const int n = config_count(precision);
    if (n == 0) return fail(MGEMM_ERR_UNSUPPORTED, "unknown precision");
    if (reps < 1) reps = 1;
    int st = check_device(nullptr);
    if (st) return st;
    hipStream_t s = (hipStream_t)stream;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        (void)hipGetLastError();
        return fail(MGEMM_ERR_HIP, "hipEventCreate");
    }
    int best = -1;
    float best_t = 0.0f;
    for (int cfg = 0; cfg < n && st == MGEMM_OK; ++cfg) {
        st = mgemm_sgemm_ex(transA, transB, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc,
                            stream, precision, cfg);                     // warm-up
        float t_min = 1e30f;
        for (int r = 0; r < reps && st == MGEMM_OK; ++r) {
            hipError_t e = hipEventRecord(e0, s);
            if (e == hipSuccess)
                st = mgemm_sgemm_ex(transA, transB, M, N, K, alpha, A, lda, B, ldb, beta, C,
                                    ldc, stream, precision, cfg);
            if (st) break;
            if (e == hipSuccess) e = hipEventRecord(e1, s);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float t = 0.0f;
            if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
            if (e != hipSuccess) {
                (void)hipGetLastError();
                st = fail(MGEMM_ERR_HIP, std::string("tuning timer: ") + hipGetErrorString(e));
                break;
            }
            if (t < t_min) t_min = t;
        }
        if (st == MGEMM_OK && (best < 0 || t_min < best_t)) {
            best = cfg;
            best_t = t_min;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st) return st;
    const int ta = trans_code(transA), tb = trans_code(transB);
    record(precision, ta, tb, M, N, K, best);
    if (best_config) *best_config = best;
    if (best_ms) *best_ms = best_t;
    return MGEMM_OK;
}

}  // extern "C"
