// tuner.cpp -- tile-configuration choice for single calls: a table of
// measured choices consulted before the built-in heuristic, and the tuner
// that fills it by timing every configuration on the caller's buffers.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <functional>
#include <map>
#include <mutex>
#include <string>
#include <tuple>

#include "host_common.hpp"
#include "mgemm.h"
#include "rules.hpp"

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

static void forget(int precision, int ta, int tb, int64_t M, int64_t N, int64_t K) {
    std::lock_guard<std::mutex> lk(g_choice_mu);
    g_choices.erase(ChoiceKey{precision, ta, tb, M, N, K});
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

namespace mgemm {

// The built-in rule's choice (no recorded measurement).
static int builtin_default_config(int precision, int ta, int tb, int64_t M, int64_t N, int64_t K) {
    switch (precision) {
        case MGEMM_PREC_FP32: return f32_default_config(ta != 0, tb != 0, M, N, K);
        case MGEMM_PREC_BF16X3: return bf16x3_default_config(M, N, K);
        case MGEMM_PREC_FP16_SCALED: return f16s_default_config(M, N, K);
        default: return -1;
    }
}

}  // namespace mgemm

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
    int dev = 0;
    int st = check_device(&dev);
    if (st) return st;
    hipStream_t s = (hipStream_t)stream;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        (void)hipGetLastError();
        return fail(MGEMM_ERR_HIP, "hipEventCreate");
    }
    // One timed round: `calls` back-to-back calls between two events, the
    // mean per call.
    auto round_of = [&](int cfg, int calls, float& ms) -> int {
        hipError_t e = hipEventRecord(e0, s);
        int r = MGEMM_OK;
        for (int c = 0; c < calls && e == hipSuccess && r == MGEMM_OK; ++c)
            r = mgemm_sgemm_ex(transA, transB, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc,
                               stream, precision, cfg);
        if (r) return r;
        if (e == hipSuccess) e = hipEventRecord(e1, s);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float t = 0.0f;
        if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return fail(MGEMM_ERR_HIP, std::string("tuning timer: ") + hipGetErrorString(e));
        }
        ms = t / calls;
        return MGEMM_OK;
    };
    // Best of `reps` rounds after a warm-up call; short products take as
    // many calls per round as fill about a millisecond (at most 64), so
    // that a round is long against the timer and the clock's drift.
    auto time_of = [&](int cfg, float& best_ms_out) -> int {
        float first = 0.0f;
        int r = round_of(cfg, 1, first);   // warm-up, and a first estimate
        const int calls = first > 0.0f ? std::max(1, std::min(64, (int)(1.0f / first))) : 64;
        float t_min = 1e30f;
        for (int k = 0; k < reps && r == MGEMM_OK; ++k) {
            float t = 0.0f;
            r = round_of(cfg, calls, t);
            if (r == MGEMM_OK && t < t_min) t_min = t;
        }
        best_ms_out = t_min;
        return r;
    };
    // An FP32 product that the library, when no choice is recorded, splits
    // at its ragged edges or runs on the thin path: that choice is the
    // default to beat (timed with no choice recorded for the shape).
    const int ta0 = trans_code(transA), tb0 = trans_code(transB);
    int64_t mm = 0, nn = 0;
    bool own = false;
    if (precision == MGEMM_PREC_FP32) {
        const ThinPlan tp = thin_plan(M, N, K, lda, ldb, ldc, ta0 != 0, tb0 != 0, device_cus(dev));
        own = f32_edge_plan(ta0 != 0, tb0 != 0, M, N, K, &mm, &nn) ||
              (tp.ok && thin_workspace_bytes(tp, M, N, K) <= F32_SPLITK_MAX_WORKSPACE);
    }
    if (own) forget(precision, ta0, tb0, M, N, K);
    int best = -1;
    float best_t = 0.0f;
    for (int cfg = 0; cfg < n && st == MGEMM_OK; ++cfg) {
        float t_min = 0.0f;
        st = time_of(cfg, t_min);
        if (st == MGEMM_OK && (best < 0 || t_min < best_t)) {
            best = cfg;
            best_t = t_min;
        }
    }
    // A choice other than the built-in default is recorded only if it also
    // beats the default by more than 2% in a head-to-head, the two timed
    // alternately three times: of near ties, the default stays.
    const int dflt = own ? -1 : builtin_default_config(precision, ta0, tb0, M, N, K);
    if (st == MGEMM_OK && best != dflt && dflt >= -1 && dflt < n) {
        float td = 1e30f, tb_ = 1e30f;
        for (int k = 0; k < 3 && st == MGEMM_OK; ++k) {
            float t = 0.0f;
            st = time_of(dflt, t);
            if (st == MGEMM_OK) td = std::min(td, t);
            if (st == MGEMM_OK) st = time_of(best, t);
            if (st == MGEMM_OK) tb_ = std::min(tb_, t);
        }
        if (st == MGEMM_OK) {
            if (tb_ < 0.98f * td) {
                best_t = tb_;
            } else {
                best = dflt;
                best_t = td;
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st) return st;
    const int ta = trans_code(transA), tb = trans_code(transB);
    if (best >= 0) record(precision, ta, tb, M, N, K, best);   // -1: the library's own path stays
    if (best_config) *best_config = best;
    if (best_ms) *best_ms = best_t;
    return MGEMM_OK;
}

}  // extern "C"
