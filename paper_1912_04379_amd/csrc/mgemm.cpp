// mgemm.cpp -- host side of the C ABI declared in include/mgemm.h:
// argument validation (BLAS order, before any HIP call), quick returns,
// device checks, configuration choice and kernel dispatch.
#include "mgemm.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <unordered_set>

#include "host_common.hpp"
#include "kernels.hpp"

namespace mgemm {

static thread_local std::string g_last_error;

int fail(int status, const std::string& msg) {
    g_last_error = msg;
    return status;
}

static int hip_fail(hipError_t e, const char* where) {
    return fail(MGEMM_ERR_HIP, std::string(where) + ": " + hipGetErrorString(e));
}

// Per-device check that the current device is a gfx950: 0 unknown,
// 1 ok, 2 wrong architecture.
static std::atomic<int> g_dev_state[64];

static std::atomic<int> g_device_count{0};

int check_device(int* out_dev) {
    // The device count does not change within a process: query it until a
    // device is seen, then keep it.
    if (g_device_count.load(std::memory_order_relaxed) <= 0) {
        int count = 0;
        hipError_t e = hipGetDeviceCount(&count);
        if (e != hipSuccess || count <= 0) {
            (void)hipGetLastError();
            return fail(MGEMM_ERR_NO_DEVICE, "no HIP device is visible");
        }
        g_device_count.store(count, std::memory_order_relaxed);
    }
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (out_dev) *out_dev = dev;
    int state = dev < 64 ? g_dev_state[dev].load(std::memory_order_relaxed) : 0;
    if (state == 0) {
        hipDeviceProp_t prop;
        e = hipGetDeviceProperties(&prop, dev);
        if (e != hipSuccess) return hip_fail(e, "hipGetDeviceProperties");
        state = std::strncmp(prop.gcnArchName, "gfx950", 6) == 0 ? 1 : 2;
        if (dev < 64) g_dev_state[dev].store(state, std::memory_order_relaxed);
        if (state == 2)
            return fail(MGEMM_ERR_ARCH, std::string("device is ") + prop.gcnArchName +
                                            ", this library is built for gfx950");
    }
    if (state == 2) return fail(MGEMM_ERR_ARCH, "device is not a gfx950");
    return MGEMM_OK;
}

// ---------------------------------------------------------------------------
// Workspace pool.  The 16-bit forms take a stream-ordered workspace per
// call from a memory pool of the library's own, one per device, whose
// release threshold is the maximum: freed workspace stays with the pool
// across synchronisations and is handed back only by mgemm_trim_workspace.
// (The device's default pool returns its memory at every synchronisation,
// so the next call would map it again: up to a few tenths of a millisecond
// for the hundreds of megabytes that packed 8192^3 operands take.)
// ---------------------------------------------------------------------------
static std::atomic<int> g_cus[64];

int device_cus(int dev) {
    if (dev < 0 || dev >= 64) return 0;
    int n = g_cus[dev].load(std::memory_order_relaxed);
    if (n > 0) return n;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    g_cus[dev].store(n, std::memory_order_relaxed);
    return n;
}

static std::mutex g_pool_mu;
static hipMemPool_t g_pools[64] = {};

static hipError_t workspace_pool(int dev, hipMemPool_t* out) {
    if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_pool_mu);
    if (!g_pools[dev]) {
        hipMemPoolProps props{};
        props.allocType = hipMemAllocationTypePinned;
        props.handleTypes = hipMemHandleTypeNone;
        props.location.type = hipMemLocationTypeDevice;
        props.location.id = dev;
        hipMemPool_t pool = nullptr;
        hipError_t e = hipMemPoolCreate(&pool, &props);
        if (e != hipSuccess) return e;
        uint64_t keep = UINT64_MAX;
        e = hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep);
        if (e != hipSuccess) {
            (void)hipMemPoolDestroy(pool);
            return e;
        }
        g_pools[dev] = pool;
    }
    *out = g_pools[dev];
    return hipSuccess;
}

int trim_workspace() {
    std::lock_guard<std::mutex> lk(g_pool_mu);
    for (hipMemPool_t pool : g_pools) {
        if (!pool) continue;
        hipError_t e = hipMemPoolTrimTo(pool, 0);
        if (e != hipSuccess) return hip_fail(e, "hipMemPoolTrimTo");
    }
    return MGEMM_OK;
}

int config_count(int precision) {
    switch (precision) {
        case MGEMM_PREC_FP32: return f32_config_count();
        case MGEMM_PREC_BF16X3: return bf16x3_config_count();
        case MGEMM_PREC_FP16_SCALED: return f16s_config_count();
        default: return 0;
    }
}

static int default_config(int precision, int ta, int tb, int64_t M, int64_t N, int64_t K) {
    const int tuned = recorded_choice(precision, ta, tb, M, N, K);
    if (tuned >= 0) return tuned;
    switch (precision) {
        case MGEMM_PREC_FP32: return f32_default_config(ta, tb, M, N, K);
        case MGEMM_PREC_BF16X3: return bf16x3_default_config(M, N, K);
        case MGEMM_PREC_FP16_SCALED: return f16s_default_config(M, N, K);
        default: return -1;
    }
}

// Workspace of one call: `fixed` (a device buffer of fixed->cap bytes that
// the caller owns) when given, else stream-ordered memory from the pool.
static hipError_t take_workspace(int dev, const FixedWorkspace* fixed, int64_t bytes,
                                 hipStream_t s, char** out) {
    if (fixed) {
        if (bytes > fixed->cap) return hipErrorOutOfMemory;
        *out = fixed->base;
        return hipSuccess;
    }
    hipMemPool_t pool = nullptr;
    hipError_t e = workspace_pool(dev, &pool);
    if (e == hipSuccess) e = hipMallocFromPoolAsync((void**)out, (size_t)bytes, pool, s);
    return e;
}

static hipError_t give_back_workspace(const FixedWorkspace* fixed, char* ws, hipStream_t s) {
    return fixed || !ws ? hipSuccess : hipFreeAsync(ws, s);
}

// Error text of a call whose workspace exceeds a fixed workspace.
static std::string too_big(int64_t bytes, int64_t cap, const char* what) {
    return std::string("the ") + what + " need " + std::to_string(bytes) +
           " bytes of workspace, more than the fixed " + std::to_string(cap);
}

// What one call did, for MGEMM_LOG.
struct Dispatch {
    const char* path = "none";   // quick return, or the kernels launched
    int cfg = -1;
    int splits = 0;
    int64_t ws_bytes = 0;
};

static int sgemm_body(char transA, char transB, int64_t M, int64_t N, int64_t K, float alpha,
                      const float* A, int64_t lda, const float* B, int64_t ldb, float beta,
                      float* C, int64_t ldc, void* stream, int precision, int config,
                      const FixedWorkspace* fixed, int act, const float* aux, Dispatch& dp) {
    std::string why;
    const int bad = validate(transA, transB, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, why);
    if (bad) return fail(bad, why);
    if (precision < 0 || precision > MGEMM_PREC_FP16_SCALED)
        return fail(MGEMM_ERR_UNSUPPORTED, "unknown precision");
    if (config < -1 || config >= config_count(precision))
        return fail(MGEMM_ERR_UNSUPPORTED, "unknown tile configuration");
    if (act < MGEMM_ACT_NONE || act > MGEMM_ACT_TANH_GRAD)
        return fail(MGEMM_ERR_UNSUPPORTED, "unknown activation");
    if (act == MGEMM_ACT_TANH_GRAD && M > 0 && N > 0 && aux == nullptr)
        return fail(MGEMM_ERR_UNSUPPORTED, "aux is NULL");
    const int ta = trans_code(transA), tb = trans_code(transB);
    // Quick returns (reference BLAS); an activation still has to be applied
    // when C itself is left as it is.
    if (M == 0 || N == 0) return MGEMM_OK;
    const bool no_product = alpha == 0.0f || K == 0;
    if (no_product && beta == 1.0f && act == MGEMM_ACT_NONE) return MGEMM_OK;
    if (overlaps(ta, tb, M, N, K, alpha, A, lda, B, ldb, C, ldc))
        return fail(MGEMM_ERR_ALIAS, "C overlaps A or B");
    if (act == MGEMM_ACT_TANH_GRAD) {
        const Extent c = extent_of(C, M, N, ldc, 0), x = extent_of(aux, M, N, ldc, 0);
        if (c.lo < x.hi && x.lo < c.hi) return fail(MGEMM_ERR_ALIAS, "C overlaps aux");
    }
    int dev = 0;
    int st = check_device(&dev);
    if (st) return st;
    FixedWorkspace fx{};
    if (fixed) {
        fx = *fixed;
        if (!fx.base && fx.resolve && (st = fx.resolve(dev, &fx.base)) != MGEMM_OK) return st;
        if (!fx.base) return fail(MGEMM_ERR_UNSUPPORTED, "fixed workspace has no address");
        fixed = &fx;
    }

    hipStream_t s = (hipStream_t)stream;
    GemmDesc d{A, B, C, M, N, K, lda, ldb, ldc, alpha, beta, nullptr, nullptr, act,
               act == MGEMM_ACT_TANH_GRAD ? aux : nullptr};
    hipError_t e;
    if (no_product) {
        dp.path = "scale_c";
        e = launch_scale_c(d, s);
        return e == hipSuccess ? MGEMM_OK : hip_fail(e, "scale kernel launch");
    }
    // The library's FP32 choice for a product a little past whole 256 x 256
    // tiles (and no choice recorded for it): the whole-tile block and the
    // thin remainders as separate products, each with its own default.
    int64_t Mm = 0, Nm = 0;
    if (precision == MGEMM_PREC_FP32 && config < 0 && act == MGEMM_ACT_NONE &&
        recorded_choice(precision, ta, tb, M, N, K) < 0 && buffer_path_ok(d) &&
        f32_edge_plan(ta, tb, M, N, K, &Mm, &Nm)) {
        dp.path = "f32_edge_split";
        dp.cfg = default_config(precision, ta, tb, Mm, Nm, K);
        auto part = [&](int64_t m, int64_t n, const float* a, const float* b, float* c, int cf) {
            Dispatch sub;
            return sgemm_body(transA, transB, m, n, K, alpha, a, lda, b, ldb, beta, c, ldc, stream,
                              precision, cf, fixed, MGEMM_ACT_NONE, nullptr, sub);
        };
        // The block on its own default; the remainders on the library's
        // choice (the thin path for at most THIN_MAX_R rows or columns).
        st = part(Mm, Nm, A, B, C, default_config(precision, ta, tb, Mm, Nm, K));
        if (!st && Mm < M)   // rows Mm..M-1 of C, every column
            st = part(M - Mm, N, ta ? A + Mm * lda : A + Mm, B, C + Mm, -1);
        if (!st && Nm < N)   // columns Nm..N-1 of the first Mm rows
            st = part(Mm, N - Nm, A, tb ? B + Nm : B + Nm * ldb, C + Nm * ldc, -1);
        return st;
    }
    // The library's FP32 choice for a matrix-vector-like product (at most
    // THIN_MAX_R columns or rows of C, no choice recorded for it): the thin
    // path, which streams the large operand once.
    if (precision == MGEMM_PREC_FP32 && config < 0 && act == MGEMM_ACT_NONE &&
        recorded_choice(precision, ta, tb, M, N, K) < 0) {
        const ThinPlan tp = thin_plan(M, N, K, lda, ldb, ldc, ta, tb, device_cus(dev));
        const int64_t bytes = thin_workspace_bytes(tp, M, N, K);
        if (tp.ok && bytes <= (fixed ? fixed->cap : F32_SPLITK_MAX_WORKSPACE)) {
            dp.path = "f32_thin";
            dp.splits = tp.splits;
            dp.ws_bytes = bytes;
            char* ws = nullptr;
            e = fault_injected() ? hipErrorOutOfMemory : take_workspace(dev, fixed, bytes, s, &ws);
            if (e != hipSuccess) {
                (void)hipGetLastError();
                return fail(MGEMM_ERR_ALLOC, "stream-ordered thin-product workspace");
            }
            e = launch_thin(ta, tb, d, tp, reinterpret_cast<float*>(ws), s);
            const hipError_t e2 = give_back_workspace(fixed, ws, s);
            if (e == hipSuccess) e = e2;
            return e == hipSuccess ? MGEMM_OK : hip_fail(e, "GEMM kernel launch");
        }
    }
    int cfg = config >= 0 ? config : default_config(precision, ta, tb, M, N, K);
    dp.cfg = cfg;
    dp.path = precision == MGEMM_PREC_FP32 ? "f32" : "in_staging";
    if (precision == MGEMM_PREC_FP32 && cfg == F32_TAIL_CONFIG) {
        dp.path = buffer_path_ok(d) ? "f32_rounds_and_tail" : "f32_64bit_addresses";
        // The 64-bit address path has no split tail: 128 x 128 tiles.
        e = buffer_path_ok(d) ? launch_f32_tail(ta, tb, d, device_cus(dev), s)
                              : launch_f32(0, ta, tb, d, s);
        return e == hipSuccess ? MGEMM_OK : hip_fail(e, "GEMM kernel launch");
    }
    if (precision == MGEMM_PREC_FP32 && cfg == F32_SPLITK_CONFIG) {
        // Split-K needs a workspace of S partial products; where it does
        // not apply (short k, 64-bit address path), 128 x 128 tiles.
        const SplitKPlan plan = f32_splitk_plan(M, N, K, device_cus(dev));
        const int64_t bytes = f32_splitk_workspace_bytes(plan, M, N);
        const bool applies = plan.splits >= 2 && buffer_path_ok(d) && M <= MAX_BUF_LD;
        if (fixed && config >= 0 && applies && bytes > fixed->cap)
            return fail(MGEMM_ERR_UNSUPPORTED, too_big(bytes, fixed->cap, "split-K partial products"));
        if (!applies || bytes > (fixed ? fixed->cap : F32_SPLITK_MAX_WORKSPACE)) {
            dp.path = "f32_unsplit";
            dp.cfg = 0;
            e = launch_f32(0, ta, tb, d, s);
            return e == hipSuccess ? MGEMM_OK : hip_fail(e, "GEMM kernel launch");
        }
        dp.path = "f32_split_k";
        dp.splits = plan.splits;
        dp.ws_bytes = bytes;
        char* ws = nullptr;
        e = fault_injected() ? hipErrorOutOfMemory : take_workspace(dev, fixed, bytes, s, &ws);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return fail(MGEMM_ERR_ALLOC, "stream-ordered split-K workspace");
        }
        e = launch_f32_splitk(ta, tb, d, plan, reinterpret_cast<float*>(ws), s);
        const hipError_t e2 = give_back_workspace(fixed, ws, s);
        if (e == hipSuccess) e = e2;
        return e == hipSuccess ? MGEMM_OK : hip_fail(e, "GEMM kernel launch");
    }
    if (precision == MGEMM_PREC_FP32) {
        e = launch_f32(cfg, ta, tb, d, s);
        return e == hipSuccess ? MGEMM_OK : hip_fail(e, "GEMM kernel launch");
    }
    const bool bf = precision == MGEMM_PREC_BF16X3;
    // Split-K (configuration LOWP_SPLITK_CONFIG): where it does not apply
    // (short k, 64-bit address path, a workspace beyond the limit), the
    // 128 x 128 in-staging tile.
    SplitKPlan split{0, 0, 0};
    int64_t split_bytes = 0;
    if (cfg == LOWP_SPLITK_CONFIG) {
        split = f32_splitk_plan(M, N, K, device_cus(dev));
        split_bytes = f32_splitk_workspace_bytes(split, M, N);
        const bool applies = split.splits >= 2 && buffer_path_ok(d) && M <= MAX_BUF_LD;
        if (fixed && config >= 0 && applies && split_bytes > fixed->cap)
            return fail(MGEMM_ERR_UNSUPPORTED,
                        too_big(split_bytes, fixed->cap, "split-K partial products"));
        if (!applies || split_bytes > (fixed ? fixed->cap : F32_SPLITK_MAX_WORKSPACE)) {
            split = SplitKPlan{0, 0, 0};
            split_bytes = 0;
            cfg = 1;
        }
    }
    bool packed = cfg >= LOWP_INSTAGE_CONFIGS && cfg < LOWP_SPLITK_CONFIG;
    if (packed && !packed_supported(bf, cfg - LOWP_INSTAGE_CONFIGS, M, N, K)) {
        // Not available for this form, or lane offsets would not fit in 31
        // bits: split while staging, with the 256 x 256 in-staging tile.
        packed = false;
        cfg = 0;
    }
    // Stream-ordered workspace: FP16 panel exponents (+ pass-1 partial
    // maxima) and/or packed operands.
    const int64_t pa = (M + 31) / 32, pb = (N + 31) / 32;
    const int64_t part_bytes = bf ? 0 : (f16_partial_floats(M, N, K) * 4 + 255) / 256 * 256;
    const int64_t exp_bytes =
        bf ? 0 : ((pa + pb) * (int64_t)sizeof(int) + 255) / 256 * 256 + part_bytes;
    int64_t pack_bytes =
        packed ? packed_workspace_bytes(bf, cfg - LOWP_INSTAGE_CONFIGS, M, N, K) : 0;
    if (fixed && packed && exp_bytes + pack_bytes > fixed->cap) {
        // The packed operands do not fit the fixed workspace.  A named
        // configuration is refused; the library's choice splits (or
        // scales) while staging instead, which needs no packed copy.
        if (config >= 0)
            return fail(MGEMM_ERR_UNSUPPORTED,
                        too_big(exp_bytes + pack_bytes, fixed->cap, "packed operands"));
        packed = false;
        cfg = 0;
        pack_bytes = 0;
    }
    if (fixed && exp_bytes > fixed->cap)
        return fail(MGEMM_ERR_UNSUPPORTED, too_big(exp_bytes, fixed->cap, "FP16 panel exponents"));
    if (fixed && split.splits && exp_bytes + split_bytes > fixed->cap) {
        // Exponents and partial products together exceed the fixed
        // workspace: a named configuration is refused, the library's choice
        // runs unsplit.
        if (config >= 0)
            return fail(MGEMM_ERR_UNSUPPORTED,
                        too_big(exp_bytes + split_bytes, fixed->cap, "split-K partial products"));
        split = SplitKPlan{0, 0, 0};
        split_bytes = 0;
        cfg = 1;
    }
    // The FP16 form's split-K pieces run on packed operands where that
    // applies and the operands fit (same results bitwise; faster than
    // scaling while staging in every piece).
    int64_t split_pack_bytes = 0;
    const int64_t split_room = (split_bytes + 255) / 256 * 256;   // packed operands start aligned
    if (!bf && split.splits && f16s_packed_splitk_supported(split, M, N, K)) {
        split_pack_bytes = f16s_packed_splitk_bytes(M, N, K);
        if (fixed && exp_bytes + split_room + split_pack_bytes > fixed->cap) split_pack_bytes = 0;
    }
    dp.cfg = cfg;
    dp.path = packed                             ? "packed"
              : split.splits && split_pack_bytes ? "lowp_split_k_packed"
              : split.splits                     ? "lowp_split_k"
                                                 : "in_staging";
    dp.splits = split.splits;
    dp.ws_bytes = exp_bytes + pack_bytes + (split_pack_bytes ? split_room + split_pack_bytes : split_bytes);
    char* ws = nullptr;
    if (dp.ws_bytes > 0) {
        e = fault_injected() ? hipErrorOutOfMemory : take_workspace(dev, fixed, dp.ws_bytes, s, &ws);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return fail(MGEMM_ERR_ALLOC, "stream-ordered workspace");
        }
    }
    e = hipSuccess;
    if (!bf) {
        d.expA = reinterpret_cast<int*>(ws);
        d.expB = reinterpret_cast<int*>(ws) + pa;
        e = launch_f16_exponents(ta, tb, d, reinterpret_cast<int*>(ws),
                                 reinterpret_cast<int*>(ws) + pa,
                                 reinterpret_cast<float*>(ws + exp_bytes - part_bytes), s);
    }
    if (e == hipSuccess) {
        if (packed)
            e = launch_packed(bf, cfg - LOWP_INSTAGE_CONFIGS, ta, tb, d, ws + exp_bytes, s);
        else if (split.splits && split_pack_bytes)
            e = launch_f16s_packed_splitk(ta, tb, d, split, ws + exp_bytes + split_room,
                                          reinterpret_cast<float*>(ws + exp_bytes), s);
        else if (split.splits)
            e = launch_lowp_splitk(bf, ta, tb, d, split, reinterpret_cast<float*>(ws + exp_bytes),
                                   s);
        else
            e = bf ? launch_bf16x3(cfg, ta, tb, d, s) : launch_f16s(cfg, ta, tb, d, s);
    }
    if (ws) {
        hipError_t e2 = give_back_workspace(fixed, ws, s);
        if (e == hipSuccess) e = e2;
    }
    return e == hipSuccess ? MGEMM_OK : hip_fail(e, "GEMM kernel launch");
}

static const char* prec_name(int precision) {
    return precision == MGEMM_PREC_FP32           ? "fp32"
           : precision == MGEMM_PREC_BF16X3       ? "bf16x3"
           : precision == MGEMM_PREC_FP16_SCALED ? "fp16s"
                                                  : "?";
}

int sgemm_impl(char transA, char transB, int64_t M, int64_t N, int64_t K, float alpha,
               const float* A, int64_t lda, const float* B, int64_t ldb, float beta, float* C,
               int64_t ldc, void* stream, int precision, int config,
               const FixedWorkspace* fixed, int act, const float* aux) {
    Dispatch dp;
    const int st = sgemm_body(transA, transB, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc,
                              stream, precision, config, fixed, act, aux, dp);
    if (log_enabled())
        log_line("sgemm%s %s %c%c M=%lld N=%lld K=%lld lda=%lld ldb=%lld ldc=%lld alpha=%g "
                 "beta=%g config=%d%s -> %s cfg=%d splits=%d workspace=%lld status=%d%s%s",
                 fixed ? "_noalloc" : "", prec_name(precision), transA ? transA : '?',
                 transB ? transB : '?', (long long)M, (long long)N, (long long)K,
                 (long long)lda, (long long)ldb, (long long)ldc, (double)alpha, (double)beta,
                 config,
                 act == MGEMM_ACT_TANH ? " act=tanh" : act == MGEMM_ACT_TANH_GRAD ? " act=tanh_grad" : "",
                 dp.path, dp.cfg, dp.splits, (long long)dp.ws_bytes, st,
                 st ? " " : "", st ? g_last_error.c_str() : "");
    return st;
}

}  // namespace mgemm

using namespace mgemm;

extern "C" {

int mgemm_trim_workspace(void) { return trim_workspace(); }

int mgemm_sgemm(char transA, char transB, int64_t M, int64_t N, int64_t K, float alpha,
                const float* A, int64_t lda, const float* B, int64_t ldb, float beta, float* C,
                int64_t ldc, void* stream) {
    return sgemm_impl(transA, transB, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, stream,
                      MGEMM_PREC_FP32, -1, nullptr);
}

int mgemm_sgemm_ex(char transA, char transB, int64_t M, int64_t N, int64_t K, float alpha,
                   const float* A, int64_t lda, const float* B, int64_t ldb, float beta,
                   float* C, int64_t ldc, void* stream, int precision, int config) {
    return sgemm_impl(transA, transB, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, stream,
                      precision, config, nullptr);
}

int mgemm_sgemm_act(char transA, char transB, int64_t M, int64_t N, int64_t K, float alpha,
                    const float* A, int64_t lda, const float* B, int64_t ldb, float beta,
                    float* C, int64_t ldc, void* stream, int precision, int config,
                    int activation, const float* aux) {
    return sgemm_impl(transA, transB, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, stream,
                      precision, config, nullptr, activation, aux);
}

int mgemm_config_count(int precision) { return config_count(precision); }

int mgemm_config_info(int precision, int config, int* bm, int* bn, int* bk, int* threads) {
    if (config < 0 || config >= config_count(precision))
        return fail(MGEMM_ERR_UNSUPPORTED, "unknown tile configuration");
    TileConfigInfo t = precision == MGEMM_PREC_FP32     ? f32_config_info(config)
                       : precision == MGEMM_PREC_BF16X3 ? bf16x3_config_info(config)
                                                        : f16s_config_info(config);
    if (bm) *bm = t.bm;
    if (bn) *bn = t.bn;
    if (bk) *bk = t.bk;
    if (threads) *threads = t.threads;
    return MGEMM_OK;
}

int mgemm_default_config(int precision, char transA, char transB, int64_t M, int64_t N,
                         int64_t K) {
    const int ta = trans_code(transA), tb = trans_code(transB);
    if (ta < 0 || tb < 0) return -1;
    return default_config(precision, ta, tb, M, N, K);
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Pre-packed op(B) (BF16x3).  The handle owns op(B) packed once in the
// 16-deep blocks of the packed engine's pipelined configurations, hi then
// lo halves; calls pack only op(A) and run the main kernel on both.
// ---------------------------------------------------------------------------
struct mgemm_packed_b {
    int precision;
    int device;
    int64_t K, N;
    char* hi;     // the allocation: packed values, then (FP16) exponents
    char* lo;     // BF16x3 lo halves (NULL for FP16 and FP32)
    int* expB;    // FP16: panel exponents of op(B) (NULL otherwise)
    int64_t bytes;
    int64_t ld;   // FP32: leading dimension of the k-contiguous K x N array
};

namespace mgemm {

static constexpr int PACKED_B_KW = 16;
// Packed configurations that read 16-deep blocks and fit the BF16x3 ring:
// the pipelined 256 x 256 and 128 x 128 tiles (16-bit configurations 10, 11).
static constexpr int PACKED_B_BIG = 6, PACKED_B_SMALL = 7;

static std::mutex g_packed_mu;
static std::unordered_set<const mgemm_packed_b*> g_packed;

static int64_t round256(int64_t b) { return (b + 255) / 256 * 256; }

// FP16 exponent bytes for P rows (or columns) of panels: the exponents and
// the pre-pass's partial maxima.
static int64_t f16_exp_bytes(int64_t P, int64_t K) {
    return round256((P + 31) / 32 * (int64_t)sizeof(int)) +
           round256(f16_partial_floats(P, 0, K) * (int64_t)sizeof(float));
}

static bool packed_b_live(const mgemm_packed_b* p) {
    std::lock_guard<std::mutex> lk(g_packed_mu);
    return p && g_packed.count(p);
}

}  // namespace mgemm

namespace mgemm {

// FP32 pre-packed B: op(B) as a column-major K x N array, k contiguous, with
// its leading dimension rounded up to a multiple of 4 floats.
static int pack_b_f32(int tb, int64_t K, int64_t N, const float* B, int64_t ldb, void* stream,
                      mgemm_packed_b** out) {
    const int64_t ld = (std::max<int64_t>(K, 1) + 3) / 4 * 4;
    if (N > 0 && ld > INT64_MAX / (int64_t)sizeof(float) / N)
        return fail(MGEMM_ERR_UNSUPPORTED, "packed B larger than the address space");
    int dev = 0;
    const int st = check_device(&dev);
    if (st) return st;
    const int64_t bytes = K > 0 && N > 0 ? ld * N * (int64_t)sizeof(float) : 0;
    mgemm_packed_b* h =
        new mgemm_packed_b{MGEMM_PREC_FP32, dev, K, N, nullptr, nullptr, nullptr, bytes, ld};
    if (bytes > 0) {
        hipError_t e = fault_injected() ? hipErrorOutOfMemory
                                        : hipMalloc((void**)&h->hi, (size_t)bytes);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            delete h;
            return fail(MGEMM_ERR_ALLOC, "packed B buffer");
        }
        e = launch_f32_pack_b(tb != 0, B, ldb, K, N, reinterpret_cast<float*>(h->hi), ld,
                              (hipStream_t)stream);
        if (e != hipSuccess) {
            (void)hipFree(h->hi);
            delete h;
            return hip_fail(e, "pack kernel launch");
        }
    }
    {
        std::lock_guard<std::mutex> lk(g_packed_mu);
        g_packed.insert(h);
    }
    *out = h;
    return MGEMM_OK;
}

}  // namespace mgemm

extern "C" {

int mgemm_pack_b(char transB, int64_t K, int64_t N, const float* B, int64_t ldb, int precision,
                 void* stream, mgemm_packed_b** out) {
    if (!out) return fail(MGEMM_ERR_UNSUPPORTED, "out is NULL");
    *out = nullptr;
    const int tb = trans_code(transB);
    if (tb < 0) return fail(-2, "transB must be N, T or C");
    if (N < 0) return fail(-4, "N < 0");
    if (K < 0) return fail(-5, "K < 0");
    if (K > 0 && N > 0 && B == nullptr) return fail(-9, "B is NULL");
    const int64_t rows_b = tb ? N : K;
    if (ldb < (rows_b > 1 ? rows_b : 1)) return fail(-10, "ldb < max(1, stored rows of B)");
    if (precision == MGEMM_PREC_FP32) return pack_b_f32(tb, K, N, B, ldb, stream, out);
    if (precision != MGEMM_PREC_BF16X3 && precision != MGEMM_PREC_FP16_SCALED)
        return fail(MGEMM_ERR_UNSUPPORTED, "unknown precision");
    const bool bf = precision == MGEMM_PREC_BF16X3;
    if (!packed_supported(bf, PACKED_B_BIG, 1, N, K) ||
        !packed_supported(bf, PACKED_B_SMALL, 1, N, K))
        return fail(MGEMM_ERR_UNSUPPORTED, "K too long for the packed engine's 32-bit offsets");
    int dev = 0;
    const int st = check_device(&dev);
    if (st) return st;
    const int64_t pack_bytes = packed_operand_bytes(bf, PACKED_B_KW, N, K);
    const int64_t bytes = round256(pack_bytes) + (bf ? 0 : f16_exp_bytes(N, K));
    mgemm_packed_b* h =
        new mgemm_packed_b{precision, dev, K, N, nullptr, nullptr, nullptr, bytes, 0};
    if (N > 0 && bytes > 0) {
        hipError_t e = fault_injected() ? hipErrorOutOfMemory
                                        : hipMalloc((void**)&h->hi, (size_t)bytes);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            delete h;
            return fail(MGEMM_ERR_ALLOC, "packed B buffer");
        }
        hipStream_t s = (hipStream_t)stream;
        if (bf) {
            h->lo = h->hi + pack_bytes / 2;
        } else {
            // op(B)'s panel exponents alone: the pre-pass with M = 0.
            h->expB = reinterpret_cast<int*>(h->hi + round256(pack_bytes));
            float* partial = reinterpret_cast<float*>(
                h->hi + round256(pack_bytes) + round256((N + 31) / 32 * (int64_t)sizeof(int)));
            const GemmDesc db{nullptr, B, nullptr, 0, N, K, 1, ldb, 1, 1.0f, 0.0f,
                              nullptr, nullptr};
            e = launch_f16_exponents(false, tb, db, nullptr, h->expB, partial, s);
        }
        if (e == hipSuccess)
            e = launch_pack_operand(bf, PACKED_B_KW, !tb, B, ldb, N, K, h->hi, h->lo, h->expB, s);
        if (e != hipSuccess) {
            (void)hipFree(h->hi);
            delete h;
            return hip_fail(e, "pack kernel launch");
        }
    }
    {
        std::lock_guard<std::mutex> lk(g_packed_mu);
        g_packed.insert(h);
    }
    *out = h;
    return MGEMM_OK;
}

int mgemm_packed_b_info(const mgemm_packed_b* Bp, int64_t* K, int64_t* N, int* precision,
                        int64_t* bytes) {
    if (!packed_b_live(Bp)) return fail(MGEMM_ERR_BAD_PLAN, "packed B is NULL or destroyed");
    if (K) *K = Bp->K;
    if (N) *N = Bp->N;
    if (precision) *precision = Bp->precision;
    if (bytes) *bytes = Bp->bytes;
    return MGEMM_OK;
}

int mgemm_sgemm_packed_b(char transA, int64_t M, float alpha, const float* A, int64_t lda,
                         const mgemm_packed_b* Bp, float beta, float* C, int64_t ldc,
                         void* stream) {
    if (!packed_b_live(Bp)) return fail(MGEMM_ERR_BAD_PLAN, "packed B is NULL or destroyed");
    const int64_t K = Bp->K, N = Bp->N;
    // The SGEMM checks with op(B) standing in as a non-NULL 'N' operand.
    std::string why;
    const int bad = validate(transA, 'N', M, N, K, alpha, A, lda,
                             reinterpret_cast<const float*>(Bp), K > 1 ? K : 1, beta, C, ldc, why);
    if (bad) return fail(bad, why);
    const int ta = trans_code(transA);
    if (M == 0 || N == 0) return MGEMM_OK;
    const bool no_product = alpha == 0.0f || K == 0;
    if (no_product && beta == 1.0f) return MGEMM_OK;
    if (!no_product) {
        const Extent a = extent_of(A, ta ? K : M, ta ? M : K, lda, 0);
        const Extent c = extent_of(C, M, N, ldc, 0);
        if (a.lo < c.hi && c.lo < a.hi) return fail(MGEMM_ERR_ALIAS, "C overlaps A");
    }
    int dev = 0;
    int st = check_device(&dev);
    if (st) return st;
    if (dev != Bp->device) return fail(MGEMM_ERR_UNSUPPORTED, "B was packed on another device");
    hipStream_t s = (hipStream_t)stream;
    GemmDesc d{A, nullptr, C, M, N, K, lda, K > 1 ? K : 1, ldc, alpha, beta, nullptr, nullptr};
    hipError_t e;
    if (no_product) {
        e = launch_scale_c(d, s);
        return e == hipSuccess ? MGEMM_OK : hip_fail(e, "scale kernel launch");
    }
    if (Bp->precision == MGEMM_PREC_FP32) {
        // An ordinary FP32 product with op(B) as the packed 'N' operand.
        return sgemm_impl(transA, 'N', M, N, K, alpha, A, lda,
                          reinterpret_cast<const float*>(Bp->hi), Bp->ld, beta, C, ldc, stream,
                          MGEMM_PREC_FP32, -1, nullptr);
    }
    const bool bf = Bp->precision == MGEMM_PREC_BF16X3;
    const int64_t t256 = ((M + 255) / 256) * ((N + 255) / 256);
    const int cfg = t256 >= 144 ? PACKED_B_BIG : PACKED_B_SMALL;
    const int64_t pack_bytes = round256(packed_operand_bytes(bf, PACKED_B_KW, M, K));
    const int64_t bytes = pack_bytes + (bf ? 0 : f16_exp_bytes(M, K));
    char* ws = nullptr;
    e = fault_injected() ? hipErrorOutOfMemory : take_workspace(dev, nullptr, bytes, s, &ws);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(MGEMM_ERR_ALLOC, "stream-ordered workspace for packed A");
    }
    if (!bf) {
        // op(A)'s panel exponents alone (the pre-pass with N = 0); op(B)'s
        // are the handle's.
        int* expA = reinterpret_cast<int*>(ws + pack_bytes);
        d.expA = expA;
        d.expB = Bp->expB;
        GemmDesc da = d;
        da.N = 0;
        float* partial = reinterpret_cast<float*>(
            ws + pack_bytes + round256((M + 31) / 32 * (int64_t)sizeof(int)));
        e = launch_f16_exponents(ta, false, da, expA, nullptr, partial, s);
    }
    if (e == hipSuccess) e = launch_packed_b_ready(bf, cfg, ta, d, ws, Bp->hi, Bp->lo, s);
    const hipError_t e2 = give_back_workspace(nullptr, ws, s);
    if (e == hipSuccess) e = e2;
    return e == hipSuccess ? MGEMM_OK : hip_fail(e, "GEMM kernel launch");
}

int mgemm_packed_b_destroy(mgemm_packed_b* Bp) {
    {
        std::lock_guard<std::mutex> lk(g_packed_mu);
        if (!Bp || !g_packed.erase(Bp))
            return fail(MGEMM_ERR_BAD_PLAN, "packed B is NULL or already destroyed");
    }
    hipError_t e = hipSuccess;
    if (Bp->hi) e = hipFree(Bp->hi);   // waits for work still reading it
    delete Bp;
    return e == hipSuccess ? MGEMM_OK : hip_fail(e, "hipFree");
}

const char* mgemm_status_string(int status) {
    if (status < 0) {
        switch (-status) {
            case 1: return "illegal argument 1 (transA)";
            case 2: return "illegal argument 2 (transB)";
            case 3: return "illegal argument 3 (M)";
            case 4: return "illegal argument 4 (N)";
            case 5: return "illegal argument 5 (K)";
            case 7: return "illegal argument 7 (A)";
            case 8: return "illegal argument 8 (lda)";
            case 9: return "illegal argument 9 (B)";
            case 10: return "illegal argument 10 (ldb)";
            case 12: return "illegal argument 12 (C)";
            case 13: return "illegal argument 13 (ldc)";
            default: return "illegal argument";
        }
    }
    switch (status) {
        case MGEMM_OK: return "success";
        case MGEMM_ERR_HIP: return "HIP runtime error";
        case MGEMM_ERR_NO_DEVICE: return "no HIP device";
        case MGEMM_ERR_ARCH: return "device is not gfx950";
        case MGEMM_ERR_ALLOC: return "device memory allocation failed";
        case MGEMM_ERR_ALIAS: return "C overlaps A or B";
        case MGEMM_ERR_UNSUPPORTED: return "unsupported precision or configuration";
        case MGEMM_ERR_BAD_PLAN: return "invalid plan";
        case MGEMM_ERR_BAD_PROBLEM: return "invalid problem in a grouped batch";
        default: return "unknown status";
    }
}

const char* mgemm_last_error(void) { return g_last_error.c_str(); }

int mgemm_version(void) { return 100; }

}  // extern "C"
