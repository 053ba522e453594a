// sgemm_lowp.hip -- the BF16x3 and scaled-FP16 forms on gfx950 16-bit MFMA:
// kernel entry, tile configurations, launchers and the FP16 exponent
// pre-pass.  The tile engine is in tile_lowp.hpp.
#include "kernels.hpp"
#include "tile_lowp.hpp"

namespace mgemm {

template <class Cfg, Form F, bool AK, bool BKC, bool BUF>
__global__ __launch_bounds__(Cfg::NT) void sgemm_lowp_kernel(GemmDesc d, uint32_t tiles_m,
                                                            uint32_t tiles_n) {
    extern __shared__ __attribute__((aligned(16))) char lowp_smem[];
    uint32_t tm, tn;
    grouped_tile<8>(xcd_remap(blockIdx.x, gridDim.x), tiles_m, tiles_n, tm, tn);
    tile_lowp<Cfg, F, AK, BKC, BUF>(d, (int64_t)tm * Cfg::BM, (int64_t)tn * Cfg::BN, lowp_smem, threadIdx.x);
}

template <class Cfg, Form F>
constexpr int lowp_smem_bytes() {
    return 2 * (F == Form::BF16X3 ? 2 : 1) * (Cfg::BM + Cfg::BN) * Cfg::ROW_BYTES;
}

template <class Cfg, Form F, bool AK, bool BKC, bool BUF>
static hipError_t launch_kernel(dim3 grid, const GemmDesc& d, uint32_t tm, uint32_t tn,
                                hipStream_t s) {
    constexpr int bytes = lowp_smem_bytes<Cfg, F>();
    auto k = sgemm_lowp_kernel<Cfg, F, AK, BKC, BUF>;
    if (bytes > 65536) {
        hipError_t e = hipFuncSetAttribute((const void*)k,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k, grid, dim3(Cfg::NT), bytes, s, d, tm, tn);
    return hipGetLastError();
}

template <class Cfg, Form F, bool BUF>
static hipError_t launch_cfg(bool ta, bool tb, const GemmDesc& d, hipStream_t s) {
    const int64_t tiles_m = (d.M + Cfg::BM - 1) / Cfg::BM;
    const int64_t tiles_n = (d.N + Cfg::BN - 1) / Cfg::BN;
    if (tiles_m * tiles_n > 0xffffffffLL) return hipErrorInvalidValue;
    dim3 grid((uint32_t)(tiles_m * tiles_n));
    const uint32_t tm = (uint32_t)tiles_m, tn = (uint32_t)tiles_n;
    if (!ta && !tb) return launch_kernel<Cfg, F, false, true, BUF>(grid, d, tm, tn, s);
    if (!ta && tb) return launch_kernel<Cfg, F, false, false, BUF>(grid, d, tm, tn, s);
    if (ta && !tb) return launch_kernel<Cfg, F, true, true, BUF>(grid, d, tm, tn, s);
    return launch_kernel<Cfg, F, true, false, BUF>(grid, d, tm, tn, s);
}

using LPCfg0 = CfgLP<256, 256, 2, 4>;  // 8 waves of 128x64
using LPCfg1 = CfgLP<128, 128, 2, 2>;  // 4 waves of 64x64
using LPCfg2 = CfgLP<256, 128, 2, 2>;  // 4 waves of 128x64
using LPCfg3 = CfgLP<64, 64, 2, 2>;    // 4 waves of 32x32 (small problems)

template <class Cfg>
static TileConfigInfo lp_info() { return {Cfg::BM, Cfg::BN, Cfg::BK, Cfg::NT}; }

static TileConfigInfo lowp_info(int cfg) {
    switch (cfg) {
        case 0: return lp_info<LPCfg0>();
        case 1: return lp_info<LPCfg1>();
        case 2: return lp_info<LPCfg2>();
        case 3: return lp_info<LPCfg3>();
        default: return {0, 0, 0, 0};
    }
}

template <Form F>
static hipError_t lowp_launch(int cfg, bool ta, bool tb, const GemmDesc& d, hipStream_t s) {
    if (cfg < 0 || cfg >= LOWP_INSTAGE_CONFIGS) return hipErrorInvalidValue;
    // A leading dimension beyond 32-bit buffer offsets takes the 64-bit
    // address path, built for the 64x64 and 128x128 tiles only (larger
    // tiles would spill registers there).
    if (!buffer_path_ok(d))
        return cfg == 3 ? launch_cfg<LPCfg3, F, false>(ta, tb, d, s)
                        : launch_cfg<LPCfg1, F, false>(ta, tb, d, s);
    switch (cfg) {
        case 0: return launch_cfg<LPCfg0, F, true>(ta, tb, d, s);
        case 1: return launch_cfg<LPCfg1, F, true>(ta, tb, d, s);
        case 2: return launch_cfg<LPCfg2, F, true>(ta, tb, d, s);
        default: return launch_cfg<LPCfg3, F, true>(ta, tb, d, s);
    }
}

// ---------------------------------------------------------------------------
// Split-K.  Piece s of every tile is an ordinary in-staging tile over k in
// [s kc, min((s+1) kc, K)) with alpha 1 and beta 0, written to slice s of the
// workspace (column-major, ld M); the FP16 unscale by the whole-K panel
// exponents is applied per piece, which is exact (a power of two).  The
// reduction kernel then adds the slices in order and applies alpha, beta.
// ---------------------------------------------------------------------------
template <class Cfg, Form F, bool AK, bool BKC>
__global__ __launch_bounds__(Cfg::NT) void sgemm_lowp_splitk_kernel(GemmDesc d, uint32_t tiles_m,
                                                                   uint32_t tiles_n, int64_t kc,
                                                                   float* ws) {
    extern __shared__ __attribute__((aligned(16))) char lowp_smem[];
    // Logical id -> (piece, tile): one XCD takes consecutive tiles of one
    // piece, which share panels of A and B.
    const uint32_t id = xcd_remap(blockIdx.x, gridDim.x);
    const uint32_t tiles = tiles_m * tiles_n;
    const uint32_t s = id / tiles;
    uint32_t tm, tn;
    grouped_tile<8>(id - s * tiles, tiles_m, tiles_n, tm, tn);
    const int64_t k0 = (int64_t)s * kc;
    GemmDesc p = d;
    p.A = d.A + (AK ? k0 : k0 * d.lda);
    p.B = d.B + (BKC ? k0 : k0 * d.ldb);
    p.K = d.K - k0 < kc ? d.K - k0 : kc;
    p.C = ws + (int64_t)s * d.M * d.N;
    p.ldc = d.M;
    p.alpha = 1.0f;
    p.beta = 0.0f;
    p.act = ACT_NONE;   // applied once, by the reduction
    tile_lowp<Cfg, F, AK, BKC, true>(p, (int64_t)tm * Cfg::BM, (int64_t)tn * Cfg::BN, lowp_smem, threadIdx.x);
}

template <class Cfg, Form F>
static hipError_t launch_splitk_pieces(bool ta, bool tb, const GemmDesc& d, const SplitKPlan& p,
                                       float* ws, hipStream_t s) {
    const uint32_t tm = (uint32_t)((d.M + Cfg::BM - 1) / Cfg::BM);
    const uint32_t tn = (uint32_t)((d.N + Cfg::BN - 1) / Cfg::BN);
    const dim3 grid(tm * tn * (uint32_t)p.splits), block(Cfg::NT);
    constexpr int bytes = lowp_smem_bytes<Cfg, F>();
    static_assert(bytes <= 65536, "split-K tiles use at most 64 KB of LDS");
    if (!ta && !tb)
        hipLaunchKernelGGL((sgemm_lowp_splitk_kernel<Cfg, F, false, true>), grid, block, bytes, s,
                           d, tm, tn, p.kc, ws);
    else if (!ta && tb)
        hipLaunchKernelGGL((sgemm_lowp_splitk_kernel<Cfg, F, false, false>), grid, block, bytes,
                           s, d, tm, tn, p.kc, ws);
    else if (ta && !tb)
        hipLaunchKernelGGL((sgemm_lowp_splitk_kernel<Cfg, F, true, true>), grid, block, bytes, s,
                           d, tm, tn, p.kc, ws);
    else
        hipLaunchKernelGGL((sgemm_lowp_splitk_kernel<Cfg, F, true, false>), grid, block, bytes, s,
                           d, tm, tn, p.kc, ws);
    return hipGetLastError();
}

hipError_t launch_lowp_splitk(bool bf16x3, bool ta, bool tb, const GemmDesc& d,
                              const SplitKPlan& p, float* ws, hipStream_t s) {
    if (!buffer_path_ok(d) || p.splits < 2 || p.kc < 32 || p.kc % 32 || d.M > MAX_BUF_LD || !ws)
        return hipErrorInvalidValue;
    if ((int64_t)(p.splits - 1) * p.kc >= d.K) return hipErrorInvalidValue;   // empty piece
    if (!bf16x3 && (!d.expA || !d.expB)) return hipErrorInvalidValue;
    hipError_t e;
    if (bf16x3)
        e = p.small_tile ? launch_splitk_pieces<LPCfg3, Form::BF16X3>(ta, tb, d, p, ws, s)
                         : launch_splitk_pieces<LPCfg1, Form::BF16X3>(ta, tb, d, p, ws, s);
    else
        e = p.small_tile ? launch_splitk_pieces<LPCfg3, Form::F16S>(ta, tb, d, p, ws, s)
                         : launch_splitk_pieces<LPCfg1, Form::F16S>(ta, tb, d, p, ws, s);
    if (e != hipSuccess) return e;
    return launch_splitk_reduce(ws, p.splits, d, s);
}

static TileConfigInfo lowp_any_info(int cfg) {
    if (cfg == LOWP_SPLITK_CONFIG) return lowp_info(1);   // 128 x 128 pieces (64 x 64 for few tiles)
    return cfg < LOWP_INSTAGE_CONFIGS ? lowp_info(cfg)
                                      : packed_config_info(cfg - LOWP_INSTAGE_CONFIGS);
}

int bf16x3_config_count() { return LOWP_INSTAGE_CONFIGS + packed_config_count() + 1; }
TileConfigInfo bf16x3_config_info(int cfg) { return lowp_any_info(cfg); }
hipError_t launch_bf16x3(int cfg, bool ta, bool tb, const GemmDesc& d, hipStream_t s) {
    return lowp_launch<Form::BF16X3>(cfg, ta, tb, d, s);
}

int f16s_config_count() { return LOWP_INSTAGE_CONFIGS + packed_config_count() + 1; }
TileConfigInfo f16s_config_info(int cfg) { return lowp_any_info(cfg); }
hipError_t launch_f16s(int cfg, bool ta, bool tb, const GemmDesc& d, hipStream_t s) {
    return lowp_launch<Form::F16S>(cfg, ta, tb, d, s);
}

// ---------------------------------------------------------------------------
// FP16 pre-pass.  The exponent of a 32-wide panel is e = 15 - p where
// amax = f 2^p, f in [0.5, 1), is the panel's largest magnitude (so amax 2^e
// lies in [2^14, 2^15)); e = 0 when amax is 0 or not finite or the panel
// holds a NaN.  Panels of op(A) are 32 rows, panels of op(B) 32 columns,
// both over the whole K.
//
// Pass 1: one work-group per (panel, 2048-deep range of k) writes the range's
// amax (NaN if the range holds a NaN) to `partial`.  P-contiguous panels:
// thread t reads row t % 32 of columns t / 32, t / 32 + 8, ... (each wave
// instruction reads two 128-byte columns; 8 loads in flight per thread).
// K-contiguous panels: 16-byte loads along each row, 4 rows at a time.
// Pass 2: one thread per panel reduces its ranges and writes e.
// ---------------------------------------------------------------------------
constexpr int64_t EXP_KRANGE = 2048;

int64_t f16_partial_floats(int64_t M, int64_t N, int64_t K) {
    const int64_t nkr = K > 0 ? (K + EXP_KRANGE - 1) / EXP_KRANGE : 1;
    return ((M + 31) / 32 + (N + 31) / 32) * nkr;
}

__global__ __launch_bounds__(256) void f16_amax_kernel(GemmDesc d, int ta, int tb,
                                                       int64_t panels_a, int64_t nkr,
                                                       float* __restrict__ partial) {
    __shared__ float red_max[4];
    __shared__ int red_nan[4];
    const int64_t pid = blockIdx.x / nkr, kr = blockIdx.x % nkr;
    const bool is_a = pid < panels_a;
    const int64_t panel = is_a ? pid : pid - panels_a;
    const float* X = is_a ? d.A : d.B;
    const int64_t ld = is_a ? d.lda : d.ldb;
    const int64_t P = is_a ? d.M : d.N;
    // op(A) rows are contiguous for A 'N'; op(B) columns are contiguous for B 'T'.
    const bool pcontig = is_a ? !ta : tb;
    const int64_t p0 = panel * 32, rows = P - p0 < 32 ? P - p0 : 32;
    const int64_t k0 = kr * EXP_KRANGE, k1 = k0 + EXP_KRANGE < d.K ? k0 + EXP_KRANGE : d.K;
    const int t = threadIdx.x;
    float amax = 0.0f;
    int nan = 0;
    auto take = [&](float x) {
        nan |= x != x;
        amax = fmaxf(amax, fabsf(x));
    };
    if (pcontig && rows == 32 && (ld & 3) == 0 && ((uintptr_t)X & 15) == 0) {
        // A whole panel with 16-byte aligned columns: 8 lanes read one
        // column's 32 rows as 16-byte loads, the 32 lane groups take every
        // 32nd k, 8 loads in flight per lane.
        const float* col = X + p0 + 4 * (t & 7);
        int64_t k = k0 + (t >> 3);
        for (; k + 224 < k1; k += 256) {
            f32x4 x[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) x[u] = *reinterpret_cast<const f32x4*>(col + (k + 32 * u) * ld);
#pragma unroll
            for (int u = 0; u < 8; ++u)
#pragma unroll
                for (int e = 0; e < 4; ++e) take(x[u][e]);
        }
        for (; k < k1; k += 32) {
            const f32x4 x = *reinterpret_cast<const f32x4*>(col + k * ld);
#pragma unroll
            for (int e = 0; e < 4; ++e) take(x[e]);
        }
    } else if (pcontig) {
        // Lane r reads row r of the panel; the 8 lane groups take every
        // 8th k, 8 loads in flight per lane.
        const int r = t & 31;
        if (r < rows) {
            const float* col = X + p0 + r;
            int64_t k = k0 + (t >> 5);
            for (; k + 56 < k1; k += 64) {
                float x[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) x[u] = col[(k + 8 * u) * ld];
#pragma unroll
                for (int u = 0; u < 8; ++u) take(x[u]);
            }
            for (; k < k1; k += 8) take(col[k * ld]);
        }
    } else {
        // Each row of the panel is contiguous over [k0, k1): 16-byte buffer
        // loads from a descriptor over exactly that range (per-element at the
        // end), 4 rows at a time.
        static_assert(EXP_KRANGE <= 2 * 1024, "two sweeps of 1024 k cover a range");
        const int len = (int)(k1 - k0);
        for (int64_t r0 = 0; r0 < rows; r0 += 4) {
            f32x4 v[4][2];
#pragma unroll
            for (int q = 0; q < 4; ++q)
#pragma unroll
                for (int i = 0; i < 2; ++i) {
                    v[q][i] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
                    if (r0 + q >= rows) continue;
                    const BufRsrc rs = make_rsrc(X + (p0 + r0 + q) * ld + k0, 4 * (int64_t)len);
                    const int kk = 4 * t + 1024 * i;
                    if (kk + 3 < len) {
                        v[q][i] = buf_load_f32x4(rs, (uint32_t)(4 * kk));
                    } else {
#pragma unroll
                        for (int e = 0; e < 4; ++e)
                            v[q][i][e] = buf_load_f32(rs, kk + e < len ? (uint32_t)(4 * (kk + e))
                                                                       : BUF_OOB);
                    }
                }
#pragma unroll
            for (int q = 0; q < 4; ++q)
#pragma unroll
                for (int i = 0; i < 2; ++i)
#pragma unroll
                    for (int e = 0; e < 4; ++e) take(v[q][i][e]);
        }
    }
    for (int o = 32; o > 0; o >>= 1) {
        amax = fmaxf(amax, __shfl_xor(amax, o));
        nan |= __shfl_xor(nan, o);
    }
    if ((t & 63) == 0) {
        red_max[t >> 6] = amax;
        red_nan[t >> 6] = nan;
    }
    __syncthreads();
    if (t == 0) {
        const float m = fmaxf(fmaxf(red_max[0], red_max[1]), fmaxf(red_max[2], red_max[3]));
        const int any_nan = red_nan[0] | red_nan[1] | red_nan[2] | red_nan[3];
        partial[blockIdx.x] = any_nan ? __builtin_nanf("") : m;
    }
}

__global__ __launch_bounds__(256) void f16_exponent_kernel(int64_t panels_a, int64_t panels,
                                                           int64_t nkr,
                                                           const float* __restrict__ partial,
                                                           int* __restrict__ expA,
                                                           int* __restrict__ expB) {
    const int64_t pid = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (pid >= panels) return;
    float m = 0.0f;
    bool nan = false;
    for (int64_t kr = 0; kr < nkr; ++kr) {
        const float v = partial[pid * nkr + kr];
        nan |= v != v;
        m = fmaxf(m, v);
    }
    int e = 0;
    if (!nan && m > 0.0f && isfinite(m)) {
        int p;
        frexpf(m, &p);
        e = 15 - p;
    }
    if (pid < panels_a) expA[pid] = e;
    else expB[pid - panels_a] = e;
}

hipError_t launch_f16_exponents(bool ta, bool tb, const GemmDesc& d, int* expA, int* expB,
                                float* partial, hipStream_t s) {
    const int64_t pa = (d.M + 31) / 32, pb = (d.N + 31) / 32;
    const int64_t nkr = d.K > 0 ? (d.K + EXP_KRANGE - 1) / EXP_KRANGE : 1;
    const int64_t nwg = (pa + pb) * nkr;
    if (nwg > 0x7fffffffLL) return hipErrorInvalidValue;
    if (nwg == 0) return hipSuccess;
    hipLaunchKernelGGL(f16_amax_kernel, dim3((uint32_t)nwg), dim3(256), 0, s, d, (int)ta,
                       (int)tb, pa, nkr, partial);
    hipLaunchKernelGGL(f16_exponent_kernel, dim3((uint32_t)((pa + pb + 255) / 256)), dim3(256), 0,
                       s, pa, pa + pb, nkr, partial, expA, expB);
    return hipGetLastError();
}

}  // namespace mgemm
