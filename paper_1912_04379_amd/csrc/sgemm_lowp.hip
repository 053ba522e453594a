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
    tile_lowp<Cfg, F, AK, BKC, BUF>(d, (int64_t)tm * Cfg::BM, (int64_t)tn * Cfg::BN, lowp_smem);
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

template <class Cfg, Form F, bool AK, bool BKC>
static hipError_t launch_one(dim3 grid, const GemmDesc& d, uint32_t tm, uint32_t tn,
                             hipStream_t s) {
    return buffer_path_ok(d) ? launch_kernel<Cfg, F, AK, BKC, true>(grid, d, tm, tn, s)
                             : launch_kernel<Cfg, F, AK, BKC, false>(grid, d, tm, tn, s);
}

template <class Cfg, Form F>
static hipError_t launch_cfg(bool ta, bool tb, const GemmDesc& d, hipStream_t s) {
    const int64_t tiles_m = (d.M + Cfg::BM - 1) / Cfg::BM;
    const int64_t tiles_n = (d.N + Cfg::BN - 1) / Cfg::BN;
    if (tiles_m * tiles_n > 0xffffffffLL) return hipErrorInvalidValue;
    dim3 grid((uint32_t)(tiles_m * tiles_n));
    const uint32_t tm = (uint32_t)tiles_m, tn = (uint32_t)tiles_n;
    if (!ta && !tb) return launch_one<Cfg, F, false, true>(grid, d, tm, tn, s);
    if (!ta && tb) return launch_one<Cfg, F, false, false>(grid, d, tm, tn, s);
    if (ta && !tb) return launch_one<Cfg, F, true, true>(grid, d, tm, tn, s);
    return launch_one<Cfg, F, true, false>(grid, d, tm, tn, s);
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
    switch (cfg) {
        case 0: return launch_cfg<LPCfg0, F>(ta, tb, d, s);
        case 1: return launch_cfg<LPCfg1, F>(ta, tb, d, s);
        case 2: return launch_cfg<LPCfg2, F>(ta, tb, d, s);
        case 3: return launch_cfg<LPCfg3, F>(ta, tb, d, s);
        default: return hipErrorInvalidValue;
    }
}

// The 256x256 tile once the chip gets at least two rounds of work-groups;
// otherwise the tile that still gives every CU several work-groups
// (measured at 2048^3: 64x64 beats 128x128, which leaves one tile per CU).
static int lowp_default(int64_t M, int64_t N) {
    auto tiles = [&](int bm, int bn) { return ((M + bm - 1) / bm) * ((N + bn - 1) / bn); };
    if (tiles(256, 256) >= 512) return 0;
    if (tiles(128, 128) >= 1024) return 1;
    return 3;
}

int bf16x3_config_count() { return 4; }
TileConfigInfo bf16x3_config_info(int cfg) { return lowp_info(cfg); }
int bf16x3_default_config(int64_t M, int64_t N, int64_t K) {
    (void)K;
    return lowp_default(M, N);
}
hipError_t launch_bf16x3(int cfg, bool ta, bool tb, const GemmDesc& d, hipStream_t s) {
    return lowp_launch<Form::BF16X3>(cfg, ta, tb, d, s);
}

int f16s_config_count() { return 4; }
TileConfigInfo f16s_config_info(int cfg) { return lowp_info(cfg); }
int f16s_default_config(int64_t M, int64_t N, int64_t K) {
    (void)K;
    return lowp_default(M, N);
}
hipError_t launch_f16s(int cfg, bool ta, bool tb, const GemmDesc& d, hipStream_t s) {
    return lowp_launch<Form::F16S>(cfg, ta, tb, d, s);
}

// ---------------------------------------------------------------------------
// FP16 pre-pass: one work-group per 32-wide panel.  Work-groups
// [0, panels_a) take 32-row panels of op(A), the rest 32-column panels of
// op(B).  amax = max |x| over the panel's P x K block (NaN if any element
// is NaN); e = 15 - p where amax = f 2^p, f in [0.5, 1) (so amax 2^e is in
// [2^14, 2^15)); e = 0 for amax == 0 or non-finite amax.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void f16_exponent_kernel(GemmDesc d, int ta, int tb,
                                                           int64_t panels_a, int* expA,
                                                           int* expB) {
    __shared__ float red[4];
    __shared__ int nan_seen;
    const int64_t pid = blockIdx.x;
    const bool is_a = pid < panels_a;
    const int64_t panel = is_a ? pid : pid - panels_a;
    const float* X = is_a ? d.A : d.B;
    const int64_t ld = is_a ? d.lda : d.ldb;
    const int64_t P = is_a ? d.M : d.N;
    // op(A) rows are contiguous for A 'N'; op(B) columns are contiguous for B 'T'.
    const bool pcontig = is_a ? !ta : tb;
    const int64_t p0 = panel * 32;
    const int64_t rows = P - p0 < 32 ? P - p0 : 32;
    const int64_t total = rows * d.K;
    if (threadIdx.x == 0) nan_seen = 0;
    __syncthreads();
    float amax = 0.0f;
    bool nan = false;
    for (int64_t e = threadIdx.x; e < total; e += 256) {
        int64_t r, k;
        if (pcontig) { r = e % rows; k = e / rows; }
        else         { k = e % d.K; r = e / d.K; }
        const float x = X[pcontig ? (p0 + r) + k * ld : k + (p0 + r) * ld];
        nan |= x != x;
        amax = fmaxf(amax, fabsf(x));
    }
    for (int o = 32; o > 0; o >>= 1) amax = fmaxf(amax, __shfl_xor(amax, o));
    if (nan) nan_seen = 1;
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = amax;
    __syncthreads();
    if (threadIdx.x == 0) {
        const float m = fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
        int e = 0;
        if (!nan_seen && m > 0.0f && isfinite(m)) {
            int p;
            frexpf(m, &p);
            e = 15 - p;
        }
        (is_a ? expA : expB)[panel] = e;
    }
}

hipError_t launch_f16_exponents(bool ta, bool tb, const GemmDesc& d, int* expA, int* expB,
                                hipStream_t s) {
    const int64_t pa = (d.M + 31) / 32, pb = (d.N + 31) / 32;
    if (pa + pb > 0x7fffffffLL) return hipErrorInvalidValue;
    hipLaunchKernelGGL(f16_exponent_kernel, dim3((uint32_t)(pa + pb)), dim3(256), 0, s, d,
                       (int)ta, (int)tb, pa, expA, expB);
    return hipGetLastError();
}

}  // namespace mgemm
