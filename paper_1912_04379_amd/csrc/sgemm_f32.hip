// sgemm_f32.hip -- FP32 GEMM on gfx950 FP32 MFMA (v_mfma_f32_32x32x2_f32):
// kernel entry, tile configurations and launchers.  The tile engine itself
// (LDS staging, MFMA main loop, epilogue) is in tile_f32.hpp.
#include "kernels.hpp"
#include "tile_f32.hpp"

namespace mgemm {

template <class Cfg, bool AK, bool BKC, bool BUF>
__global__ __launch_bounds__(Cfg::NT, Cfg::WPE) void sgemm_f32_kernel(GemmDesc d, uint32_t tiles_m,
                                                           uint32_t tiles_n) {
    __shared__ __attribute__((aligned(16))) float smem[Cfg::SMEM_FLOATS];
    uint32_t tm, tn;
    grouped_tile<8>(xcd_remap(blockIdx.x, gridDim.x), tiles_m, tiles_n, tm, tn);
    tile_f32<Cfg, AK, BKC, BUF>(d, (int64_t)tm * Cfg::BM, (int64_t)tn * Cfg::BN, smem);
}

template <class Cfg, bool BUF>
static hipError_t launch_cfg(bool ta, bool tb, const GemmDesc& d, hipStream_t s) {
    const int64_t tiles_m = (d.M + Cfg::BM - 1) / Cfg::BM;
    const int64_t tiles_n = (d.N + Cfg::BN - 1) / Cfg::BN;
    const int64_t tiles = tiles_m * tiles_n;
    if (tiles_m > 0xffffffffLL || tiles_n > 0xffffffffLL || tiles > 0xffffffffLL)
        return hipErrorInvalidValue;
    const dim3 grid((uint32_t)tiles), block(Cfg::NT);
    const uint32_t tm = (uint32_t)tiles_m, tn = (uint32_t)tiles_n;
    // op(A) is K-contiguous for A 'T'; op(B) is K-contiguous for B 'N'.
    if (!ta && !tb)
        hipLaunchKernelGGL((sgemm_f32_kernel<Cfg, false, true, BUF>), grid, block,
                           Cfg::PAD_BYTES, s, d, tm, tn);
    else if (!ta && tb)
        hipLaunchKernelGGL((sgemm_f32_kernel<Cfg, false, false, BUF>), grid, block,
                           Cfg::PAD_BYTES, s, d, tm, tn);
    else if (ta && !tb)
        hipLaunchKernelGGL((sgemm_f32_kernel<Cfg, true, true, BUF>), grid, block,
                           Cfg::PAD_BYTES, s, d, tm, tn);
    else
        hipLaunchKernelGGL((sgemm_f32_kernel<Cfg, true, false, BUF>), grid, block,
                           Cfg::PAD_BYTES, s, d, tm, tn);
    return hipGetLastError();
}

using F32Cfg0 = CfgF32<128, 128, 16, 2, 2>;  // 4 waves of 64x64
using F32Cfg1 = CfgF32<64, 64, 16, 2, 2>;    // 4 waves of 32x32 (small problems)
using F32Cfg2 = CfgF32<128, 128, 32, 2, 2>;  // deeper slab
using F32Cfg3 = CfgF32<256, 128, 16, 2, 2>;  // 4 waves of 128x64
using F32Cfg4 = CfgF32<128, 128, 16, 2, 2, 2, 2>;  // as 0, at most 2 work-groups per CU
using F32Cfg5 = CfgF32<256, 128, 16, 2, 2, 2>;  // as 3, held to 2 waves per SIMD
using F32Cfg6 = CfgF32<128, 256, 16, 2, 2, 2>;  // 4 waves of 64x128, 2 waves per SIMD
using F32Cfg7 = CfgF32<128, 128, 32, 2, 2, 2, 2>;  // as 2, at most 2 work-groups per CU
// 8 waves of 128x64 at 2 waves per SIMD, one work-group per CU (144 KB of
// LDS): a third fewer global loads per flop than 256x128.
using F32Cfg8 = CfgF32<256, 256, 32, 2, 4, 2>;

template <class Cfg>
static TileConfigInfo info_of() { return {Cfg::BM, Cfg::BN, Cfg::BK, Cfg::NT}; }

// ---------------------------------------------------------------------------
// Configuration 10: 256 x 256 x 32 tiles in whole rounds, 128 x 128 tiles in
// the tail.  With one 256 x 256 work-group per CU, T tiles take
// ceil(T / CUs) rounds, and a last round of r < CUs tiles leaves the other
// CUs idle for a whole tile's time.  Here the whole rounds run as usual and
// the r tail tiles are computed as 128 x 128 quarters (configuration 0's
// tile, several work-groups per CU), about a quarter of a round's time when
// r is at most a third of the CUs and no more than half of it up to r ~
// 0.6 CUs.  Ordinary tiles throughout: no workspace, no atomics.
// ---------------------------------------------------------------------------
using BigCfg = F32Cfg8;
using TailCfg = F32Cfg0;

template <class Cfg, bool AK, bool BKC>
__global__ __launch_bounds__(Cfg::NT, Cfg::WPE) void sgemm_f32_tail_kernel(GemmDesc d,
                                                                         uint32_t tiles_m,
                                                                         uint32_t tiles_n,
                                                                         uint32_t first_tile) {
    constexpr int R = BigCfg::BM / Cfg::BM;
    static_assert(R * Cfg::BM == BigCfg::BM && R * Cfg::BN == BigCfg::BN, "quarters");
    __shared__ __attribute__((aligned(16))) float smem[Cfg::SMEM_FLOATS];
    const uint32_t w = xcd_remap(blockIdx.x, gridDim.x);
    const uint32_t t = w / (R * R), q = w % (R * R);
    uint32_t tm, tn;
    grouped_tile<8>(first_tile + t, tiles_m, tiles_n, tm, tn);
    const int64_t m0 = (int64_t)tm * BigCfg::BM + (int64_t)(q % R) * Cfg::BM;
    const int64_t n0 = (int64_t)tn * BigCfg::BN + (int64_t)(q / R) * Cfg::BN;
    if (m0 >= d.M || n0 >= d.N) return;   // a quarter past the edge of C
    tile_f32<Cfg, AK, BKC, true>(d, m0, n0, smem);
}

hipError_t launch_f32_tail(bool ta, bool tb, const GemmDesc& d, int cus, hipStream_t s) {
    if (!buffer_path_ok(d) || cus < 1) return hipErrorInvalidValue;
    const int64_t tiles_m = (d.M + BigCfg::BM - 1) / BigCfg::BM;
    const int64_t tiles_n = (d.N + BigCfg::BN - 1) / BigCfg::BN;
    const int64_t tiles = tiles_m * tiles_n;
    constexpr int64_t R2 = (BigCfg::BM / TailCfg::BM) * (BigCfg::BN / TailCfg::BN);
    if (tiles * R2 > 0xffffffffLL) return hipErrorInvalidValue;
    const int64_t tail = tiles % cus, whole = tiles - tail;
    const uint32_t tm = (uint32_t)tiles_m, tn = (uint32_t)tiles_n;
    // Whole rounds: the ordinary kernel over the first `whole` tiles of the
    // rasterised order (its grid size bounds the tile ids it takes).
    if (whole > 0) {
        using Cfg = BigCfg;
        const dim3 grid((uint32_t)whole), block(Cfg::NT);
        if (!ta && !tb)
            hipLaunchKernelGGL((sgemm_f32_kernel<Cfg, false, true, true>), grid, block, 0, s, d, tm, tn);
        else if (!ta && tb)
            hipLaunchKernelGGL((sgemm_f32_kernel<Cfg, false, false, true>), grid, block, 0, s, d, tm, tn);
        else if (ta && !tb)
            hipLaunchKernelGGL((sgemm_f32_kernel<Cfg, true, true, true>), grid, block, 0, s, d, tm, tn);
        else
            hipLaunchKernelGGL((sgemm_f32_kernel<Cfg, true, false, true>), grid, block, 0, s, d, tm, tn);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (tail == 0) return hipSuccess;
    using Cfg = TailCfg;
    const dim3 grid((uint32_t)(tail * R2)), block(Cfg::NT);
    const uint32_t first = (uint32_t)whole;
    if (!ta && !tb)
        hipLaunchKernelGGL((sgemm_f32_tail_kernel<Cfg, false, true>), grid, block, Cfg::PAD_BYTES, s, d, tm, tn, first);
    else if (!ta && tb)
        hipLaunchKernelGGL((sgemm_f32_tail_kernel<Cfg, false, false>), grid, block, Cfg::PAD_BYTES, s, d, tm, tn, first);
    else if (ta && !tb)
        hipLaunchKernelGGL((sgemm_f32_tail_kernel<Cfg, true, true>), grid, block, Cfg::PAD_BYTES, s, d, tm, tn, first);
    else
        hipLaunchKernelGGL((sgemm_f32_tail_kernel<Cfg, true, false>), grid, block, Cfg::PAD_BYTES, s, d, tm, tn, first);
    return hipGetLastError();
}

// Configuration 9 is the small-product kernel (sgemm_small.hip);
// configuration 10 the 256 x 256 x 32 tile with a 128 x 128 tail (above).
constexpr int F32_SMALL_CONFIG = 9;

int f32_config_count() { return 11; }

TileConfigInfo f32_config_info(int cfg) {
    switch (cfg) {
        case 0: return info_of<F32Cfg0>();
        case 1: return info_of<F32Cfg1>();
        case 2: return info_of<F32Cfg2>();
        case 3: return info_of<F32Cfg3>();
        case 4: return info_of<F32Cfg4>();
        case 5: return info_of<F32Cfg5>();
        case 6: return info_of<F32Cfg6>();
        case 7: return info_of<F32Cfg7>();
        case 8: return info_of<F32Cfg8>();
        case F32_SMALL_CONFIG: return {16, 16, 16, 256};
        case F32_TAIL_CONFIG: return info_of<BigCfg>();
        default: return {0, 0, 0, 0};
    }
}

hipError_t launch_f32(int cfg, bool ta, bool tb, const GemmDesc& d, hipStream_t s) {
    if (cfg < 0 || cfg >= f32_config_count()) return hipErrorInvalidValue;
    // A leading dimension beyond 32-bit buffer offsets takes the 64-bit
    // address path, built for the 64x64 and 128x128 tiles only (larger
    // tiles would spill registers there).
    if (!buffer_path_ok(d))
        return cfg == 1 || cfg == F32_SMALL_CONFIG ? launch_cfg<F32Cfg1, false>(ta, tb, d, s)
                                                   : launch_cfg<F32Cfg0, false>(ta, tb, d, s);
    switch (cfg) {
        case 0: return launch_cfg<F32Cfg0, true>(ta, tb, d, s);
        case 1: return launch_cfg<F32Cfg1, true>(ta, tb, d, s);
        case 2: return launch_cfg<F32Cfg2, true>(ta, tb, d, s);
        case 3: return launch_cfg<F32Cfg3, true>(ta, tb, d, s);
        case 4: return launch_cfg<F32Cfg4, true>(ta, tb, d, s);
        case 5: return launch_cfg<F32Cfg5, true>(ta, tb, d, s);
        case 6: return launch_cfg<F32Cfg6, true>(ta, tb, d, s);
        case 7: return launch_cfg<F32Cfg7, true>(ta, tb, d, s);
        case 8: return launch_cfg<F32Cfg8, true>(ta, tb, d, s);
        case F32_SMALL_CONFIG: return launch_small(ta, tb, d, s);
        default: return hipErrorInvalidValue;   // configuration 10: launch_f32_tail
    }
}

// ---------------------------------------------------------------------------
// C <- beta C, for alpha == 0 or K == 0.  beta == 0 writes zeros and never
// reads C.  Grid-stride over rows (x) and columns (y) of C.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void scale_c_kernel(float* C, int64_t M, int64_t N,
                                                      int64_t ldc, float beta) {
    for (int64_t n = blockIdx.y; n < N; n += gridDim.y)
        for (int64_t m = (int64_t)blockIdx.x * 256 + threadIdx.x; m < M;
             m += (int64_t)gridDim.x * 256) {
            float* c = C + m + n * ldc;
            *c = beta == 0.0f ? 0.0f : beta * *c;
        }
}

hipError_t launch_scale_c(const GemmDesc& d, hipStream_t s) {
    const int64_t gx = (d.M + 255) / 256 < 64 ? (d.M + 255) / 256 : 64;
    const int64_t gy = d.N < 4096 ? d.N : 4096;
    hipLaunchKernelGGL(scale_c_kernel, dim3((uint32_t)gx, (uint32_t)gy), dim3(256), 0, s,
                       d.C, d.M, d.N, d.ldc, d.beta);
    return hipGetLastError();
}

}  // namespace mgemm
