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
    tile_f32<Cfg, AK, BKC, BUF>(d, (int64_t)tm * Cfg::BM, (int64_t)tn * Cfg::BN, smem, threadIdx.x);
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
// 4 waves of 32x32 with 32-deep slabs (configuration 12): twice the MFMAs
// per slab of configuration 1, so that with few work-groups per CU each
// slab's MFMAs cover more of the next slab's load latency; 3-11% faster
// than configuration 1 from 512^3 to 8192^3.
using F32Cfg12 = CfgF32<64, 64, 32, 2, 2>;

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
    tile_f32<Cfg, AK, BKC, true>(d, m0, n0, smem, threadIdx.x);
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

// ---------------------------------------------------------------------------
// Configuration 11: split-K.  A product with few tiles and a long k range
// leaves most CUs idle and runs each tile's K/2 MFMAs as one serial chain.
// Cutting k into S pieces gives S times the work-groups and chains S times
// shorter; each piece is an ordinary tile (alpha 1, beta 0) into its own
// slice of a workspace, and a second kernel adds the slices in a fixed
// order and applies the epilogue, so results do not depend on timing.
// ---------------------------------------------------------------------------
template <class Cfg, bool AK, bool BKC>
__global__ __launch_bounds__(Cfg::NT, Cfg::WPE) void sgemm_f32_splitk_kernel(
    GemmDesc d, uint32_t tiles_m, uint32_t tiles_n, int64_t kc, float* ws) {
    __shared__ __attribute__((aligned(16))) float smem[Cfg::SMEM_FLOATS];
    // Logical id -> (piece, tile): the work-groups of one XCD take
    // consecutive tiles of one piece, which share panels of A and B.
    const uint32_t id = xcd_remap(blockIdx.x, gridDim.x);
    const uint32_t tiles = tiles_m * tiles_n;
    const uint32_t s = id / tiles;
    uint32_t tm, tn;
    grouped_tile<8>(id - s * tiles, tiles_m, tiles_n, tm, tn);
    const int64_t k0 = (int64_t)s * kc;
    GemmDesc p = d;
    // op(A)'s k runs along columns of A 'N' and rows of A 'T'; op(B)'s along
    // rows of B 'N' and columns of B 'T'.
    p.A = d.A + (AK ? k0 : k0 * d.lda);
    p.B = d.B + (BKC ? k0 : k0 * d.ldb);
    p.K = d.K - k0 < kc ? d.K - k0 : kc;
    p.C = ws + (int64_t)s * d.M * d.N;
    p.ldc = d.M;
    p.alpha = 1.0f;
    p.beta = 0.0f;
    p.act = ACT_NONE;   // applied once, by the reduction
    tile_f32<Cfg, AK, BKC, true>(p, (int64_t)tm * Cfg::BM, (int64_t)tn * Cfg::BN, smem, threadIdx.x);
}

// C <- act(alpha * sum_s ws[s] + beta * C), s in increasing order; beta ==
// 0 never reads C.  Grid-stride over the M*N outputs, m fastest.
__global__ __launch_bounds__(256) void splitk_reduce_kernel(const float* __restrict__ ws,
                                                            int splits, int64_t M, int64_t N,
                                                            float* C, int64_t ldc, float alpha,
                                                            float beta, int act,
                                                            const float* __restrict__ aux) {
    const int64_t mn = M * N;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < mn;
         i += (int64_t)gridDim.x * 256) {
        float sum = ws[i];
        for (int s = 1; s < splits; ++s) sum += ws[(int64_t)s * mn + i];
        const int64_t n = i / M, m = i - n * M;
        float* c = C + m + n * ldc;
        const float v = beta == 0.0f ? alpha * sum : fmaf(beta, *c, alpha * sum);
        *c = activate(act, v, act == ACT_TANH_GRAD ? aux[m + n * ldc] : 0.0f);
    }
}

template <class Cfg>
static void launch_splitk_pieces(bool ta, bool tb, const GemmDesc& d, const SplitKPlan& p,
                                 float* ws, hipStream_t s) {
    const uint32_t tm = (uint32_t)((d.M + Cfg::BM - 1) / Cfg::BM);
    const uint32_t tn = (uint32_t)((d.N + Cfg::BN - 1) / Cfg::BN);
    const dim3 grid(tm * tn * (uint32_t)p.splits), block(Cfg::NT);
    if (!ta && !tb)
        hipLaunchKernelGGL((sgemm_f32_splitk_kernel<Cfg, false, true>), grid, block,
                           Cfg::PAD_BYTES, s, d, tm, tn, p.kc, ws);
    else if (!ta && tb)
        hipLaunchKernelGGL((sgemm_f32_splitk_kernel<Cfg, false, false>), grid, block,
                           Cfg::PAD_BYTES, s, d, tm, tn, p.kc, ws);
    else if (ta && !tb)
        hipLaunchKernelGGL((sgemm_f32_splitk_kernel<Cfg, true, true>), grid, block,
                           Cfg::PAD_BYTES, s, d, tm, tn, p.kc, ws);
    else
        hipLaunchKernelGGL((sgemm_f32_splitk_kernel<Cfg, true, false>), grid, block,
                           Cfg::PAD_BYTES, s, d, tm, tn, p.kc, ws);
}

hipError_t launch_f32_splitk(bool ta, bool tb, const GemmDesc& d, const SplitKPlan& p,
                             float* ws, hipStream_t s) {
    // The workspace slices are the C of ordinary tiles: ld M within the
    // buffer path's limit.
    if (!buffer_path_ok(d) || p.splits < 2 || p.kc < 32 || d.M > MAX_BUF_LD || !ws)
        return hipErrorInvalidValue;
    if ((int64_t)(p.splits - 1) * p.kc >= d.K) return hipErrorInvalidValue;   // empty piece
    // Few tiles: 64 x 64 with 32-deep slabs (4-8% faster pieces than 16-deep
    // at 256^2 x 65536, 512^2 x 16384 and 768^2 x 6144; the 128 x 128 pieces
    // lose 1% with 32-deep slabs and keep 16).
    if (p.small_tile)
        launch_splitk_pieces<F32Cfg12>(ta, tb, d, p, ws, s);
    else
        launch_splitk_pieces<F32Cfg0>(ta, tb, d, p, ws, s);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_splitk_reduce(ws, p.splits, d, s);
}

hipError_t launch_splitk_reduce(const float* ws, int splits, const GemmDesc& d, hipStream_t s) {
    const int64_t mn = d.M * d.N;
    int64_t blocks = (mn + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(splitk_reduce_kernel, dim3((uint32_t)blocks), dim3(256), 0, s, ws,
                       splits, d.M, d.N, d.C, d.ldc, d.alpha, d.beta, d.act, d.aux);
    return hipGetLastError();
}

// Configuration 9 is the small-product kernel (sgemm_small.hip);
// configuration 10 the 256 x 256 x 32 tile with a 128 x 128 tail (above);
// configuration 11 split-K (above); configuration 12 the 64 x 64 x 32 tile.
constexpr int F32_SMALL_CONFIG = 9;

int f32_config_count() { return 13; }

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
        case F32_SPLITK_CONFIG: return info_of<F32Cfg0>();   // 64 x 64 for few tiles
        case F32_DEEP64_CONFIG: return info_of<F32Cfg12>();
        default: return {0, 0, 0, 0};
    }
}

hipError_t launch_f32(int cfg, bool ta, bool tb, const GemmDesc& d, hipStream_t s) {
    if (cfg < 0 || cfg >= f32_config_count()) return hipErrorInvalidValue;
    // A leading dimension beyond 32-bit buffer offsets takes the 64-bit
    // address path, built for the 64x64 and 128x128 tiles only (larger
    // tiles would spill registers there).
    if (!buffer_path_ok(d))
        return cfg == 1 || cfg == F32_SMALL_CONFIG || cfg == F32_DEEP64_CONFIG
                   ? launch_cfg<F32Cfg1, false>(ta, tb, d, s)
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
        case F32_DEEP64_CONFIG: return launch_cfg<F32Cfg12, true>(ta, tb, d, s);
        default: return hipErrorInvalidValue;   // 10: launch_f32_tail, 11: launch_f32_splitk
    }
}

// ---------------------------------------------------------------------------
// C <- beta C, for alpha == 0 or K == 0.  beta == 0 writes zeros and never
// reads C.  Grid-stride over rows (x) and columns (y) of C.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void scale_c_kernel(float* C, int64_t M, int64_t N,
                                                      int64_t ldc, float beta, int act,
                                                      const float* __restrict__ aux) {
    for (int64_t n = blockIdx.y; n < N; n += gridDim.y)
        for (int64_t m = (int64_t)blockIdx.x * 256 + threadIdx.x; m < M;
             m += (int64_t)gridDim.x * 256) {
            float* c = C + m + n * ldc;
            const float v = beta == 0.0f ? 0.0f : beta * *c;
            *c = activate(act, v, act == ACT_TANH_GRAD ? aux[m + n * ldc] : 0.0f);
        }
}

hipError_t launch_scale_c(const GemmDesc& d, hipStream_t s) {
    const int64_t gx = (d.M + 255) / 256 < 64 ? (d.M + 255) / 256 : 64;
    const int64_t gy = d.N < 4096 ? d.N : 4096;
    hipLaunchKernelGGL(scale_c_kernel, dim3((uint32_t)gx, (uint32_t)gy), dim3(256), 0, s,
                       d.C, d.M, d.N, d.ldc, d.beta, d.act, d.aux);
    return hipGetLastError();
}

}  // namespace mgemm
