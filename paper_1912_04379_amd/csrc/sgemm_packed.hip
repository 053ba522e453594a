// sgemm_packed.hip -- the BF16x3 and scaled-FP16 forms through pre-packed
// operands: pack kernels (FP32 op(X) -> zero-padded 32 x 32 blocks of 16-bit
// values, k contiguous) and the launchers of the direct-to-LDS tile engine
// in tile_packed.hpp.
#include "kernels.hpp"
#include "tile_packed.hpp"

namespace mgemm {

// ---------------------------------------------------------------------------
// Pack: one work-group (256 threads) per 32-row x 128-k group of op(X) per
// iteration; thread t owns 4 consecutive k of one row in each of the 4
// 32-k regions of the group, and issues all 16 loads before it stores.
// K-contiguous sources (A 'T', B 'N') number the threads k-fastest (8
// threads read one 128-byte row segment, 16 bytes each); P-contiguous
// sources number them p-fastest (each load reads 32 consecutive rows of one
// column).  A region lands in one 32 x 32 block (KW = 32) or two 32 x 16
// blocks (KW = 16), each row-major with k contiguous; the group's blocks
// are one contiguous range per array, which P-contiguous sources assemble
// in LDS and write in order.  Elements outside P x K are written as zeros.  BUF: raw buffer loads rebased to each
// group's first element (elements outside P x K get an out-of-range offset
// and read 0); otherwise predicated 64-bit loads (leading dimensions above
// the buffer limit).
// ---------------------------------------------------------------------------
constexpr int PACK_KG = 128;   // k per group

template <Form F, bool KC, int KW, bool BUF>
__global__ __launch_bounds__(256) void pack_kernel(const float* __restrict__ X, int64_t ld,
                                                   int64_t P, int64_t K, int64_t extent,
                                                   int64_t kb, int64_t kgroups, int64_t ngroups,
                                                   char* __restrict__ hi, char* __restrict__ lo,
                                                   const int* __restrict__ expo) {
    constexpr int RB = 2 * KW;
    constexpr int GROUP_BYTES = 32 * PACK_KG * 2;   // one array's share of a group
    __shared__ __attribute__((aligned(16))) char stage_hi[KC ? 16 : GROUP_BYTES];
    __shared__ __attribute__((aligned(16))) char stage_lo[KC || F != Form::BF16X3 ? 16 : GROUP_BYTES];
    const int t = threadIdx.x;
    const int r = KC ? t >> 3 : t & 31;
    const int kq = KC ? t & 7 : t >> 5;
    for (int64_t g = blockIdx.x; g < ngroups; g += gridDim.x) {
        const int64_t pb = g / kgroups, kg0 = (g - pb * kgroups) * PACK_KG;
        const int64_t p = pb * 32 + r;
        f32x4 v[4];
        if constexpr (BUF) {
            const int64_t first = KC ? kg0 + pb * 32 * ld : pb * 32 + kg0 * ld;
            const BufRsrc rs = make_rsrc(X + first, 4 * (extent - first));
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int kk = 32 * j + 4 * kq;       // k relative to the group
                const int64_t k = kg0 + kk;
                if (KC && p < P && k + 3 < K) {
                    v[j] = buf_load_f32x4(rs, (uint32_t)(4 * (kk + (int64_t)r * ld)));
                } else {
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const bool in = p < P && k + e < K;
                        const uint32_t o = KC ? (uint32_t)(4 * (kk + e + (int64_t)r * ld))
                                              : (uint32_t)(4 * (r + (int64_t)(kk + e) * ld));
                        v[j][e] = buf_load_f32(rs, in ? o : BUF_OOB);
                    }
                }
            }
        } else {
#pragma unroll
            for (int j = 0; j < 4; ++j)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int64_t k = kg0 + 32 * j + 4 * kq + e;
                    float x = 0.0f;
                    if (p < P && k < K) x = X[KC ? k + p * ld : p + k * ld];
                    v[j][e] = x;
                }
        }
        if constexpr (KC) {
            // Eight threads cover one 64-byte row segment: stores are
            // contiguous as they are.
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int64_t k = kg0 + 32 * j + 4 * kq;
                const int64_t blk = k / KW;
                if (blk >= kb) continue;               // past the last KW block
                const int64_t off = ((pb * kb + blk) * 32 + r) * RB + (k % KW) * 2;
                if constexpr (F == Form::BF16X3) {
                    u32x2 h2, l2;
                    split_bf16x4(v[j], h2, l2);
                    *reinterpret_cast<u32x2*>(hi + off) = h2;
                    *reinterpret_cast<u32x2*>(lo + off) = l2;
                } else {
                    *reinterpret_cast<u32x2*>(hi + off) = scale_f16x4(v[j], expo[pb]);
                }
            }
        } else {
            // Threads run along rows here, so their 8-byte pieces would be
            // scattered one per row; the group's blocks (one contiguous
            // GROUP_BYTES range per array) are assembled in LDS first and
            // then written with 16-byte stores that walk it in order.
            const int64_t blk0 = kg0 / KW;
            const int live = (int)((kb - blk0) < PACK_KG / KW ? (kb - blk0) : PACK_KG / KW) * 32 * RB;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int kk = 32 * j + 4 * kq;
                const int off = ((kk / KW) * 32 + r) * RB + (kk % KW) * 2;
                if constexpr (F == Form::BF16X3) {
                    u32x2 h2, l2;
                    split_bf16x4(v[j], h2, l2);
                    *reinterpret_cast<u32x2*>(stage_hi + off) = h2;
                    *reinterpret_cast<u32x2*>(stage_lo + off) = l2;
                } else {
                    *reinterpret_cast<u32x2*>(stage_hi + off) = scale_f16x4(v[j], expo[pb]);
                }
            }
            __syncthreads();
            const int64_t base = (pb * kb + blk0) * 32 * RB;
#pragma unroll
            for (int q = 0; q < GROUP_BYTES / (256 * 16); ++q) {
                const int o = (q * 256 + t) * 16;
                if (o >= live) continue;               // past the last KW block
                *reinterpret_cast<u32x4*>(hi + base + o) = *reinterpret_cast<const u32x4*>(stage_hi + o);
                if constexpr (F == Form::BF16X3)
                    *reinterpret_cast<u32x4*>(lo + base + o) = *reinterpret_cast<const u32x4*>(stage_lo + o);
            }
            __syncthreads();                           // the stage is reused
        }
    }
}

template <Form F, int KW>
static hipError_t launch_pack(bool kcontig, const float* X, int64_t ld, int64_t P, int64_t K,
                              char* hi, char* lo, const int* expo, hipStream_t s) {
    const int64_t pb = (P + 31) / 32, kb = (K + KW - 1) / KW;
    const int64_t kgroups = (K + PACK_KG - 1) / PACK_KG;
    const int64_t n = pb * kgroups;
    if (n == 0) return hipSuccess;
    const int64_t extent = kcontig ? stored_extent(K, P, ld) : stored_extent(P, K, ld);
    const uint32_t grid = (uint32_t)(n < 65536 ? n : 65536);
    const bool buf = ld <= MAX_BUF_LD;
    auto k = kcontig ? (buf ? pack_kernel<F, true, KW, true> : pack_kernel<F, true, KW, false>)
                     : (buf ? pack_kernel<F, false, KW, true> : pack_kernel<F, false, KW, false>);
    hipLaunchKernelGGL(k, dim3(grid), dim3(256), 0, s, X, ld, P, K, extent, kb, kgroups, n, hi, lo,
                       expo);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Main kernel and configurations.
// ---------------------------------------------------------------------------
template <class Cfg, Form F, bool BUF>
__global__ __launch_bounds__(Cfg::NT, Cfg::WPE) void packed_kernel(GemmDesc d, PackedArgs pk,
                                                        uint32_t tiles_m, uint32_t tiles_n) {
    extern __shared__ __attribute__((aligned(16))) char packed_smem[];
    uint32_t tm, tn;
    grouped_tile<8>(xcd_remap(blockIdx.x, gridDim.x), tiles_m, tiles_n, tm, tn);
    if constexpr (Cfg::PIPELINED)
        tile_packed_pp<Cfg, F, BUF>(d, pk, (int64_t)tm * Cfg::BM, (int64_t)tn * Cfg::BN,
                                    packed_smem, 0, pk.kb);
    else
        tile_packed<Cfg, F, BUF>(d, pk, (int64_t)tm * Cfg::BM, (int64_t)tn * Cfg::BN,
                                 packed_smem);
}

// KW = 32: the in-staging engine's LDS layout (configuration 0 matches its
// 256 x 256 tile bitwise); KW = 16: half-depth stages, so a 4-deep ring of
// the 256 x 256 BF16x3 tile fits in 128 KB of LDS.
using PKCfg0 = CfgPK<256, 256, 2, 4, 2, 32>;   // 8 waves of 128x64, 2 stages of 32 k
using PKCfg1 = CfgPK<256, 256, 2, 4, 4, 16>;   // 8 waves of 128x64, 4 stages of 16 k
using PKCfg2 = CfgPK<128, 128, 2, 2, 3, 32>;   // 4 waves of 64x64, 3 stages of 32 k
using PKCfg3 = CfgPK<256, 256, 2, 4, 4, 32>;   // FP16 only: 4 stages of 32 k (128 KB)
// Two work-groups per CU (72 KB of LDS each for BF16x3): their barriers are
// independent, so one keeps the MFMA pipes busy while the other waits.
using PKCfg4 = CfgPK<256, 128, 2, 2, 3, 16>;   // 4 waves of 128x64, 3 stages of 16 k
using PKCfg5 = CfgPK<128, 256, 2, 2, 3, 16>;   // 4 waves of 64x128, 3 stages of 16 k
// As 1 with fragment double buffering (tile_packed_pp).
using PKCfg6 = CfgPK<256, 256, 2, 4, 4, 16, 2, true>;
// As 2 in 4 x 16-k stages with fragment double buffering (64 KB BF16x3).
using PKCfg7 = CfgPK<128, 128, 2, 2, 4, 16, 2, true>;
// FP16 only: as 6 in 4 x 32-k stages (128 KB), half the barriers per MFMA.
using PKCfg8 = CfgPK<256, 256, 2, 4, 4, 32, 2, true>;
constexpr int PACKED_CONFIGS = LOWP_PACKED_CONFIGS;

// Calls f(Cfg{}) for configuration `cfg` (0 <= cfg < PACKED_CONFIGS).
template <class Fn>
static auto with_packed_cfg(int cfg, Fn&& f) {
    switch (cfg) {
        case 0: return f(PKCfg0{});
        case 1: return f(PKCfg1{});
        case 2: return f(PKCfg2{});
        case 3: return f(PKCfg3{});
        case 4: return f(PKCfg4{});
        case 5: return f(PKCfg5{});
        case 6: return f(PKCfg6{});
        case 7: return f(PKCfg7{});
        default: return f(PKCfg8{});
    }
}

template <class Cfg, Form F, bool BUF>
static hipError_t launch_tiles(const GemmDesc& d, const PackedArgs& pk, hipStream_t s) {
    const int64_t tiles_m = (d.M + Cfg::BM - 1) / Cfg::BM;
    const int64_t tiles_n = (d.N + Cfg::BN - 1) / Cfg::BN;
    if (tiles_m * tiles_n > 0xffffffffLL) return hipErrorInvalidValue;
    constexpr int bytes = PackedStage<Cfg, F>::SMEM;
    auto k = packed_kernel<Cfg, F, BUF>;
    hipError_t e = hipFuncSetAttribute((const void*)k,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k, dim3((uint32_t)(tiles_m * tiles_n)), dim3(Cfg::NT), bytes, s, d, pk,
                       (uint32_t)tiles_m, (uint32_t)tiles_n);
    return hipGetLastError();
}

template <class Cfg, Form F>
static hipError_t launch_main(const GemmDesc& d, const PackedArgs& pk, hipStream_t s) {
    if (buffer_path_ok(d)) return launch_tiles<Cfg, F, true>(d, pk, s);
    // A leading dimension of C beyond 32-bit buffer offsets: the epilogue
    // takes 64-bit addresses, built for one smaller tile per block depth
    // (the packed operands do not change; larger tiles would spill there).
    using G = typename std::conditional<Cfg::KW == 16, PKCfg4, PKCfg2>::type;
    return launch_tiles<G, F, false>(d, pk, s);
}

int packed_config_count() { return PACKED_CONFIGS; }

TileConfigInfo packed_config_info(int cfg) {
    if (cfg < 0 || cfg >= PACKED_CONFIGS) return {0, 0, 0, 0};
    return with_packed_cfg(cfg, [](auto c) {
        using C = decltype(c);
        return TileConfigInfo{C::BM, C::BN, C::BK, C::NT};
    });
}

static int packed_kw(int cfg) {
    return with_packed_cfg(cfg, [](auto c) { return decltype(c)::KW; });
}

// LDS ring of the configuration for the form fits in one CU.
static bool packed_fits(bool bf16x3, int cfg) {
    return with_packed_cfg(cfg, [&](auto c) {
        using C = decltype(c);
        return (bf16x3 ? PackedStage<C, Form::BF16X3>::SMEM : PackedStage<C, Form::F16S>::SMEM) <=
               160 * 1024;
    });
}

// Bytes of device workspace for the packed operands.
int64_t packed_workspace_bytes(bool bf16x3, int cfg, int64_t M, int64_t N, int64_t K) {
    const int kw = packed_kw(cfg);
    const int64_t kb = (K + kw - 1) / kw, blk = 64LL * kw;
    const int64_t a = ((M + 31) / 32) * kb * blk, b = ((N + 31) / 32) * kb * blk;
    return (bf16x3 ? 2 : 1) * (a + b);
}

// True when the configuration exists for the form and every lane offset of
// the main loop fits in 31 bits (8 row blocks x the K extent of a block row).
bool packed_supported(bool bf16x3, int cfg, int64_t M, int64_t N, int64_t K) {
    (void)M;
    (void)N;
    if (cfg < 0 || cfg >= PACKED_CONFIGS || !packed_fits(bf16x3, cfg)) return false;
    const int kw = packed_kw(cfg);
    return 8 * ((K + kw - 1) / kw) * 64LL * kw < (1LL << 31);
}

hipError_t launch_packed(bool bf16x3, int cfg, bool ta, bool tb, const GemmDesc& d,
                         char* workspace, hipStream_t s) {
    const int kw = packed_kw(cfg);
    const int64_t kb = (d.K + kw - 1) / kw, blk = 64LL * kw;
    const int64_t pba = (d.M + 31) / 32, pbb = (d.N + 31) / 32;
    const int64_t a = pba * kb * blk, b = pbb * kb * blk;
    PackedArgs pk{};
    pk.kb = kb;
    pk.pb_a = pba;
    pk.pb_b = pbb;
    char* a_hi = workspace;
    char* b_hi = workspace + a;
    char* a_lo = bf16x3 ? workspace + a + b : nullptr;
    char* b_lo = bf16x3 ? workspace + 2 * a + b : nullptr;
    pk.a_hi = a_hi;
    pk.b_hi = b_hi;
    pk.a_lo = a_lo;
    pk.b_lo = b_lo;
    // op(A) is K-contiguous for A 'T'; op(B) is K-contiguous for B 'N'.
    hipError_t e;
    if (bf16x3 && kw == 32) {
        e = launch_pack<Form::BF16X3, 32>(ta, d.A, d.lda, d.M, d.K, a_hi, a_lo, nullptr, s);
        if (e == hipSuccess)
            e = launch_pack<Form::BF16X3, 32>(!tb, d.B, d.ldb, d.N, d.K, b_hi, b_lo, nullptr, s);
    } else if (bf16x3) {
        e = launch_pack<Form::BF16X3, 16>(ta, d.A, d.lda, d.M, d.K, a_hi, a_lo, nullptr, s);
        if (e == hipSuccess)
            e = launch_pack<Form::BF16X3, 16>(!tb, d.B, d.ldb, d.N, d.K, b_hi, b_lo, nullptr, s);
    } else if (kw == 32) {
        e = launch_pack<Form::F16S, 32>(ta, d.A, d.lda, d.M, d.K, a_hi, nullptr, d.expA, s);
        if (e == hipSuccess)
            e = launch_pack<Form::F16S, 32>(!tb, d.B, d.ldb, d.N, d.K, b_hi, nullptr, d.expB, s);
    } else {
        e = launch_pack<Form::F16S, 16>(ta, d.A, d.lda, d.M, d.K, a_hi, nullptr, d.expA, s);
        if (e == hipSuccess)
            e = launch_pack<Form::F16S, 16>(!tb, d.B, d.ldb, d.N, d.K, b_hi, nullptr, d.expB, s);
    }
    if (e != hipSuccess) return e;
    if (cfg < 0 || cfg >= PACKED_CONFIGS || !packed_fits(bf16x3, cfg)) return hipErrorInvalidValue;
    return with_packed_cfg(cfg, [&](auto c) {
        using C = decltype(c);
        if constexpr (PackedStage<C, Form::BF16X3>::SMEM <= 160 * 1024) {
            if (bf16x3) return launch_main<C, Form::BF16X3>(d, pk, s);
        }
        return launch_main<C, Form::F16S>(d, pk, s);
    });
}

// One packed operand: op(X) as P x K (P = M for A, N for B) in kw-deep
// blocks, hi then lo (BF16x3), or the FP16 values (panel exponents `expo`).
int64_t packed_operand_bytes(bool bf16x3, int kw, int64_t P, int64_t K) {
    const int64_t kb = (K + kw - 1) / kw;
    return (bf16x3 ? 2 : 1) * ((P + 31) / 32) * kb * 64LL * kw;
}

hipError_t launch_pack_operand(bool bf16x3, int kw, bool kcontig, const float* X, int64_t ld,
                               int64_t P, int64_t K, char* hi, char* lo, const int* expo,
                               hipStream_t s) {
    if (kw != 16 && kw != 32) return hipErrorInvalidValue;
    if (bf16x3)
        return kw == 32 ? launch_pack<Form::BF16X3, 32>(kcontig, X, ld, P, K, hi, lo, nullptr, s)
                        : launch_pack<Form::BF16X3, 16>(kcontig, X, ld, P, K, hi, lo, nullptr, s);
    return kw == 32 ? launch_pack<Form::F16S, 32>(kcontig, X, ld, P, K, hi, nullptr, expo, s)
                    : launch_pack<Form::F16S, 16>(kcontig, X, ld, P, K, hi, nullptr, expo, s);
}

int packed_config_kw(int cfg) {
    return cfg >= 0 && cfg < PACKED_CONFIGS ? packed_kw(cfg) : 0;
}

// op(A) packed into a_ws (packed_operand_bytes(bf16x3, kw, M, K)), op(B)
// already packed at b_hi / b_lo in the configuration's block depth; then
// the main kernel.  d.B is not read.
hipError_t launch_packed_b_ready(bool bf16x3, int cfg, bool ta, const GemmDesc& d, char* a_ws,
                                 const char* b_hi, const char* b_lo, hipStream_t s) {
    if (cfg < 0 || cfg >= PACKED_CONFIGS || !packed_fits(bf16x3, cfg)) return hipErrorInvalidValue;
    const int kw = packed_kw(cfg);
    const int64_t kb = (d.K + kw - 1) / kw, blk = 64LL * kw;
    const int64_t pba = (d.M + 31) / 32, a = pba * kb * blk;
    PackedArgs pk{};
    pk.kb = kb;
    pk.pb_a = pba;
    pk.pb_b = (d.N + 31) / 32;
    pk.a_hi = a_ws;
    pk.a_lo = bf16x3 ? a_ws + a : nullptr;
    pk.b_hi = b_hi;
    pk.b_lo = b_lo;
    hipError_t e = launch_pack_operand(bf16x3, kw, ta, d.A, d.lda, d.M, d.K, a_ws,
                                       bf16x3 ? a_ws + a : nullptr, d.expA, s);
    if (e != hipSuccess) return e;
    return with_packed_cfg(cfg, [&](auto c) {
        using C = decltype(c);
        if constexpr (PackedStage<C, Form::BF16X3>::SMEM <= 160 * 1024) {
            if (bf16x3) return launch_main<C, Form::BF16X3>(d, pk, s);
        }
        return launch_main<C, Form::F16S>(d, pk, s);
    });
}

// ---------------------------------------------------------------------------
// Split-K of the scaled-FP16 form over packed operands.  Piece s of every
// tile runs the pipelined packed 128 x 128 tile over the k blocks
// [s kbp, min((s+1) kbp, kb)) into slice s of the workspace (alpha 1, beta 0,
// no activation, unscaled by the panel exponents of the whole K, which are
// powers of two); the split-K reduction then adds the slices in order.  The
// pieces take the same MFMAs in the same order as the in-staging pieces, so
// the results are the same bitwise.
// ---------------------------------------------------------------------------
using PKSplitCfg = PKCfg7;

__global__ __launch_bounds__(PKSplitCfg::NT, PKSplitCfg::WPE) void f16s_packed_splitk_kernel(
    GemmDesc d, PackedArgs pk, uint32_t tiles_m, uint32_t tiles_n, int64_t kbp, float* ws) {
    extern __shared__ __attribute__((aligned(16))) char packed_smem[];
    using C = PKSplitCfg;
    // Logical id -> (piece, tile): one XCD takes consecutive tiles of one
    // piece, which share panels of A and B.
    const uint32_t id = xcd_remap(blockIdx.x, gridDim.x);
    const uint32_t tiles = tiles_m * tiles_n;
    const uint32_t s = id / tiles;
    uint32_t tm, tn;
    grouped_tile<8>(id - s * tiles, tiles_m, tiles_n, tm, tn);
    const int64_t kb0 = (int64_t)s * kbp;
    const int64_t cnt = pk.kb - kb0 < kbp ? pk.kb - kb0 : kbp;
    GemmDesc p = d;
    p.C = ws + (int64_t)s * d.M * d.N;
    p.ldc = d.M;
    p.alpha = 1.0f;
    p.beta = 0.0f;
    p.act = ACT_NONE;   // applied once, by the reduction
    tile_packed_pp<C, Form::F16S, true>(p, pk, (int64_t)tm * C::BM, (int64_t)tn * C::BN,
                                        packed_smem, kb0, cnt);
}

int64_t f16s_packed_splitk_bytes(int64_t M, int64_t N, int64_t K) {
    return packed_operand_bytes(false, PKSplitCfg::KW, M, K) +
           packed_operand_bytes(false, PKSplitCfg::KW, N, K);
}

bool f16s_packed_splitk_supported(const SplitKPlan& p, int64_t M, int64_t N, int64_t K) {
    constexpr int cfg = 7;
    static_assert(std::is_same<PKSplitCfg, PKCfg7>::value, "split-K pieces use configuration 7");
    return p.splits >= 2 && !p.small_tile && p.kc % PKSplitCfg::KW == 0 &&
           packed_supported(false, cfg, M, N, K);
}

hipError_t launch_f16s_packed_splitk(bool ta, bool tb, const GemmDesc& d, const SplitKPlan& p,
                                     char* pack_ws, float* slices, hipStream_t s) {
    using C = PKSplitCfg;
    constexpr int kw = C::KW;
    if (!f16s_packed_splitk_supported(p, d.M, d.N, d.K) || !buffer_path_ok(d) ||
        d.M > MAX_BUF_LD || !d.expA || !d.expB || !pack_ws || !slices)
        return hipErrorInvalidValue;
    if ((int64_t)(p.splits - 1) * p.kc >= d.K) return hipErrorInvalidValue;   // empty piece
    const int64_t kb = (d.K + kw - 1) / kw;
    PackedArgs pk{};
    pk.kb = kb;
    pk.pb_a = (d.M + 31) / 32;
    pk.pb_b = (d.N + 31) / 32;
    char* a = pack_ws;
    char* b = pack_ws + packed_operand_bytes(false, kw, d.M, d.K);
    pk.a_hi = a;
    pk.b_hi = b;
    // op(A) is K-contiguous for A 'T'; op(B) is K-contiguous for B 'N'.
    hipError_t e = launch_pack<Form::F16S, kw>(ta, d.A, d.lda, d.M, d.K, a, nullptr, d.expA, s);
    if (e == hipSuccess)
        e = launch_pack<Form::F16S, kw>(!tb, d.B, d.ldb, d.N, d.K, b, nullptr, d.expB, s);
    if (e != hipSuccess) return e;
    const int64_t tiles_m = (d.M + C::BM - 1) / C::BM, tiles_n = (d.N + C::BN - 1) / C::BN;
    const int64_t grid = tiles_m * tiles_n * p.splits;
    if (grid > 0xffffffffLL) return hipErrorInvalidValue;
    constexpr int bytes = PackedStage<C, Form::F16S>::SMEM;
    e = hipFuncSetAttribute((const void*)f16s_packed_splitk_kernel,
                            hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(f16s_packed_splitk_kernel, dim3((uint32_t)grid), dim3(C::NT), bytes, s, d, pk,
                       (uint32_t)tiles_m, (uint32_t)tiles_n, p.kc / kw, slices);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_splitk_reduce(slices, p.splits, d, s);
}

}  // namespace mgemm
