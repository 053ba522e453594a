// tile_lowp.hpp -- the BF16x3 and scaled-FP16 MFMA tile engine.
//
//
//   BF16x3:  each FP32 operand x is split while it is staged into LDS:
//            hi = bf16(x), lo = bf16(x - hi), both rounded to nearest even
//            (x - hi is exact in FP32).  The product is accumulated as
//            hi*hi + hi*lo + lo*hi; lo*lo (relative size 2^-16) is dropped.
//   FP16s:   a pre-pass finds, for every 32-row panel of op(A) and every
//            32-column panel of op(B), the power of two 2^e that puts the
//            panel's largest magnitude in [2^14, 2^15).  Staging stores
//            fp16(x * 2^e) (the scaling is exact, the conversion rounds to
//            nearest even) and the epilogue multiplies each accumulator by
//            2^-(eA + eB) with ldexp (exact).
//
// Tile engine (same roles as the FP32 kernel): one work-group per BM x BN
// tile of C; BK-deep slabs of op(A) and op(B) staged through two LDS buffers
// while the next slab is fetched into registers; each wave keeps an
// (FM*32) x (FN*32) block of C in MFMA accumulators for the whole K loop.
//
// LDS layout of one operand slab: P rows of BK 16-bit values (64-byte rows
// for BK = 32), k contiguous.  A row is four 16-byte chunks of 8 k values;
// chunk c of row p sits at chunk slot c ^ ((p >> 2) & 3), so the 16 lanes
// that read one 16-byte chunk of 16 consecutive rows hit 16 distinct slots
// (no bank conflicts) without padding.
#pragma once
#include <type_traits>

#include "tile_common.hpp"

namespace mgemm {

enum class Form { BF16X3, F16S };

template <int BM_, int BN_, int WGM_, int WGN_>
struct CfgLP {
    static constexpr int BM = BM_, BN = BN_, BK = 32;
    static constexpr int WGM = WGM_, WGN = WGN_;
    static constexpr int NT = 64 * WGM * WGN;
    static constexpr int WM = BM / WGM, WN = BN / WGN;
    static constexpr int FM = WM / 32, FN = WN / 32;
    static constexpr int ROW_BYTES = BK * 2;  // 64
    static_assert(WM % 32 == 0 && WN % 32 == 0, "wave tile must be 32-aligned");
};

// Byte offset of 16-byte chunk c (0..3) of row p in a swizzled slab.
__device__ inline int chunk_off(int p, int c) {
    return p * 64 + ((c ^ ((p >> 2) & 3)) << 4);
}

// hi = bf16(x) and lo = bf16(x - hi) for four values, packed two per dword.
__device__ inline void split_bf16x4(const f32x4& v, u32x2& hi, u32x2& lo) {
#pragma unroll
    for (int e = 0; e < 4; e += 2) {
        const __bf16 h0 = (__bf16)v[e], h1 = (__bf16)v[e + 1];
        const __bf16 l0 = (__bf16)(v[e] - (float)h0);
        const __bf16 l1 = (__bf16)(v[e + 1] - (float)h1);
        hi[e / 2] = (uint32_t)__builtin_bit_cast(uint16_t, h0) |
                    ((uint32_t)__builtin_bit_cast(uint16_t, h1) << 16);
        lo[e / 2] = (uint32_t)__builtin_bit_cast(uint16_t, l0) |
                    ((uint32_t)__builtin_bit_cast(uint16_t, l1) << 16);
    }
}

// fp16(x * 2^e) for four values, packed two per dword.
__device__ inline u32x2 scale_f16x4(const f32x4& v, int e) {
    u32x2 q;
#pragma unroll
    for (int i = 0; i < 4; i += 2) {
        const _Float16 a = (_Float16)ldexpf(v[i], e);
        const _Float16 b = (_Float16)ldexpf(v[i + 1], e);
        q[i / 2] = (uint32_t)__builtin_bit_cast(uint16_t, a) |
                   ((uint32_t)__builtin_bit_cast(uint16_t, b) << 16);
    }
    return q;
}

// Write one register-staged slab (BP rows) into LDS.  `hi` / `lo` are the
// two arrays of the BF16x3 form; the FP16 form uses `hi` only, with the
// exponent of each 32-row panel from `expo` (indexed from panel p0/32).
template <Form F, class Loader, int NT>
__device__ inline void stage_lowp(const Loader& ld, char* hi, char* lo,
                                  const int* __restrict__ expo, int64_t panel0, int64_t panels,
                                  int tid) {
#pragma unroll
    for (int q = 0; q < Loader::PER_THREAD; ++q) {
        int p, kq;
        Loader::group_pos(tid + q * NT, p, kq);
        const int off = chunk_off(p, kq >> 1) + ((kq & 1) << 3);
        if constexpr (F == Form::BF16X3) {
            u32x2 h, l;
            split_bf16x4(ld.v[q], h, l);
            *reinterpret_cast<u32x2*>(hi + off) = h;
            *reinterpret_cast<u32x2*>(lo + off) = l;
        } else {
            const int64_t pan = panel0 + (p >> 5);
            const int e = pan < panels ? expo[pan] : 0;
            *reinterpret_cast<u32x2*>(hi + off) = scale_f16x4(ld.v[q], e);
        }
    }
}

// MF: this wave reads fragments, issues MFMAs and stores its block (false:
// a wave whose block of C lies wholly outside C; it still stages its share
// of every slab and meets every barrier).
template <class Cfg, Form F, bool AK, bool BKC, bool BUF, bool MF>
__device__ inline void tile_lowp_body(const GemmDesc& d, int64_t m0, int64_t n0, char* smem,
                                      int tid) {
    constexpr int BM = Cfg::BM, BN = Cfg::BN, BK = Cfg::BK, NT = Cfg::NT;
    constexpr int FM = Cfg::FM, FN = Cfg::FN;
    constexpr int ARR = (BM + BN) * Cfg::ROW_BYTES;                 // one array, one stage
    constexpr int STAGE = (F == Form::BF16X3 ? 2 : 1) * ARR;
    const int lane = tid & 63, wave = tid >> 6;
    const int l32 = lane & 31, h = lane >> 5;
    const int wm = (wave % Cfg::WGM) * Cfg::WM;
    const int wn = (wave / Cfg::WGM) * Cfg::WN;
    const int64_t pan_a = (d.M + 31) / 32, pan_b = (d.N + 31) / 32;

    using LA = typename std::conditional<BUF, SlabLoaderB<BM, BK, NT, AK>,
                                         SlabLoaderG<BM, BK, NT, AK>>::type;
    using LB = typename std::conditional<BUF, SlabLoaderB<BN, BK, NT, BKC>,
                                         SlabLoaderG<BN, BK, NT, BKC>>::type;
    using Epi = typename std::conditional<BUF, EpilogueB, EpilogueG>::type;
    const Panel pa{d.A, d.lda, d.M, d.K,
                   AK ? stored_extent(d.K, d.M, d.lda) : stored_extent(d.M, d.K, d.lda), m0};
    const Panel pb{d.B, d.ldb, d.N, d.K,
                   BKC ? stored_extent(d.K, d.N, d.ldb) : stored_extent(d.N, d.K, d.ldb), n0};
    LA la;
    LB lb;
    la.init(pa, tid);
    lb.init(pb, tid);

    f32x16 acc[FM][FN];
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j)
            acc[i][j] = f32x16{};

    // Stage layout: [hi: A rows, B rows][lo: A rows, B rows]
    auto stage_ptr = [&](int s) { return smem + s * STAGE; };
    auto put = [&](int s) {
        char* base = stage_ptr(s);
        char* lo = base + ARR;
        stage_lowp<F, LA, NT>(la, base, lo, d.expA, m0 / 32, pan_a, tid);
        stage_lowp<F, LB, NT>(lb, base + BM * 64, lo + BM * 64, d.expB, n0 / 32, pan_b, tid);
    };

    // MFMAs of the slab in LDS stage `cur`.
    auto compute = [&](int cur) {
        const char* Ah = stage_ptr(cur);
        const char* Bh = Ah + BM * 64;
        const char* Al = Ah + ARR;
        const char* Bl = Al + BM * 64;
        // Two MFMA k-steps of 16 per slab.  In step ks, lanes with h = 0
        // supply k = 16 ks + 0..7 and lanes with h = 1 supply 16 ks + 8..15
        // (chunk 2 ks + h of their row).
#pragma unroll
        for (int ks = 0; ks < 2; ++ks) {
            const int c = 2 * ks + h;
            if constexpr (F == Form::BF16X3) {
                bf16x8 ah[FM], al[FM], bh[FN], bl[FN];
#pragma unroll
                for (int i = 0; i < FM; ++i) {
                    const int o = chunk_off(wm + 32 * i + l32, c);
                    ah[i] = *reinterpret_cast<const bf16x8*>(Ah + o);
                    al[i] = *reinterpret_cast<const bf16x8*>(Al + o);
                }
#pragma unroll
                for (int j = 0; j < FN; ++j) {
                    const int o = chunk_off(wn + 32 * j + l32, c);
                    bh[j] = *reinterpret_cast<const bf16x8*>(Bh + o);
                    bl[j] = *reinterpret_cast<const bf16x8*>(Bl + o);
                }
                // rows of D = n (op(B)), columns of D = m (op(A)).  Every
                // accumulator takes lo*hi, then hi*lo, then hi*hi; the loops
                // run term-major so that consecutive MFMAs are independent.
#pragma unroll
                for (int i = 0; i < FM; ++i)
#pragma unroll
                    for (int j = 0; j < FN; ++j)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(bl[j], ah[i],
                                                                            acc[i][j], 0, 0, 0);
#pragma unroll
                for (int i = 0; i < FM; ++i)
#pragma unroll
                    for (int j = 0; j < FN; ++j)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(bh[j], al[i],
                                                                            acc[i][j], 0, 0, 0);
#pragma unroll
                for (int i = 0; i < FM; ++i)
#pragma unroll
                    for (int j = 0; j < FN; ++j)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(bh[j], ah[i],
                                                                            acc[i][j], 0, 0, 0);
            } else {
                f16x8 aq[FM], bq[FN];
#pragma unroll
                for (int i = 0; i < FM; ++i)
                    aq[i] = *reinterpret_cast<const f16x8*>(Ah + chunk_off(wm + 32 * i + l32, c));
#pragma unroll
                for (int j = 0; j < FN; ++j)
                    bq[j] = *reinterpret_cast<const f16x8*>(Bh + chunk_off(wn + 32 * j + l32, c));
#pragma unroll
                for (int i = 0; i < FM; ++i)
#pragma unroll
                    for (int j = 0; j < FN; ++j)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_f16(bq[j], aq[i],
                                                                           acc[i][j], 0, 0, 0);
            }
        }
    };

    // The K loop is split into straight-line pieces (full-slab loads, the
    // one partial slab, the last slab) so that no iteration joins two load
    // sequences, which would make the compiler wait for every load in
    // flight before the MFMAs.  The loads of slab kt+1 are kept ahead of
    // the MFMAs of slab kt.
    const int64_t nk = (d.K + BK - 1) / BK;   // >= 1: K == 0 never reaches here
    const int64_t nfull = d.K / BK;
    la.load(pa, 0, tid);
    lb.load(pb, 0, tid);
    put(0);
    __syncthreads();

    int64_t kt = 0;
    auto step = [&](auto kind_tag) {
        constexpr int kind = decltype(kind_tag)::value;   // 0 full, 1 partial, 2 last
        const int cur = (int)(kt & 1);
        if constexpr (kind == 0) {
            la.template load<true>(pa, (kt + 1) * BK);
            lb.template load<true>(pb, (kt + 1) * BK);
        } else if constexpr (kind == 1) {
            la.template load<false>(pa, (kt + 1) * BK);
            lb.template load<false>(pb, (kt + 1) * BK);
        }
        __builtin_amdgcn_sched_barrier(0);
        if constexpr (MF) compute(cur);
        if constexpr (kind != 2) {
            put(cur ^ 1);
            __syncthreads();
            ++kt;
        }
    };
    while (kt + 1 < nfull) step(std::integral_constant<int, 0>{});
    if (kt + 1 < nk) step(std::integral_constant<int, 1>{});
    step(std::integral_constant<int, 2>{});

    if constexpr (!MF) return;
    Epi epi(d, m0, n0);
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) {
            int sh = 0;
            if constexpr (F == Form::F16S) {
                const int64_t pa = (m0 + wm + 32 * i) / 32, pb = (n0 + wn + 32 * j) / 32;
                sh = -((pa < pan_a ? d.expA[pa] : 0) + (pb < pan_b ? d.expB[pb] : 0));
            }
            f32x16 v = acc[i][j];
            if constexpr (F == Form::F16S) {
#pragma unroll
                for (int r = 0; r < 16; ++r) v[r] = ldexpf(v[r], sh);
            }
            epi.store_block(wm + 32 * i + l32, wn + 32 * j, lane, v);
        }
}

// One tile.  SKIP (for tiles that are mostly edge, as in a batch of small
// products): a wave whose rows or columns of the tile all lie beyond M or N
// takes the body without fragment reads, MFMAs or stores.  The test is
// wave-uniform.
template <class Cfg, Form F, bool AK, bool BKC, bool BUF, bool SKIP = false>
__device__ inline void tile_lowp(const GemmDesc& d, int64_t m0, int64_t n0, char* smem, int tid) {
    if constexpr (!SKIP) {
        tile_lowp_body<Cfg, F, AK, BKC, BUF, true>(d, m0, n0, smem, tid);
    } else {
        const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
        const int64_t wm = (wave % Cfg::WGM) * Cfg::WM, wn = (wave / Cfg::WGM) * Cfg::WN;
        if (m0 + wm < d.M && n0 + wn < d.N)
            tile_lowp_body<Cfg, F, AK, BKC, BUF, true>(d, m0, n0, smem, tid);
        else
            tile_lowp_body<Cfg, F, AK, BKC, BUF, false>(d, m0, n0, smem, tid);
    }
}

}  // namespace mgemm
