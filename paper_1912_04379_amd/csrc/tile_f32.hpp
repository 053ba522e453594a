// tile_f32.hpp -- the FP32 MFMA tile engine (one BM x BN tile of C).
//
// C <- alpha op(A) op(B) + beta C, FP32 in, FP32 accumulate, FP32 out.
// The paper's recipe (Sections 2 and 3) -- accumulate in registers as long
// as possible, reuse every loaded operand several times, stage blocks of
// A and B close to the arithmetic, prefetch the next block while computing
// the current one -- maps onto gfx950 as:
//   * registers:  each wave owns an (FM*32) x (FN*32) block of C held in
//                 MFMA accumulators for the whole K loop; each operand value
//                 read from LDS feeds FN (or FM) MFMAs;
//   * L1 block:   a BM x BK slab of op(A) and a BK x BN slab of op(B) in LDS;
//   * prefetch:   the next slab is loaded from global memory into registers
//                 while the MFMAs run on the current LDS buffer (two LDS
//                 buffers, one barrier per slab);
//   * L2 block:   XCD-aware, band-ordered tile rasterisation.
#pragma once
#include <type_traits>

#include "tile_common.hpp"

namespace mgemm {

// WPE: waves per SIMD the kernel is compiled for (0 = the compiler's choice;
// otherwise registers are held to 512 / WPE per lane).  OCC: at most this
// many work-groups per CU (0 = no cap), enforced by reserving LDS at launch
// (a whole number of rounds of work-groups avoids a part-empty last round).
template <int BM_, int BN_, int BK_, int WGM_, int WGN_, int WPE_ = 0, int OCC_ = 0>
struct CfgF32 {
    static constexpr int BM = BM_, BN = BN_, BK = BK_, WPE = WPE_, OCC = OCC_;
    static constexpr int WGM = WGM_, WGN = WGN_;
    static constexpr int NT = 64 * WGM * WGN;
    static constexpr int WM = BM / WGM, WN = BN / WGN;
    static constexpr int FM = WM / 32, FN = WN / 32;
    static constexpr int S = BK + 4;  // LDS row stride (floats): 16-byte
                                      // aligned rows, conflict-free b128 reads
    static constexpr int STAGE = (BM + BN) * S;
    static constexpr int SMEM_FLOATS = 2 * STAGE;
    // Dynamic LDS reserved (unused) so that OCC + 1 work-groups do not fit
    // in a CU's 160 KB.
    static constexpr int LDS_CU = 160 * 1024;
    static constexpr int CAP_BYTES = OCC > 0 ? LDS_CU / (OCC + 1) + 1024 : 0;
    static constexpr int PAD_BYTES =
        CAP_BYTES > SMEM_FLOATS * 4 ? CAP_BYTES - SMEM_FLOATS * 4 : 0;
    static_assert(WM % 32 == 0 && WN % 32 == 0, "wave tile must be 32-aligned");
    static_assert(BK % 8 == 0, "BK must be a multiple of 8");
};

template <class Loader, int BK>
__device__ inline void stage_to_lds(const Loader& ld, float* Xs, int tid, int nt) {
    constexpr int S = BK + 4;
#pragma unroll
    for (int q = 0; q < Loader::PER_THREAD; ++q) {
        int p, kq;
        Loader::group_pos(tid + q * nt, p, kq);
        *reinterpret_cast<f32x4*>(Xs + p * S + 4 * kq) = ld.v[q];
    }
}

// One BM x BN tile of C at (m0, n0).  AK / BKC: op(A) / op(B) contiguous
// along K in memory (A 'T' / B 'N').  BUF: buffer loads and stores (every
// leading dimension <= MAX_BUF_LD) or plain global accesses.
template <class Cfg, bool AK, bool BKC, bool BUF>
__device__ inline void tile_f32(const GemmDesc& d, int64_t m0, int64_t n0, float* smem) {
    constexpr int BM = Cfg::BM, BN = Cfg::BN, BK = Cfg::BK, NT = Cfg::NT, S = Cfg::S;
    constexpr int FM = Cfg::FM, FN = Cfg::FN;
    using LA = typename std::conditional<BUF, SlabLoaderB<BM, BK, NT, AK>,
                                         SlabLoaderG<BM, BK, NT, AK>>::type;
    using LB = typename std::conditional<BUF, SlabLoaderB<BN, BK, NT, BKC>,
                                         SlabLoaderG<BN, BK, NT, BKC>>::type;
    using Epi = typename std::conditional<BUF, EpilogueB, EpilogueG>::type;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int l32 = lane & 31, h = lane >> 5;
    const int wm = (wave % Cfg::WGM) * Cfg::WM;
    const int wn = (wave / Cfg::WGM) * Cfg::WN;

    // op(A) is M x K: stored M x K ('N') or K x M ('T'); likewise op(B) as N x K.
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

    const int64_t nk = (d.K + BK - 1) / BK;
    la.load(pa, 0, tid);
    lb.load(pb, 0, tid);
    stage_to_lds<LA, BK>(la, smem, tid, NT);
    stage_to_lds<LB, BK>(lb, smem + BM * S, tid, NT);
    __syncthreads();

    for (int64_t kt = 0; kt < nk; ++kt) {
        float* cur = smem + (kt & 1) * Cfg::STAGE;
        float* nxt = smem + ((kt + 1) & 1) * Cfg::STAGE;
        const bool more = kt + 1 < nk;
        if (more) {
            la.load(pa, (kt + 1) * BK, tid);
            lb.load(pb, (kt + 1) * BK, tid);
        }
        const float* As = cur;
        const float* Bs = cur + BM * S;
        // MFMA step (c, e): lanes with h = 0 supply k = 4c + e, lanes with
        // h = 1 supply k = BK/2 + 4c + e; every k of the slab is used once.
#pragma unroll
        for (int c = 0; c < BK / 8; ++c) {
            f32x4 a[FM], b[FN];
            const int ko = h * (BK / 2) + 4 * c;
#pragma unroll
            for (int i = 0; i < FM; ++i)
                a[i] = *reinterpret_cast<const f32x4*>(As + (wm + 32 * i + l32) * S + ko);
#pragma unroll
            for (int j = 0; j < FN; ++j)
                b[j] = *reinterpret_cast<const f32x4*>(Bs + (wn + 32 * j + l32) * S + ko);
#pragma unroll
            for (int e = 0; e < 4; ++e)
#pragma unroll
                for (int i = 0; i < FM; ++i)
#pragma unroll
                    for (int j = 0; j < FN; ++j)
                        // rows of D = n (from op(B)), columns of D = m (op(A))
                        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(
                            b[j][e], a[i][e], acc[i][j], 0, 0, 0);
        }
        if (more) {
            stage_to_lds<LA, BK>(la, nxt, tid, NT);
            stage_to_lds<LB, BK>(lb, nxt + BM * S, tid, NT);
        }
        __syncthreads();
    }

    Epi epi(d, m0, n0);
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r)
                epi.store(wm + 32 * i + l32, wn + 32 * j + mfma32_row(r, lane), acc[i][j][r]);
}

}  // namespace mgemm
