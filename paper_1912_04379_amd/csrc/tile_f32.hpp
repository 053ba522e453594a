// tile_f32.hpp -- the FP32 MFMA tile engine (one BM x BN tile of C).
//
// C <- alpha op(A) op(B) + beta C, FP32 in, FP32 accumulate, FP32 out.
// The paper's recipe (Sections 2 and 3) -- keep every partial sum in a
// register for the whole k loop, reuse every loaded operand several times,
// stage blocks of A and B close to the arithmetic, prefetch the next block
// while computing the current one -- maps onto gfx950 as:
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
template <int BM_, int BN_, int BK_, int WGM_, int WGN_, int WPE_ = 0, int OCC_ = 0,
          bool IL_ = true>
struct CfgF32 {
    static constexpr int BM = BM_, BN = BN_, BK = BK_, WPE = WPE_, OCC = OCC_;
    static constexpr bool IL = IL_;   // interleave LDS writes / loads with MFMAs
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

// Operand fragments of one MFMA k-chunk c (8 consecutive k of the slab,
// 4 per half-wave): lanes with h = 0 hold k = 4c + e, lanes with h = 1 hold
// k = BK/2 + 4c + e (e = 0..3).  Every k of the slab is used once; the
// order of k inside one slab is free.
template <class Cfg>
struct FragF32 {
    f32x4 a[Cfg::FM], b[Cfg::FN];

    __device__ inline void read(const float* As, const float* Bs, int wm, int wn, int l32,
                                int h, int c) {
        constexpr int S = Cfg::S;
        const int ko = h * (Cfg::BK / 2) + 4 * c;
#pragma unroll
        for (int i = 0; i < Cfg::FM; ++i)
            a[i] = *reinterpret_cast<const f32x4*>(As + (wm + 32 * i + l32) * S + ko);
#pragma unroll
        for (int j = 0; j < Cfg::FN; ++j)
            b[j] = *reinterpret_cast<const f32x4*>(Bs + (wn + 32 * j + l32) * S + ko);
    }

    __device__ inline void mfma(f32x16 (&acc)[Cfg::FM][Cfg::FN]) const {
#pragma unroll
        for (int e = 0; e < 4; ++e)
#pragma unroll
            for (int i = 0; i < Cfg::FM; ++i)
#pragma unroll
                for (int j = 0; j < Cfg::FN; ++j)
                    // rows of D = n (from op(B)), columns of D = m (op(A))
                    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(b[j][e], a[i][e],
                                                                     acc[i][j], 0, 0, 0);
    }
};

// What one K-loop step does besides its MFMAs: stage the next slab into
// the other LDS buffer (and then load the slab after it, a whole slab of
// MFMAs ahead: in full, partially, or not at all), or nothing (last slab).
enum class Step { STAGE_LOAD_FULL, STAGE_LOAD_PART, STAGE, LAST };

// One BM x BN tile of C at (m0, n0).  AK / BKC: op(A) / op(B) contiguous
// along K in memory (A 'T' / B 'N').  BUF: buffer loads and stores (every
// leading dimension <= MAX_BUF_LD) or plain global accesses.
//
// Software pipeline, per slab kt (LDS buffer kt & 1; NC = BK/8 k-chunks):
//   MFMAs of chunks 0..NC-2, each while the next chunk's fragments load;
//   write slab kt+1 (in registers) to the other buffer; issue the global
//   loads of slab kt+2; barrier on LDS only; read chunk 0 of slab kt+1;
//   MFMAs of chunk NC-1 (which hide that read and the barrier skew).
// The loop is split into straight-line pieces (full-slab loads, the one
// partial slab, no load, last slab) so that no step joins two load
// sequences: a join makes the compiler wait for every load in flight.
//
// MF: this wave reads fragments and issues MFMAs (false: a wave whose block
// of C lies wholly outside C, which still stages its share of every slab
// and meets every barrier, but computes and stores nothing).
template <class Cfg, bool AK, bool BKC, bool BUF, bool MF>
__device__ inline void tile_f32_body(const GemmDesc& d, int64_t m0, int64_t n0, float* smem,
                                     int tid) {
    constexpr int BM = Cfg::BM, BK = Cfg::BK, NT = Cfg::NT, S = Cfg::S;
    constexpr int FM = Cfg::FM, FN = Cfg::FN, NC = BK / 8;
    static_assert(NC >= 2, "the pipeline needs two k-chunks per slab");
    using LA = typename std::conditional<BUF, SlabLoaderB<BM, BK, NT, AK>,
                                         SlabLoaderG<BM, BK, NT, AK>>::type;
    using LB = typename std::conditional<BUF, SlabLoaderB<Cfg::BN, BK, NT, BKC>,
                                         SlabLoaderG<Cfg::BN, BK, NT, BKC>>::type;
    using Epi = typename std::conditional<BUF, EpilogueB, EpilogueG>::type;
    const int lane = tid & 63, wave = tid >> 6;
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

    const int64_t nk = (d.K + BK - 1) / BK;   // >= 1: K == 0 never reaches here
    const int64_t nfull = d.K / BK;
    auto load = [&](int64_t slab, bool full) {
        if (full) {
            la.template load<true>(pa, slab * BK);
            lb.template load<true>(pb, slab * BK);
        } else {
            la.template load<false>(pa, slab * BK);
            lb.template load<false>(pb, slab * BK);
        }
    };
    load(0, nfull > 0);
    stage_to_lds<LA, BK>(la, smem, tid, NT);
    stage_to_lds<LB, BK>(lb, smem + BM * S, tid, NT);
    if (nk > 1) load(1, nfull > 1);
    lds_barrier();

    FragF32<Cfg> f[2];
    if constexpr (MF) f[0].read(smem, smem + BM * S, wm, wn, l32, h, 0);

    // Instruction counts of one step, for the interleaving below.
    constexpr int N_MFMA = 4 * FM * FN;                    // per k-chunk
    constexpr int N_READ = FM + FN;                        // per k-chunk
    constexpr int N_WRITE = LA::PER_THREAD + LB::PER_THREAD;
    constexpr int N_VMEM = (AK ? 1 : 4) * LA::PER_THREAD + (BKC ? 1 : 4) * LB::PER_THREAD;
    // Small wave tiles have too few MFMAs per chunk to interleave with.
    constexpr bool IL = Cfg::IL && N_WRITE + (N_VMEM + 1) / 2 <= N_MFMA;

    int64_t kt = 0;
    auto step = [&](auto kind_tag) {
        constexpr Step kind = decltype(kind_tag)::value;
        const float* cur = smem + (kt & 1) * Cfg::STAGE;
        float* nxt = smem + ((kt + 1) & 1) * Cfg::STAGE;
#pragma unroll
        for (int c = 0; c + 2 < NC; ++c) {
            if constexpr (MF) f[(c + 1) & 1].read(cur, cur + BM * S, wm, wn, l32, h, c + 1);
            if constexpr (MF) f[c & 1].mfma(acc);
            // Issue the next chunk's reads before this chunk's MFMAs, so that
            // all of them hide the reads' latency (left alone, the scheduler
            // sinks the reads to the last few MFMAs).
            __builtin_amdgcn_sched_group_barrier(0x100, N_READ, 0);   // DS read
            __builtin_amdgcn_sched_group_barrier(0x008, N_MFMA, 0);   // MFMA
        }
        if constexpr (kind == Step::LAST) {
            if constexpr (NC > 1) {
                if constexpr (MF) f[(NC - 1) & 1].read(cur, cur + BM * S, wm, wn, l32, h, NC - 1);
                if constexpr (MF) f[NC & 1].mfma(acc);
            }
            if constexpr (MF) f[(NC - 1) & 1].mfma(acc);
        } else {
            __builtin_amdgcn_sched_barrier(0);
            // Chunk NC-2's MFMAs, with the read of chunk NC-1, the writes of
            // slab kt+1 to LDS and the loads of slab kt+2 issued between
            // them (their issue then costs no MFMA time).
            if constexpr (NC > 1)
                if constexpr (MF) f[(NC - 1) & 1].read(cur, cur + BM * S, wm, wn, l32, h, NC - 1);
            stage_to_lds<LA, BK>(la, nxt, tid, NT);
            stage_to_lds<LB, BK>(lb, nxt + BM * S, tid, NT);
            if constexpr (kind == Step::STAGE_LOAD_FULL) {
                la.template load<true>(pa, (kt + 2) * BK);
                lb.template load<true>(pb, (kt + 2) * BK);
            } else if constexpr (kind == Step::STAGE_LOAD_PART) {
                la.template load<false>(pa, (kt + 2) * BK);
                lb.template load<false>(pb, (kt + 2) * BK);
            }
            if constexpr (NC > 1) {
                if constexpr (MF) f[NC & 1].mfma(acc);
                if constexpr (IL) {
                    __builtin_amdgcn_sched_group_barrier(0x100, N_READ, 0);   // DS read
#pragma unroll
                    for (int i = 0; i < N_WRITE; ++i) {
                        __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);    // MFMA
                        __builtin_amdgcn_sched_group_barrier(0x200, 1, 0);    // DS write
                    }
                    if constexpr (kind != Step::STAGE) {
#pragma unroll
                        for (int i = 0; i < (N_VMEM + 1) / 2; ++i) {
                            __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
                            __builtin_amdgcn_sched_group_barrier(0x020, 2, 0);  // VMEM read
                        }
                    }
                }
            }
            __builtin_amdgcn_sched_barrier(0);
            lds_barrier();
            if constexpr (MF) f[NC & 1].read(nxt, nxt + BM * S, wm, wn, l32, h, 0);
            // Keep the last chunk's MFMAs after the read of the next slab.
            __builtin_amdgcn_sched_barrier(0);
            if constexpr (MF) f[(NC - 1) & 1].mfma(acc);
            ++kt;
        }
    };
    using SF = std::integral_constant<Step, Step::STAGE_LOAD_FULL>;
    using SP = std::integral_constant<Step, Step::STAGE_LOAD_PART>;
    using SS = std::integral_constant<Step, Step::STAGE>;
    using SL = std::integral_constant<Step, Step::LAST>;
    while (kt + 2 < nfull) step(SF{});   // slab kt+2 is full
    if (kt + 2 < nk) step(SP{});         // slab kt+2 is the partial one
    if (kt + 1 < nk) step(SS{});
    step(SL{});

    if constexpr (MF) {
        Epi epi(d, m0, n0);
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
            for (int j = 0; j < FN; ++j)
                epi.store_block(wm + 32 * i + l32, wn + 32 * j, lane, acc[i][j]);
    }
}

// One tile.  SKIP (for tiles that are mostly edge, as in a batch of small
// products): a wave whose rows or columns of the tile all lie beyond M or N
// takes the body without fragment reads, MFMAs or stores, so the MFMA pipes
// of its SIMD serve the other work-group's waves.  The test is wave-uniform.
template <class Cfg, bool AK, bool BKC, bool BUF, bool SKIP = false>
__device__ inline void tile_f32(const GemmDesc& d, int64_t m0, int64_t n0, float* smem, int tid) {
    if constexpr (!SKIP) {
        tile_f32_body<Cfg, AK, BKC, BUF, true>(d, m0, n0, smem, tid);
    } else {
        const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
        const int64_t wm = (wave % Cfg::WGM) * Cfg::WM, wn = (wave / Cfg::WGM) * Cfg::WN;
        if (m0 + wm < d.M && n0 + wn < d.N)
            tile_f32_body<Cfg, AK, BKC, BUF, true>(d, m0, n0, smem, tid);
        else
            tile_f32_body<Cfg, AK, BKC, BUF, false>(d, m0, n0, smem, tid);
    }
}

}  // namespace mgemm
