// tile_packed.hpp -- 16-bit MFMA tile engine fed straight from pre-packed
// operands into a multi-stage LDS ring (gfx950 buffer_load_dwordx4 ... lds).
//
// Packed operand layout (written by the pack kernels in sgemm_packed.hip):
// op(X), P x K, as 16-bit values in blocks of 32 rows x KW k (KW = 32 or 16;
// one 2*KW-byte row per p, k contiguous); block (pb, kb) starts at byte
// (pb * KB + kb) * 64 * KW with KB = ceil(K / KW).  Rows >= P and k >= K
// hold zeros, so the main loop needs no masking.  The BF16x3 form has two such
// arrays per operand (hi, lo); the FP16 form one (x * 2^e of its 32-row
// panel, e from the exponent pre-pass).
//
// Main loop.  A work-group owns a BM x BN tile of C.  Its K loop walks
// KW-deep slabs; slab s of every array goes to LDS stage s mod NS by direct
// memory-to-LDS loads issued NS-1 slabs ahead (no registers, no VALU).
// Each slab iteration is: wait for this slab's own loads (s_waitcnt vmcnt
// with the later slabs still in flight), barrier, issue the loads of slab
// s+NS-1 into the stage that the previous iteration finished reading, then
// KW/16 MFMA k-steps on stage s.  In LDS a row of KW values is split into
// 16-byte chunks of 8 k; chunk c of row p sits at slot c ^ swz(p), with
// swz(p) = (p >> 2) & 3 for 64-byte rows (the in-staging engine's layout)
// and (p >> 3) & 1 for 32-byte rows, so that the 16 lanes reading one chunk
// of 16 consecutive rows hit 16 distinct 16-byte slots (no bank conflicts).
// Lane i of a load fetches the chunk whose swizzled slot is i: a permutation
// inside one block, so the loads stay fully coalesced.
#pragma once
#include <type_traits>

#include "tile_lowp.hpp"

namespace mgemm {

// Device view of the packed operands of one product.
struct PackedArgs {
    const char* a_hi;
    const char* a_lo;   // BF16x3 only
    const char* b_hi;
    const char* b_lo;   // BF16x3 only
    int64_t kb;         // 32-wide k blocks
    int64_t pb_a, pb_b; // 32-row blocks of op(A) and op(B)
};

// WPE: waves per SIMD the kernel is compiled for (registers <= 512 / WPE);
// 2 with 4-wave work-groups means two work-groups share each CU.
// PIPELINED: the fragment-double-buffered main loop (tile_packed_pp), with
// SPLIT8 eighths of each stage's MFMAs issued before its barrier.
template <int BM_, int BN_, int WGM_, int WGN_, int NS_, int KW_, int WPE_ = 2,
          bool PIPELINED_ = false, int SPLIT8_ = 4>
struct CfgPK {
    static constexpr int BM = BM_, BN = BN_, BK = KW_, NS = NS_, KW = KW_, WPE = WPE_;
    static constexpr bool PIPELINED = PIPELINED_;
    static constexpr int SPLIT8 = SPLIT8_;
    static constexpr int WGM = WGM_, WGN = WGN_;
    static constexpr int NT = 64 * WGM * WGN, NWAVES = WGM * WGN;
    static constexpr int WM = BM / WGM, WN = BN / WGN;
    static constexpr int FM = WM / 32, FN = WN / 32;
    static constexpr int ROW_BYTES = 2 * KW;            // one row of a block
    static constexpr int CPR = KW / 8;                  // 16-byte chunks per row
    static constexpr int BLOCK = 32 * ROW_BYTES;        // one 32-row block
    static_assert(KW == 16 || KW == 32, "k-width of a packed block");
    static_assert(WM % 32 == 0 && WN % 32 == 0, "wave tile must be 32-aligned");
    static_assert(BM % 32 == 0 && BN % 32 == 0, "tiles are whole 32-row blocks");
};

// Swizzled slot of logical chunk c of row p (an involution in c).
template <int KW>
__device__ inline int pk_slot(int p, int c) {
    return KW == 32 ? c ^ ((p >> 2) & 3) : c ^ ((p >> 3) & 1);
}

template <class Cfg, Form F>
struct PackedStage {
    static constexpr int ARRAYS = F == Form::BF16X3 ? 2 : 1;
    static constexpr int ARR = (Cfg::BM + Cfg::BN) * Cfg::ROW_BYTES;   // one array
    static constexpr int BYTES = ARRAYS * ARR;
    static constexpr int CHUNKS = BYTES / 1024;                 // 1 KB per wave-wide load
    static constexpr int PER_WAVE = CHUNKS / Cfg::NWAVES;
    static_assert(CHUNKS % Cfg::NWAVES == 0, "stage must split evenly over waves");
    static constexpr int SMEM = Cfg::NS * BYTES;
};

#define MGEMM_LDS(p) ((__attribute__((address_space(3))) void*)(p))

// Wait until at most N of this wave's vector-memory operations are in
// flight, then barrier.  The memory clobber keeps the compiler from moving
// LDS reads of the next stage above it.
template <int N>
__device__ inline void wait_vm_and_barrier() {
    static_assert(N >= 0 && N < 64, "vmcnt range");
    asm volatile("s_waitcnt vmcnt(%0)\n\ts_barrier" ::"n"(N) : "memory");
}

// Global -> LDS loads of one stage.  A stage is [hi: A rows | B rows]
// [lo: A rows | B rows] (FP16: the hi half only), cut into 1 KB pieces of
// RPC rows of one array; wave w loads pieces w*PW .. w*PW+PW-1.  Which
// array a piece belongs to depends only on the wave, so its base pointer
// (advanced to the tile's first block) and the bytes left from there are
// worked out once, as scalars; a stage then costs one descriptor per piece
// and no selects or branches.  The packed path guarantees fewer than 2^31
// blocks, so stage numbers are 32-bit.
template <class Cfg, Form F>
struct PackedIssuer {
    using St = PackedStage<Cfg, F>;
    static constexpr int PW = St::PER_WAVE, RPC = 1024 / Cfg::ROW_BYTES;
    const char* base[PW];
    int64_t bytes[PW];
    uint32_t goff[PW];   // lane's byte offset from the piece's first block
    int kb, wave;

    // Stages 0 .. cnt-1 are the blocks kb0 .. kb0+cnt-1 of the operands (the
    // whole K: kb0 = 0, cnt = pk.kb).
    __device__ inline PackedIssuer(const PackedArgs& pk, int64_t m0, int64_t n0, int wave_,
                                   int lane, int64_t kb0, int64_t cnt) {
        constexpr int BM = Cfg::BM, GROUPS = (Cfg::BM + Cfg::BN) / RPC;
        kb = (int)cnt;
        wave = wave_;
#pragma unroll
        for (int t = 0; t < PW; ++t) {
            const int j = wave * PW + t;
            const int within = j % GROUPS;                 // row group inside one array
            const bool is_a = within < BM / RPC;
            const bool lo = j >= GROUPS;
            const int rg = is_a ? within : within - BM / RPC;
            const int p = rg * RPC + lane / Cfg::CPR;      // tile-relative row
            const int c = pk_slot<Cfg::KW>(p, lane % Cfg::CPR);   // logical chunk of this slot
            goff[t] = (uint32_t)((int64_t)(p >> 5) * pk.kb * Cfg::BLOCK + (p & 31) * Cfg::ROW_BYTES +
                                 c * 16);
            const char* arr = is_a ? (lo ? pk.a_lo : pk.a_hi) : (lo ? pk.b_lo : pk.b_hi);
            const int64_t first = ((is_a ? m0 : n0) / 32 * pk.kb + kb0) * Cfg::BLOCK;
            base[t] = arr + first;
            bytes[t] = (is_a ? pk.pb_a : pk.pb_b) * pk.kb * Cfg::BLOCK - first;
        }
    }

    // Loads of stage s into LDS slot s % NS.  Stages past the end of K get
    // an empty range: every lane reads 0.
    __device__ inline void issue(char* smem, int s) const {
        char* stage = smem + (int)((unsigned)s % Cfg::NS) * St::BYTES;
        const bool live = s < kb;
#pragma unroll
        for (int t = 0; t < PW; ++t) {
            const int64_t o = (int64_t)s * Cfg::BLOCK;
            const BufRsrc r = make_rsrc(base[t] + o, live ? bytes[t] - o : 0);
            char* dst = stage + (wave * PW + t) * 1024;
            __builtin_amdgcn_raw_ptr_buffer_load_lds(r, MGEMM_LDS(dst), 16, goff[t], 0, 0, 0);
        }
    }
};

template <class Cfg, Form F, bool BUF>
__device__ inline void tile_packed(const GemmDesc& d, const PackedArgs& pk, int64_t m0,
                                   int64_t n0, char* smem) {
    using St = PackedStage<Cfg, F>;
    constexpr int BM = Cfg::BM, NS = Cfg::NS, FM = Cfg::FM, FN = Cfg::FN;
    constexpr int PW = St::PER_WAVE, KW = Cfg::KW, RB = Cfg::ROW_BYTES;
    using Epi = typename std::conditional<BUF, EpilogueB, EpilogueG>::type;
    const int tid = threadIdx.x, lane = tid & 63;
    // tid >> 6 is the same on every lane of a wave; say so, so that the
    // buffer descriptors and LDS destinations derived from it stay scalar.
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int l32 = lane & 31, h = lane >> 5;
    const int wm = (wave % Cfg::WGM) * Cfg::WM;
    const int wn = (wave / Cfg::WGM) * Cfg::WN;
    const int64_t pan_a = (d.M + 31) / 32, pan_b = (d.N + 31) / 32;

    const PackedIssuer<Cfg, F> ld(pk, m0, n0, wave, lane, 0, pk.kb);
    auto issue = [&](int64_t st) { ld.issue(smem, (int)st); };

    f32x16 acc[FM][FN];
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j)
            acc[i][j] = f32x16{};

    const int64_t nk = pk.kb;
#pragma unroll
    for (int s = 0; s < NS - 1; ++s) issue(s);

    for (int64_t kt = 0; kt < nk; ++kt) {
        // Loads of slabs kt+1 .. kt+NS-2 may stay in flight.
        wait_vm_and_barrier<(NS - 2) * PW>();
        issue(kt + NS - 1);   // into the stage read in iteration kt-1
        const char* Ah = smem + (int)(kt % NS) * St::BYTES;
        const char* Bh = Ah + BM * RB;
        const char* Al = Ah + St::ARR;
        const char* Bl = Al + BM * RB;
        // Byte offset of logical chunk c of row p inside one array.
        auto co = [](int p, int c) { return p * RB + (pk_slot<KW>(p, c) << 4); };
#pragma unroll
        for (int ks = 0; ks < KW / 16; ++ks) {
            const int c = 2 * ks + h;
            if constexpr (F == Form::BF16X3) {
                bf16x8 ah[FM], al[FM], bh[FN], bl[FN];
#pragma unroll
                for (int i = 0; i < FM; ++i) {
                    const int o = co(wm + 32 * i + l32, c);
                    ah[i] = *reinterpret_cast<const bf16x8*>(Ah + o);
                    al[i] = *reinterpret_cast<const bf16x8*>(Al + o);
                }
#pragma unroll
                for (int j = 0; j < FN; ++j) {
                    const int o = co(wn + 32 * j + l32, c);
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
                    aq[i] = *reinterpret_cast<const f16x8*>(Ah + co(wm + 32 * i + l32, c));
#pragma unroll
                for (int j = 0; j < FN; ++j)
                    bq[j] = *reinterpret_cast<const f16x8*>(Bh + co(wn + 32 * j + l32, c));
#pragma unroll
                for (int i = 0; i < FM; ++i)
#pragma unroll
                    for (int j = 0; j < FN; ++j)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_f16(bq[j], aq[i],
                                                                           acc[i][j], 0, 0, 0);
            }
        }
    }
    // Drain the (empty) loads issued past the end before the work-group ends
    // or the LDS is reused.
    wait_vm_and_barrier<0>();

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

// ---------------------------------------------------------------------------
// Software-pipelined variant: two register sets of MFMA fragments, so that
// the next stage's fragments are read while the current stage's MFMAs run.
// Iteration kt:
//   1. the first SPLIT8/8 of stage kt's MFMAs (fragments already in
//      registers);
//   2. wait for stage kt+1's loads, barrier (every wave has now read stage
//      kt's fragments, so its LDS buffer is free);
//   3. issue the loads of stage kt+NS into that buffer;
//   4. read stage kt+1's fragments into the other register set, overlapped
//      with the rest of stage kt's MFMAs.
// A stage is one or two 16-deep k steps (KW 16 or 32); every accumulator
// still takes lo*hi, hi*lo, hi*hi per 16-deep k step in k order, so results
// equal the other packed configurations bitwise.
// ---------------------------------------------------------------------------
template <class Cfg, Form F>
struct PPFrags {
    static constexpr int FM = Cfg::FM, FN = Cfg::FN, KS = Cfg::KW / 16;
    bf16x8 ah[KS][FM], al[KS][FM], bh[KS][FN], bl[KS][FN];     // BF16x3
    f16x8 aq[KS][FM], bq[KS][FN];                               // FP16
};

template <class Cfg, Form F, bool BUF>
__device__ inline void tile_packed_pp(const GemmDesc& d, const PackedArgs& pk, int64_t m0,
                                      int64_t n0, char* smem, int64_t kb0, int64_t cnt) {
    using St = PackedStage<Cfg, F>;
    constexpr int BM = Cfg::BM, NS = Cfg::NS, FM = Cfg::FM, FN = Cfg::FN;
    constexpr int PW = St::PER_WAVE, KW = Cfg::KW, RB = Cfg::ROW_BYTES;
    static_assert(KW == 16 || KW == 32, "one or two 16-deep MFMA steps per stage");
    constexpr int KS = KW / 16;
    static_assert(NS >= 3, "at least three stages");
    using Epi = typename std::conditional<BUF, EpilogueB, EpilogueG>::type;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int l32 = lane & 31, h = lane >> 5;
    const int wm = (wave % Cfg::WGM) * Cfg::WM;
    const int wn = (wave / Cfg::WGM) * Cfg::WN;
    const int64_t pan_a = (d.M + 31) / 32, pan_b = (d.N + 31) / 32;

    const PackedIssuer<Cfg, F> ld(pk, m0, n0, wave, lane, kb0, cnt);
    auto issue = [&](int64_t st) { ld.issue(smem, (int)st); };
    auto co = [](int p, int c) { return p * RB + (pk_slot<KW>(p, c) << 4); };
    auto read = [&](int s, PPFrags<Cfg, F>& f) {
        const char* Ah = smem + (int)((unsigned)s % NS) * St::BYTES;
        const char* Bh = Ah + BM * RB;
        const char* Al = Ah + St::ARR;
        const char* Bl = Al + BM * RB;
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
            const int c = 2 * ks + h;
#pragma unroll
            for (int i = 0; i < FM; ++i) {
                const int o = co(wm + 32 * i + l32, c);
                if constexpr (F == Form::BF16X3) {
                    f.ah[ks][i] = *reinterpret_cast<const bf16x8*>(Ah + o);
                    f.al[ks][i] = *reinterpret_cast<const bf16x8*>(Al + o);
                } else {
                    f.aq[ks][i] = *reinterpret_cast<const f16x8*>(Ah + o);
                }
            }
#pragma unroll
            for (int j = 0; j < FN; ++j) {
                const int o = co(wn + 32 * j + l32, c);
                if constexpr (F == Form::BF16X3) {
                    f.bh[ks][j] = *reinterpret_cast<const bf16x8*>(Bh + o);
                    f.bl[ks][j] = *reinterpret_cast<const bf16x8*>(Bl + o);
                } else {
                    f.bq[ks][j] = *reinterpret_cast<const f16x8*>(Bh + o);
                }
            }
        }
    };

    f32x16 acc[FM][FN];
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j)
            acc[i][j] = f32x16{};

    // MFMA number q (0 .. NQ-1) of one stage: k-step-major, then term-major
    // over (term, i, j), so every accumulator sees its k steps in order.
    constexpr int TERMS = F == Form::BF16X3 ? 3 : 1;
    constexpr int PER_KS = TERMS * FM * FN;
    constexpr int NQ = KS * PER_KS;
    auto mfma_range = [&](const PPFrags<Cfg, F>& f, auto lo_c, auto hi_c) {
        constexpr int LO = decltype(lo_c)::value, HI = decltype(hi_c)::value;
#pragma unroll
        for (int q = LO; q < HI; ++q) {
            const int ks = q / PER_KS, r = q % PER_KS;
            const int term = r / (FM * FN), i = (r / FN) % FM, j = r % FN;
            if constexpr (F == Form::BF16X3) {
                if (term == 0)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(f.bl[ks][j], f.ah[ks][i], acc[i][j], 0, 0, 0);
                else if (term == 1)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(f.bh[ks][j], f.al[ks][i], acc[i][j], 0, 0, 0);
                else
                    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(f.bh[ks][j], f.ah[ks][i], acc[i][j], 0, 0, 0);
            } else {
                acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_f16(f.bq[ks][j], f.aq[ks][i], acc[i][j], 0, 0, 0);
            }
        }
    };
    // MFMAs issued before the barrier: any number >= 1 keeps the reads of
    // stage k complete before stage k's buffer is reloaded (a wave reaches
    // the barrier only after its first MFMA of stage k, which waits for them).
    constexpr int SPLIT = NQ * Cfg::SPLIT8 / 8 < 1 ? 1 : NQ * Cfg::SPLIT8 / 8;
    static_assert(SPLIT >= 1 && SPLIT <= NQ, "split point");
    using Split = std::integral_constant<int, SPLIT>;
    using Zero = std::integral_constant<int, 0>;
    using All = std::integral_constant<int, NQ>;

    const int nk = (int)cnt;   // the packed path keeps block counts below 2^31
#pragma unroll
    for (int s = 0; s < NS; ++s) issue(s);
    PPFrags<Cfg, F> fr[2];
    wait_vm_and_barrier<(NS - 1) * PW>();     // stage 0 has landed
    read(0, fr[0]);

    for (int kt = 0; kt < nk; kt += 2) {
        // Two iterations per trip so that the register set is a constant.
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int k = kt + u;
            if (k >= nk) break;
            PPFrags<Cfg, F>& cur = fr[u];
            PPFrags<Cfg, F>& nxt = fr[u ^ 1];
            mfma_range(cur, Zero{}, Split{});
            __builtin_amdgcn_sched_barrier(0);
            wait_vm_and_barrier<(NS - 2) * PW>();   // stage k+1 has landed
            issue(k + NS);                          // into stage k's buffer
            if (k + 1 < nk) read(k + 1, nxt);
            __builtin_amdgcn_sched_barrier(0);
            mfma_range(cur, Split{}, All{});
        }
    }
    wait_vm_and_barrier<0>();

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

}  // namespace mgemm
