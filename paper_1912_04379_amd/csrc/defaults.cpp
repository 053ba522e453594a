// defaults.cpp -- built-in tile-configuration rules for single calls, used
// when no measured choice is recorded for the product, and the split-K
// plan.  Host code only, free of HIP (rules.hpp).
#include <stdint.h>

#include "rules.hpp"

namespace mgemm {

// Default-configuration model.  A tile configuration that runs at `rate` once
// every CU is busy delivers, on an M x N product, rate x (useful share of the
// work-group slots it occupies): M*N over rounds x slots x BM*BN, where a
// round fills every slot once (one work-group per CU unless stated).  This
// counts both the slots left idle in the last round and the padding of edge
// tiles.  MI355X has 256 CUs.
static constexpr int64_t NUM_CUS = 256;
static int64_t tile_count(int64_t M, int64_t N, int bm, int bn) {
    return ((M + bm - 1) / bm) * ((N + bn - 1) / bn);
}
static double slot_share(int64_t M, int64_t N, int bm, int bn, int64_t slots = NUM_CUS) {
    const int64_t rounds = (tile_count(M, N, bm, bn) + slots - 1) / slots;
    return rounds == 0 ? 0.0
                       : (double)M * (double)N / ((double)rounds * slots * bm * bn);
}

// Split-K plan: 128 x 128 tiles when there are at least CUs/4 of them,
// else 64 x 64; S pieces of kc (a multiple of 32).
SplitKPlan f32_splitk_plan(int64_t M, int64_t N, int64_t K, int cus) {
    SplitKPlan p{0, 0, 0};
    if (M < 1 || N < 1 || K < 1 || cus < 1) return p;
    const int64_t t128 = ((M + 127) / 128) * ((N + 127) / 128);
    const int64_t t64 = ((M + 63) / 64) * ((N + 63) / 64);
    p.small_tile = t128 * 4 >= cus ? 0 : 1;
    const int64_t tiles = p.small_tile ? t64 : t128;
    // About two work-groups per CU, pieces of at least 256 k.
    int64_t s = (2 * (int64_t)cus + tiles - 1) / tiles;
    if (s > 32) s = 32;
    int64_t kc = (K + s - 1) / s;
    kc = (kc + 31) / 32 * 32;
    if (kc < 256) kc = 256;
    s = (K + kc - 1) / kc;
    if (s < 2 || tiles * s > 0xffffffffLL) return p;
    p.splits = (int)s;
    p.kc = kc;
    return p;
}

int64_t f32_splitk_workspace_bytes(const SplitKPlan& p, int64_t M, int64_t N) {
    return (int64_t)p.splits * M * N * 4;
}

int f32_default_config(bool ta, bool tb, int64_t M, int64_t N, int64_t K) {
    // At most one 128x128 tile per CU and a long enough k range: split-K
    // (configuration 11).  Measured NN on MI355X, TFLOP/s, split-K against
    // the best unsplit choice: 256 x 256 x 65536, 85 against 18 (the
    // small-product kernel); 512 x 512 x 2048, 37 against 22 (64x64
    // tiles); 1000 x 1000 x 4000, 93 against 82; 1024 x 1024 x 3072, 92
    // against 88; 1024 x 4096 x 8192, 133 against 124; 2048 x 2048 x 4096,
    // 123 against 119.  The pieces get too short below K = 2048 for products
    // split into 64x64 tiles, below 3072 for 128x128 tiles (1024^2 x 2048:
    // 76 against 87), and below 4096 where the small-product kernel applies
    // (256 x 256 x 2048: 7 against 14).
    {
        const int64_t t128 = tile_count(M, N, 128, 128), t64 = tile_count(M, N, 64, 64);
        const int64_t kmin = t64 <= 32 ? 4096 : (t128 * 4 < NUM_CUS ? 2048 : 3072);
        if (t128 <= NUM_CUS && K >= kmin) {
            const SplitKPlan p = f32_splitk_plan(M, N, K, (int)NUM_CUS);
            if (p.splits >= 2 && f32_splitk_workspace_bytes(p, M, N) <= F32_SPLITK_MAX_WORKSPACE)
                return F32_SPLITK_CONFIG;
        }
    }

    // Few 64x64 tiles and a k range worth splitting: the small-product
    // kernel (16x16 tiles, k split over 4 waves).  Measured kernel times:
    // 5.7 us vs 8.9 us for 64x64 tiles at 256^3, 34 us vs 89 us at
    // 256 x 256 x 4096; at 64^3 its fixed cost makes it 1.5 us slower, and
    // from 64 tiles of 64x64 up (512^3: 19 us vs 15 us) it loses.
    if (tile_count(M, N, 64, 64) <= 32 && K >= 128) return 9;

    // Otherwise, candidates with their steady rates measured on MI355X
    // (TFLOP/s, large square products): 256x256 with 32-deep slabs (only
    // for K >= 4096: its longer prologue and epilogue cost more on shorter
    // products), 256x128 at 2 waves per SIMD (128x256 for TT, whose operand
    // layouts favour it), 128x128, and 64x64 with 32-deep slabs.  Each is
    // scored by the slot-share model, less 10% while it has fewer tiles than
    // it needs resident per CU to hide its load latency.  Against measured
    // sweeps (512^3 to 8192^3, odd and rectangular shapes, all four
    // transposes) the pick is the fastest configuration or within 6% of it.
    // The 64x64x32 tile replaced 64x64x16 (rate 125, 6 resident) here: 3-11%
    // faster at every size from 512^3 to 8192^3, it also wins at 2048^3
    // (127 against 123 for 128x128) and 5120^3 (133 against 127 for the
    // rounds with a 128x128 tail).
    struct Cand {
        int cfg, bm, bn;
        double rate;
        int64_t resident, min_k;
    };
    const Cand cands[4] = {
        Cand{8, 256, 256, 148.5, 1, 4096},
        ta && tb ? Cand{6, 128, 256, 147.0, 2, 0} : Cand{5, 256, 128, 147.0, 2, 0},
        Cand{0, 128, 128, 142.0, 3, 0},
        Cand{F32_DEEP64_CONFIG, 64, 64, 131.0, 4, 0},
    };
    int best = F32_DEEP64_CONFIG;
    double best_score = -1.0;
    for (const Cand& c : cands) {
        if (K < c.min_k) continue;
        double score = c.rate * slot_share(M, N, c.bm, c.bn);
        if (tile_count(M, N, c.bm, c.bn) < c.resident * NUM_CUS) score *= 0.9;
        if (score > best_score) {
            best_score = score;
            best = c.cfg;
        }
    }
    // Configuration 10: 256x256 tiles in whole rounds and 128x128 quarters
    // for a part-filled last round.  The tail of r tiles takes about a
    // quarter of a round per ceil(4r / CUs) quarters on a CU; 4% is lost to
    // the second launch and the smaller tile (measured 143, 136 and 127
    // TFLOP/s at 6144^3, 7168^3 and 5120^3).
    if (K >= 4096) {
        const int64_t t = tile_count(M, N, 256, 256), tail = t % NUM_CUS;
        if (tail > 0) {
            const double rounds = (double)(t - tail) / NUM_CUS +
                                  0.25 * (double)((4 * tail + NUM_CUS - 1) / NUM_CUS);
            const double pad = (double)M * (double)N / ((double)t * 256.0 * 256.0);
            const double score = 148.5 * 0.96 * pad * ((double)t / NUM_CUS) / rounds;
            if (score > best_score) best = 10;
        }
    }
    return best;
}

// Ragged edges a little past a multiple of 256.  Measured NN on MI355X,
// TFLOP/s, whole product (the rule's pick) against the whole-tile block plus
// the two remainders (each on its own default: split-K for these thin
// products): 4097^3 124.2 against 135.0, 4128^3 128.4 against 138.8,
// 5121^3 116.2 against 127.6, 6145^3 130.1 against 138.5, 8193^3 132.0
// against 140.7, 2049^2 x 16384 105.1 against 123.2, 8193 x 4097 x 2048
// 128.1 against 134.2, 3073^2 x 8192 121.1 against 123.7.  The remainders
// cost about a pass over A and B plus two launches, so smaller blocks lose
// (4097^2 x 1024 -3.4%, 3073^3 -1.1%, 4100^2 x 512 -7.1%): the block must
// hold at least 2^37 flops (about 0.9 ms).
bool f32_edge_plan(bool ta, bool tb, int64_t M, int64_t N, int64_t K, int64_t* Mm,
                   int64_t* Nm) {
    (void)ta;
    (void)tb;
    const int64_t rm = M % 256, rn = N % 256;
    if (rm > 64 || rn > 64 || (rm == 0 && rn == 0)) return false;
    const int64_t mm = M - rm, nn = N - rn;
    if (mm < 256 || nn < 256 || K < 1) return false;
    if (2.0 * (double)mm * (double)nn * (double)K < 137438953472.0) return false;   // 2^37
    *Mm = mm;
    *Nm = nn;
    return true;
}

// The split-K plan applies (at least two pieces) and its partial products
// fit the workspace limit.
static bool lowp_split_fits(int64_t M, int64_t N, int64_t K) {
    const SplitKPlan p = f32_splitk_plan(M, N, K, (int)NUM_CUS);
    return p.splits >= 2 && f32_splitk_workspace_bytes(p, M, N) <= F32_SPLITK_MAX_WORKSPACE;
}

// In-staging tiles, for products too shallow to repay pre-packing: 256x256
// once the chip gets at least two rounds of work-groups, otherwise the tile
// that still gives every CU several work-groups.
static int lowp_default(int64_t M, int64_t N) {
    if (tile_count(M, N, 256, 256) >= 512) return 0;
    if (tile_count(M, N, 128, 128) >= 1024) return 1;
    return 3;
}

int bf16x3_default_config(int64_t M, int64_t N, int64_t K) {
    // From measured sweeps on MI355X (1024^3 to 8192^3, odd and rectangular
    // shapes, all four transposes).  Configuration 10 is the pipelined
    // packed 256x256 tile (4 x 16-k stages), 11 the pipelined packed
    // 128x128 tile.  Pre-packing costs one extra read of A and B and a write
    // of their two halves: repaid once both M and N reach ~4.5k, where the
    // 256x256 tile wins if its tiles fill the chip evenly and K is deep
    // enough for its longer prologue, and the 128x128 tile otherwise.  Below
    // that, from 144 tiles of 256x256, the in-staging 256x256 tile or the
    // packed 128x128 tile by slot share; then, by tile count, packed 128x128
    // for deep products, in-staging 128x128 for shallow ones, in-staging
    // 64x64 below one round of 128x128 tiles.
    const int64_t t256 = tile_count(M, N, 256, 256), t128 = tile_count(M, N, 128, 128);
    // Few tiles and a long k range: split-K.  Measured NN, TFLOP/s, split
    // against the best unsplit configuration: 512^2 x 16384 139 against 27;
    // 1024^2 x 8192 223 against 106; 256^2 x 65536 128 against 7; 1024^2 x
    // 2048 114 against 99; 2048 x 1024 x 3072 205 against 168; 1024 x 4096 x
    // 8192 262 against 252; it loses at 2048^2 x 4096 (254 against 265).
    if (((t128 <= NUM_CUS / 2 && K >= 2048) || (t128 <= NUM_CUS && K >= 8192)) &&
        lowp_split_fits(M, N, K))
        return LOWP_SPLITK_CONFIG;
    if (t256 >= NUM_CUS && (M < N ? M : N) >= 4608 && K >= 512)
        return K >= 2048 && slot_share(M, N, 256, 256) >= 0.85 ? LOWP_INSTAGE_CONFIGS + 6
                                                               : LOWP_INSTAGE_CONFIGS + 7;
    if (t256 >= 144) {
        // In-staging 256x256 (one work-group per CU, 400 TFLOP/s in full
        // rounds) against the pipelined packed 128x128 (two per CU, 377), by
        // slot share.  Measured: 6144 x 3072 x 3072, 288 tiles of 256x256
        // (a round and an eighth), 258 against 339; 3072^2 x 8192, 144 tiles
        // (one part-filled round for both), 300 against 293; 12288 x 1024 x
        // 4096, 347 against 308.
        if (K >= 512 && 377.0 * slot_share(M, N, 128, 128, 2 * NUM_CUS) >
                            400.0 * slot_share(M, N, 256, 256))
            return LOWP_INSTAGE_CONFIGS + 7;
        return 0;
    }
    if (t128 >= 192 && K >= 512) return LOWP_INSTAGE_CONFIGS + 7;
    if (t128 > NUM_CUS) return 1;
    return 3;
}

int f16s_default_config(int64_t M, int64_t N, int64_t K) {
    // Pre-packing costs FP16 only one extra read of A and B and a half-size
    // write, and its direct-to-LDS main loop beats the in-staging one at
    // every measured size from 1024^3 up (1.15x there, up to 2.6x at 2048^3
    // to 3001^3): packed tiles unless K is too short to repay the pass.
    // Between the pipelined packed 256x256 tile in 32-deep stages (906
    // TFLOP/s at 8192^3) and the pipelined packed 128x128 tile (about 850),
    // the slot-share model picks; the larger tile's longer prologue needs K
    // of 3072 or more.
    // Few tiles and a long k range: split-K.  Measured NN, TFLOP/s, split
    // against the best unsplit configuration: 512^2 x 16384 95 against 44;
    // 1024^2 x 8192 240 against 140; 256^2 x 65536 80 against 13; 1000^2 x
    // 4000 132 against 105; 1024^2 x 2048 83 against 79.  From a quarter
    // round of 128 x 128 tiles up the pieces run on packed operands, which
    // beat the packed 128 x 128 tile for K >= 3072 up to about 150 tiles
    // (1152^2 x 4096 181 against 150, 1280^2 x 8192 290 against 212,
    // 1536^2 x 4096 270 against 251, 2048 x 1024 x 3072 214 against 198)
    // and lose below (1280^2 x 2048 129 against 134, 1536^2 x 2048 174
    // against 186) and at a full round (2048^2 x 4096 377 against 400).
    const int64_t t128 = tile_count(M, N, 128, 128);
    if (((t128 <= NUM_CUS / 4 && K >= 2048) || (t128 <= 5 * NUM_CUS / 8 && K >= 3072)) &&
        lowp_split_fits(M, N, K))
        return LOWP_SPLITK_CONFIG;
    if (K < 512) return lowp_default(M, N);
    const double big = 906.0 * slot_share(M, N, 256, 256);
    const double mid = 850.0 * slot_share(M, N, 128, 128);
    return K >= 3072 && big > mid ? LOWP_INSTAGE_CONFIGS + 8 : LOWP_INSTAGE_CONFIGS + 7;
}

ThinPlan thin_plan(int64_t M, int64_t N, int64_t K, int64_t lda, int64_t ldb, int64_t ldc,
                   bool ta, bool tb, int cus) {
    ThinPlan p{0, 0, 0, 0, 0};
    if (K < 256 || M < 1 || N < 1 || cus < 1) return p;
    // The buffer path: leading dimensions, and the slices' ld M, within its
    // limit.
    if (lda > THIN_MAX_LD || ldb > THIN_MAX_LD || ldc > THIN_MAX_LD || M > THIN_MAX_LD) return p;
    const bool cols = N <= THIN_MAX_R;   // few columns of C: the large operand is op(A)
    const bool rows = !cols && M <= THIN_MAX_R;
    if (!cols && !rows) return p;
    const int64_t P = cols ? M : N;
    if (P < 256) return p;
    // 32-bit byte offsets from the bases of A and B as referenced.
    const int64_t aext = ta ? K + (M - 1) * lda : M + (K - 1) * lda;
    const int64_t bext = tb ? N + (K - 1) * ldb : K + (N - 1) * ldb;
    if (4 * aext >= THIN_MAX_RANGE || 4 * bext >= THIN_MAX_RANGE) return p;
    const bool kcontig = cols ? ta : !tb;
    const int64_t r = cols ? N : M;
    // Five to eight columns on the k-contiguous kernel run below the rate
    // of split-K unless the large operand is big.
    if (kcontig && r > 4 && P * K < THIN_GATHER_MIN) return p;
    const int64_t per = kcontig ? THIN_ROWS_K : THIN_ROWS_I;
    const int64_t blocks = (P + per - 1) / per;
    // About eight work-groups per CU, so that the loads in flight cover the
    // memory latency with short chains per work-group; pieces a multiple of
    // 64 k, at most 64 of them.
    int64_t S = (8 * (int64_t)cus + blocks - 1) / blocks;
    if (S > 64) S = 64;
    int64_t kc = (K + S - 1) / S;
    kc = (kc + 63) / 64 * 64;
    S = (K + kc - 1) / kc;
    p.splits = (int)S;
    p.kc = kc;
    p.rows = rows ? 1 : 0;
    const bool strided = cols ? (tb && ldb != 1) : (!ta && lda != 1);
    p.gather = strided && kcontig && (r >= 2 || P * K >= THIN_GATHER_MIN) ? 1 : 0;
    p.ok = 1;
    return p;
}

int64_t thin_workspace_bytes(const ThinPlan& p, int64_t M, int64_t N, int64_t K) {
    if (!p.ok) return 0;
    const int64_t r = p.rows ? M : N;
    return 4 * ((int64_t)p.splits * M * N + (p.gather ? K * r : 0));
}

}  // namespace mgemm
