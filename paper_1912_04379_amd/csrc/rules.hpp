// rules.hpp -- the library's host-side decision rules, free of any HIP
// type: tile-configuration defaults, the split-K plan, and the list
// schedule of grouped plans.  Internal; built into the library and, on its
// own, into the host-only sanitizer check.
#pragma once
#include <stdint.h>

#include <utility>
#include <vector>

namespace mgemm {

// FP32 configuration 10: 256 x 256 x 32 tiles in whole rounds of one per
// CU, 128 x 128 tiles in the tail.
constexpr int F32_TAIL_CONFIG = 10;
// FP32 configuration 11: split-K.  The k range is cut into S pieces of kc
// (the last one shorter); piece s of every tile is an ordinary tile product
// written to workspace + s*M*N (column-major, ld M), and a second kernel
// adds the S partial products in order s = 0..S-1 and applies alpha, beta.
constexpr int F32_SPLITK_CONFIG = 11;
// FP32 configuration 12: 64 x 64 tiles with 32-deep slabs (4 waves of
// 32 x 32), the default for products of about one to a few 64 x 64 tiles
// per CU.
constexpr int F32_DEEP64_CONFIG = 12;
struct SplitKPlan {
    int small_tile;   // 0: 128 x 128 x 16 tiles, 1: 64 x 64 x 32
    int splits;       // S >= 2, or 0 when splitting does not apply
    int64_t kc;       // k per piece, a multiple of 32
};
SplitKPlan f32_splitk_plan(int64_t M, int64_t N, int64_t K, int cus);
// Largest split-K workspace taken (1 GiB); larger products run unsplit.
constexpr int64_t F32_SPLITK_MAX_WORKSPACE = 1LL << 30;
int64_t f32_splitk_workspace_bytes(const SplitKPlan& p, int64_t M, int64_t N);

// Configurations 0..3 of the 16-bit forms split or scale while staging;
// configuration LOWP_INSTAGE_CONFIGS + c is packed configuration c.
constexpr int LOWP_INSTAGE_CONFIGS = 4;
// Packed configurations of the 16-bit forms, and the split-K configuration
// that follows them (the k range cut as for FP32 configuration 11, the
// pieces run as in-staging tiles).
constexpr int LOWP_PACKED_CONFIGS = 9;
constexpr int LOWP_SPLITK_CONFIG = LOWP_INSTAGE_CONFIGS + LOWP_PACKED_CONFIGS;

// Built-in configuration of a single call (no recorded choice).
int f32_default_config(bool transA, bool transB, int64_t M, int64_t N, int64_t K);
// FP32 products whose M and N are each a multiple of 256 or at most 64 past
// one, with at least one of them past: when the whole-tile block Mm x Nm
// holds at least 2^37 flops, it runs on its own and the thin remainders
// (rows Mm..M-1 of C, then columns Nm..N-1 of its first Mm rows) as separate
// products.  Returns false, leaving Mm and Nm alone, when the product stays
// whole.
bool f32_edge_plan(bool transA, bool transB, int64_t M, int64_t N, int64_t K, int64_t* Mm,
                   int64_t* Nm);
// FP32 products with at most THIN_MAX_R columns of C (or rows: then taken
// through the transpose), at least 256 of the other and K >= 256, whose
// operands stay within 32-bit buffer offsets (leading dimensions, M and the
// referenced extents) -- with a k-contiguous large operand and more than 4
// of them, only when it holds at least THIN_GATHER_MIN elements -- the
// library's choice is the thin path, the large
// operand P x K streamed once in S pieces of kc along k (about eight
// work-groups of THIN_ROWS_I or THIN_ROWS_K rows per CU) into S*M*N floats
// of workspace, then the split-K reduction.
constexpr int THIN_MAX_R = 8;
constexpr int THIN_ROWS_I = 64;   // rows per work-group, row-contiguous large operand
constexpr int THIN_ROWS_K = 16;   // rows per work-group, k-contiguous large operand
constexpr int64_t THIN_MAX_LD = (1LL << 21) - 64;       // the buffer path's ld limit
constexpr int64_t THIN_MAX_RANGE = 0x7ffffff0LL;         // bytes one buffer resource spans
// With a k-contiguous large operand, a small operand whose k elements are
// not adjacent in memory (op(B) with transB, or op(A)^T without transA) is
// first gathered into K*r floats in k-major order after the partial sums,
// when r >= 2 or the large operand holds at least THIN_GATHER_MIN elements:
// the streaming kernel's lanes would otherwise touch a cache line per k and
// column.  (The row-contiguous kernel reads few k at a time and gains
// nothing from it.)
constexpr int64_t THIN_GATHER_MIN = 1LL << 25;
struct ThinPlan {
    int ok;       // the thin path applies
    int rows;     // few rows of C (the product taken through its transpose)
    int splits;   // S
    int64_t kc;   // k per piece, a multiple of 64
    int gather;   // the small operand is gathered first
};
ThinPlan thin_plan(int64_t M, int64_t N, int64_t K, int64_t lda, int64_t ldb, int64_t ldc,
                   bool transA, bool transB, int cus);
// S*M*N partial sums, then the gathered small operand (K*r) if any.
int64_t thin_workspace_bytes(const ThinPlan& p, int64_t M, int64_t N, int64_t K);
int bf16x3_default_config(int64_t M, int64_t N, int64_t K);
int f16s_default_config(int64_t M, int64_t N, int64_t K);

// Longest-processing-time-first list schedule: items taken in the order
// given (the caller sorts them by decreasing cost), each to the work-group
// with the least assigned cost so far, ties to the lowest number.  Returns
// the work-group of every item; G >= 1.
std::vector<uint32_t> lpt_schedule(const std::vector<double>& cost_in_order, uint32_t G);

// The work queues of one grouped launch: problem i has ntiles[i] tiles of
// cost tile_cost[i] each.  Problems (cut into contiguous runs of tiles when
// one costs more than a queue's share) go to the nq queues by the list
// schedule above; each queue holds its (problem, tile) pairs costliest
// first.  Every tile appears in exactly one queue.
std::vector<std::vector<std::pair<uint32_t, uint32_t>>> queue_partition(
    const std::vector<uint32_t>& ntiles, const std::vector<double>& tile_cost, uint32_t nq);

}  // namespace mgemm
