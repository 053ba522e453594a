// sgemm_small.hip -- FP32 GEMM for small products (v_mfma_f32_16x16x4_f32).
//
// When C has too few 64 x 64 tiles to occupy the CUs, the time of a call is
// the serial chain of each tile: its loads' latency plus K/2 dependent
// 32x32x2 MFMAs.  Here each work-group owns a 16 x 16 tile of C (many more
// work-groups), and its 4 waves each sum a quarter of the k range, so the
// chain is a quarter as long and the 16x16x4 MFMA retires 4 k per step.  The
// four partial tiles are added in LDS in a fixed order, so results do not
// depend on timing.  Operands go from memory straight to registers: a tile
// this small has no reuse for LDS staging to pay for.
//
// MFMA roles as in the other FP32 kernels: srcA carries op(B) (rows of D
// are columns n of C), srcB carries op(A) (columns of D are rows m of C), so
// the 16 lanes of a row of D hold 16 consecutive m of one column of C.
// Lane l of a 16x16 block holds D rows 4*(l/16) + r (r = 0..3), column l%16.
#include "kernels.hpp"

namespace mgemm {

namespace {

constexpr int SM_TILE = 16;      // C tile edge
constexpr int SM_KG = 16;        // k per group: 4 MFMA steps of 4
constexpr int SM_BATCH = 4;      // groups in flight per buffer

// Operand values of one batch of k groups for one lane: element e of
// a[g] / b[g] is k = kb(g) + 4*(lane/16) + e.
struct SmallFrags {
    f32x4 a[SM_BATCH], b[SM_BATCH];
};

// One operand, op(X) as P x K (rows p of op(X) are rows of A or columns of
// B): KC when op(X) is contiguous along k in memory (A 'T', B 'N').
template <bool KC>
struct SmallOperand {
    const float* X;
    int64_t ld, K, extent;   // extent: referenced elements of X
    int64_t p0;              // the tile's first row of op(X)
    int dp;                  // this lane's row, relative to p0 (0..15)
    bool p_ok;               // ... and whether it exists

    // Loads of k group g (groups >= glim give zeros without a memory
    // access).  The descriptor is based at the tile's first element of the
    // group so every offset stays below 2^27 bytes (ld <= MAX_BUF_LD).
    __device__ inline f32x4 load(int64_t g, int64_t glim, int q) const {
        f32x4 v;
        const int64_t kb = g * SM_KG;
        const bool live = g < glim;
        const int64_t first = live ? (KC ? kb + p0 * ld : p0 + kb * ld) : 0;
        const BufRsrc r = make_rsrc(X + first, live ? 4 * (extent - first) : 0);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int kk = 4 * q + e;
            const bool ok = live && p_ok && kb + kk < K;
            const int64_t off = KC ? kk + (int64_t)dp * ld : dp + (int64_t)kk * ld;
            v[e] = buf_load_f32(r, ok ? (uint32_t)(4 * off) : BUF_OOB);
        }
        return v;
    }
};

}  // namespace

template <bool AK, bool BKC>
__global__ __launch_bounds__(256) void sgemm_small_kernel(GemmDesc d, uint32_t tiles_m) {
    __shared__ f32x4 part[3][64];
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int l16 = lane & 15, q = lane >> 4;
    const int64_t m0 = (int64_t)(blockIdx.x % tiles_m) * SM_TILE;
    const int64_t n0 = (int64_t)(blockIdx.x / tiles_m) * SM_TILE;

    const SmallOperand<AK> opa{d.A, d.lda, d.K,
                               AK ? stored_extent(d.K, d.M, d.lda) : stored_extent(d.M, d.K, d.lda),
                               m0, l16, m0 + l16 < d.M};
    const SmallOperand<BKC> opb{d.B, d.ldb, d.K,
                                BKC ? stored_extent(d.K, d.N, d.ldb) : stored_extent(d.N, d.K, d.ldb),
                                n0, l16, n0 + l16 < d.N};

    // This wave's k groups [g0, g1): a quarter of them.
    const int64_t groups = (d.K + SM_KG - 1) / SM_KG;
    const int64_t g0 = groups * wave / 4, g1 = groups * (wave + 1) / 4;

    auto load_batch = [&](int64_t g, SmallFrags& f) {
#pragma unroll
        for (int i = 0; i < SM_BATCH; ++i) {
            f.a[i] = opa.load(g + i, g1, q);
            f.b[i] = opb.load(g + i, g1, q);
        }
    };
    f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
    auto mfma_batch = [&](const SmallFrags& f) {
#pragma unroll
        for (int i = 0; i < SM_BATCH; ++i)
#pragma unroll
            for (int e = 0; e < 4; ++e)
                acc = __builtin_amdgcn_mfma_f32_16x16x4f32(f.b[i][e], f.a[i][e], acc, 0, 0, 0);
    };

    // Two buffers: the loads of the next batch are in flight during the
    // MFMAs of this one.  Batches past g1 load zeros and add nothing.
    SmallFrags f0, f1;
    load_batch(g0, f0);
    for (int64_t g = g0; g < g1; g += 2 * SM_BATCH) {
        load_batch(g + SM_BATCH, f1);
        mfma_batch(f0);
        if (g + SM_BATCH >= g1) break;
        load_batch(g + 2 * SM_BATCH, f0);
        mfma_batch(f1);
    }

    // Partial tiles of waves 1..3 to LDS; wave 0 adds them in wave order
    // and writes C <- alpha * sum + beta * C (beta == 0 never reads C).
    if (wave > 0) part[wave - 1][lane] = acc;
    __syncthreads();
    if (wave != 0) return;
#pragma unroll
    for (int w = 0; w < 3; ++w) acc += part[w][lane];
    const int64_t first = m0 + n0 * d.ldc;
    const BufRsrc rc = make_rsrc(d.C + first, 4 * (stored_extent(d.M, d.N, d.ldc) - first));
    uint32_t off[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int n = 4 * q + r;
        off[r] = m0 + l16 < d.M && n0 + n < d.N ? (uint32_t)(4 * (l16 + (int64_t)n * d.ldc))
                                                : BUF_OOB;
    }
    f32x4 v;
    if (d.beta != 0.0f) {
        float c[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) c[r] = buf_load_f32(rc, off[r]);
#pragma unroll
        for (int r = 0; r < 4; ++r) v[r] = fmaf(d.beta, c[r], d.alpha * acc[r]);
    } else {
#pragma unroll
        for (int r = 0; r < 4; ++r) v[r] = d.alpha * acc[r];
    }
    if (d.act != ACT_NONE) {
        const BufRsrc ra = make_rsrc(d.act == ACT_TANH_GRAD ? d.aux + first : d.C + first,
                                     d.act == ACT_TANH_GRAD
                                         ? 4 * (stored_extent(d.M, d.N, d.ldc) - first)
                                         : 0);
#pragma unroll
        for (int r = 0; r < 4; ++r)
            v[r] = activate(d.act, v[r], d.act == ACT_TANH_GRAD ? buf_load_f32(ra, off[r]) : 0.0f);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) buf_store_f32(rc, off[r], v[r]);
}

hipError_t launch_small(bool ta, bool tb, const GemmDesc& d, hipStream_t s) {
    if (!buffer_path_ok(d)) return hipErrorInvalidValue;
    const int64_t tiles_m = (d.M + SM_TILE - 1) / SM_TILE;
    const int64_t tiles_n = (d.N + SM_TILE - 1) / SM_TILE;
    if (tiles_m * tiles_n > 0xffffffffLL) return hipErrorInvalidValue;
    const dim3 grid((uint32_t)(tiles_m * tiles_n)), block(256);
    const uint32_t tm = (uint32_t)tiles_m;
    // op(A) is K-contiguous for A 'T'; op(B) is K-contiguous for B 'N'.
    if (!ta && !tb)
        hipLaunchKernelGGL((sgemm_small_kernel<false, true>), grid, block, 0, s, d, tm);
    else if (!ta && tb)
        hipLaunchKernelGGL((sgemm_small_kernel<false, false>), grid, block, 0, s, d, tm);
    else if (ta && !tb)
        hipLaunchKernelGGL((sgemm_small_kernel<true, true>), grid, block, 0, s, d, tm);
    else
        hipLaunchKernelGGL((sgemm_small_kernel<true, false>), grid, block, 0, s, d, tm);
    return hipGetLastError();
}

}  // namespace mgemm
