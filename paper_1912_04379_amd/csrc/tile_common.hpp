// tile_common.hpp -- pieces shared by the gfx950 GEMM kernels: operand
// descriptors, work-group -> tile rasterisation, global -> register slab
// loads with ragged-edge masking, and the alpha/beta epilogue.
//
// Data layout (column-major, BLAS): element (r, c) of a stored array X is
// X[r + c*ld].  op(A) is M x K, op(B) is K x N.  For staging, each operand
// is seen as a "panel" P x K where P is M (for op(A)) or N (for op(B)):
//   * op(A) 'N' and op(B) 'T' are contiguous along P in memory;
//   * op(A) 'T' and op(B) 'N' are contiguous along K.
// Every slab is written to LDS as Xs[p][k], k contiguous, so a lane of an
// MFMA reads several consecutive k of one row with one wide LDS read.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mgemm {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef short i16x4 __attribute__((ext_vector_type(4)));
typedef unsigned u32x2 __attribute__((ext_vector_type(2)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

// One GEMM: C <- alpha op(A) op(B) + beta C.
struct GemmDesc {
    const float* A;
    const float* B;
    float* C;
    int64_t M, N, K;
    int64_t lda, ldb, ldc;
    float alpha, beta;
    // FP16-scaled form only: per-32-row exponents of op(A), per-32-column
    // exponents of op(B) (NULL otherwise).
    const int* expA;
    const int* expB;
};

// ---------------------------------------------------------------------------
// Rasterisation.  The hardware hands work-group w to XCD (w mod 8); each XCD
// has its own L2.  `xcd_remap` renumbers the work-groups so that each XCD
// runs one contiguous range of logical tile ids, and `grouped_tile` walks
// the tiles in bands of GROUP_M tile-rows so that tiles running at the same
// time on one XCD share op(A) row panels and op(B) column panels.
// ---------------------------------------------------------------------------
constexpr int NUM_XCD = 8;

__device__ inline uint32_t xcd_remap(uint32_t wg, uint32_t nwg) {
    const uint32_t q = nwg / NUM_XCD, r = nwg % NUM_XCD;
    const uint32_t x = wg % NUM_XCD, i = wg / NUM_XCD;
    const uint32_t start = x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q;
    return start + i;
}

template <int GROUP_M>
__device__ inline void grouped_tile(uint32_t id, uint32_t tiles_m, uint32_t tiles_n,
                                    uint32_t& tm, uint32_t& tn) {
    const uint32_t per_group = GROUP_M * tiles_n;
    const uint32_t g = id / per_group;
    const uint32_t first = g * GROUP_M;
    const uint32_t size = min(tiles_m - first, (uint32_t)GROUP_M);
    const uint32_t in = id - g * per_group;
    tm = first + in % size;
    tn = in / size;
}

// ---------------------------------------------------------------------------
// Slab loads.  A slab is BP x BK of a panel starting at (p0, k0).  It is
// cut into groups of 4 consecutive k at one p; thread t owns the groups
// t, t+NT, t+2NT, ...  K-contiguous panels number the groups k-fastest
// (lanes walk along k in memory); P-contiguous panels number them
// p-fastest (each of the 4 dword loads of a group is coalesced across
// lanes along p).  Elements outside P x K read as 0.
// ---------------------------------------------------------------------------
template <int BP, int BK, int NT, bool KCONTIG>
struct SlabLoader {
    static constexpr int GROUPS = BP * BK / 4;
    static constexpr int PER_THREAD = GROUPS / NT;
    static_assert(GROUPS % NT == 0, "slab must split evenly over threads");
    static_assert(BK % 4 == 0, "BK must be a multiple of 4");

    f32x4 v[PER_THREAD];

    __device__ static inline void group_pos(int g, int& p, int& kq) {
        if (KCONTIG) { kq = g % (BK / 4); p = g / (BK / 4); }
        else         { p = g % BP;        kq = g / BP; }
    }

    // X: the operand base pointer; P, K: panel extents; ld: leading dim.
    __device__ inline void load(const float* __restrict__ X, int64_t ld,
                                int64_t P, int64_t K, int64_t p0, int64_t k0,
                                int tid) {
#pragma unroll
        for (int q = 0; q < PER_THREAD; ++q) {
            int p, kq;
            group_pos(tid + q * NT, p, kq);
            const int64_t gp = p0 + p;
            const int64_t gk = k0 + 4 * kq;
            const bool prow = gp < P;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int64_t k = gk + e;
                float x = 0.0f;
                if (prow && k < K) {
                    const int64_t off = KCONTIG ? (k + gp * ld) : (gp + k * ld);
                    x = X[off];
                }
                v[q][e] = x;
            }
        }
    }
};

// ---------------------------------------------------------------------------
// Epilogue.  The MFMA computes D[n][m] (rows of D are columns of C) so that
// the 32 lanes of a 32x32 block hold 32 consecutive m of one column of C:
// column-major stores are then 128-byte coalesced.  Register r of lane l in
// a 32x32 block holds row 8*(r/4) + 4*(l/32) + (r%4) and column l%32.
// ---------------------------------------------------------------------------
__device__ inline int mfma32_row(int r, int lane) {
    return 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
}

__device__ inline void store_c(const GemmDesc& d, int64_t m, int64_t n, float acc,
                               float scale) {
    if (m < d.M && n < d.N) {
        float* c = d.C + m + n * d.ldc;
        float v = d.alpha * (acc * scale);
        if (d.beta != 0.0f) v = fmaf(d.beta, *c, v);
        *c = v;
    }
}

}  // namespace mgemm
