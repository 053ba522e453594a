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
    // Activation applied to v = alpha acc + beta C before it is stored
    // (ACT_NONE, ACT_TANH or ACT_TANH_GRAD); aux: ACT_TANH_GRAD's second
    // operand, M x N with C's leading dimension.
    int act;
    const float* aux;
};

// Fused activations of the epilogue.  ACT_TANH: tanh(v).  ACT_TANH_GRAD:
// v (1 - y^2), the derivative of tanh at the point whose tanh is y, times v.
constexpr int ACT_NONE = 0, ACT_TANH = 1, ACT_TANH_GRAD = 2;

__device__ inline float activate(int act, float v, float y) {
    if (act == ACT_TANH) return tanhf(v);
    if (act == ACT_TANH_GRAD) return v * (1.0f - y * y);
    return v;
}

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
//
// Two implementations with the same interface:
//   SlabLoaderB  raw buffer loads.  The buffer descriptor is rebased to the
//                slab's first element each slab (scalar work); lanes keep
//                32-bit byte offsets computed once; a lane outside the
//                panel uses an offset beyond the descriptor's range, which
//                the hardware returns as 0 -- no branches.  Needs every
//                in-slab offset below 2^31 bytes (ld <= MAX_BUF_LD).
//   SlabLoaderG  plain 64-bit global loads with per-element predicates, for
//                any leading dimension.
// ---------------------------------------------------------------------------
constexpr int64_t MAX_BUF_LD = (1LL << 21) - 64;
constexpr uint32_t BUF_OOB = 0x80000000u;      // offset that is always out of range
constexpr int64_t BUF_MAX_RANGE = 0x7ffffff0LL;

typedef __amdgpu_buffer_rsrc_t BufRsrc;

// Descriptor for `bytes` bytes at `base` (clamped below 2^31).
__device__ inline BufRsrc make_rsrc(const void* base, int64_t bytes) {
    const int64_t n = bytes <= 0 ? 0 : (bytes > BUF_MAX_RANGE ? BUF_MAX_RANGE : bytes);
    // dword 3 = 0x00020000: 32-bit data format, the raw (untyped) buffer
    // setting for gfx9-family parts.
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)n,
                                             0x00020000);
}

__device__ inline float buf_load_f32(BufRsrc r, uint32_t off) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}

__device__ inline f32x4 buf_load_f32x4(BufRsrc r, uint32_t off) {
    return __builtin_bit_cast(f32x4, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0));
}

__device__ inline void buf_store_f32(BufRsrc r, uint32_t off, float v) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, off, 0, 0);
}

// One operand panel: stored array X (column-major, leading dimension ld,
// `extent` referenced elements from X), panel extents P x K, first panel
// row p0.
struct Panel {
    const float* X;
    int64_t ld, P, K, extent, p0;
};

template <int BP, int BK, int NT, bool KCONTIG>
struct SlabGeom {
    static constexpr int GROUPS = BP * BK / 4;
    static constexpr int PER_THREAD = GROUPS / NT;
    static_assert(GROUPS % NT == 0, "slab must split evenly over threads");
    static_assert(BK % 4 == 0, "BK must be a multiple of 4");

    __device__ static inline void group_pos(int g, int& p, int& kq) {
        if (KCONTIG) { kq = g % (BK / 4); p = g / (BK / 4); }
        else         { p = g % BP;        kq = g / BP; }
    }
};

template <int BP, int BK, int NT, bool KCONTIG>
struct SlabLoaderB : SlabGeom<BP, BK, NT, KCONTIG> {
    using G = SlabGeom<BP, BK, NT, KCONTIG>;
    f32x4 v[G::PER_THREAD];
    // Byte offset of element e = 0 of each group from the slab's first
    // element, or BUF_OOB for a group outside the panel.  BUF_OOB plus any
    // in-slab step (< 2^31 - 2^30) stays at or above 2^31, beyond every
    // descriptor's range, so masked groups never need a second select.
    uint32_t off[G::PER_THREAD];
    int kbase[G::PER_THREAD];      // k of element 0 relative to the slab

    __device__ inline void init(const Panel& pn, int tid) {
#pragma unroll
        for (int q = 0; q < G::PER_THREAD; ++q) {
            int p, kq;
            G::group_pos(tid + q * NT, p, kq);
            kbase[q] = 4 * kq;
            const uint32_t o = KCONTIG ? (uint32_t)(4 * (4 * kq + (int64_t)p * pn.ld))
                                       : (uint32_t)(4 * (p + (int64_t)(4 * kq) * pn.ld));
            off[q] = pn.p0 + p < pn.P ? o : BUF_OOB;
        }
    }

    // FULL: the slab lies inside K (k0 + BK <= K), only the panel edge is
    // masked (in off).  Otherwise k >= K is masked too.
    template <bool FULL>
    __device__ inline void load(const Panel& pn, int64_t k0) {
        // The slab's first element and the bytes left in the array from it.
        const int64_t first = KCONTIG ? k0 + pn.p0 * pn.ld : pn.p0 + k0 * pn.ld;
        const BufRsrc r = make_rsrc(pn.X + first, 4 * (pn.extent - first));
        const uint32_t kstep = KCONTIG ? 4u : (uint32_t)(4 * pn.ld);   // bytes per k
        if constexpr (FULL) {
#pragma unroll
            for (int q = 0; q < G::PER_THREAD; ++q) {
                if constexpr (KCONTIG) {
                    v[q] = buf_load_f32x4(r, off[q]);
                } else {
#pragma unroll
                    for (int e = 0; e < 4; ++e) v[q][e] = buf_load_f32(r, off[q] + e * kstep);
                }
            }
        } else {
            const int krem = (int)(pn.K - k0);
#pragma unroll
            for (int q = 0; q < G::PER_THREAD; ++q)
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    v[q][e] = buf_load_f32(r, kbase[q] + e < krem ? off[q] + e * kstep : BUF_OOB);
        }
    }

    // Either form, chosen at run time.
    __device__ inline void load(const Panel& pn, int64_t k0, int tid) {
        (void)tid;
        if (k0 + BK <= pn.K) load<true>(pn, k0);
        else load<false>(pn, k0);
    }
};

template <int BP, int BK, int NT, bool KCONTIG>
struct SlabLoaderG : SlabGeom<BP, BK, NT, KCONTIG> {
    using G = SlabGeom<BP, BK, NT, KCONTIG>;
    f32x4 v[G::PER_THREAD];

    int tid_;

    __device__ inline void init(const Panel&, int tid) { tid_ = tid; }

    template <bool FULL>
    __device__ inline void load(const Panel& pn, int64_t k0) {
#pragma unroll
        for (int q = 0; q < G::PER_THREAD; ++q) {
            int p, kq;
            G::group_pos(tid_ + q * NT, p, kq);
            const int64_t gp = pn.p0 + p;
            const int64_t gk = k0 + 4 * kq;
            const bool prow = gp < pn.P;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int64_t k = gk + e;
                float x = 0.0f;
                if (prow && (FULL || k < pn.K))
                    x = pn.X[KCONTIG ? (k + gp * pn.ld) : (gp + k * pn.ld)];
                v[q][e] = x;
            }
        }
    }

    __device__ inline void load(const Panel& pn, int64_t k0, int tid) {
        (void)tid;
        if (k0 + BK <= pn.K) load<true>(pn, k0);
        else load<false>(pn, k0);
    }
};

// Work-group barrier that waits for this wave's LDS accesses only: global
// loads stay in flight across it (__syncthreads would wait for them too).
// The wait goes through the builtin (encoding: lgkmcnt 0, vmcnt and expcnt
// at their maximum) so that the compiler's own wait insertion knows the
// LDS / scalar-load counter is drained; the "memory" clobber on the
// barrier keeps memory accesses from moving across it.
__device__ inline void lds_barrier() {
    __builtin_amdgcn_s_waitcnt(0xc07f);
    asm volatile("s_barrier" ::: "memory");
}

// Referenced elements of a stored rows x cols array with leading dim ld.
__device__ __host__ inline int64_t stored_extent(int64_t rows, int64_t cols, int64_t ld) {
    return rows > 0 && cols > 0 ? (cols - 1) * ld + rows : 0;
}

// ---------------------------------------------------------------------------
// Epilogue.  The MFMA computes D[n][m] (rows of D are columns of C) so that
// the 32 lanes of a 32x32 block hold 32 consecutive m of one column of C:
// column-major stores are then 128-byte coalesced.  Register r of lane l in
// a 32x32 block holds row 8*(r/4) + 4*(l/32) + (r%4) and column l%32.
//
// C <- alpha * acc + beta * C; beta == 0 never reads C.  EpilogueB masks
// with out-of-range buffer offsets (a dropped store, a load of 0);
// EpilogueG with predicates.
// ---------------------------------------------------------------------------
__device__ inline int mfma32_row(int r, int lane) {
    return 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
}

struct EpilogueB {
    BufRsrc r, raux;
    int64_t mrem, nrem, ldc;
    float alpha, beta;
    int act;
    __device__ inline EpilogueB(const GemmDesc& d, int64_t m0, int64_t n0) {
        const int64_t first = m0 + n0 * d.ldc;
        const int64_t bytes = 4 * (stored_extent(d.M, d.N, d.ldc) - first);
        r = make_rsrc(d.C + first, bytes);
        act = d.act;
        raux = make_rsrc(act == ACT_TANH_GRAD ? d.aux + first : d.C + first,
                         act == ACT_TANH_GRAD ? bytes : 0);
        mrem = d.M - m0;
        nrem = d.N - n0;
        ldc = d.ldc;
        alpha = d.alpha;
        beta = d.beta;
    }
    // One 32x32 MFMA block of this lane: column m and rows n0b +
    // mfma32_row(0..15, lane), relative to the tile origin.  The 16 loads of
    // C are issued together, then the 16 stores: one memory round trip per
    // block, not per element (a load cannot move above an earlier store to
    // C, so element-wise code would wait for each load in turn).
    __device__ inline void store_block(int m, int n0b, int lane, const f32x16& acc) {
        uint32_t off[16];
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            const int n = n0b + mfma32_row(e, lane);
            off[e] = m < mrem && n < nrem ? (uint32_t)(4 * (m + (int64_t)n * ldc)) : BUF_OOB;
        }
        f32x16 v;
        if (beta != 0.0f) {
            float c[16];
#pragma unroll
            for (int e = 0; e < 16; ++e) c[e] = buf_load_f32(r, off[e]);
#pragma unroll
            for (int e = 0; e < 16; ++e) v[e] = fmaf(beta, c[e], alpha * acc[e]);
        } else {
#pragma unroll
            for (int e = 0; e < 16; ++e) v[e] = alpha * acc[e];
        }
        if (act == ACT_TANH_GRAD) {
            // aux is read through its own descriptor at the offsets of C.
            float y[16];
#pragma unroll
            for (int e = 0; e < 16; ++e) y[e] = buf_load_f32(raux, off[e]);
#pragma unroll
            for (int e = 0; e < 16; ++e) v[e] = activate(act, v[e], y[e]);
        } else if (act != ACT_NONE) {
#pragma unroll
            for (int e = 0; e < 16; ++e) v[e] = activate(act, v[e], 0.0f);
        }
#pragma unroll
        for (int e = 0; e < 16; ++e) buf_store_f32(r, off[e], v[e]);
    }
};

struct EpilogueG {
    float* C;
    const float* aux;
    int64_t mrem, nrem, ldc;
    float alpha, beta;
    int act;
    __device__ inline EpilogueG(const GemmDesc& d, int64_t m0, int64_t n0) {
        C = d.C + m0 + n0 * d.ldc;
        act = d.act;
        aux = act == ACT_TANH_GRAD ? d.aux + m0 + n0 * d.ldc : nullptr;
        mrem = d.M - m0;
        nrem = d.N - n0;
        ldc = d.ldc;
        alpha = d.alpha;
        beta = d.beta;
    }
    // As EpilogueB::store_block, in four groups of 4 (64-bit addresses).
    __device__ inline void store_block(int m, int n0b, int lane, const f32x16& acc) {
        float* col = C + m;
#pragma unroll
        for (int g = 0; g < 4; ++g) {
            bool ok[4];
            float v[4];
#pragma unroll
            for (int e = 0; e < 4; ++e)
                ok[e] = m < mrem && n0b + mfma32_row(4 * g + e, lane) < nrem;
            if (beta != 0.0f) {
                float c[4];
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    c[e] = ok[e] ? col[(int64_t)(n0b + mfma32_row(4 * g + e, lane)) * ldc] : 0.0f;
#pragma unroll
                for (int e = 0; e < 4; ++e) v[e] = fmaf(beta, c[e], alpha * acc[4 * g + e]);
            } else {
#pragma unroll
                for (int e = 0; e < 4; ++e) v[e] = alpha * acc[4 * g + e];
            }
            if (act != ACT_NONE) {
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const float y = act == ACT_TANH_GRAD && ok[e]
                                        ? aux[m + (int64_t)(n0b + mfma32_row(4 * g + e, lane)) * ldc]
                                        : 0.0f;
                    v[e] = activate(act, v[e], y);
                }
            }
#pragma unroll
            for (int e = 0; e < 4; ++e)
                if (ok[e]) col[(int64_t)(n0b + mfma32_row(4 * g + e, lane)) * ldc] = v[e];
        }
    }
};

// True when every leading dimension allows the buffer (32-bit offset) path.
__host__ __device__ inline bool buffer_path_ok(const GemmDesc& d) {
    return d.lda <= MAX_BUF_LD && d.ldb <= MAX_BUF_LD && d.ldc <= MAX_BUF_LD;
}

}  // namespace mgemm
