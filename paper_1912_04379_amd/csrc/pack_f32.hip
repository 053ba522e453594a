// pack_f32.hip -- FP32 pre-packed B: op(B) transposed once into the
// k-contiguous layout that the FP32 kernels load with 16-byte loads.
#include "kernels.hpp"

namespace mgemm {

// ---------------------------------------------------------------------------
// FP32 pre-packed B: op(B) copied once into a k-contiguous K x N array, so
// that every later product loads it as an 'N' operand (16-byte loads along
// k).  64 x 64 tiles of op(B) per work-group, grid-stride over the tiles.
// For B stored N x K ('T') the tile goes through LDS (row stride 65 floats:
// the column reads hit 64 distinct banks), so that both the loads (along n)
// and the stores (along k) are coalesced; for B stored K x N it is a copy.
// ---------------------------------------------------------------------------
template <bool TB>
__global__ __launch_bounds__(256) void f32_pack_b_kernel(const float* __restrict__ B, int64_t ldb,
                                                         int64_t K, int64_t N,
                                                         float* __restrict__ out, int64_t ldp,
                                                         int64_t tiles_k, int64_t tiles) {
    __shared__ float t[64][65];
    const int c = threadIdx.x & 63, r = threadIdx.x >> 6;
    for (int64_t b = blockIdx.x; b < tiles; b += gridDim.x) {
        const int64_t k0 = (b % tiles_k) * 64, n0 = (b / tiles_k) * 64;
        if constexpr (TB) {
            // t[k][n] = op(B)(k0 + k, n0 + n) = B[(n0 + n) + (k0 + k) ldb]
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const int kl = r + 4 * i;
                const int64_t k = k0 + kl, n = n0 + c;
                t[kl][c] = k < K && n < N ? B[n + k * ldb] : 0.0f;
            }
            __syncthreads();
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const int nl = r + 4 * i;
                const int64_t k = k0 + c, n = n0 + nl;
                if (k < K && n < N) out[k + n * ldp] = t[c][nl];
            }
            __syncthreads();   // t is reused by the next tile
        } else {
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const int64_t k = k0 + c, n = n0 + r + 4 * i;
                if (k < K && n < N) out[k + n * ldp] = B[k + n * ldb];
            }
        }
    }
}

hipError_t launch_f32_pack_b(bool tb, const float* B, int64_t ldb, int64_t K, int64_t N,
                             float* out, int64_t ldp, hipStream_t s) {
    if (K <= 0 || N <= 0) return hipSuccess;
    if (ldp < K) return hipErrorInvalidValue;
    const int64_t tiles_k = (K + 63) / 64, tiles = tiles_k * ((N + 63) / 64);
    const uint32_t grid = (uint32_t)(tiles < 65536 ? tiles : 65536);
    if (tb)
        hipLaunchKernelGGL(f32_pack_b_kernel<true>, dim3(grid), dim3(256), 0, s, B, ldb, K, N,
                           out, ldp, tiles_k, tiles);
    else
        hipLaunchKernelGGL(f32_pack_b_kernel<false>, dim3(grid), dim3(256), 0, s, B, ldb, K, N,
                           out, ldp, tiles_k, tiles);
    return hipGetLastError();
}

}  // namespace mgemm
