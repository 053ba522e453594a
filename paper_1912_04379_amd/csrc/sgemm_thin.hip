// sgemm_thin.hip -- FP32 products with at most THIN_MAX_R columns of C (and,
// through the transpose, rows): matrix-vector-like, bound by reading the
// large operand once.  The large operand X (P x K) is streamed with
// coalesced loads, cut along k into S pieces so that every CU has several
// work-groups of loads in flight; the small operand Y (K x r) is read
// through the cache (for the k-contiguous kernel, from a k-major copy
// gathered first when its k elements are not adjacent, as the plan in
// defaults.cpp decides).  Piece s writes its partial sums to slice s of a
// workspace, and the split-K reduction adds the slices in the order
// s = 0..S-1 and applies alpha and beta: results do not depend on timing.
#include <hip/hip_runtime.h>

#include "kernels.hpp"
#include "tile_common.hpp"

namespace mgemm {

// out[i, j] = sum over the piece's k of X[i, k] Y[k, j], i < P, j < r:
//   X[i, k] at X + i + k*xld (i contiguous) or X + k + i*xld (k contiguous),
//   Y[k, j] at Y + k*yks + j*yjs,
//   slice s of the partial sums at ws + s*P*r, element (i, j) at i*wis + j*wjs.
struct ThinArgs {
    const float* X;
    const float* Y;
    float* ws;
    int64_t P, K, xld, yks, yjs, wis, wjs, kc;
    int64_t xbytes, ybytes;   // bytes referenced from X and from Y
    // How the k-contiguous kernel reads 4 consecutive k of Y: 0 one element
    // at a time, 1 16 bytes per column (yks == 1), 2 16 bytes at a time
    // over the 4r adjacent elements (yks == r, yjs == 1).
    int ymode;
};

// The plan's limits are the buffer path's.
static_assert(THIN_MAX_LD == MAX_BUF_LD && THIN_MAX_RANGE == BUF_MAX_RANGE,
              "thin plan limits");
constexpr int THIN_UNROLL = 4;

// i-contiguous X: a lane loads 4 consecutive rows (16 bytes); 16 lanes cover
// the work-group's 64 rows at one k, the 4 lane groups of a wave 4 k, the 4
// waves 16 k.  Partial sums over the lanes that share rows are added in LDS
// in a fixed order.
template <int R>
__global__ __launch_bounds__(256) void thin_icontig_kernel(ThinArgs t) {
    __shared__ float red[16][THIN_ROWS_I][R];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int rq = lane & 15, kl = 4 * wave + (lane >> 4);   // kl: 0..15
    const int64_t i0 = (int64_t)blockIdx.x * THIN_ROWS_I, s = blockIdx.y;
    const int64_t k0 = s * t.kc, k1 = k0 + t.kc < t.K ? k0 + t.kc : t.K;
    const int64_t i = i0 + 4 * rq;
    const BufRsrc rx = make_rsrc(t.X, t.xbytes), ry = make_rsrc(t.Y, t.ybytes);
    float acc[4][R];
#pragma unroll
    for (int e = 0; e < 4; ++e)
#pragma unroll
        for (int j = 0; j < R; ++j) acc[e][j] = 0.0f;
    const bool whole = i + 3 < t.P;
    for (int64_t kb = k0 + kl; kb < k1; kb += 16 * THIN_UNROLL) {
        f32x4 x[THIN_UNROLL];
        float y[THIN_UNROLL][R];
#pragma unroll
        for (int u = 0; u < THIN_UNROLL; ++u) {
            const int64_t k = kb + 16 * u;
            const bool kin = k < k1;
            if (whole) {
                x[u] = buf_load_f32x4(rx, kin ? (uint32_t)(4 * (i + k * t.xld)) : BUF_OOB);
            } else {
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    x[u][e] = buf_load_f32(
                        rx, kin && i + e < t.P ? (uint32_t)(4 * (i + e + k * t.xld)) : BUF_OOB);
            }
#pragma unroll
            for (int j = 0; j < R; ++j)
                y[u][j] = buf_load_f32(ry, kin ? (uint32_t)(4 * (k * t.yks + j * t.yjs)) : BUF_OOB);
        }
#pragma unroll
        for (int u = 0; u < THIN_UNROLL; ++u)
#pragma unroll
            for (int e = 0; e < 4; ++e)
#pragma unroll
                for (int j = 0; j < R; ++j) acc[e][j] = fmaf(x[u][e], y[u][j], acc[e][j]);
    }
#pragma unroll
    for (int e = 0; e < 4; ++e)
#pragma unroll
        for (int j = 0; j < R; ++j) red[kl][4 * rq + e][j] = acc[e][j];
    __syncthreads();
    // Thread p < 64 * R adds the 16 k-lane sums of its (row, column) in order.
    for (int p = tid; p < THIN_ROWS_I * R; p += 256) {
        const int row = p / R, j = p % R;
        float v = 0.0f;
#pragma unroll
        for (int q = 0; q < 16; ++q) v += red[q][row][j];
        if (i0 + row < t.P) t.ws[s * t.P * R + (i0 + row) * t.wis + j * t.wjs] = v;
    }
}

// k-contiguous X: each wave takes 4 of the work-group's 16 rows at once; its
// lanes load 16 bytes (4 consecutive k) of each row, 256 k per wave, the
// loads of Y shared by the 4 rows, and each sum is reduced across the lanes
// in a fixed butterfly order.
template <int R, int YM>
__global__ __launch_bounds__(256) void thin_kcontig_kernel(ThinArgs t) {
    // Fewer loads in flight per lane as r grows, so that the registers stay
    // within 128.
    constexpr int U = R == 1 ? THIN_UNROLL : (R <= 4 ? 2 : 1);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t i0 = (int64_t)blockIdx.x * THIN_ROWS_K + 4 * wave, s = blockIdx.y;
    const int64_t k0 = s * t.kc, k1 = k0 + t.kc < t.K ? k0 + t.kc : t.K;
    const BufRsrc rx = make_rsrc(t.X, t.xbytes), ry = make_rsrc(t.Y, t.ybytes);
    if (i0 >= t.P) return;   // uniform in the wave; no barrier follows
    bool live[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) live[q] = i0 + q < t.P;
    float acc[4][R];
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int j = 0; j < R; ++j) acc[q][j] = 0.0f;
    for (int64_t kb = k0 + 4 * lane; kb < k1; kb += 256 * U) {
        f32x4 x[U][4];
        float y[U][4][R];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t k = kb + 256 * u;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                if (k + 3 < k1) {
                    x[u][q] = buf_load_f32x4(
                        rx, live[q] ? (uint32_t)(4 * (k + (i0 + q) * t.xld)) : BUF_OOB);
                } else {
#pragma unroll
                    for (int e = 0; e < 4; ++e)
                        x[u][q][e] = buf_load_f32(
                            rx, live[q] && k + e < k1 ? (uint32_t)(4 * (k + e + (i0 + q) * t.xld))
                                                      : BUF_OOB);
                }
            }
            if (YM == 1 && k + 3 < k1) {
#pragma unroll
                for (int j = 0; j < R; ++j) {
                    const f32x4 v = buf_load_f32x4(ry, (uint32_t)(4 * (k + j * t.yjs)));
#pragma unroll
                    for (int e = 0; e < 4; ++e) y[u][e][j] = v[e];
                }
            } else if (YM == 2 && k + 3 < k1) {
#pragma unroll
                for (int q = 0; q < R; ++q) {
                    const f32x4 v = buf_load_f32x4(ry, (uint32_t)(4 * (k * R + 4 * q)));
#pragma unroll
                    for (int c = 0; c < 4; ++c) y[u][(4 * q + c) / R][(4 * q + c) % R] = v[c];
                }
            } else {
#pragma unroll
                for (int e = 0; e < 4; ++e)
#pragma unroll
                    for (int j = 0; j < R; ++j)
                        y[u][e][j] = buf_load_f32(
                            ry, k + e < k1 ? (uint32_t)(4 * ((k + e) * t.yks + j * t.yjs))
                                           : BUF_OOB);
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int q = 0; q < 4; ++q)
#pragma unroll
                for (int e = 0; e < 4; ++e)
#pragma unroll
                    for (int j = 0; j < R; ++j)
                        acc[q][j] = fmaf(x[u][q][e], y[u][e][j], acc[q][j]);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int j = 0; j < R; ++j) {
            float v = acc[q][j];
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
            if (lane == 0 && live[q]) t.ws[s * t.P * R + (i0 + q) * t.wis + j * t.wjs] = v;
        }
}

// Yc[k*r + j] = Y[k*yks + j*yjs] for k < K, j < r: the small operand in
// k-major order, so that the streaming kernels read it in whole lines.
__global__ __launch_bounds__(256) void thin_gather_kernel(const float* Y, int64_t yks,
                                                          int64_t yjs, int64_t K, int r,
                                                          float* Yc) {
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p >= K * r) return;
    const int64_t k = p / r, j = p - k * r;
    Yc[p] = Y[k * yks + j * yjs];
}

template <int R>
static void launch_thin_r(bool kcontig, const ThinArgs& t, int64_t S, hipStream_t s) {
    if (kcontig) {
        // One way of reading Y per kernel, so that the registers of the
        // others are not held.
        const dim3 grid((uint32_t)((t.P + THIN_ROWS_K - 1) / THIN_ROWS_K), (uint32_t)S);
        if (t.ymode == 1)
            hipLaunchKernelGGL((thin_kcontig_kernel<R, 1>), grid, dim3(256), 0, s, t);
        else if (t.ymode == 2)
            hipLaunchKernelGGL((thin_kcontig_kernel<R, 2>), grid, dim3(256), 0, s, t);
        else
            hipLaunchKernelGGL((thin_kcontig_kernel<R, 0>), grid, dim3(256), 0, s, t);
    } else {
        const dim3 grid((uint32_t)((t.P + THIN_ROWS_I - 1) / THIN_ROWS_I), (uint32_t)S);
        hipLaunchKernelGGL(thin_icontig_kernel<R>, grid, dim3(256), 0, s, t);
    }
}

hipError_t launch_thin(bool ta, bool tb, const GemmDesc& d, const ThinPlan& p, float* ws,
                       hipStream_t s) {
    if (!p.ok || !ws || !buffer_path_ok(d) || d.act != ACT_NONE) return hipErrorInvalidValue;
    const int64_t M = d.M, N = d.N, K = d.K;
    ThinArgs t{};
    int r;
    bool kcontig;
    if (!p.rows) {
        // C (M x r) = op(A) (M x K) op(B) (K x r).
        r = (int)N;
        t.X = d.A;
        t.xld = d.lda;
        kcontig = ta;
        t.Y = d.B;
        t.yks = tb ? d.ldb : 1;
        t.yjs = tb ? 1 : d.ldb;
        t.P = M;
        t.wis = 1;
        t.wjs = M;
        t.xbytes = 4 * (ta ? K + (M - 1) * d.lda : M + (K - 1) * d.lda);
        t.ybytes = 4 * (tb ? N + (K - 1) * d.ldb : K + (N - 1) * d.ldb);
    } else {
        // C^T (N x r) = op(B)^T (N x K) op(A)^T (K x r); the slices keep
        // C's own orientation (r x N, ld r).
        r = (int)M;
        t.X = d.B;
        t.xld = d.ldb;
        kcontig = !tb;
        t.Y = d.A;
        t.yks = ta ? 1 : d.lda;
        t.yjs = ta ? d.lda : 1;
        t.P = N;
        t.wis = M;
        t.wjs = 1;
        t.xbytes = 4 * (tb ? N + (K - 1) * d.ldb : K + (N - 1) * d.ldb);
        t.ybytes = 4 * (ta ? K + (M - 1) * d.lda : M + (K - 1) * d.lda);
    }
    t.ws = ws;
    t.K = K;
    t.kc = p.kc;
    if (r < 1 || r > THIN_MAX_R) return hipErrorInvalidValue;
    if (p.gather) {
        // After the S slices of partial sums.
        float* yc = ws + (int64_t)p.splits * M * N;
        const int64_t n = K * r;
        hipLaunchKernelGGL(thin_gather_kernel, dim3((uint32_t)((n + 255) / 256)), dim3(256), 0, s,
                           t.Y, t.yks, t.yjs, K, r, yc);
        t.Y = yc;
        t.yks = r;
        t.yjs = 1;
        t.ybytes = 4 * n;
    }
    t.ymode = t.yks == 1 ? 1 : (t.yks == r && t.yjs == 1 ? 2 : 0);
    switch (r) {
        case 1: launch_thin_r<1>(kcontig, t, p.splits, s); break;
        case 2: launch_thin_r<2>(kcontig, t, p.splits, s); break;
        case 3: launch_thin_r<3>(kcontig, t, p.splits, s); break;
        case 4: launch_thin_r<4>(kcontig, t, p.splits, s); break;
        case 5: launch_thin_r<5>(kcontig, t, p.splits, s); break;
        case 6: launch_thin_r<6>(kcontig, t, p.splits, s); break;
        case 7: launch_thin_r<7>(kcontig, t, p.splits, s); break;
        default: launch_thin_r<8>(kcontig, t, p.splits, s); break;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // The slices are M x N column-major (ld M) in either orientation.
    return launch_splitk_reduce(ws, p.splits, d, s);
}

}  // namespace mgemm
