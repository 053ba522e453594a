// kernels.hpp -- internal interface between the host library (mgemm.cpp)
// and the kernel translation units.  Not part of the public C ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rules.hpp"
#include "tile_common.hpp"

namespace mgemm {

struct TileConfigInfo {
    int bm, bn, bk, threads;
};

// FP32 MFMA path.
int f32_config_count();
TileConfigInfo f32_config_info(int cfg);
hipError_t launch_f32(int cfg, bool transA, bool transB, const GemmDesc& d,
                      hipStream_t stream);
// FP32 small-product kernel (16 x 16 tiles, k split over 4 waves); needs
// buffer_path_ok(d).
hipError_t launch_small(bool transA, bool transB, const GemmDesc& d, hipStream_t stream);
// FP32 configuration 10 (F32_TAIL_CONFIG): 256 x 256 x 32 tiles in whole
// rounds of one per CU (`cus` CUs), 128 x 128 tiles in the tail; needs
// buffer_path_ok(d).
hipError_t launch_f32_tail(bool transA, bool transB, const GemmDesc& d, int cus,
                           hipStream_t stream);
// FP32 configuration 11 (F32_SPLITK_CONFIG, plan in rules.hpp).
// Needs buffer_path_ok(d), p.splits >= 2 and f32_splitk_workspace_bytes()
// of workspace.
hipError_t launch_f32_splitk(bool transA, bool transB, const GemmDesc& d, const SplitKPlan& p,
                             float* workspace, hipStream_t stream);
// The second kernel of every split-K path: C <- alpha * sum of the `splits`
// M x N slices of `ws` (ld M), added in order s = 0..splits-1, + beta * C.
hipError_t launch_splitk_reduce(const float* ws, int splits, const GemmDesc& d,
                                hipStream_t stream);

// BF16x3 split path.
int bf16x3_config_count();
TileConfigInfo bf16x3_config_info(int cfg);
hipError_t launch_bf16x3(int cfg, bool transA, bool transB, const GemmDesc& d,
                         hipStream_t stream);

// Scaled FP16 path: exponent pre-pass and main kernel.
int f16s_config_count();
TileConfigInfo f16s_config_info(int cfg);
// FP16 exponent pre-pass; `partial` is scratch of f16_partial_floats().
int64_t f16_partial_floats(int64_t M, int64_t N, int64_t K);
hipError_t launch_f16_exponents(bool transA, bool transB, const GemmDesc& d,
                                int* expA, int* expB, float* partial, hipStream_t stream);
hipError_t launch_f16s(int cfg, bool transA, bool transB, const GemmDesc& d,
                       hipStream_t stream);
// The thin path (plan in rules.hpp): the large operand streamed once in S
// pieces of kc along k into S*M*N floats of workspace, then
// launch_splitk_reduce (see sgemm_thin.hip).
hipError_t launch_thin(bool transA, bool transB, const GemmDesc& d, const ThinPlan& p,
                       float* workspace, hipStream_t stream);

// Split-K of either 16-bit form (the LOWP_SPLITK_CONFIG configuration): the
// pieces of plan p run as in-staging tiles (64 x 64 when p.small_tile, else
// 128 x 128) into `workspace` (S*M*N floats), then launch_splitk_reduce.
// For the FP16 form d.expA / d.expB already hold the panel exponents of the
// whole K.  Needs buffer_path_ok(d), d.M <= MAX_BUF_LD and p.splits >= 2.
hipError_t launch_lowp_splitk(bool bf16x3, bool transA, bool transB, const GemmDesc& d,
                              const SplitKPlan& p, float* workspace, hipStream_t stream);
// The same split of the FP16 form with its pieces on packed operands (the
// pipelined packed 128 x 128 tile), bitwise equal to launch_lowp_splitk:
// op(A) and op(B) are packed once into `pack_ws` (f16s_packed_splitk_bytes)
// and the pieces go to `slices` (S*M*N floats).  Applies where
// f16s_packed_splitk_supported (128 x 128 pieces, kc a multiple of the
// block depth, lane offsets within 31 bits).
int64_t f16s_packed_splitk_bytes(int64_t M, int64_t N, int64_t K);
bool f16s_packed_splitk_supported(const SplitKPlan& p, int64_t M, int64_t N, int64_t K);
hipError_t launch_f16s_packed_splitk(bool transA, bool transB, const GemmDesc& d,
                                     const SplitKPlan& p, char* pack_ws, float* slices,
                                     hipStream_t stream);

// Pre-packed 16-bit path (direct-to-LDS engine).  Configuration c of this
// family is configuration LOWP_INSTAGE_CONFIGS + c of the BF16x3 and FP16
// forms (those whose BF16x3 LDS ring exceeds a CU are FP16 only).  The caller provides `workspace` of
// packed_workspace_bytes(); for the FP16 form d.expA / d.expB must already
// hold the panel exponents.
int packed_config_count();
TileConfigInfo packed_config_info(int cfg);
int64_t packed_workspace_bytes(bool bf16x3, int cfg, int64_t M, int64_t N, int64_t K);
bool packed_supported(bool bf16x3, int cfg, int64_t M, int64_t N, int64_t K);
hipError_t launch_packed(bool bf16x3, int cfg, bool transA, bool transB, const GemmDesc& d,
                         char* workspace, hipStream_t stream);
// One operand packed on its own (the pre-packed B entry points): bytes of
// op(X) as P x K in kw-deep blocks, the pack launch (kcontig: op(X) is
// contiguous along k), the block depth of a packed configuration (0 for an
// unknown one), and the main kernel with op(B) already packed.
int64_t packed_operand_bytes(bool bf16x3, int kw, int64_t P, int64_t K);
// FP32 pre-packed B: op(B) (K x N; B stored K x N for !tb, N x K for tb,
// leading dimension ldb) into a column-major K x N array at `out` with
// leading dimension ldp >= K (k contiguous, the FP32 kernels' 16-byte-load
// layout).  Rows k >= K of `out` are not written.
hipError_t launch_f32_pack_b(bool tb, const float* B, int64_t ldb, int64_t K, int64_t N,
                             float* out, int64_t ldp, hipStream_t s);
hipError_t launch_pack_operand(bool bf16x3, int kw, bool kcontig, const float* X, int64_t ld,
                               int64_t P, int64_t K, char* hi, char* lo, const int* expo,
                               hipStream_t stream);
int packed_config_kw(int cfg);
hipError_t launch_packed_b_ready(bool bf16x3, int cfg, bool transA, const GemmDesc& d,
                                 char* a_workspace, const char* b_hi, const char* b_lo,
                                 hipStream_t stream);

// C <- beta*C (beta == 0 writes zeros without reading C).
hipError_t launch_scale_c(const GemmDesc& d, hipStream_t stream);

}  // namespace mgemm
