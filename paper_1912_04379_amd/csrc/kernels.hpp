// kernels.hpp -- internal interface between the host library (mgemm.cpp)
// and the kernel translation units.  Not part of the public C ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "tile_common.hpp"

namespace mgemm {

struct TileConfigInfo {
    int bm, bn, bk, threads;
};

// FP32 MFMA path.
int f32_config_count();
TileConfigInfo f32_config_info(int cfg);
int f32_default_config(int64_t M, int64_t N, int64_t K);
hipError_t launch_f32(int cfg, bool transA, bool transB, const GemmDesc& d,
                      hipStream_t stream);

// BF16x3 split path.
int bf16x3_config_count();
TileConfigInfo bf16x3_config_info(int cfg);
int bf16x3_default_config(int64_t M, int64_t N, int64_t K);
hipError_t launch_bf16x3(int cfg, bool transA, bool transB, const GemmDesc& d,
                         hipStream_t stream);

// Scaled FP16 path: exponent pre-pass and main kernel.
int f16s_config_count();
TileConfigInfo f16s_config_info(int cfg);
int f16s_default_config(int64_t M, int64_t N, int64_t K);
hipError_t launch_f16_exponents(bool transA, bool transB, const GemmDesc& d,
                                int* expA, int* expB, hipStream_t stream);
hipError_t launch_f16s(int cfg, bool transA, bool transB, const GemmDesc& d,
                       hipStream_t stream);

// C <- beta*C (beta == 0 writes zeros without reading C).
hipError_t launch_scale_c(const GemmDesc& d, hipStream_t stream);

}  // namespace mgemm
