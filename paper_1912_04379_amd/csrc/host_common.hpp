// host_common.hpp -- helpers of the host library shared by its translation
// units (validation, device checks, error reporting).  Internal.
#pragma once
#include <stdint.h>

#include <string>

namespace mgemm {

// Record `msg` as the calling thread's last error and return `status`.
int fail(int status, const std::string& msg);

// 0 for 'N'/'n', 1 for 'T'/'t'/'C'/'c', -1 otherwise.
int trans_code(char t);

// BLAS-order argument check; returns 0 or -(position of the bad argument)
// and a reason in `why`.  Makes no HIP call.
int validate(char transA, char transB, int64_t M, int64_t N, int64_t K, float alpha,
             const float* A, int64_t lda, const float* B, int64_t ldb, float beta,
             const float* C, int64_t ldc, std::string& why);

// True when the referenced part of C overlaps that of A or B.
bool overlaps(int ta, int tb, int64_t M, int64_t N, int64_t K, float alpha, const float* A,
              int64_t lda, const float* B, int64_t ldb, const float* C, int64_t ldc);

// MGEMM_OK when the current device is a gfx950; otherwise an error status.
int check_device(int* out_dev);

// Number of tile configurations of a precision.
int config_count(int precision);

// Configuration recorded by the tuner for exactly this product, or -1.
int recorded_choice(int precision, int ta, int tb, int64_t M, int64_t N, int64_t K);

}  // namespace mgemm
