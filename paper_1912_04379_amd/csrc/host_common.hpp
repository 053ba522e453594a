// host_common.hpp -- helpers of the host library shared by its translation
// units (validation, device checks, error reporting).  Internal.
#pragma once
#include <stdint.h>

#include <functional>
#include <string>
#include <vector>

#include "mgemm.h"

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

// Byte range [lo, hi) of the referenced part of a stored array, and the
// problem it belongs to.
struct Extent {
    uintptr_t lo, hi;
    int64_t owner;
};
Extent extent_of(const void* p, int64_t rows, int64_t cols, int64_t ld, int64_t owner);

// A grouped batch's aliasing rule: no C extent (cs) may overlap another, or
// any operand extent (ab).  Returns the owner of an offending C (with
// *kind = 1 for C against C, 2 for C against an operand), or -1.
int64_t batch_alias(std::vector<Extent> cs, const std::vector<Extent>& ab, int* kind);

// MGEMM_OK when the current device is a gfx950; otherwise an error status.
int check_device(int* out_dev);

// Compute units of device dev (cached; 0 if unknown).
int device_cus(int dev);

// Number of tile configurations of a precision.
int config_count(int precision);

// Configuration recorded by the tuner for exactly this product, or -1.
int recorded_choice(int precision, int ta, int tb, int64_t M, int64_t N, int64_t K);

// Every recorded single-call choice: fn(precision, ta, tb, M, N, K, config).
void for_each_choice(
    const std::function<void(int, int, int, int64_t, int64_t, int64_t, int)>& fn);

// Tuning cache file (tune_cache.cpp): the current device's key, a grouped
// batch's key, and lookup / append of a batch's bucket configurations.
void device_key(std::string& arch, int& cus);
uint64_t batch_key(const mgemm_problem* probs, int64_t count);
bool grouped_cache_lookup(const char* path, int precision, uint64_t key, int* configs);
bool grouped_cache_store(const char* path, int precision, uint64_t key, const int* configs);

// A device buffer of `cap` bytes that a call uses as its workspace instead
// of memory from the library's pool.  When `base` is NULL, `resolve` gives
// it for the current device `dev` (called once the arguments have been
// checked; returns MGEMM_OK or an error status).
struct FixedWorkspace {
    char* base;
    int64_t cap;
    int (*resolve)(int dev, char** base);
};

// The SGEMM entry points' common body: validation, quick returns,
// configuration choice and launches.  `fixed` == nullptr takes workspace
// from the pool; otherwise configurations whose workspace exceeds
// fixed->cap run as they would without one (see mgemm_sgemm_ex_noalloc).
// `act` / `aux`: the fused activation (MGEMM_ACT_*) and its second operand.
int sgemm_impl(char transA, char transB, int64_t M, int64_t N, int64_t K, float alpha,
               const float* A, int64_t lda, const float* B, int64_t ldb, float beta, float* C,
               int64_t ldc, void* stream, int precision, int config,
               const FixedWorkspace* fixed, int act = MGEMM_ACT_NONE,
               const float* aux = nullptr);

// True when MGEMM_FAULT=alloc asks every workspace, packed-operand or plan
// allocation to fail (a test hook for the MGEMM_ERR_ALLOC paths).
bool fault_injected();

// MGEMM_LOG: whether call logging is on, and one printf-style line of it.
bool log_enabled();
void log_line(const char* fmt, ...) __attribute__((format(printf, 1, 2)));

}  // namespace mgemm
