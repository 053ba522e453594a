// noalloc.hip -- mgemm_sgemm_ex_noalloc: the SGEMM entry point for callers
// that cannot allocate device memory.  Its workspace is one file-scope
// device array per GPU, fixed at load time; the call itself allocates
// nothing.
//
// In host code the array's name is a host-side stand-in for the symbol,
// not a device address.  Its device address is fetched once per device,
// with that device current, by hipGetSymbolAddress and kept in a per-device
// table; only that address is handed to kernels.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "host_common.hpp"

namespace mgemm {

static __device__ __align__(256) char scratch[MGEMM_NOALLOC_SCRATCH_BYTES];

static std::mutex g_scratch_mu;
static char* g_scratch_ptr[64] = {};

// FixedWorkspace::resolve for the static array: the device address of this
// device's copy of `scratch` (the calling device is current).
static int scratch_address(int dev, char** out) {
    if (dev < 0 || dev >= 64)
        return fail(MGEMM_ERR_UNSUPPORTED, "device index beyond the scratch table");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            return fail(MGEMM_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") +
                                           hipGetErrorString(e));
        }
        g_scratch_ptr[dev] = static_cast<char*>(p);
    }
    *out = g_scratch_ptr[dev];
    return MGEMM_OK;
}

}  // namespace mgemm

using namespace mgemm;

extern "C" int mgemm_sgemm_ex_noalloc(char transA, char transB, int64_t M, int64_t N, int64_t K,
                                      float alpha, const float* A, int64_t lda, const float* B,
                                      int64_t ldb, float beta, float* C, int64_t ldc,
                                      void* stream, int precision, int config) {
    const FixedWorkspace fixed{nullptr, MGEMM_NOALLOC_SCRATCH_BYTES, scratch_address};
    return sgemm_impl(transA, transB, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, stream,
                      precision, config, &fixed);
}
