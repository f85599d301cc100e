// Allocation-free GEMM entry point (sgemm_form_noalloc, include/fewfit.h).
//
// For callers that cannot allocate device memory (code under HIP graph
// capture, tight serving loops, harnesses that forbid hipMalloc): the
// scratch buffers that sgemm_form()'s kernels use (K-split slices of
// partial products, the FP16 forms' block maxima and exponents, the
// pre-split forms' pieces) come from one fixed device array, `scratch`,
// instead of the library's allocated workspaces.
//
// In host code `scratch` names a host-side stand-in, not the device array:
// its device address is fetched once per device with hipGetSymbolAddress
// (with that device current) and only that address is handed to kernels.
// The array lives in this translation unit's own code object, so a process
// holds it on a device only once this entry point has run there.

#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/fewfit.h"
#include "runtime_internal.h"

#define FF_EXPORT extern "C" __attribute__((visibility("default")))

namespace {

constexpr size_t kScratchBytes = FF_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 16;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void* g_scratch[kMaxDevices];  // device address of `scratch`, per device

// Device address of the array on the current device (fetched on the first
// call there), or nullptr with the error recorded.
void* scratch_address(int& rc)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) {
        rc = fewfit_internal::set_error(FF_ERR_HIP, "sgemm_form_noalloc: hipGetDevice failed");
        return nullptr;
    }
    if (dev < 0 || dev >= kMaxDevices) {
        rc = fewfit_internal::set_error(FF_ERR_ARG, "sgemm_form_noalloc: device beyond the supported 16");
        return nullptr;
    }
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_scratch[dev] == nullptr) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || p == nullptr) {
            rc = fewfit_internal::set_error(FF_ERR_HIP, "sgemm_form_noalloc: hipGetSymbolAddress of the scratch "
                                                        "array failed");
            return nullptr;
        }
        g_scratch[dev] = p;
    }
    rc = FF_OK;
    return g_scratch[dev];
}

}  // namespace

FF_EXPORT int sgemm_form_noalloc(int form, int64_t M, int64_t N, int64_t K, float alpha, const float* A,
                                 int64_t lda, const float* B, int64_t ldb, float beta, float* C, int64_t ldc,
                                 void* stream)
{
    int rc = FF_OK;
    void* p = scratch_address(rc);
    if (p == nullptr) return rc;
    return fewfit_internal::gemm_scratch(form, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, stream, p,
                                         kScratchBytes);
}
