// Runtime entry points shared between libfewfit's translation units that
// are not part of its C ABI.
#pragma once

#include <cstddef>
#include <cstdint>

namespace fewfit_internal {

// Record an error for fewfit_last_error() and return `code`.
int set_error(int code, const char* msg);

// sgemm_form() with every scratch buffer its kernels use taken from the
// device memory [scratch, scratch + bytes) on the current device instead of
// the library's allocated workspaces: the FP16 maxima and exponents first,
// then the pre-split pieces, then the K-split slices.  Same dispatch, split
// count and kernels as sgemm_form(), so the same results bit for bit.
// FF_ERR_TOO_LARGE, before any launch, when the call needs more than
// `bytes`.  Neither waits on nor records the workspace ordering event.
int gemm_scratch(int form, int64_t M, int64_t N, int64_t K, float alpha, const float* A, int64_t lda,
                 const float* B, int64_t ldb, float beta, float* C, int64_t ldc, void* stream, void* scratch,
                 size_t bytes);

}  // namespace fewfit_internal
