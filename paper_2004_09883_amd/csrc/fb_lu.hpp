// fb_lu.hpp -- the LU function block: shared between fb_lu.hip and the C ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fb {

constexpr int LU_NB = 16;            // panel width (columns factored per panel)
constexpr int64_t LU_MAX_N = 2048;   // the panel kernel holds 4 rows per thread of one 512-thread workgroup

// Blocked LU with partial pivoting of the row-major n x n matrix a (row
// stride lda) in place; ipiv[j] = row swapped with row j at step j; info[0]
// = first j + 1 with a zero pivot, else 0.  Stream-ordered, no allocation.
hipError_t launch_lu(double *a, int64_t n, int64_t lda, int32_t *ipiv, int32_t *info, hipStream_t st);

}  // namespace fb
