// Dense FP64 kernels of the exact GCV tier (kernels_dense.hip).
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>

namespace dbl {

// K = A^T A (lower triangle; diagonal tiles written whole) for a dense n x n
// column-major FP64 A, on the FP64 matrix cores.  A and K must not overlap.
hipError_t launch_gram64(const double* A, double* K, int n, hipStream_t stream);
// Blocks of that launch (128 x 128 tiles on and below the diagonal).
int gram_tiles(int n);
// out[c] = sum_{r < rows} M[r + c ld] v[r] for c < cols (M^T v), FP64, each
// entry summed in a fixed order.
hipError_t launch_gemv_t64(const double* M, size_t ld, int rows, int cols, const double* v,
                           double* out, hipStream_t stream);

}  // namespace dbl
