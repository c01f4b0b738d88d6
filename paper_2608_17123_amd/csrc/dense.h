// Dense FP64 kernels of the exact GCV tier (kernels_dense.hip).
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>

#include "launch.h"

namespace dbl {

// K = A^T A (lower triangle; diagonal tiles written whole) for a dense n x n
// column-major FP64 A, on the FP64 matrix cores.  A and K must not overlap.
hipError_t launch_gram64(const double* A, double* K, int n, hipStream_t stream);
// Blocks of that launch (128 x 128 tiles on and below the diagonal).
int gram_tiles(int n);
// The DCT products of the spectral tier on grids of at least 128 (m a multiple
// of 128): out = A B, or A B^T with transpose_b (every job of the launch
// alike); one block per 128 x 128 output tile of every job (job and tile
// tables as for the 64 x 64 kernel, jobs added with m / 128 tiles per axis);
// the same result as that kernel, bit for bit.
hipError_t launch_gemm128(const LaunchArgs& la, int transpose_b);
// out[c] = sum_{r < rows} M[r + c ld] v[r] for c < cols (M^T v), FP64, each
// entry summed in a fixed order.
hipError_t launch_gemv_t64(const double* M, size_t ld, int rows, int cols, const double* v,
                           double* out, hipStream_t stream);

}  // namespace dbl
