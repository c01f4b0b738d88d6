// Fused CGLS phase kernels for general (non-separable) operators on 32 x 32
// output tiles, grids of at least 32: the bodies of cgls_sep.h with the
// convolution over 2-D class tap lists (GEN).  Every sum and partial is the
// generic kernels' (same pixel set and order per thread, same tap order), so
// the two paths agree bit for bit, as the separable ones do.
#include "cgls_sep.h"

namespace dbl {

template <typename T, typename S, int RB, int MINW>
__global__ void __launch_bounds__(NTHREADS, MINW)
    k_cgls_p1_gen(const Job* __restrict__ jobs, const uint32_t* __restrict__ tiles) {
  p1_sep_body<T, S, RB, true>(jobs, tiles);
}
template <typename T, typename S, int RB, int MINW>
__global__ void __launch_bounds__(NTHREADS, MINW)
    k_cgls_p2_gen(const Job* __restrict__ jobs, const uint32_t* __restrict__ tiles) {
  p2_sep_body<T, S, RB, true>(jobs, tiles);
}

// Dynamic LDS bytes: haloed tile, the staged interior list (offsets, then
// values) and in phase 2 the tile's gradient part.
size_t cgls_gen_lds(int phase, int precision, int rb) {
  const size_t esz = precision == 1 ? 8 : 4;
  const size_t xs = (size_t)(TE + 2 * rb) * (TE + 2 * rb + 1);
  const size_t gt = (size_t)(2 * rb + 1) * (2 * rb + 1), gti = (gt + 1) & ~size_t(1);
  return esz * xs + 4 * gti + esz * gt + (phase == 2 ? esz * TE * TE : 0);
}

// One variant per bucket: without a tighter bound the FP32 kernels already
// take 76-84 VGPRs (5-6 waves per SIMD, no spills); the 8-wave bound of the
// separable kernels would spill here.
#define DBL_GEN_CASE(KERNEL, T, S, R)                                                     \
  case R:                                                                                 \
    hipLaunchKernelGGL((KERNEL<T, S, R, waves_per_simd<T, R>()>), dim3(la.ntiles),         \
                       dim3(NTHREADS), lds, la.stream, la.jobs, la.tiles);                \
    break;
#define DBL_GEN_DISPATCH(KERNEL, T, S)                                                    \
  switch (rb) {                                                                           \
    DBL_GEN_CASE(KERNEL, T, S, 2)                                                         \
    DBL_GEN_CASE(KERNEL, T, S, 4)                                                         \
    DBL_GEN_CASE(KERNEL, T, S, 8)                                                         \
    DBL_GEN_CASE(KERNEL, T, S, 12)                                                        \
    DBL_GEN_CASE(KERNEL, T, S, 16)                                                        \
    default: return hipErrorInvalidValue;                                                 \
  }

hipError_t launch_cgls_p1_gen(const LaunchArgs& la, int precision, int rb) {
  const size_t lds = cgls_gen_lds(1, precision, rb);
  if (precision == 1) { DBL_GEN_DISPATCH(k_cgls_p1_gen, double, double) }
  else if (precision == 2) { DBL_GEN_DISPATCH(k_cgls_p1_gen, float, bf16s) }
  else { DBL_GEN_DISPATCH(k_cgls_p1_gen, float, float) }
  return hipGetLastError();
}
hipError_t launch_cgls_p2_gen(const LaunchArgs& la, int precision, int rb) {
  const size_t lds = cgls_gen_lds(2, precision, rb);
  if (precision == 1) { DBL_GEN_DISPATCH(k_cgls_p2_gen, double, double) }
  else if (precision == 2) { DBL_GEN_DISPATCH(k_cgls_p2_gen, float, bf16s) }
  else { DBL_GEN_DISPATCH(k_cgls_p2_gen, float, float) }
  return hipGetLastError();
}
#undef DBL_GEN_DISPATCH
#undef DBL_GEN_CASE

}  // namespace dbl
