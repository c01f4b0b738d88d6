// Fused CGLS phase kernels for separable operators on 32 x 32 output tiles,
// one radius bucket per launch (the bodies and their layout: cgls_sep.h).
#include "cgls_sep.h"

namespace dbl {

// Register bounds as for the generic phase kernels: MINW waves per SIMD.
template <typename T, typename S, int RB, int MINW>
__global__ void __launch_bounds__(NTHREADS, MINW)
    k_cgls_p1_sep(const Job* __restrict__ jobs, const uint32_t* __restrict__ tiles) {
  p1_sep_body<T, S, RB>(jobs, tiles);
}
template <typename T, typename S, int RB, int MINW>
__global__ void __launch_bounds__(NTHREADS, MINW)
    k_cgls_p2_sep(const Job* __restrict__ jobs, const uint32_t* __restrict__ tiles) {
  p2_sep_body<T, S, RB>(jobs, tiles);
}

// Dynamic LDS bytes: haloed tile, pass-A result, both tap rows, and in phase
// 2 the tile's gradient part.
size_t cgls_sep_lds(int phase, int precision, int rb) {
  const size_t esz = precision == 1 ? 8 : 4;
  const size_t e = (size_t)(TE + 2 * rb) * (TE + 2 * rb + 1) + (size_t)(TE + 2 * rb) * (TE + 1) +
                   2 * (2 * rb + 1);
  return esz * (e + (phase == 2 ? TE * TE : 0));
}

// Launch over the radius buckets: the register-bounded (wide) variant for
// launches of more tiles than fit the chip at the unconstrained register use,
// as for the generic kernels.
#define DBL_SEP_CASE(KERNEL, T, S, R)                                                     \
  case R:                                                                                 \
    if (wide)                                                                             \
      hipLaunchKernelGGL((KERNEL<T, S, R, sep_wide_waves<T, R>()>), dim3(la.ntiles),       \
                         dim3(NTHREADS), lds, la.stream, la.jobs, la.tiles);              \
    else                                                                                  \
      hipLaunchKernelGGL((KERNEL<T, S, R, waves_per_simd<T, R>()>), dim3(la.ntiles),       \
                         dim3(NTHREADS), lds, la.stream, la.jobs, la.tiles);              \
    break;
#define DBL_SEP_DISPATCH(KERNEL, T, S)                                                    \
  switch (rb) {                                                                           \
    DBL_SEP_CASE(KERNEL, T, S, 2)                                                         \
    DBL_SEP_CASE(KERNEL, T, S, 4)                                                         \
    DBL_SEP_CASE(KERNEL, T, S, 8)                                                         \
    DBL_SEP_CASE(KERNEL, T, S, 12)                                                        \
    DBL_SEP_CASE(KERNEL, T, S, 16)                                                        \
    default: return hipErrorInvalidValue;                                                 \
  }

hipError_t launch_cgls_p1_sep(const LaunchArgs& la, int precision, int rb, bool wide) {
  const size_t lds = cgls_sep_lds(1, precision, rb);
  if (precision == 1) { DBL_SEP_DISPATCH(k_cgls_p1_sep, double, double) }
  else if (precision == 2) { DBL_SEP_DISPATCH(k_cgls_p1_sep, float, bf16s) }
  else { DBL_SEP_DISPATCH(k_cgls_p1_sep, float, float) }
  return hipGetLastError();
}
hipError_t launch_cgls_p2_sep(const LaunchArgs& la, int precision, int rb, bool wide) {
  const size_t lds = cgls_sep_lds(2, precision, rb);
  if (precision == 1) { DBL_SEP_DISPATCH(k_cgls_p2_sep, double, double) }
  else if (precision == 2) { DBL_SEP_DISPATCH(k_cgls_p2_sep, float, bf16s) }
  else { DBL_SEP_DISPATCH(k_cgls_p2_sep, float, float) }
  return hipGetLastError();
}
#undef DBL_SEP_DISPATCH
#undef DBL_SEP_CASE

}  // namespace dbl
