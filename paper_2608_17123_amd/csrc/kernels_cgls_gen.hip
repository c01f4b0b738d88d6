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

// Launches that mix radius buckets (batched solves): each block runs the body
// of its own job's bucket, the bucket above the operator's radius (read once
// per block, so the branch is the same for all its threads), which is the
// halo the job's own one-bucket launch takes: every job computes what it
// computes alone, bit for bit.  Buckets up to RBMAX in {4, 8, 12}; the LDS of
// a launch is that of RBMAX.
namespace {

template <int PH, typename T, typename S, int RB>
__device__ __forceinline__ void gen_phase(const Job* __restrict__ jobs,
                                          const uint32_t* __restrict__ tiles) {
  if constexpr (PH == 1) p1_sep_body<T, S, RB, true>(jobs, tiles);
  else p2_sep_body<T, S, RB, true>(jobs, tiles);
}

template <int PH, typename T, typename S, int RBMAX>
__device__ __forceinline__ void gen_multi_body(const Job* __restrict__ jobs,
                                               const uint32_t* __restrict__ tiles) {
  static_assert(RBMAX == 4 || RBMAX == 8 || RBMAX == 12, "mixed launches cover buckets 2 .. 12");
  const Job* job = jobs + (tiles[blockIdx.x] >> 16);
  const int R = __builtin_amdgcn_readfirstlane(gview(job->op)->R);
  if (R <= 2) {
    gen_phase<PH, T, S, 2>(jobs, tiles);
  } else if (RBMAX == 4 || R <= 4) {
    gen_phase<PH, T, S, 4>(jobs, tiles);
  } else if constexpr (RBMAX >= 8) {
    if (RBMAX == 8 || R <= 8) gen_phase<PH, T, S, 8>(jobs, tiles);
    else if constexpr (RBMAX == 12) gen_phase<PH, T, S, 12>(jobs, tiles);
  }
}

}  // namespace

template <typename T, typename S, int RBMAX, int MINW>
__global__ void __launch_bounds__(NTHREADS, MINW)
    k_cgls_p1_gmulti(const Job* __restrict__ jobs, const uint32_t* __restrict__ tiles) {
  gen_multi_body<1, T, S, RBMAX>(jobs, tiles);
}
template <typename T, typename S, int RBMAX, int MINW>
__global__ void __launch_bounds__(NTHREADS, MINW)
    k_cgls_p2_gmulti(const Job* __restrict__ jobs, const uint32_t* __restrict__ tiles) {
  gen_multi_body<2, T, S, RBMAX>(jobs, tiles);
}

bool cgls_gen_multi_bucket(int rbmax) { return rbmax == 4 || rbmax == 8 || rbmax == 12; }

#define DBL_GMULTI_CASE(KERNEL, T, S, R)                                                  \
  case R:                                                                                 \
    hipLaunchKernelGGL((KERNEL<T, S, R, waves_per_simd<T, R>()>), dim3(la.ntiles),         \
                       dim3(NTHREADS), lds, la.stream, la.jobs, la.tiles);                \
    break;
#define DBL_GMULTI_DISPATCH(KERNEL, T, S)                                                 \
  switch (rbmax) {                                                                        \
    DBL_GMULTI_CASE(KERNEL, T, S, 4)                                                      \
    DBL_GMULTI_CASE(KERNEL, T, S, 8)                                                      \
    DBL_GMULTI_CASE(KERNEL, T, S, 12)                                                     \
    default: return hipErrorInvalidValue;                                                 \
  }

hipError_t launch_cgls_gen_multi(const LaunchArgs& la, int phase, int precision, int rbmax) {
  const size_t lds = cgls_gen_lds(phase, precision, rbmax);
  if (phase == 1) {
    if (precision == 1) { DBL_GMULTI_DISPATCH(k_cgls_p1_gmulti, double, double) }
    else if (precision == 2) { DBL_GMULTI_DISPATCH(k_cgls_p1_gmulti, float, bf16s) }
    else { DBL_GMULTI_DISPATCH(k_cgls_p1_gmulti, float, float) }
  } else {
    if (precision == 1) { DBL_GMULTI_DISPATCH(k_cgls_p2_gmulti, double, double) }
    else if (precision == 2) { DBL_GMULTI_DISPATCH(k_cgls_p2_gmulti, float, bf16s) }
    else { DBL_GMULTI_DISPATCH(k_cgls_p2_gmulti, float, float) }
  }
  return hipGetLastError();
}
#undef DBL_GMULTI_DISPATCH
#undef DBL_GMULTI_CASE

}  // namespace dbl
