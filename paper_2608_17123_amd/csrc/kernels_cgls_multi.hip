// CGLS phase kernels for launches that mix radius buckets.  Each block runs
// the body of its own job's bucket (the bucket its tables are padded to,
// read once per block, so the branch is the same for all its threads): a job
// computes exactly what a launch of its bucket alone computes, bit for bit,
// while the groups of several buckets share one launch instead of running
// one after another on a chip that each of them alone leaves half idle.
// Buckets up to RBMAX in {4, 8, 12}; the registers and the LDS of a launch
// are those of RBMAX.
#include "cgls_sep.h"

namespace dbl {
namespace {

template <int PH, typename T, typename S, int RB>
__device__ __forceinline__ void phase_body(const Job* __restrict__ jobs,
                                           const uint32_t* __restrict__ tiles) {
  if constexpr (PH == 1) p1_sep_body<T, S, RB>(jobs, tiles);
  else p2_sep_body<T, S, RB>(jobs, tiles);
}

template <int PH, typename T, typename S, int RBMAX>
__device__ __forceinline__ void multi_body(const Job* __restrict__ jobs,
                                           const uint32_t* __restrict__ tiles) {
  static_assert(RBMAX == 4 || RBMAX == 8 || RBMAX == 12, "mixed launches cover buckets 2 .. 12");
  const Job* job = jobs + (tiles[blockIdx.x] >> 16);
  const int rb = __builtin_amdgcn_readfirstlane(gview(job->op)->rb);
  if (rb == 2) {
    phase_body<PH, T, S, 2>(jobs, tiles);
  } else if (RBMAX == 4 || rb == 4) {
    phase_body<PH, T, S, 4>(jobs, tiles);
  } else if constexpr (RBMAX >= 8) {
    if (RBMAX == 8 || rb == 8) phase_body<PH, T, S, 8>(jobs, tiles);
    else if constexpr (RBMAX == 12) phase_body<PH, T, S, 12>(jobs, tiles);
  }
}

}  // namespace

template <typename T, typename S, int RBMAX, int MINW>
__global__ void __launch_bounds__(NTHREADS, MINW)
    k_cgls_p1_multi(const Job* __restrict__ jobs, const uint32_t* __restrict__ tiles) {
  multi_body<1, T, S, RBMAX>(jobs, tiles);
}
template <typename T, typename S, int RBMAX, int MINW>
__global__ void __launch_bounds__(NTHREADS, MINW)
    k_cgls_p2_multi(const Job* __restrict__ jobs, const uint32_t* __restrict__ tiles) {
  multi_body<2, T, S, RBMAX>(jobs, tiles);
}

bool cgls_multi_bucket(int rbmax) { return rbmax == 4 || rbmax == 8 || rbmax == 12; }

// Waves per SIMD.  A mixed launch gathers enough tiles to fill the chip, so
// its kernels are register-bounded like the one-bucket kernels of large
// launches (measured faster than the unbounded ones at every mixed stage of
// the 256-image batch).  Branching between bucket bodies keeps some values
// live across all of them, so the FP32 8-wave bound of the one-bucket
// kernels (64 VGPRs) would spill here: 7 waves (72 VGPRs) up to bucket 8, 6
// (80) with bucket 12, no spills; FP64 as elsewhere.
template <typename T, int RBMAX>
constexpr int multi_wide_waves() {
  return sizeof(T) == 4 ? (RBMAX <= 8 ? 7 : 6) : 2;
}

#define DBL_MULTI_CASE(KERNEL, T, S, R)                                                   \
  case R:                                                                                 \
    hipLaunchKernelGGL((KERNEL<T, S, R, multi_wide_waves<T, R>()>), dim3(la.ntiles),       \
                       dim3(NTHREADS), lds, la.stream, la.jobs, la.tiles);                \
    break;
#define DBL_MULTI_DISPATCH(KERNEL, T, S)                                                  \
  switch (rbmax) {                                                                        \
    DBL_MULTI_CASE(KERNEL, T, S, 4)                                                       \
    DBL_MULTI_CASE(KERNEL, T, S, 8)                                                       \
    DBL_MULTI_CASE(KERNEL, T, S, 12)                                                      \
    default: return hipErrorInvalidValue;                                                 \
  }

hipError_t launch_cgls_multi(const LaunchArgs& la, int phase, int precision, int rbmax) {
  const size_t lds = cgls_sep_lds(phase, precision, rbmax);
  if (phase == 1) {
    if (precision == 1) { DBL_MULTI_DISPATCH(k_cgls_p1_multi, double, double) }
    else if (precision == 2) { DBL_MULTI_DISPATCH(k_cgls_p1_multi, float, bf16s) }
    else { DBL_MULTI_DISPATCH(k_cgls_p1_multi, float, float) }
  } else {
    if (precision == 1) { DBL_MULTI_DISPATCH(k_cgls_p2_multi, double, double) }
    else if (precision == 2) { DBL_MULTI_DISPATCH(k_cgls_p2_multi, float, bf16s) }
    else { DBL_MULTI_DISPATCH(k_cgls_p2_multi, float, float) }
  }
  return hipGetLastError();
}
#undef DBL_MULTI_DISPATCH
#undef DBL_MULTI_CASE

}  // namespace dbl
