// Mean structural similarity (SSIM), the second quality measure of Sec. 5,
// of images against a reference image: per pixel the Gaussian-window local
// means, variances and covariance of the two images (edge pixels replicated
// outside the image), combined with c1 = (0.01 L)^2 and c2 = (0.03 L)^2, and
// averaged over the image.  Everything runs in FP64 from the stored values.
//
// k_ssim: one block per 32 x 32 output tile.  The tile and its halo of both
// images (clamped indices: replication) are staged in LDS as FP64; thread
// (row r, column group g) slides down the halo columns of its four output
// columns, forms the five window sums along axis 0 for each halo column in
// registers and adds them, weighted, to the outputs they reach along axis 1
// (the window is the outer product of two 1-D windows).  The block's SSIM
// total goes to one FP64 partial; k_ssim_fin adds a job's partials in a
// fixed order and divides by m^2.
//
// Job fields: m; v[0] the reference (FP64, column-major), v[1] the image
// (T), v[2] the 2R + 1 window taps (FP64), v[3] the job's result (one
// double); i0 = R; p0 = c1, p1 = c2; pw the tile partials (k_ssim); pr[0] the
// same partials and i1 their count (k_ssim_fin).
#include "common.h"
#include "metrics.h"

namespace dbl {

constexpr int SS_TE = 32;        // output tile edge
constexpr int SS_CPT = 4;        // output columns per thread
constexpr int SS_RMAX = 16;      // largest window radius
static_assert(SS_TE * (SS_TE / SS_CPT) == NTHREADS, "one thread per (row, column group)");

__host__ __device__ constexpr int ssim_ld(int R) { return SS_TE + 2 * R; }
size_t ssim_lds(int R) { return 2 * sizeof(double) * (size_t)ssim_ld(R) * ssim_ld(R); }

template <typename T>
__global__ void __launch_bounds__(NTHREADS) k_ssim(const Job* __restrict__ jobs,
                                                   const uint32_t* __restrict__ tiles) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ double gs[2 * SS_RMAX + 1];
  __shared__ double red[4];
  const Job* job; int ti, tj, tix;
  decode_tile(jobs, tiles, job, ti, tj, tix);
  const int m = job->m, R = job->i0, LD = ssim_ld(R), NW = 2 * R + 1;
  const int i0 = ti * SS_TE, j0 = tj * SS_TE;
  const double* __restrict__ ref = static_cast<const double*>(job->v[0]);
  const T* __restrict__ x = static_cast<const T*>(job->v[1]);
  const double* __restrict__ taps = static_cast<const double*>(job->v[2]);
  double* As = reinterpret_cast<double*>(smem);
  double* Bs = As + LD * LD;
  for (int k = threadIdx.x; k < NW; k += NTHREADS) gs[k] = taps[k];
  // haloed tile, column-major with leading dimension LD; rows and columns
  // outside [0, m) take the nearest edge pixel
  for (int o = threadIdx.x; o < LD * LD; o += NTHREADS) {
    const int r = o % LD, c = o / LD;
    const int gi = min(max(i0 - R + r, 0), m - 1), gj = min(max(j0 - R + c, 0), m - 1);
    const size_t g = gi + (size_t)gj * m;
    As[o] = ref[g];
    Bs[o] = (double)x[g];
  }
  __syncthreads();
  const int r = threadIdx.x % SS_TE, c0 = (threadIdx.x / SS_TE) * SS_CPT;
  // acc[u][*]: window sums of a, b, a^2, b^2, a b at output (r, c0 + u)
  double acc[SS_CPT][5];
#pragma unroll
  for (int u = 0; u < SS_CPT; ++u)
#pragma unroll
    for (int s = 0; s < 5; ++s) acc[u][s] = 0.0;
  for (int c = 0; c < SS_CPT - 1 + NW; ++c) {
    const double* Ac = As + (c0 + c) * LD + r;
    const double* Bc = Bs + (c0 + c) * LD + r;
    double sa = 0.0, sb = 0.0, saa = 0.0, sbb = 0.0, sab = 0.0;
    for (int k = 0; k < NW; ++k) {
      const double a = Ac[k], b = Bc[k], w = gs[k];
      const double wa = w * a, wb = w * b;
      sa += wa;
      sb += wb;
      saa = fma(wa, a, saa);
      sbb = fma(wb, b, sbb);
      sab = fma(wa, b, sab);
    }
    // halo column c0 + c reaches output column c0 + u with tap c - u
#pragma unroll
    for (int u = 0; u < SS_CPT; ++u) {
      const int k = c - u;
      if (k < 0 || k >= NW) continue;
      const double w = gs[k];
      acc[u][0] = fma(w, sa, acc[u][0]);
      acc[u][1] = fma(w, sb, acc[u][1]);
      acc[u][2] = fma(w, saa, acc[u][2]);
      acc[u][3] = fma(w, sbb, acc[u][3]);
      acc[u][4] = fma(w, sab, acc[u][4]);
    }
  }
  const double c1 = job->p0, c2 = job->p1;
  double tot = 0.0;
#pragma unroll
  for (int u = 0; u < SS_CPT; ++u) {
    if (i0 + r >= m || j0 + c0 + u >= m) continue;
    const double ma = acc[u][0], mb = acc[u][1];
    const double va = acc[u][2] - ma * ma, vb = acc[u][3] - mb * mb, cv = acc[u][4] - ma * mb;
    tot += ((2.0 * ma * mb + c1) * (2.0 * cv + c2)) / ((ma * ma + mb * mb + c1) * (va + vb + c2));
  }
  double v[1] = {tot};
  put_partials<1>(job->pw, tix, v, red);
}

// One block per job: the mean over the image.
__global__ void __launch_bounds__(NTHREADS) k_ssim_fin(const Job* __restrict__ jobs,
                                                       const uint32_t* __restrict__ tiles) {
  __shared__ double red[4];
  __shared__ double bc;
  const Job* job = jobs + (tiles[blockIdx.x] >> 16);
  const double s = sum_partials<1>(job->pr[0], job->i1, 0, red, &bc);
  if (threadIdx.x == 0)
    *static_cast<double*>(job->v[3]) = s / ((double)job->m * (double)job->m);
}

hipError_t launch_ssim(const LaunchArgs& la, int precision, int R) {
  if (R < 0 || R > SS_RMAX) return hipErrorInvalidValue;
  const size_t lds = ssim_lds(R);
  if (precision == 1)
    hipLaunchKernelGGL(k_ssim<double>, dim3(la.ntiles), dim3(NTHREADS), lds, la.stream, la.jobs,
                       la.tiles);
  else
    hipLaunchKernelGGL(k_ssim<float>, dim3(la.ntiles), dim3(NTHREADS), lds, la.stream, la.jobs,
                       la.tiles);
  return hipGetLastError();
}

hipError_t launch_ssim_fin(const LaunchArgs& la) {
  hipLaunchKernelGGL(k_ssim_fin, dim3(la.ntiles), dim3(NTHREADS), 0, la.stream, la.jobs,
                     la.tiles);
  return hipGetLastError();
}

}  // namespace dbl
