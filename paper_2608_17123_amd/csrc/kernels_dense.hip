// Dense FP64 kernels of the exact GCV tier (Sec. 3: the pencil of A^T A and
// A^T A + D^T D on one level, n = m^2 unknowns, up to n = 16384).
//
// k_gram64_mfma: K = A^T A for a dense n x n column-major A, lower triangle
// (tiles on and below the diagonal; a diagonal tile is written whole), on the
// FP64 matrix cores (v_mfma_f64_16x16x4f64).  One block per 128 x 128 tile:
// each 16-row slab of the two column panels it needs (columns i0.. and j0..
// of A) is staged in LDS (the next one loaded into registers meanwhile), and wave w computes the 64 x 64 quadrant (rows
// 64 (w % 2), columns 64 (w / 2)) as 4 x 4 accumulators of 16 x 16, four
// k-steps of 4 per slab.  Operand lanes as for the DCT GEMM: the A fragment of
// a lane is (row 16 u + lane % 16, k 4 q + lane / 16) of A^T, the B fragment
// (k 4 q + lane / 16, column 16 v + lane % 16) of A; result element e of a
// lane is row lane / 16 + 4 e, column lane % 16 of its 16 x 16 block (the
// FP64 instruction interleaves its result rows; checked on the device).  The
// tile list is cut into eight contiguous chunks, one per XCD (blocks are
// dealt to the XCDs round robin), so the blocks sharing an L2 work on
// neighbouring tiles, which share column panels.
//
// k_gemv_t64: out[c] = sum_r M[r + c ld] v[r] (M^T v) for the columns c of a
// column-major M, one block per column, FP64 with a fixed-order block sum.
#include "common.h"
#include "dense.h"

namespace dbl {

typedef double dbl4 __attribute__((ext_vector_type(4)));

constexpr int GR_TS = 128;  // tile edge
constexpr int GR_KS = 16;   // slab depth
constexpr int GR_LD = GR_TS + 1;

__device__ __forceinline__ void gram_tile_of(int t, int& ti, int& tj) {
  // t -> (ti, tj), ti >= tj, t = ti (ti + 1) / 2 + tj
  int i = (int)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
  while ((long long)i * (i + 1) / 2 > t) --i;
  while ((long long)(i + 1) * (i + 2) / 2 <= t) ++i;
  ti = i;
  tj = t - i * (i + 1) / 2;
}

__global__ void __launch_bounds__(NTHREADS, 2) k_gram64_mfma(const double* __restrict__ A,
                                                          double* __restrict__ K, int n,
                                                          int ntile) {
  __shared__ double As[GR_KS][GR_LD];
  __shared__ double Bs[GR_KS][GR_LD];
  // XCD chunks: block b runs on XCD b % 8 and takes position b / 8 of its chunk
  const int b = blockIdx.x, q = ntile / 8, rem = ntile % 8, x = b % 8;
  const int t = x * q + min(x, rem) + b / 8;
  int ti, tj;
  gram_tile_of(t, ti, tj);
  const int i0 = ti * GR_TS, j0 = tj * GR_TS;
  const bool diag = ti == tj;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int wr = 64 * (wid & 1), wc = 64 * (wid >> 1);
  const int fr = lane & 15, fk = lane >> 4;
  dbl4 acc[4][4];
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[u][v] = dbl4{0.0, 0.0, 0.0, 0.0};
  // Slab rows k0 .. k0 + 15 of the column panels; 16 consecutive rows of a
  // column are contiguous, so element p of a thread is row idx % 16 of
  // column idx / 16, idx = threadIdx.x + p NTHREADS.  The next slab is loaded
  // into registers while the MFMAs run on the current one (the barriers
  // around the LDS exchange order LDS only, so those loads stay in flight).
  constexpr int PER = GR_KS * GR_TS / NTHREADS;
  double pa[PER], pb[PER];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int p = 0; p < PER; ++p) {
      const int idx = threadIdx.x + p * NTHREADS, k = idx % GR_KS, r = idx / GR_KS;
      const int gk = k0 + k;
      pa[p] = (gk < n && i0 + r < n) ? A[gk + (size_t)(i0 + r) * n] : 0.0;
      if (!diag) pb[p] = (gk < n && j0 + r < n) ? A[gk + (size_t)(j0 + r) * n] : 0.0;
    }
  };
  fetch(0);
  for (int k0 = 0; k0 < n; k0 += GR_KS) {
#pragma unroll
    for (int p = 0; p < PER; ++p) {
      const int idx = threadIdx.x + p * NTHREADS, k = idx % GR_KS, r = idx / GR_KS;
      As[k][r] = pa[p];
      if (!diag) Bs[k][r] = pb[p];
    }
    lds_barrier();
    if (k0 + GR_KS < n) fetch(k0 + GR_KS);
    const double(*Bp)[GR_LD] = diag ? As : Bs;
#pragma unroll
    for (int s = 0; s < GR_KS / 4; ++s) {
      const int k = 4 * s + fk;
      double a[4], bb[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        a[u] = As[k][wr + 16 * u + fr];
        bb[u] = Bp[k][wc + 16 * u + fr];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v)
          acc[u][v] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u], bb[v], acc[u][v], 0, 0, 0);
    }
    lds_barrier();
  }
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int r = i0 + wr + 16 * u + fk + 4 * e, c = j0 + wc + 16 * v + fr;
        if (r < n && c < n) K[r + (size_t)c * n] = acc[u][v][e];
      }
}

__global__ void __launch_bounds__(NTHREADS) k_gemv_t64(const double* __restrict__ M, size_t ld,
                                                       int rows, const double* __restrict__ v,
                                                       double* __restrict__ out) {
  __shared__ double red[4];
  const double* __restrict__ col = M + (size_t)blockIdx.x * ld;
  double s = 0.0;
  for (int r = threadIdx.x; r < rows; r += NTHREADS) s = fma(col[r], v[r], s);
  double t[1] = {s};
  block_sum<1>(t, red);
  if (threadIdx.x == 0) out[blockIdx.x] = t[0];
}

// k_gemm128_mfma: the DCT products of the spectral GCV tier on grids of at
// least 128 (m a multiple of 128): out = A B (i0 = 0) or A B^T (i0 = 1), m x m
// FP64 column-major, v[0] = A, v[1] = B, v[2] = out (the launch's jobs all
// take the same form, which is a template parameter); one block per 128 x 128
// output tile of a job (job and tile tables as for every batched launch).
// The tile work is the Gram kernel's (slabs of 16 in LDS, the next one
// prefetched, 4 x 4 accumulators per wave); every output element takes its
// k terms in the same order as in the 64 x 64 kernel (slabs of 16, four
// steps of 4), so both give the same result bit for bit.
template <bool TB>
__global__ void __launch_bounds__(NTHREADS, 2) k_gemm128_mfma(const Job* __restrict__ jobs,
                                                             const uint32_t* __restrict__ tiles) {
  __shared__ double As[GR_KS][GR_LD];
  __shared__ double Bs[GR_KS][GR_LD];
  const Job* job; int ti, tj, tix;
  decode_tile(jobs, tiles, job, ti, tj, tix);
  const int m = job->m;
  const int i0 = ti * GR_TS, j0 = tj * GR_TS;
  const double* __restrict__ A = static_cast<const double*>(job->v[0]);
  const double* __restrict__ B = static_cast<const double*>(job->v[1]);
  double* __restrict__ C = static_cast<double*>(job->v[2]);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int wr = 64 * (wid & 1), wc = 64 * (wid >> 1);
  const int fr = lane & 15, fk = lane >> 4;
  dbl4 acc[4][4];
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[u][v] = dbl4{0.0, 0.0, 0.0, 0.0};
  // element p of a thread: A (and B^T) rows are contiguous along the tile
  // (row idx % 128 of slab row idx / 128); B columns along k (k idx % 16 of
  // column idx / 16)
  constexpr int PER = GR_KS * GR_TS / NTHREADS;
  double pa[PER], pb[PER];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int p = 0; p < PER; ++p) {
      const int idx = threadIdx.x + p * NTHREADS;
      const int r = idx % GR_TS, k = idx / GR_TS;
      pa[p] = A[(i0 + r) + (size_t)(k0 + k) * m];
      if constexpr (TB) {
        pb[p] = B[(j0 + r) + (size_t)(k0 + k) * m];
      } else {
        const int kb = idx % GR_KS, rb = idx / GR_KS;
        pb[p] = B[(k0 + kb) + (size_t)(j0 + rb) * m];
      }
    }
  };
  fetch(0);
  for (int k0 = 0; k0 < m; k0 += GR_KS) {
#pragma unroll
    for (int p = 0; p < PER; ++p) {
      const int idx = threadIdx.x + p * NTHREADS;
      As[idx / GR_TS][idx % GR_TS] = pa[p];
      if constexpr (TB) Bs[idx / GR_TS][idx % GR_TS] = pb[p];
      else Bs[idx % GR_KS][idx / GR_KS] = pb[p];
    }
    lds_barrier();
    if (k0 + GR_KS < m) fetch(k0 + GR_KS);
#pragma unroll
    for (int s = 0; s < GR_KS / 4; ++s) {
      const int k = 4 * s + fk;
      double a[4], bb[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        a[u] = As[k][wr + 16 * u + fr];
        bb[u] = Bs[k][wc + 16 * u + fr];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v)
          acc[u][v] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u], bb[v], acc[u][v], 0, 0, 0);
    }
    lds_barrier();
  }
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int r = i0 + wr + 16 * u + fk + 4 * e, c = j0 + wc + 16 * v + fr;
        C[r + (size_t)c * m] = acc[u][v][e];
      }
}

hipError_t launch_gemm128(const LaunchArgs& la, int transpose_b) {
  if (transpose_b)
    hipLaunchKernelGGL(k_gemm128_mfma<true>, dim3(la.ntiles), dim3(NTHREADS), 0, la.stream,
                       la.jobs, la.tiles);
  else
    hipLaunchKernelGGL(k_gemm128_mfma<false>, dim3(la.ntiles), dim3(NTHREADS), 0, la.stream,
                       la.jobs, la.tiles);
  return hipGetLastError();
}

int gram_tiles(int n) {
  const int t = (n + GR_TS - 1) / GR_TS;
  return t * (t + 1) / 2;
}

hipError_t launch_gram64(const double* A, double* K, int n, hipStream_t stream) {
  if (n <= 0) return hipErrorInvalidValue;
  const int nt = gram_tiles(n);
  hipLaunchKernelGGL(k_gram64_mfma, dim3(nt), dim3(NTHREADS), 0, stream, A, K, n, nt);
  return hipGetLastError();
}

hipError_t launch_gemv_t64(const double* M, size_t ld, int rows, int cols, const double* v,
                           double* out, hipStream_t stream) {
  if (rows <= 0 || cols <= 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_gemv_t64, dim3(cols), dim3(NTHREADS), 0, stream, M, ld, rows, v, out);
  return hipGetLastError();
}

}  // namespace dbl
