// GCV kernels (Sec. 3, eqs. (xgamma), (GCV)), spectral tier: the GCV
// function of the subproblem evaluated in the orthonormal 2-D DCT-II basis,
// which diagonalises L^T L (Neumann Laplacian) exactly and the blur for its
// reflexive-boundary counterpart.  All arithmetic is FP64.
//
//   s_k  = a_k^2                 a_k: cosine symbol of the interior kernel
//   lp_k = wbar^2 (l(k0) + l(k1)), l(k) = 4 sin^2(pi k / (2 m))
//   e_k  = (a_k c^_k - lp_k b^_k)^2, b^ = DCT(b), c^ = DCT(L^T c)
//   resid(g) = g^2 sum_k e_k / (s_k + g lp_k)^2,  trace(g) = sum_k s_k / (s_k + g lp_k)
//   GCV(g) = resid(g) / (n - trace(g))^2
//
// The minimiser follows the paper's recipe: a log-spaced grid (bounds from
// the smallest and largest s/lp, lower bound clamped to 14 decades below the
// upper), then Brent's method (golden section with parabolic steps) on the
// interval around the grid minimum, xtol 1e-8 in log10(g), at most 100 steps.
// EXACT tier (levels with n <= 4096): the data are the generalised
// eigenvalues nu_k of the pencil (A^T A, A^T A + D^T D) with B-orthonormal
// eigenvectors V, f = V^T A^T b, g = V^T D^T c and ||b||^2 (built on the
// host side by gcv.cpp), and with den_k = nu_k + g (1 - nu_k),
// y_k = (f_k + g g_k) / den_k:
//   resid(g) = ||b||^2 - 2 sum f_k y_k + sum nu_k y_k^2,
//   trace(g) = sum nu_k / den_k,  GCV(g) = resid(g) / (n - trace(g))^2,
// grid bounds from log10(nu / (1 - nu)) over 0 < nu < 1 - 1e-10.  The same
// grid and Brent kernels evaluate both tiers (Job flag F_EXACT).
// Brent runs as a device state machine over a fixed number of launches: each
// launch sums the previous evaluation's per-tile partials (every block, same
// order), advances the state identically in every block, persists it (tile 0
// of the job) in the copy the next launch reads, and evaluates GCV at the new
// point.  State copies and partial arrays alternate between launches, so no
// block ever reads what another block of the same launch writes.
#include <algorithm>

#include "launch.h"
#include "stencil.h"

namespace dbl {

// v slots for GCV jobs
enum : int {
  G_B = 0,     // level data b (device precision)
  G_W = 1,     // IRLS weights or null
  G_C1 = 2,    // shift c = c1 - c2 (or c1), or null
  G_C2 = 3,
  G_IN = 4,    // FP64 n
  G_TMP = 5,   // FP64 n
  G_BH = 6,    // FP64 n: DCT(b)
  G_E = 7,     // FP64 n: DCT(L^T c), then e_k
  G_SYM = 8,   // FP64 n: symbol a_k
  G_LAM = 9,   // FP64 m: l(k)
  G_KINT = 10, // FP64 interior kernel (2r0+1) x (2r1+1), column-major
  G_DCT = 11,  // FP64 m x m DCT-II matrix, column-major
  G_DONE = 12  // optional FP64 flag, written by every Brent step: 1 once the
               // job's minimisation has ended (the host stops launching steps
               // when every flag of a launch reads 1)
};

constexpr int DBL_GCV_GRID_MAX_DEV = 64;
// Grid points evaluated per block reduction.  Each point keeps its own
// summation order, so the values do not depend on this grouping.
constexpr int GRID_GROUP = 4;

// GCV from the summed terms: spectral resid = gam^2 res; exact resid = bb + res.
__device__ __forceinline__ double gcv_from(const Job* job, double gam, double res, double tr,
                                           int n) {
  const double d = (double)n - tr;
  if (job->flags & F_EXACT) return (job->scal[S_G_BB] + res) / (d * d);
  return gam * gam * res / (d * d);
}

// ------------------------------------------------------ EXACT tier prep --
// n x n identity, column-major: the input columns of the dense-operator
// launch (A applied to every unit vector).
__global__ void __launch_bounds__(NTHREADS) k_gcv_eye(double* __restrict__ I, int n) {
  const size_t tot = (size_t)n * n;
  for (size_t q = blockIdx.x * (size_t)NTHREADS + threadIdx.x; q < tot;
       q += (size_t)gridDim.x * NTHREADS)
    I[q] = (q % (size_t)(n + 1) == 0) ? 1.0 : 0.0;
}

// M += D^T D for D = diag(w) L (w null: D = L) on an m x m grid.  Thread p
// owns column p of M: its diagonal (the sum of the squared weights of the
// differences that touch pixel p) and minus the squared weight at each grid
// neighbour, so no two threads write the same entry.
template <typename T>
__global__ void __launch_bounds__(NTHREADS) k_gcv_add_dtd(double* __restrict__ M,
                                                          const T* __restrict__ w, int m) {
  const int n = m * m, nx = (m - 1) * m;
  auto om = [&](int k) {
    const double v = w ? (double)w[k] : 1.0;
    return v * v;
  };
  for (int p = blockIdx.x * NTHREADS + threadIdx.x; p < n; p += gridDim.x * NTHREADS) {
    const int i = p % m, j = p / m;
    double* col = M + (size_t)p * n;
    double diag = 0.0;
    if (i > 0) { const double o = om(i - 1 + j * (m - 1)); diag += o; col[p - 1] -= o; }
    if (i < m - 1) { const double o = om(i + j * (m - 1)); diag += o; col[p + 1] -= o; }
    if (j > 0) { const double o = om(nx + p - m); diag += o; col[p - m] -= o; }
    if (j < m - 1) { const double o = om(nx + p); diag += o; col[p + m] -= o; }
    col[p] += diag;
  }
}

// -------------------------------------------------------------- symbol ----
// a[k0 + k1 m] = sum_{a,b} K[a,b] cos(pi k0 a / m) cos(pi k1 b / m).
// Job: m, i0 = r0, i1 = r1.  The inner sums over a, which do not depend on
// k1, are formed once per tile row and kernel column (T[u, b]), then combined
// along b for every column of the tile: the same additions in the same order
// as summing each coefficient on its own.
__global__ void __launch_bounds__(NTHREADS) k_gcv_symbol(const Job* __restrict__ jobs,
                                                         const uint32_t* __restrict__ tiles) {
  __shared__ double c0[64 * 33], c1[64 * 33], T[64 * 33];
  const Job* job; int ti, tj, tix;
  decode_tile(jobs, tiles, job, ti, tj, tix);
  const int m = job->m;
  int i0, j0, TI, TJ;
  tile_geom<float>(m, ti, tj, i0, j0, TI, TJ);
  const int r0 = job->i0, r1 = job->i1, n0 = 2 * r0 + 1, n1 = 2 * r1 + 1;
  const double* __restrict__ K = static_cast<const double*>(job->v[G_KINT]);
  double* __restrict__ sym = static_cast<double*>(job->v[G_SYM]);
  const double w = 3.14159265358979323846 / m;
  // cos(pi k a / m) for the tile's frequencies and every kernel offset
  for (int q = threadIdx.x; q < TI * n0; q += NTHREADS)
    c0[q] = cos(w * (double)(i0 + (q & (TI - 1))) * (double)((q >> (__ffs(TI) - 1)) - r0));
  for (int q = threadIdx.x; q < TJ * n1; q += NTHREADS)
    c1[q] = cos(w * (double)(j0 + (q & (TJ - 1))) * (double)((q >> (__ffs(TJ) - 1)) - r1));
  __syncthreads();
  for (int q = threadIdx.x; q < TI * n1; q += NTHREADS) {
    const int u = (q & (TI - 1)), b = (q >> (__ffs(TI) - 1));
    double inner = 0.0;
    for (int a = 0; a < n0; ++a) inner = fma(K[a + (size_t)b * n0], c0[u + a * TI], inner);
    T[u + b * TI] = inner;
  }
  __syncthreads();
  for (int o = threadIdx.x; o < TI * TJ; o += NTHREADS) {
    const int u = (o & (TI - 1)), v = (o >> (__ffs(TI) - 1));
    double acc = 0.0;
    for (int b = 0; b < n1; ++b) acc = fma(T[u + b * TI], c1[v + b * TJ], acc);
    sym[(i0 + u) + (size_t)(j0 + v) * m] = acc;
  }
}

// ---------------------------------------------------------------- prep ----
// i0 = 0: in = (double) b.  i0 = 1: in = L^T c (c = c1 - c2), plus, when G_W
// holds IRLS weights, the partial sums of u and u^2 for u = w^-2 over the
// nonzero weights (the surrogate's weight scale wbar^2 = sum u / sum u^2: the
// weights are max(|L x|, eps)^(-1/2), so u recovers max(|L x|, eps) and the
// ratio is the Rayleigh quotient ||diag(w) u||^2 / ||u||^2).
template <typename T>
__global__ void __launch_bounds__(NTHREADS) k_gcv_prep(const Job* __restrict__ jobs,
                                                       const uint32_t* __restrict__ tiles) {
  __shared__ double red[8];
  const Job* job; int ti, tj, tix;
  decode_tile(jobs, tiles, job, ti, tj, tix);
  const int m = job->m;
  int i0, j0, TI, TJ;
  tile_geom<float>(m, ti, tj, i0, j0, TI, TJ);
  double* __restrict__ in = static_cast<double*>(job->v[G_IN]);
  const size_t nx = (size_t)(m - 1) * m;
  double su = 0.0, su2 = 0.0;
  auto add_w = [&](double v) {
    const double w2 = v * v;
    if (w2 > 0.0) {
      const double u = 1.0 / w2;
      su += u;
      su2 += u * u;
    }
  };
  if (job->i0 == 0) {
    const T* __restrict__ b = static_cast<const T*>(job->v[G_B]);
    for (int o = threadIdx.x; o < TI * TJ; o += NTHREADS) {
      const size_t g = (i0 + (o & (TI - 1))) + (size_t)(j0 + (o >> (__ffs(TI) - 1))) * m;
      in[g] = (double)b[g];
    }
    return;
  }
  const T* __restrict__ c1 = static_cast<const T*>(job->v[G_C1]);
  const T* __restrict__ c2 = static_cast<const T*>(job->v[G_C2]);
  const T* __restrict__ w = static_cast<const T*>(job->v[G_W]);
  auto cv = [&](size_t k) -> double {
    return c1 ? (double)c1[k] - (c2 ? (double)c2[k] : 0.0) : 0.0;
  };
  for (int o = threadIdx.x; o < TI * TJ; o += NTHREADS) {
    const int gi = i0 + (o & (TI - 1)), gj = j0 + (o >> (__ffs(TI) - 1));
    const size_t g = gi + (size_t)gj * m;
    double a = 0.0;
    if (c1) {
      if (gi >= 1) a += cv(gi - 1 + (size_t)gj * (m - 1));
      if (gi < m - 1) a -= cv(gi + (size_t)gj * (m - 1));
      if (gj >= 1) a += cv(nx + g - m);
      if (gj < m - 1) a -= cv(nx + g);
    }
    in[g] = a;
    if (w) {
      if (gi < m - 1) add_w((double)w[gi + (size_t)gj * (m - 1)]);
      if (gj < m - 1) add_w((double)w[nx + g]);
    }
  }
  if (w) {
    double vv[2] = {su, su2};
    put_partials<2>(job->pw, tix, vv, red);
  }
}

// ---------------------------------------------------- boundary completion --
// The level operator blurs with zero boundaries, the surrogate models a
// reflexive one.  One pass writes out = b + E(Y), with E(Y) the reflexive-
// boundary blur of Y minus its zero-boundary blur: at a pixel within the
// kernel radius of an edge, the taps of the interior kernel K (convolution
// orientation, column-major (2 r0 + 1) x (2 r1 + 1)) whose source lies
// outside the grid, applied to the half-sample symmetric reflection of Y.
// Two passes (Y = b, then Y = the first result) complete the data before its
// transform.  A thread reads b and writes out only at its own pixel, so out
// may be b; Y is never written.  Job: m, i0 = r0, i1 = r1, v[0] = b,
// v[1] = Y, v[2] = out, v[G_KINT] = K (all FP64).
__device__ __forceinline__ int mirror_index(int s, int m) {
  // ..., 1, 0 | 0, 1, ..., m - 1 | m - 1, ...: one reflection per step, a
  // single step for offsets at most m outside the grid; two steps shift s by
  // 2m towards the grid, so the loop ends for every m >= 1
  while (s < 0 || s >= m) s = s < 0 ? -1 - s : 2 * m - 1 - s;
  return s;
}

// Every source pixel that a tile's band reads (reflected or not) lies in the
// tile grown by the kernel radius and clipped to the grid, so a band tile
// stages that region of Y, and K, in LDS; tiles with no band pixel copy b.
constexpr int CMP_RMAX = 16;                  // interior kernel radius bound
constexpr int CMP_EDGE = 32 + 2 * CMP_RMAX;   // staged region edge (32-pixel tiles)

__global__ void __launch_bounds__(NTHREADS) k_gcv_complete(const Job* __restrict__ jobs,
                                                           const uint32_t* __restrict__ tiles) {
  __shared__ double ys[CMP_EDGE * CMP_EDGE];
  __shared__ double ks[(2 * CMP_RMAX + 1) * (2 * CMP_RMAX + 1)];
  const Job* job; int ti, tj, tix;
  decode_tile(jobs, tiles, job, ti, tj, tix);
  const int m = job->m;
  int i0, j0, TI, TJ;
  tile_geom<float>(m, ti, tj, i0, j0, TI, TJ);
  const int r0 = job->i0, r1 = job->i1, n0 = 2 * r0 + 1, n1 = 2 * r1 + 1;
  const double* b = static_cast<const double*>(job->v[0]);
  const double* Y = static_cast<const double*>(job->v[1]);
  double* out = static_cast<double*>(job->v[2]);
  const double* __restrict__ K = static_cast<const double*>(job->v[G_KINT]);
  const int lg = __ffs(TI) - 1;
  const bool band = i0 < r0 || i0 + TI > m - r0 || j0 < r1 || j0 + TJ > m - r1;
  if (!band || r0 > CMP_RMAX || r1 > CMP_RMAX || TI > 32 || TJ > 32) {
    // (the host never launches radii above the bound)
    for (int o = threadIdx.x; o < TI * TJ; o += NTHREADS) {
      const size_t g = (i0 + (o & (TI - 1))) + (size_t)(j0 + (o >> lg)) * m;
      out[g] = b[g];
    }
    return;
  }
  const int a0 = max(0, i0 - r0), a1 = min(m, i0 + TI + r0);
  const int c0 = max(0, j0 - r1), c1 = min(m, j0 + TJ + r1);
  const int H = a1 - a0, W = c1 - c0;
  const bool single = r0 <= m && r1 <= m;
  for (int q = threadIdx.x; q < H * W; q += NTHREADS) {
    const int u = q % H, v = q / H;
    ys[q] = Y[(a0 + u) + (size_t)(c0 + v) * m];
  }
  for (int q = threadIdx.x; q < n0 * n1; q += NTHREADS) ks[q] = K[q];
  __syncthreads();
  for (int o = threadIdx.x; o < TI * TJ; o += NTHREADS) {
    const int gi = i0 + (o & (TI - 1)), gj = j0 + (o >> lg);
    const size_t g = gi + (size_t)gj * m;
    double acc = b[g];
    if (gi < r0 || gi >= m - r0 || gj < r1 || gj >= m - r1) {
      // source row si = gi - aa lies below the grid for aa <= gi - m and
      // above it for aa > gi; a column outside takes every row.  With
      // r0, r1 <= m one reflection suffices and the staged row is linear in
      // aa on each of the three ranges: 2m - 1 - si, si, -1 - si.
      const int hi_lo = min(r0, gi - m), lo_hi = max(-r0, gi + 1);
      double e = 0.0;
      for (int bb = -r1; bb <= r1; ++bb) {
        const int sj = gj - bb;
        const bool col_out = sj < 0 || sj >= m;
        const int kc = (bb + r1) * n0 + r0;                  // ks[kc + aa] = K[aa, bb]
        const int yc = (mirror_index(sj, m) - c0) * H - a0;  // ys[yc + row]
        if (single) {
          const int yb = yc + 2 * m - 1 - gi, ym = yc + gi, ya = yc - gi - 1;
          for (int aa = -r0; aa <= hi_lo; ++aa) e += ks[kc + aa] * ys[yb + aa];
          if (col_out)
            for (int aa = max(-r0, gi - m + 1); aa <= min(r0, gi); ++aa)
              e += ks[kc + aa] * ys[ym - aa];
          for (int aa = lo_hi; aa <= r0; ++aa) e += ks[kc + aa] * ys[ya + aa];
        } else {
          for (int aa = -r0; aa <= r0; ++aa) {
            const int si = gi - aa;
            if (col_out || si < 0 || si >= m) e += ks[kc + aa] * ys[yc + mirror_index(si, m)];
          }
        }
      }
      acc += e;
    }
    out[g] = acc;
  }
}

// ---------------------------------------------------------------- GEMM ----
// out = A * B (i0 = 0) or A * B^T (i0 = 1); m x m FP64, column-major.
// v[0] = A, v[1] = B, v[2] = out.  64 x 64 output tiles.
// On the FP64 matrix cores (v_mfma_f64_16x16x4f64): the block stages
// 16-deep slabs of A and B in LDS; wave w computes the
// 32 x 32 quarter (rows 32 (w % 2), columns 32 (w / 2)) of the 64 x 64 tile
// as four 16 x 16 accumulators, four k-steps of 4 per slab.  Operand lanes:
// A fragment a = A[row 16 rb + lane % 16][k 4 q + lane / 16], B fragment
// b = B[k 4 q + lane / 16][column 16 cb + lane % 16]; result element v of a
// lane is D[lane / 16 + 4 v][lane % 16] of its 16 x 16 block (the FP64
// instruction interleaves its result rows).  Stores are guarded by the tile
// size (a grid below 64 is one partial tile).
typedef double dbl4 __attribute__((ext_vector_type(4)));

__global__ void __launch_bounds__(NTHREADS) k_gemm64_mfma(const Job* __restrict__ jobs,
                                                          const uint32_t* __restrict__ tiles) {
  __shared__ double As[16][65];
  __shared__ double Bs[16][65];
  const Job* job; int ti, tj, tix;
  decode_tile(jobs, tiles, job, ti, tj, tix);
  const int m = job->m;
  const int TS = m < 64 ? m : 64;
  const int i0 = ti * TS, j0 = tj * TS;
  const double* __restrict__ A = static_cast<const double*>(job->v[0]);
  const double* __restrict__ B = static_cast<const double*>(job->v[1]);
  double* __restrict__ C = static_cast<double*>(job->v[2]);
  const bool tb = job->i0 != 0;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int wr = 32 * (wid & 1), wc = 32 * (wid >> 1);  // the wave's quarter
  const int fr = lane & 15, fk = lane >> 4;              // fragment row / column, k
  dbl4 acc[2][2];
#pragma unroll
  for (int u = 0; u < 2; ++u)
#pragma unroll
    for (int v = 0; v < 2; ++v) acc[u][v] = dbl4{0.0, 0.0, 0.0, 0.0};
  // The next 16-deep slab is loaded into registers while the MFMAs run on
  // the current one (LDS-only barriers keep those loads in flight).
  constexpr int PER = 16 * 64 / NTHREADS;
  double pa[PER], pb[PER];
  auto fetch = [&](int k0) {
    const int kk = m - k0 < 16 ? m - k0 : 16;
#pragma unroll
    for (int p = 0; p < PER; ++p) {
      const int idx = threadIdx.x + p * NTHREADS, r = idx % 64, k = idx / 64;
      const bool in = r < TS && k < kk;
      pa[p] = in ? A[(i0 + r) + (size_t)(k0 + k) * m] : 0.0;
      pb[p] = in ? (tb ? B[(j0 + r) + (size_t)(k0 + k) * m] : B[(k0 + k) + (size_t)(j0 + r) * m])
                 : 0.0;
    }
  };
  fetch(0);
  for (int k0 = 0; k0 < m; k0 += 16) {
#pragma unroll
    for (int p = 0; p < PER; ++p) {
      const int idx = threadIdx.x + p * NTHREADS, r = idx % 64, k = idx / 64;
      As[k][r] = pa[p];
      Bs[k][r] = pb[p];
    }
    lds_barrier();
    if (k0 + 16 < m) fetch(k0 + 16);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int k = 4 * q + fk;
      double a[2], b[2];
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        a[u] = As[k][wr + 16 * u + fr];
        b[u] = Bs[k][wc + 16 * u + fr];
      }
#pragma unroll
      for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int v = 0; v < 2; ++v)
          acc[u][v] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u], b[v], acc[u][v], 0, 0, 0);
    }
    lds_barrier();
  }
#pragma unroll
  for (int u = 0; u < 2; ++u)
#pragma unroll
    for (int v = 0; v < 2; ++v)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int r = wr + 16 * u + fk + 4 * e, c = wc + 16 * v + fr;
        if (r < TS && c < TS) C[(i0 + r) + (size_t)(j0 + c) * m] = acc[u][v][e];
      }
}

// ---------------------------------------------------------------- data ----
// e_k = (a c^ - lp b^)^2 in place of c^ (or with c^ = 0 when i0 == 0), and
// the grid bounds from min / max of log10(s / lp) over lp > 0, s > 0.
__global__ void __launch_bounds__(NTHREADS) k_gcv_data(const Job* __restrict__ jobs,
                                                       const uint32_t* __restrict__ tiles) {
  __shared__ double red[8];
  __shared__ double bc;
  const Job* job; int ti, tj, tix;
  decode_tile(jobs, tiles, job, ti, tj, tix);
  const int m = job->m;
  int i0, j0, TI, TJ;
  tile_geom<float>(m, ti, tj, i0, j0, TI, TJ);
  const double* __restrict__ sym = static_cast<const double*>(job->v[G_SYM]);
  const double* __restrict__ lam = static_cast<const double*>(job->v[G_LAM]);
  const double* __restrict__ bh = static_cast<const double*>(job->v[G_BH]);
  double* __restrict__ e = static_cast<double*>(job->v[G_E]);
  const bool shift = job->i0 != 0;
  const bool exact = job->flags & F_EXACT;
  // IRLS weight scale wbar^2 = sum u / sum u^2 from the prep partials (1
  // without weights or without a nonzero weight)
  double wb2 = 1.0;
  if (job->pr[0]) {
    const double s1 = sum_partials<2>(job->pr[0], job->nti * job->ntj, 0, red, &bc);
    const double s2 = sum_partials<2>(job->pr[0], job->nti * job->ntj, 1, red, &bc);
    if (s2 > 0.0) wb2 = s1 / s2;
  }
  if (tix == 0 && threadIdx.x == 0) job->scal[S_G_WBAR] = wb2;
  double lo = 1e300, hi = -1e300;
  for (int o = threadIdx.x; o < TI * TJ && exact; o += NTHREADS) {
    // nu in the symbol slot: bounds from nu / (1 - nu) over 0 < nu < 1 - 1e-10
    const size_t g = (i0 + (o & (TI - 1))) + (size_t)(j0 + (o >> (__ffs(TI) - 1))) * m;
    const double nu = fmin(fmax(sym[g], 0.0), 1.0);
    if (nu > 0.0 && nu < 1.0 - 1e-10) {
      const double r = nu / (1.0 - nu);
      if (r > 0.0 && r < 1e308) {
        const double t = log10(r);
        lo = fmin(lo, t);
        hi = fmax(hi, t);
      }
    }
  }
  for (int o = threadIdx.x; o < TI * TJ && !exact; o += NTHREADS) {
    const int k0 = i0 + (o & (TI - 1)), k1 = j0 + (o >> (__ffs(TI) - 1));
    const size_t g = k0 + (size_t)k1 * m;
    const double a = sym[g];
    const double lp = wb2 * (lam[k0] + lam[k1]);
    const double ch = shift ? e[g] : 0.0;
    const double r = a * ch - lp * bh[g];
    e[g] = r * r;
    const double s = a * a;
    if (lp > 0.0 && s > 0.0) {
      const double t = log10(s / lp);
      lo = fmin(lo, t);
      hi = fmax(hi, t);
    }
  }
  // block min / max, stored as this tile's partials (min, max)
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    lo = fmin(lo, __shfl_xor(lo, off, 64));
    hi = fmax(hi, __shfl_xor(hi, off, 64));
  }
  if (lane == 0) { red[wid] = lo; red[4 + wid] = hi; }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < 4; ++w) { lo = fmin(lo, red[w]); hi = fmax(hi, red[4 + w]); }
    job->pw[2 * tix] = lo;
    job->pw[2 * tix + 1] = hi;
  }
}

// 1 / d for d > 0 in the normal range: the hardware reciprocal (relative
// error about 2^-23) refined by two Newton-Raphson steps r <- r + r (1 - d r),
// each of which doubles the correct bits, so the result is within an ulp or
// so of the rounded quotient; five instructions where IEEE division takes
// about eleven.  The GCV sums are bound by these reciprocals (one per
// frequency and parameter).
__device__ __forceinline__ double recip_pos(double d) {
  double r = __builtin_amdgcn_rcp(d);
  double e = fma(-d, r, 1.0);
  r = fma(r, e, r);
  e = fma(-d, r, 1.0);
  return fma(r, e, r);
}

// Per-thread view of the frequencies of one tile: at most Q per thread (4
// for the 32 x 32 tiles of the multi-block kernels, 16 for one block over a
// grid of up to 64 x 64).  Entry q is frequency threadIdx.x + q * NT of the
// tile; every index is known at compile time so the arrays stay in registers.
template <int Q>
struct FreqRegs {
  double s[Q], lp[Q], e[Q];
  int cnt;
};

template <int NT = NTHREADS, int Q>
__device__ __forceinline__ void load_freqs(const Job* job, int i0, int j0, int TI, int TJ,
                                           FreqRegs<Q>& f) {
  const int m = job->m;
  const double* __restrict__ sym = static_cast<const double*>(job->v[G_SYM]);
  const double* __restrict__ lam = static_cast<const double*>(job->v[G_LAM]);
  const double* __restrict__ e = static_cast<const double*>(job->v[G_E]);
  const double wb2 = job->scal[S_G_WBAR];
  const bool exact = job->flags & F_EXACT;
  const double* __restrict__ fv = static_cast<const double*>(job->v[G_BH]);
  f.cnt = 0;
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int o = threadIdx.x + q * NT;
    f.s[q] = f.lp[q] = f.e[q] = 0.0;
    if (o >= TI * TJ) continue;
    const int k0 = i0 + (o & (TI - 1)), k1 = j0 + (o >> (__ffs(TI) - 1));
    const size_t g = k0 + (size_t)k1 * m;
    if (exact) {  // (nu, f, g) in the (s, lp, e) registers
      f.s[q] = fmin(fmax(sym[g], 0.0), 1.0);
      f.lp[q] = fv[g];
      f.e[q] = e[g];
    } else {
      const double a = sym[g];
      f.s[q] = a * a;
      f.lp[q] = wb2 * (lam[k0] + lam[k1]);
      f.e[q] = e[g];
    }
    f.cnt = q + 1;
  }
}

template <int Q>
__device__ __forceinline__ void eval_freqs(const Job* job, const FreqRegs<Q>& f, double gam,
                                           double& res, double& tr) {
  res = 0.0;
  tr = 0.0;
  if (job->flags & F_EXACT) {
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      if (q < f.cnt) {
        const double nu = f.s[q];
        const double den = nu + gam * (1.0 - nu);
        if (den > 0.0) {
          const double inv = recip_pos(den);
          const double y = (f.lp[q] + gam * f.e[q]) * inv;
          res += nu * y * y - 2.0 * f.lp[q] * y;
          tr += nu * inv;
        }
      }
    }
    return;
  }
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    if (q < f.cnt) {
      const double den = f.s[q] + gam * f.lp[q];
      if (den > 0.0) {
        const double inv = recip_pos(den);
        res += f.e[q] * inv * inv;
        tr += f.s[q] * inv;
      }
    }
  }
}

// eval_freqs at G parameters at once (v[2g], v[2g+1] = res, tr at gam[g]; g
// with gam[g] < 0 are skipped and left at zero).  Each parameter's terms are
// added in the same order as by eval_freqs.
template <int G, int Q>
__device__ __forceinline__ void eval_freqs_multi(const Job* job, const FreqRegs<Q>& f,
                                                 const double (&gam)[G], double (&v)[2 * G]) {
#pragma unroll
  for (int k = 0; k < 2 * G; ++k) v[k] = 0.0;
  const bool exact = job->flags & F_EXACT;
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    if (q >= f.cnt) break;
    const double s = f.s[q], lp = f.lp[q], e = f.e[q];
#pragma unroll
    for (int g = 0; g < G; ++g) {
      if (gam[g] < 0.0) continue;
      if (exact) {
        const double den = s + gam[g] * (1.0 - s);
        if (den > 0.0) {
          const double inv = recip_pos(den);
          const double y = (lp + gam[g] * e) * inv;
          v[2 * g] += s * y * y - 2.0 * lp * y;
          v[2 * g + 1] += s * inv;
        }
      } else {
        const double den = s + gam[g] * lp;
        if (den > 0.0) {
          const double inv = recip_pos(den);
          v[2 * g] += e * inv * inv;
          v[2 * g + 1] += s * inv;
        }
      }
    }
  }
}

// One step of Brent's minimisation without derivatives (golden section with
// parabolic interpolation) on the state st, given f(st[BR_U]): updates the
// bracket and the best points, then sets st[BR_U] to the next point.
// Returns true when the bracket meets the tolerance or maxit steps are done.
__device__ __forceinline__ bool brent_step(double* st, double fu, double xtol, int maxit) {
  const double u = st[BR_U];
  const double golden = 0.5 * (3.0 - sqrt(5.0));
  const double sqeps = sqrt(2.220446049250313e-16);
  double a = st[BR_A], b = st[BR_B], x = st[BR_X], w = st[BR_W], v = st[BR_V];
  double fx = st[BR_FX], fw = st[BR_FW], fv = st[BR_FV], d = st[BR_D], e = st[BR_E];
  int it = (int)st[BR_IT];
  if (it < 0) {
    fx = fw = fv = fu;
    it = 0;
  } else {
    if (fu <= fx) {
      if (u >= x) a = x; else b = x;
      v = w; fv = fw; w = x; fw = fx; x = u; fx = fu;
    } else {
      if (u < x) a = u; else b = u;
      if (fu <= fw || w == x) { v = w; fv = fw; w = u; fw = fu; }
      else if (fu <= fv || v == x || v == w) { v = u; fv = fu; }
    }
    it += 1;
  }
  bool done = it >= maxit;
  double unext = x;
  if (!done) {
    const double xm = 0.5 * (a + b);
    const double tol = sqeps * fabs(x) + xtol / 3.0;
    const double tol2 = 2.0 * tol;
    if (fabs(x - xm) <= tol2 - 0.5 * (b - a)) {
      done = true;
    } else {
      bool use_golden = true;
      if (fabs(e) > tol) {
        double r = (x - w) * (fx - fv);
        double q = (x - v) * (fx - fw);
        double p = (x - v) * q - (x - w) * r;
        q = 2.0 * (q - r);
        if (q > 0.0) p = -p;
        q = fabs(q);
        const double e_prev = e;
        e = d;
        if (fabs(p) < fabs(0.5 * q * e_prev) && p > q * (a - x) && p < q * (b - x)) {
          d = p / q;
          const double uu = x + d;
          if ((uu - a) < tol2 || (b - uu) < tol2) d = xm >= x ? tol : -tol;
          use_golden = false;
        }
      }
      if (use_golden) {
        e = x >= xm ? (a - x) : (b - x);
        d = golden * e;
      }
      unext = fabs(d) >= tol ? x + d : (d > 0.0 ? x + tol : x - tol);
    }
  }
  st[BR_A] = a; st[BR_B] = b; st[BR_X] = x; st[BR_W] = w; st[BR_V] = v;
  st[BR_FX] = fx; st[BR_FW] = fw; st[BR_FV] = fv; st[BR_D] = d; st[BR_E] = e;
  st[BR_IT] = (double)it;
  st[BR_U] = unext;
  st[BR_DONE] = done ? 1.0 : 0.0;
  return done;
}

// Bracket around the lowest-index grid minimum and Brent's start state.
__device__ __forceinline__ void brent_start(double* st, double tlo, double thi, int npts, int jb) {
  const double step = (thi - tlo) / (npts - 1);
  const double a = tlo + step * (jb > 0 ? jb - 1 : 0);
  const double b = tlo + step * (jb < npts - 1 ? jb + 1 : npts - 1);
  const double golden = 0.5 * (3.0 - sqrt(5.0));
  const double x = a + golden * (b - a);
  for (int q = 0; q < BR_SIZE; ++q) st[q] = 0.0;
  st[BR_A] = a;
  st[BR_B] = b;
  st[BR_X] = x;
  st[BR_W] = x;
  st[BR_V] = x;
  st[BR_U] = x;
  st[BR_IT] = -1.0;    // the first evaluation is the start point
  st[BR_PHASE] = 0.0;  // nothing evaluated yet
  st[BR_DONE] = 0.0;
}

// ---------------------------------------------------------------- grid ----
// Job::i1 = number of grid points; pr[0] = (min, max) partials of k_gcv_data.
// Writes 2 partials (residual sum, trace) per grid point per tile.
__global__ void __launch_bounds__(NTHREADS) k_gcv_grid(const Job* __restrict__ jobs,
                                                       const uint32_t* __restrict__ tiles) {
  __shared__ double red[2 * GRID_GROUP * 4];
  __shared__ double gam_s[DBL_GCV_GRID_MAX_DEV];
  __shared__ double bl, bh_;
  const Job* job; int ti, tj, tix;
  decode_tile(jobs, tiles, job, ti, tj, tix);
  const int m = job->m, npts = job->i1, nt = job->nti * job->ntj;
  int i0, j0, TI, TJ;
  tile_geom<float>(m, ti, tj, i0, j0, TI, TJ);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  // bounds: min / max of log10(s / lp) over the job (order-free)
  double lo = 1e300, hi = -1e300;
  for (int t = threadIdx.x; t < nt; t += NTHREADS) {
    lo = fmin(lo, job->pr[0][2 * t]);
    hi = fmax(hi, job->pr[0][2 * t + 1]);
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    lo = fmin(lo, __shfl_xor(lo, off, 64));
    hi = fmax(hi, __shfl_xor(hi, off, 64));
  }
  if (lane == 0) { red[wid] = lo; red[4 + wid] = hi; }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < 4; ++w) { lo = fmin(lo, red[w]); hi = fmax(hi, red[4 + w]); }
    bl = fmax(lo, hi - 14.0);
    bh_ = hi;
  }
  __syncthreads();
  const double tlo = bl, thi = bh_;
  if (tix == 0 && threadIdx.x == 0) {
    job->scal[S_G_TLO] = tlo;
    job->scal[S_G_THI] = thi;
  }
  for (int p = threadIdx.x; p < npts; p += NTHREADS)
    gam_s[p] = pow(10.0, tlo + (thi - tlo) * p / (npts - 1));
  FreqRegs<4> f;  // 32 x 32 tile over 256 threads
  load_freqs(job, i0, j0, TI, TJ, f);
  __syncthreads();
  for (int p0 = 0; p0 < npts; p0 += GRID_GROUP) {
    double v[2 * GRID_GROUP], gg[GRID_GROUP];
#pragma unroll
    for (int g = 0; g < GRID_GROUP; ++g) gg[g] = p0 + g < npts ? gam_s[p0 + g] : -1.0;
    eval_freqs_multi(job, f, gg, v);
#pragma unroll
    for (int k = 0; k < 2 * GRID_GROUP; ++k) v[k] = wave_sum(v[k]);
    __syncthreads();
    if (lane == 0)
#pragma unroll
      for (int k = 0; k < 2 * GRID_GROUP; ++k) red[k * 4 + wid] = v[k];
    __syncthreads();
    const int g = threadIdx.x;
    if (g < GRID_GROUP && p0 + g < npts) {
      const int p = p0 + g;
      double a = 0.0, b = 0.0;
      for (int w = 0; w < 4; ++w) { a += red[(2 * g) * 4 + w]; b += red[(2 * g + 1) * 4 + w]; }
      job->pw[(size_t)tix * 2 * npts + 2 * p] = a;
      job->pw[(size_t)tix * 2 * npts + 2 * p + 1] = b;
    }
  }
}

// One block per job: grid GCV values from the partials (pr[0], i1 tiles,
// i0 points), lowest-index minimum, Brent's bracket and start state.
constexpr int GF_GROUP = 8;  // grid points summed per pass over the partials
__global__ void __launch_bounds__(NTHREADS) k_gcv_gridfin(const Job* __restrict__ jobs,
                                                          const uint32_t* __restrict__ tiles) {
  const Job* job = jobs + (tiles[blockIdx.x] >> 16);
  const int npts = job->i0, nt = job->i1, n = job->m * job->m;
  double* sc = job->scal;
  const double tlo = sc[S_G_TLO], thi = sc[S_G_THI];
  __shared__ double vals[DBL_GCV_GRID_MAX_DEV];
  __shared__ double red[2 * GF_GROUP * (NTHREADS / 64)];
  // eight points at a time: thread t adds tiles t, t + NTHREADS, ... (their
  // 16 values are contiguous), then a fixed-order block sum
  const double* __restrict__ part = job->pr[0];
  for (int p0 = 0; p0 < npts; p0 += GF_GROUP) {
    const int np = npts - p0 < GF_GROUP ? npts - p0 : GF_GROUP;
    double v[2 * GF_GROUP];
#pragma unroll
    for (int q = 0; q < 2 * GF_GROUP; ++q) v[q] = 0.0;
    for (int t = threadIdx.x; t < nt; t += NTHREADS) {
      const double* row = part + (size_t)t * 2 * npts + 2 * p0;
#pragma unroll
      for (int q = 0; q < 2 * GF_GROUP; ++q)
        if (q < 2 * np) v[q] += row[q];
    }
    block_sum<2 * GF_GROUP>(v, red);
    if (threadIdx.x == 0)
      for (int g = 0; g < np; ++g) {
        const int p = p0 + g;
        const double t = tlo + (thi - tlo) * p / (npts - 1);
        vals[p] = gcv_from(job, pow(10.0, t), v[2 * g], v[2 * g + 1], n);
        sc[S_GRID + p] = vals[p];
      }
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  int jb = 0;
  double best = vals[0];
  for (int p = 1; p < npts; ++p)
    if (vals[p] < best) { best = vals[p]; jb = p; }
  brent_start(sc + S_BR, tlo, thi, npts, jb);  // copy 0: read by the first Brent launch
}

// --------------------------------------------------------------- Brent ----
// Launch parity is Job::i0 (0 / 1): read state copy i0 and partials pr[0]
// (previous evaluation), write state copy 1 - i0 and partials pw.
// Job::i1 = max Brent steps; p0 = xtol.
__global__ void __launch_bounds__(NTHREADS) k_gcv_brent(const Job* __restrict__ jobs,
                                                        const uint32_t* __restrict__ tiles) {
  __shared__ double red[8];
  __shared__ double bc;
  const Job* job; int ti, tj, tix;
  decode_tile(jobs, tiles, job, ti, tj, tix);
  double* sc = job->scal;
  const int par = job->i0;
  const double* in = sc + S_BR + par * BR_SIZE;
  double* out = sc + S_BR + (1 - par) * BR_SIZE;
  const bool owner = (tix == 0 && threadIdx.x == 0);
  double* dflag = static_cast<double*>(job->v[G_DONE]);
  double st[BR_SIZE];
#pragma unroll
  for (int q = 0; q < BR_SIZE; ++q) st[q] = in[q];
  if (st[BR_DONE] != 0.0) {
    if (owner) {
      for (int q = 0; q < BR_SIZE; ++q) out[q] = st[q];
      if (dflag) *dflag = 1.0;
    }
    return;
  }
  const int m = job->m, n = m * m, nt = job->nti * job->ntj;
  bool done = false;
  if (st[BR_PHASE] == 0.0) {
    st[BR_PHASE] = 1.0;  // evaluate at U (= the start point) below
  } else {
    // the previous launch evaluated GCV at U: total its partials
    const double res = sum_partials<2>(job->pr[0], nt, 0, red, &bc);
    const double tr = sum_partials<2>(job->pr[0], nt, 1, red, &bc);
    const double fu = gcv_from(job, pow(10.0, st[BR_U]), res, tr, n);
    done = brent_step(st, fu, job->p0, job->i1);
  }
  if (owner) {
    for (int q = 0; q < BR_SIZE; ++q) out[q] = st[q];
    if (done) {
      const double g = pow(10.0, st[BR_X]);
      sc[S_GAMMA] = g;
      sc[S_SQRTG] = sqrt(g);
      sc[S_G_FBEST] = st[BR_FX];
    }
    if (dflag) *dflag = done ? 1.0 : 0.0;
  }
  if (done) return;
  // evaluate GCV at U: per-tile partials (residual sum, trace)
  int i0, j0, TI, TJ;
  tile_geom<float>(m, ti, tj, i0, j0, TI, TJ);
  FreqRegs<4> f;  // 32 x 32 tile over 256 threads
  load_freqs(job, i0, j0, TI, TJ, f);
  double res, tr;
  eval_freqs(job, f, pow(10.0, st[BR_U]), res, tr);
  double vv[2] = {res, tr};
  put_partials<2>(job->pw, tix, vv, red);
}

// ----------------------------------------------------------- one block --
// Levels of at most 64 x 64: every frequency of a job fits in one block's
// registers (16 per thread), so the grid bounds, the grid, the bracket and
// all Brent steps run in one launch, one block per job.  (At 128 x 128 a
// 1024-thread block is slower than the multi-launch path: measured.)  The steps are those
// of k_gcv_grid / k_gcv_gridfin / k_gcv_brent; the sums over frequencies are
// block sums instead of per-tile partials.  Job: i0 = grid points, i1 = tiles
// of the data launch, pr[0] = its (min, max) partials, p0 = xtol, p1 = max
// Brent steps.  Every thread holds the same Brent state (the block sums are
// identical in all threads), so all threads leave the loop together.
template <int NT>
__global__ void __launch_bounds__(NT) k_gcv_solo(const Job* __restrict__ jobs,
                                                 const uint32_t* __restrict__ tiles) {
  __shared__ double red[2 * GRID_GROUP * (NT / 64)];
  __shared__ double vals[DBL_GCV_GRID_MAX_DEV];
  __shared__ double gam_s[DBL_GCV_GRID_MAX_DEV];
  const Job* job = jobs + (tiles[blockIdx.x] >> 16);
  double* sc = job->scal;
  const int m = job->m, n = m * m, npts = job->i0, nt = job->i1;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  constexpr int NW = NT / 64;
  // grid bounds from the data partials
  double lo = 1e300, hi = -1e300;
  for (int t = threadIdx.x; t < nt; t += NT) {
    lo = fmin(lo, job->pr[0][2 * t]);
    hi = fmax(hi, job->pr[0][2 * t + 1]);
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    lo = fmin(lo, __shfl_xor(lo, off, 64));
    hi = fmax(hi, __shfl_xor(hi, off, 64));
  }
  if (lane == 0) { red[wid] = lo; red[NW + wid] = hi; }
  __syncthreads();
  for (int w = 0; w < NW; ++w) { lo = fmin(lo, red[w]); hi = fmax(hi, red[NW + w]); }
  const double thi = hi, tlo = fmax(lo, hi - 14.0);
  FreqRegs<64 * 64 / NT> f;
  load_freqs<NT>(job, 0, 0, m, m, f);
  auto gcv_at = [&](double t) {
    double v[2];
    eval_freqs(job, f, pow(10.0, t), v[0], v[1]);
    block_allsum<2, NT>(v, red);
    return gcv_from(job, pow(10.0, t), v[0], v[1], n);
  };
  for (int p = threadIdx.x; p < npts; p += NT)
    gam_s[p] = pow(10.0, tlo + (thi - tlo) * p / (npts - 1));
  __syncthreads();
  for (int p0 = 0; p0 < npts; p0 += GRID_GROUP) {
    double v[2 * GRID_GROUP], gg[GRID_GROUP];
#pragma unroll
    for (int g = 0; g < GRID_GROUP; ++g) gg[g] = p0 + g < npts ? gam_s[p0 + g] : -1.0;
    eval_freqs_multi(job, f, gg, v);
    block_allsum<2 * GRID_GROUP, NT>(v, red);
    if (threadIdx.x == 0)
      for (int g = 0; g < GRID_GROUP && p0 + g < npts; ++g) {
        const double val = gcv_from(job, gam_s[p0 + g], v[2 * g], v[2 * g + 1], n);
        vals[p0 + g] = val;
        sc[S_GRID + p0 + g] = val;
      }
  }
  __syncthreads();
  int jb = 0;
  double best = vals[0];
  for (int p = 1; p < npts; ++p)
    if (vals[p] < best) { best = vals[p]; jb = p; }
  double st[BR_SIZE];
  brent_start(st, tlo, thi, npts, jb);
  const double xtol = job->p0;
  const int maxit = (int)job->p1;
  bool done = false;
  while (!done) done = brent_step(st, gcv_at(st[BR_U]), xtol, maxit);
  if (threadIdx.x == 0) {
    const double g = pow(10.0, st[BR_X]);
    sc[S_G_TLO] = tlo;
    sc[S_G_THI] = thi;
    sc[S_GAMMA] = g;
    sc[S_SQRTG] = sqrt(g);
    sc[S_G_FBEST] = st[BR_FX];
  }
}

// -------------------------------------------------------------- launchers --

#define GLAUNCH(KERNEL, la)                                                             \
  hipLaunchKernelGGL((KERNEL), dim3((la).ntiles), dim3(NTHREADS), 0, (la).stream,      \
                     (la).jobs, (la).tiles)

hipError_t launch_gcv_prep(const LaunchArgs& la, int precision) {
  if (precision == 1) GLAUNCH(k_gcv_prep<double>, la);
  else GLAUNCH(k_gcv_prep<float>, la);
  return hipGetLastError();
}
hipError_t launch_gcv_complete(const LaunchArgs& la) {
  GLAUNCH(k_gcv_complete, la);
  return hipGetLastError();
}
hipError_t launch_gemm64(const LaunchArgs& la) { GLAUNCH(k_gemm64_mfma, la); return hipGetLastError(); }
hipError_t launch_gcv_symbol(const LaunchArgs& la) {
  GLAUNCH(k_gcv_symbol, la);
  return hipGetLastError();
}
hipError_t launch_gcv_eye(double* I, int n, hipStream_t stream) {
  const size_t tot = (size_t)n * n;
  const int blocks = (int)std::min<size_t>((tot + NTHREADS - 1) / NTHREADS, 4096);
  hipLaunchKernelGGL(k_gcv_eye, dim3(blocks), dim3(NTHREADS), 0, stream, I, n);
  return hipGetLastError();
}

hipError_t launch_gcv_add_dtd(double* M, const void* w, int precision, int m,
                              hipStream_t stream) {
  const int blocks = (m * m + NTHREADS - 1) / NTHREADS;
  if (precision == 1)
    hipLaunchKernelGGL((k_gcv_add_dtd<double>), dim3(blocks), dim3(NTHREADS), 0, stream, M,
                       static_cast<const double*>(w), m);
  else
    hipLaunchKernelGGL((k_gcv_add_dtd<float>), dim3(blocks), dim3(NTHREADS), 0, stream, M,
                       static_cast<const float*>(w), m);
  return hipGetLastError();
}

// Threads of the one-block GCV: 8 frequencies of a 64 x 64 grid per thread,
// all in registers.
constexpr int SOLO_NT = 512;

hipError_t launch_gcv_solo(const LaunchArgs& la) {
  if (la.m_max > 64) return hipErrorInvalidValue;  // 8 frequencies per thread
  hipLaunchKernelGGL(k_gcv_solo<SOLO_NT>, dim3(la.ntiles), dim3(SOLO_NT), 0, la.stream,
                     la.jobs, la.tiles);
  return hipGetLastError();
}
hipError_t launch_gcv_data(const LaunchArgs& la) { GLAUNCH(k_gcv_data, la); return hipGetLastError(); }
hipError_t launch_gcv_grid(const LaunchArgs& la, int) { GLAUNCH(k_gcv_grid, la); return hipGetLastError(); }
hipError_t launch_gcv_brent(const LaunchArgs& la) { GLAUNCH(k_gcv_brent, la); return hipGetLastError(); }
hipError_t launch_gcv_gridfin(const LaunchArgs& la) {
  GLAUNCH(k_gcv_gridfin, la);
  return hipGetLastError();
}

}  // namespace dbl
