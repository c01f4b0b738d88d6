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
// Brent runs as a device state machine: each launch evaluates GCV at the
// current point (all blocks), the job's last block advances the state.
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
  G_DCT = 11   // FP64 m x m DCT-II matrix, column-major
};

__device__ __forceinline__ double gcv_from(double gam, double res, double tr, int n) {
  const double d = (double)n - tr;
  return gam * gam * res / (d * d);
}

// -------------------------------------------------------------- symbol ----
// a[k0 + k1 m] = sum_{a,b} K[a,b] cos(pi k0 a / m) cos(pi k1 b / m).
// Job: m, i0 = r0, i1 = r1.
__global__ void __launch_bounds__(NTHREADS) k_gcv_symbol(const Job* __restrict__ jobs,
                                                         const uint32_t* __restrict__ tiles) {
  const Job* job; int ti, tj, tix;
  decode_tile(jobs, tiles, job, ti, tj, tix);
  const int m = job->m;
  int i0, j0, TI, TJ;
  tile_geom<float>(m, ti, tj, i0, j0, TI, TJ);
  const int r0 = job->i0, r1 = job->i1, n0 = 2 * r0 + 1;
  const double* __restrict__ K = static_cast<const double*>(job->v[G_KINT]);
  double* __restrict__ sym = static_cast<double*>(job->v[G_SYM]);
  const double w = 3.14159265358979323846 / m;
  for (int o = threadIdx.x; o < TI * TJ; o += NTHREADS) {
    const int k0 = i0 + o % TI, k1 = j0 + o / TI;
    double acc = 0.0;
    for (int b = -r1; b <= r1; ++b) {
      double inner = 0.0;
      for (int a = -r0; a <= r0; ++a) inner += K[(a + r0) + (size_t)(b + r1) * n0] * cos(w * k0 * a);
      acc += inner * cos(w * k1 * b);
    }
    sym[k0 + (size_t)k1 * m] = acc;
  }
}

// ---------------------------------------------------------------- prep ----
// i0 = 0: in = (double) b.  i0 = 1: in = L^T c (c = c1 - c2), plus the sum of
// squared IRLS weights when G_W is set (scal[S_G_WBAR] = sum w^2 / n_L).
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
  double wsq = 0.0;
  if (job->i0 == 0) {
    const T* __restrict__ b = static_cast<const T*>(job->v[G_B]);
    for (int o = threadIdx.x; o < TI * TJ; o += NTHREADS) {
      const size_t g = (i0 + o % TI) + (size_t)(j0 + o / TI) * m;
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
    const int gi = i0 + o % TI, gj = j0 + o / TI;
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
      if (gi < m - 1) { const double v = w[gi + (size_t)gj * (m - 1)]; wsq += v * v; }
      if (gj < m - 1) { const double v = w[nx + g]; wsq += v * v; }
    }
  }
  double vv[1] = {wsq}, tot[1];
  if (job_reduce<1>(job, tix, vv, red, tot))
    put_scal(job->scal, S_G_WBAR, w ? tot[0] / (2.0 * (double)m * (m - 1)) : 1.0);
}

// ---------------------------------------------------------------- GEMM ----
// out = A * B (i0 = 0) or A * B^T (i0 = 1); m x m FP64, column-major.
// v[0] = A, v[1] = B, v[2] = out.  64 x 64 output tiles, 4 x 4 per thread.
__global__ void __launch_bounds__(NTHREADS) k_gemm64(const Job* __restrict__ jobs,
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
  const int tr = threadIdx.x % 16, tc = threadIdx.x / 16;  // 16 x 16 threads
  double acc[4][4] = {};
  for (int k0 = 0; k0 < m; k0 += 16) {
    const int kk = m - k0 < 16 ? m - k0 : 16;
    for (int idx = threadIdx.x; idx < 16 * 64; idx += NTHREADS) {
      const int r = idx % 64, k = idx / 64;  // A(i0 + r, k0 + k)
      As[k][r] = (r < TS && k < kk) ? A[(i0 + r) + (size_t)(k0 + k) * m] : 0.0;
      const int c = idx % 64, k2 = idx / 64;
      double bv = 0.0;
      if (c < TS && k2 < kk)
        bv = tb ? B[(j0 + c) + (size_t)(k0 + k2) * m] : B[(k0 + k2) + (size_t)(j0 + c) * m];
      Bs[k2][c] = bv;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      double a[4], b[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        a[u] = As[k][tr + 16 * u];
        b[u] = Bs[k][tc + 16 * u];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[u][v] = fma(a[u], b[v], acc[u][v]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = tr + 16 * u, c = tc + 16 * v;
      if (r < TS && c < TS) C[(i0 + r) + (size_t)(j0 + c) * m] = acc[u][v];
    }
}

// ---------------------------------------------------------------- data ----
// e_k = (a c^ - lp b^)^2 in place of c^ (or with c^ = 0 when i0 == 0), and
// the grid bounds from min / max of log10(s / lp) over lp > 0, s > 0.
__global__ void __launch_bounds__(NTHREADS) k_gcv_data(const Job* __restrict__ jobs,
                                                       const uint32_t* __restrict__ tiles) {
  __shared__ double red[8];
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
  const double wb2 = job->scal[S_G_WBAR];
  double lo = 1e300, hi = -1e300;
  for (int o = threadIdx.x; o < TI * TJ; o += NTHREADS) {
    const int k0 = i0 + o % TI, k1 = j0 + o / TI;
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
  // min / max through the sum reduction: reduce (-lo, hi) with max below.
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    lo = fmin(lo, __shfl_xor(lo, off, 64));
    hi = fmax(hi, __shfl_xor(hi, off, 64));
  }
  __shared__ double sl[4], sh[4];
  __shared__ int s_last;
  if (lane == 0) { sl[wid] = lo; sh[wid] = hi; }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < 4; ++w) { lo = fmin(lo, sl[w]); hi = fmax(hi, sh[w]); }
    __hip_atomic_store(job->part + 2 * tix, lo, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(job->part + 2 * tix + 1, hi, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __threadfence();
    const unsigned prev = atomicAdd(job->cnt, 1u);
    s_last = prev == unsigned(job->nti * job->ntj - 1);
  }
  __syncthreads();
  if (!s_last || threadIdx.x != 0) return;
  __threadfence();
  const int nt = job->nti * job->ntj;
  double L = 1e300, Hh = -1e300;
  for (int t = 0; t < nt; ++t) {
    L = fmin(L, __hip_atomic_load(job->part + 2 * t, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    Hh = fmax(Hh, __hip_atomic_load(job->part + 2 * t + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
  }
  (void)red;
  put_scal(job->scal, S_G_THI, Hh);
  put_scal(job->scal, S_G_TLO, fmax(L, Hh - 14.0));
  __hip_atomic_store(job->cnt, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Per-thread view of the frequencies of one tile (at most 16 per thread).
struct FreqRegs {
  double s[16], lp[16], e[16];
  int cnt;
};

__device__ __forceinline__ void load_freqs(const Job* job, int i0, int j0, int TI, int TJ,
                                           FreqRegs& f) {
  const int m = job->m;
  const double* __restrict__ sym = static_cast<const double*>(job->v[G_SYM]);
  const double* __restrict__ lam = static_cast<const double*>(job->v[G_LAM]);
  const double* __restrict__ e = static_cast<const double*>(job->v[G_E]);
  const double wb2 = job->scal[S_G_WBAR];
  f.cnt = 0;
  for (int o = threadIdx.x; o < TI * TJ; o += NTHREADS) {
    const int k0 = i0 + o % TI, k1 = j0 + o / TI;
    const size_t g = k0 + (size_t)k1 * m;
    const double a = sym[g];
    f.s[f.cnt] = a * a;
    f.lp[f.cnt] = wb2 * (lam[k0] + lam[k1]);
    f.e[f.cnt] = e[g];
    ++f.cnt;
  }
}

__device__ __forceinline__ void eval_freqs(const FreqRegs& f, double gam, double& res,
                                           double& tr) {
  res = 0.0;
  tr = 0.0;
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    if (q < f.cnt) {
      const double den = f.s[q] + gam * f.lp[q];
      if (den > 0.0) {
        res += f.e[q] / (den * den);
        tr += f.s[q] / den;
      }
    }
  }
}

// ---------------------------------------------------------------- grid ----
// Job::i1 = number of grid points.  Partials: 2 per point per tile.
__global__ void __launch_bounds__(NTHREADS) k_gcv_grid(const Job* __restrict__ jobs,
                                                       const uint32_t* __restrict__ tiles) {
  __shared__ double red[2 * 4];
  __shared__ int s_last;
  const Job* job; int ti, tj, tix;
  decode_tile(jobs, tiles, job, ti, tj, tix);
  const int m = job->m, npts = job->i1;
  int i0, j0, TI, TJ;
  tile_geom<float>(m, ti, tj, i0, j0, TI, TJ);
  FreqRegs f;
  load_freqs(job, i0, j0, TI, TJ, f);
  const double tlo = job->scal[S_G_TLO], thi = job->scal[S_G_THI];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  for (int p = 0; p < npts; ++p) {
    const double t = tlo + (thi - tlo) * p / (npts - 1);
    double res, tr;
    eval_freqs(f, pow(10.0, t), res, tr);
    res = wave_sum(res);
    tr = wave_sum(tr);
    if (lane == 0) { red[wid] = res; red[4 + wid] = tr; }
    __syncthreads();
    if (threadIdx.x == 0) {
      double a = 0.0, b = 0.0;
      for (int w = 0; w < 4; ++w) { a += red[w]; b += red[4 + w]; }
      __hip_atomic_store(job->part + (size_t)tix * 2 * npts + 2 * p, a, __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(job->part + (size_t)tix * 2 * npts + 2 * p + 1, b, __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    __threadfence();
    const unsigned prev = atomicAdd(job->cnt, 1u);
    s_last = prev == unsigned(job->nti * job->ntj - 1);
  }
  __syncthreads();
  if (!s_last) return;
  __threadfence();
  // last block: one thread per grid point sums the tiles in order
  const int nt = job->nti * job->ntj;
  double* sc = job->scal;
  const int n = m * m;
  if (threadIdx.x < npts) {
    const int p = threadIdx.x;
    double a = 0.0, b = 0.0;
    for (int t = 0; t < nt; ++t) {
      a += __hip_atomic_load(job->part + (size_t)t * 2 * npts + 2 * p, __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
      b += __hip_atomic_load(job->part + (size_t)t * 2 * npts + 2 * p + 1, __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
    }
    const double t = tlo + (thi - tlo) * p / (npts - 1);
    sc[S_GRID + p] = gcv_from(pow(10.0, t), a, b, n);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int jb = 0;
    double best = sc[S_GRID];
    for (int p = 1; p < npts; ++p)
      if (sc[S_GRID + p] < best) { best = sc[S_GRID + p]; jb = p; }
    const double step = (thi - tlo) / (npts - 1);
    const double a = tlo + step * (jb > 0 ? jb - 1 : 0);
    const double b = tlo + step * (jb < npts - 1 ? jb + 1 : npts - 1);
    const double golden = 0.5 * (3.0 - sqrt(5.0));
    const double x = a + golden * (b - a);
    put_scal(sc, S_G_A, a);
    put_scal(sc, S_G_B, b);
    put_scal(sc, S_G_X, x);
    put_scal(sc, S_G_W, x);
    put_scal(sc, S_G_V, x);
    put_scal(sc, S_G_D, 0.0);
    put_scal(sc, S_G_E, 0.0);
    put_scal(sc, S_G_U, x);
    put_scal(sc, S_G_IT, -1.0);  // -1: the next evaluation is the start point
    put_scal(sc, S_G_DONE, 0.0);
    put_scal(sc, S_G_NEV, 0.0);
    __hip_atomic_store(job->cnt, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// --------------------------------------------------------------- Brent ----
// One evaluation per launch.  Job::i1 = max Brent steps; p0 = xtol.
__global__ void __launch_bounds__(NTHREADS) k_gcv_brent(const Job* __restrict__ jobs,
                                                        const uint32_t* __restrict__ tiles) {
  __shared__ double red[8];
  const Job* job; int ti, tj, tix;
  decode_tile(jobs, tiles, job, ti, tj, tix);
  double* sc = job->scal;
  if (sc[S_G_DONE] != 0.0) return;
  const int m = job->m;
  int i0, j0, TI, TJ;
  tile_geom<float>(m, ti, tj, i0, j0, TI, TJ);
  FreqRegs f;
  load_freqs(job, i0, j0, TI, TJ, f);
  const double u = sc[S_G_U];
  double res, tr;
  eval_freqs(f, pow(10.0, u), res, tr);
  double vv[2] = {res, tr}, tot[2];
  if (!job_reduce<2>(job, tix, vv, red, tot)) return;
  // ---- state machine (thread 0 of the job's last block) ----
  const int n = m * m;
  const double fu = gcv_from(pow(10.0, u), tot[0], tot[1], n);
  const double golden = 0.5 * (3.0 - sqrt(5.0));
  const double sqeps = sqrt(2.220446049250313e-16);
  const double xtol = job->p0;
  const int maxit = job->i1;
  double a = sc[S_G_A], b = sc[S_G_B], x = sc[S_G_X], w = sc[S_G_W], v = sc[S_G_V];
  double fx = sc[S_G_FX], fw = sc[S_G_FW], fv = sc[S_G_FV], d = sc[S_G_D], e = sc[S_G_E];
  int it = (int)sc[S_G_IT];
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
  put_scal(sc, S_G_A, a);
  put_scal(sc, S_G_B, b);
  put_scal(sc, S_G_X, x);
  put_scal(sc, S_G_W, w);
  put_scal(sc, S_G_V, v);
  put_scal(sc, S_G_FX, fx);
  put_scal(sc, S_G_FW, fw);
  put_scal(sc, S_G_FV, fv);
  put_scal(sc, S_G_D, d);
  put_scal(sc, S_G_E, e);
  put_scal(sc, S_G_IT, (double)it);
  put_scal(sc, S_G_NEV, sc[S_G_NEV] + 1.0);
  if (done) {
    const double g = pow(10.0, x);
    put_scal(sc, S_GAMMA, g);
    put_scal(sc, S_SQRTG, sqrt(g));
    put_scal(sc, S_G_FBEST, fx);
    put_scal(sc, S_G_DONE, 1.0);
  } else {
    put_scal(sc, S_G_U, unext);
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
hipError_t launch_gemm64(const LaunchArgs& la) { GLAUNCH(k_gemm64, la); return hipGetLastError(); }
hipError_t launch_gcv_symbol(const LaunchArgs& la) {
  GLAUNCH(k_gcv_symbol, la);
  return hipGetLastError();
}
hipError_t launch_gcv_data(const LaunchArgs& la) { GLAUNCH(k_gcv_data, la); return hipGetLastError(); }
hipError_t launch_gcv_grid(const LaunchArgs& la, int) { GLAUNCH(k_gcv_grid, la); return hipGetLastError(); }
hipError_t launch_gcv_brent(const LaunchArgs& la) { GLAUNCH(k_gcv_brent, la); return hipGetLastError(); }

}  // namespace dbl
