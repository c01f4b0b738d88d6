// Operator kernels: blur A^(i) / A^(i)^T, gradient L / L^T, periodic wavelet
// restriction, prolongation, four-band DWT and the Approach D block transfer.
// Each kernel walks a tile table over a list of jobs (common.h).
#include "launch.h"
#include "stencil.h"

namespace dbl {

// ------------------------------------------------------------- filters ----
// Low-pass filters of Sec. 4 and the high-pass partner g_k = (-1)^k h_{k-1-k}.
__device__ __forceinline__ double wl_h(int wav, int k) {
  if (wav == 0) return 0.70710678118654752440;
  // (1 + s3, 3 + s3, 3 - s3, 1 - s3) / (4 sqrt 2)
  const double s3 = 1.73205080756887729353, d = 5.65685424949238019520;
  switch (k) {
    case 0: return (1.0 + s3) / d;
    case 1: return (3.0 + s3) / d;
    case 2: return (3.0 - s3) / d;
    default: return (1.0 - s3) / d;
  }
}
__device__ __forceinline__ int wl_len(int wav) { return wav == 0 ? 2 : 4; }
__device__ __forceinline__ double wl_g(int wav, int k) {
  const int K = wl_len(wav);
  return ((k & 1) ? -1.0 : 1.0) * wl_h(wav, K - 1 - k);
}

// ---------------------------------------------------------------- blur ----
// v[0] = input, v[1] = output; flags & F_ADJ selects A^T.
template <typename T, int RB>
__global__ void __launch_bounds__(NTHREADS, sizeof(T) == 4 ? 3 : 2) k_apply_sep(const Job* __restrict__ jobs,
                                                        const uint32_t* __restrict__ tiles) {
  extern __shared__ __align__(16) unsigned char smem[];
  const Job* job; int ti, tj, tix;
  decode_tile(jobs, tiles, job, ti, tj, tix);
  const int m = job->m;
  int i0, j0, TI, TJ;
  tile_geom<T>(m, ti, tj, i0, j0, TI, TJ);
  T* Xs = reinterpret_cast<T*>(smem);
  T* Zs = Xs + (TI + 2 * RB) * sep_lx(TJ, RB);
  const T* __restrict__ in = static_cast<const T*>(job->v[0]);
  T* __restrict__ out = static_cast<T*>(job->v[1]);
  load_tile<T, true>(Xs, sep_lx(TJ, RB), i0, j0, TI, TJ, RB, m, [&](int g) { return in[g]; });
  __syncthreads();
  const LevelOp& op = *job->op;
  const bool adj = job->flags & F_ADJ;
  sep_tile<T, RB>(Xs, RB, Zs, adj ? op.a0 : op.f0, adj ? op.a1 : op.f1, i0, j0, TI, TJ, m,
                  [&](int i, int j, T v) { out[(i0 + i) + (size_t)(j0 + j) * m] = v; });
}

template <typename T>
__global__ void __launch_bounds__(NTHREADS) k_apply_gen(const Job* __restrict__ jobs,
                                                        const uint32_t* __restrict__ tiles) {
  extern __shared__ __align__(16) unsigned char smem[];
  const Job* job; int ti, tj, tix;
  decode_tile(jobs, tiles, job, ti, tj, tix);
  const int m = job->m;
  int i0, j0, TI, TJ;
  tile_geom<T>(m, ti, tj, i0, j0, TI, TJ);
  const LevelOp& op = *job->op;
  const int H = op.R;
  T* Xs = reinterpret_cast<T*>(smem);
  T* s_v = Xs + col_lds_elems(TI, TJ, H);
  short2* s_e = reinterpret_cast<short2*>(s_v + (2 * H + 1) * (2 * H + 1));
  const T* __restrict__ in = static_cast<const T*>(job->v[0]);
  T* __restrict__ out = static_cast<T*>(job->v[1]);
  load_tile<T, false>(Xs, col_lx(TI, H), i0, j0, TI, TJ, H, m, [&](int g) { return in[g]; });
  __syncthreads();
  const bool adj = job->flags & F_ADJ;
  gen_tile<T>(Xs, H, adj ? op.a2 : op.f2, s_e, s_v, i0, j0, TI, TJ, m,
              [&](int i, int j, T v) { out[(i0 + i) + (size_t)(j0 + j) * m] = v; });
}

// ------------------------------------------------------------ gradient ----
// v[0] = x (m x m), v[1] = q (n_L): q = L x.
template <typename T>
__global__ void __launch_bounds__(NTHREADS) k_grad(const Job* __restrict__ jobs,
                                                   const uint32_t* __restrict__ tiles) {
  const Job* job; int ti, tj, tix;
  decode_tile(jobs, tiles, job, ti, tj, tix);
  const int m = job->m;
  int i0, j0, TI, TJ;
  tile_geom<T>(m, ti, tj, i0, j0, TI, TJ);
  const T* __restrict__ x = static_cast<const T*>(job->v[0]);
  T* __restrict__ q = static_cast<T*>(job->v[1]);
  const size_t nx = (size_t)(m - 1) * m;
  for (int o = threadIdx.x; o < TI * TJ; o += NTHREADS) {
    const int i = i0 + (o & (TI - 1)), j = j0 + (o >> (__ffs(TI) - 1));
    const T xc = x[i + (size_t)j * m];
    if (i < m - 1) q[i + (size_t)j * (m - 1)] = x[i + 1 + (size_t)j * m] - xc;
    if (j < m - 1) q[nx + i + (size_t)j * m] = x[i + (size_t)(j + 1) * m] - xc;
  }
}

// v[0] = q (n_L), v[1] = y (m x m): y = L^T q = vec(D^T Qx + Qy D).
template <typename T>
__global__ void __launch_bounds__(NTHREADS) k_gradT(const Job* __restrict__ jobs,
                                                    const uint32_t* __restrict__ tiles) {
  const Job* job; int ti, tj, tix;
  decode_tile(jobs, tiles, job, ti, tj, tix);
  const int m = job->m;
  int i0, j0, TI, TJ;
  tile_geom<T>(m, ti, tj, i0, j0, TI, TJ);
  const T* __restrict__ q = static_cast<const T*>(job->v[0]);
  T* __restrict__ y = static_cast<T*>(job->v[1]);
  const T* __restrict__ qy = q + (size_t)(m - 1) * m;
  for (int o = threadIdx.x; o < TI * TJ; o += NTHREADS) {
    const int i = i0 + (o & (TI - 1)), j = j0 + (o >> (__ffs(TI) - 1));
    T a = T(0);
    if (i >= 1) a += q[i - 1 + (size_t)j * (m - 1)];
    if (i < m - 1) a -= q[i + (size_t)j * (m - 1)];
    if (j >= 1) a += qy[i + (size_t)(j - 1) * m];
    if (j < m - 1) a -= qy[i + (size_t)j * m];
    y[i + (size_t)j * m] = a;
  }
}

// ------------------------------------------------------------- wavelets ----
// Jobs carry m = fine size; flags = wavelet id.  Restriction / forward DWT
// tiles cover the coarse grid, prolongation / inverse / transfer tiles the
// fine grid.

// v[0] = fine X, v[1] = coarse out (LL only) or 4 bands when p0 != 0.
template <typename T>
__global__ void __launch_bounds__(NTHREADS) k_dwt_fwd(const Job* __restrict__ jobs,
                                                      const uint32_t* __restrict__ tiles) {
  const Job* job; int ti, tj, tix;
  decode_tile(jobs, tiles, job, ti, tj, tix);
  const int m = job->m, mc = m >> 1, msk = m - 1;
  int i0, j0, TI, TJ;
  tile_geom<T>(mc, ti, tj, i0, j0, TI, TJ);
  const int wav = job->flags, K = wl_len(wav);
  const bool four = job->p0 != 0.0;
  const T* __restrict__ x = static_cast<const T*>(job->v[0]);
  T* __restrict__ y = static_cast<T*>(job->v[1]);
  const size_t nc = (size_t)mc * mc;
  for (int o = threadIdx.x; o < TI * TJ; o += NTHREADS) {
    const int a0 = i0 + (o & (TI - 1)), a1 = j0 + (o >> (__ffs(TI) - 1));
    double ll = 0, lh = 0, hl = 0, hh = 0;
    for (int b = 0; b < K; ++b) {
      const size_t col = (size_t)((2 * a1 + b) & msk) * m;
      double lo = 0, hi = 0;
      for (int a = 0; a < K; ++a) {
        const double v = (double)x[((2 * a0 + a) & msk) + col];
        lo += wl_h(wav, a) * v;
        hi += wl_g(wav, a) * v;
      }
      ll += wl_h(wav, b) * lo;
      if (four) {
        lh += wl_g(wav, b) * lo;
        hl += wl_h(wav, b) * hi;
        hh += wl_g(wav, b) * hi;
      }
    }
    const size_t k = a0 + (size_t)a1 * mc;
    y[k] = (T)ll;
    if (four) {
      y[nc + k] = (T)lh;
      y[2 * nc + k] = (T)hl;
      y[3 * nc + k] = (T)hh;
    }
  }
}

// v[0] = coarse LL (or 4 bands when p0 != 0), v[1] = fine out.
template <typename T>
__global__ void __launch_bounds__(NTHREADS) k_dwt_inv(const Job* __restrict__ jobs,
                                                      const uint32_t* __restrict__ tiles) {
  const Job* job; int ti, tj, tix;
  decode_tile(jobs, tiles, job, ti, tj, tix);
  const int m = job->m, mc = m >> 1, cm = mc - 1;
  int i0, j0, TI, TJ;
  tile_geom<T>(m, ti, tj, i0, j0, TI, TJ);
  const int wav = job->flags, K2 = wl_len(wav) / 2;
  const bool four = job->p0 != 0.0;
  const T* __restrict__ c = static_cast<const T*>(job->v[0]);
  T* __restrict__ x = static_cast<T*>(job->v[1]);
  const size_t nc = (size_t)mc * mc;
  for (int o = threadIdx.x; o < TI * TJ; o += NTHREADS) {
    const int f0 = i0 + (o & (TI - 1)), f1 = j0 + (o >> (__ffs(TI) - 1));
    double acc = 0;
    for (int t1 = 0; t1 < K2; ++t1) {
      const int c1 = ((f1 >> 1) - t1) & cm, k1 = (f1 & 1) + 2 * t1;
      for (int t0 = 0; t0 < K2; ++t0) {
        const int c0 = ((f0 >> 1) - t0) & cm, k0 = (f0 & 1) + 2 * t0;
        const size_t k = c0 + (size_t)c1 * mc;
        acc += wl_h(wav, k0) * wl_h(wav, k1) * (double)c[k];
        if (four) {
          acc += wl_h(wav, k0) * wl_g(wav, k1) * (double)c[nc + k];
          acc += wl_g(wav, k0) * wl_h(wav, k1) * (double)c[2 * nc + k];
          acc += wl_g(wav, k0) * wl_g(wav, k1) * (double)c[3 * nc + k];
        }
      }
    }
    x[f0 + (size_t)f1 * m] = (T)acc;
  }
}

// Approach D transfer.  v[0] = coarse gradient vector (mc), v[1] = fine one.
// Qx_f = W~1 Qx_c W1^T, Qy_f = W1 Qy_c W~1^T (W~1: W1 without its last row
// and last column).
template <typename T>
__global__ void __launch_bounds__(NTHREADS) k_dtransfer(const Job* __restrict__ jobs,
                                                        const uint32_t* __restrict__ tiles) {
  const Job* job; int ti, tj, tix;
  decode_tile(jobs, tiles, job, ti, tj, tix);
  const int m = job->m, mc = m >> 1, cm = mc - 1;
  int i0, j0, TI, TJ;
  tile_geom<T>(m, ti, tj, i0, j0, TI, TJ);
  const int wav = job->flags, K2 = wl_len(wav) / 2;
  const T* __restrict__ qc = static_cast<const T*>(job->v[0]);
  T* __restrict__ qf = static_cast<T*>(job->v[1]);
  const T* __restrict__ qyc = qc + (size_t)(mc - 1) * mc;
  T* __restrict__ qyf = qf + (size_t)(m - 1) * m;
  for (int o = threadIdx.x; o < TI * TJ; o += NTHREADS) {
    const int f0 = i0 + (o & (TI - 1)), f1 = j0 + (o >> (__ffs(TI) - 1));
    if (f0 < m - 1) {  // row block: rows of W~1 x columns of W1
      double acc = 0;
      for (int t1 = 0; t1 < K2; ++t1) {
        const int c1 = ((f1 >> 1) - t1) & cm, k1 = (f1 & 1) + 2 * t1;
        for (int t0 = 0; t0 < K2; ++t0) {
          const int c0 = ((f0 >> 1) - t0) & cm, k0 = (f0 & 1) + 2 * t0;
          if (c0 < mc - 1)
            acc += wl_h(wav, k0) * wl_h(wav, k1) * (double)qc[c0 + (size_t)c1 * (mc - 1)];
        }
      }
      qf[f0 + (size_t)f1 * (m - 1)] = (T)acc;
    }
    if (f1 < m - 1) {  // column block: W1 rows x W~1 columns
      double acc = 0;
      for (int t1 = 0; t1 < K2; ++t1) {
        const int c1 = ((f1 >> 1) - t1) & cm, k1 = (f1 & 1) + 2 * t1;
        if (c1 >= mc - 1) continue;
        for (int t0 = 0; t0 < K2; ++t0) {
          const int c0 = ((f0 >> 1) - t0) & cm, k0 = (f0 & 1) + 2 * t0;
          acc += wl_h(wav, k0) * wl_h(wav, k1) * (double)qyc[c0 + (size_t)c1 * mc];
        }
      }
      qyf[f0 + (size_t)f1 * m] = (T)acc;
    }
  }
}

// -------------------------------------------------------------- launchers --

template <typename T>
static hipError_t launch_apply(const LaunchArgs& la, int sep, int rb, int H) {
  const int ts = tile_edge(la.m_max);
  if (sep) {
    const size_t lds = sizeof(T) * sep_lds_elems(ts, ts, rb);
    switch (rb) {
#define CASE(R)                                                                      \
  case R:                                                                            \
    hipLaunchKernelGGL((k_apply_sep<T, R>), dim3(la.ntiles), dim3(NTHREADS), lds,   \
                       la.stream, la.jobs, la.tiles);                                \
    break;
      CASE(2) CASE(4) CASE(8) CASE(12) CASE(16)
#undef CASE
      default: return hipErrorInvalidValue;
    }
  } else {
    const size_t lds = sizeof(T) * col_lds_elems(ts, ts, H) +
                       (sizeof(T) + sizeof(short2)) * (2 * H + 1) * (2 * H + 1);
    hipLaunchKernelGGL((k_apply_gen<T>), dim3(la.ntiles), dim3(NTHREADS), lds, la.stream,
                       la.jobs, la.tiles);
  }
  return hipGetLastError();
}

hipError_t launch_apply_A(const LaunchArgs& la, int precision, int sep, int rb, int H) {
  return precision == 1 ? launch_apply<double>(la, sep, rb, H)
                        : launch_apply<float>(la, sep, rb, H);
}

#define SIMPLE_LAUNCHER(NAME, KERNEL)                                                   \
  hipError_t NAME(const LaunchArgs& la, int precision) {                               \
    if (precision == 1)                                                                \
      hipLaunchKernelGGL((KERNEL<double>), dim3(la.ntiles), dim3(NTHREADS), 0,         \
                         la.stream, la.jobs, la.tiles);                                \
    else                                                                               \
      hipLaunchKernelGGL((KERNEL<float>), dim3(la.ntiles), dim3(NTHREADS), 0,          \
                         la.stream, la.jobs, la.tiles);                                \
    return hipGetLastError();                                                          \
  }

SIMPLE_LAUNCHER(launch_grad, k_grad)
SIMPLE_LAUNCHER(launch_gradT, k_gradT)
SIMPLE_LAUNCHER(launch_dwt_fwd, k_dwt_fwd)
SIMPLE_LAUNCHER(launch_dwt_inv, k_dwt_inv)
SIMPLE_LAUNCHER(launch_dtransfer, k_dtransfer)

}  // namespace dbl
