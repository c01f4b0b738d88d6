// Solver kernels: the two fused CGLS phases on the augmented system of eq.
// (augmented), their start, the per-outer-iteration auxiliary updates of
// Algs. 1-3 (IRLS weights, MM shift, SB shrink and Bregman update) and the
// per-outer-iteration statistics (relative change of eq. (stop), objective).
//
// CGLS on [A; sqrt(g) D] x ~ [b; sqrt(g) c], x0 = 0, FP64 scalars:
//   init : x = 0, p = 0, r1 = b, r2 = sqrt(g) c
//   p2(first): s = A^T r1 + sqrt(g) D^T r2,  gs = |s|^2,  beta = 0
//   repeat:
//   p1   : p = s + beta p;  q1 = A p;  q2 = sqrt(g) D p;  alpha = gs / |q|^2
//   p2   : x += alpha p;  r -= alpha q;  s = A^T r1 + sqrt(g) D^T r2;
//          beta = |s|^2 / gs
// p, r1 and r2 are double-buffered (read one copy, write the other) because
// the stencils read neighbours that other blocks update in the same launch.
// S is the storage type of the state vectors p, s, r1, r2, q1, q2 (T, or
// bfloat16 with FP32 arithmetic); norms are taken of the stored values.
// The norms are per-tile FP64 partials: p1 writes |q|^2 partials and sums the
// |s|^2 partials of the previous p2 (beta); p2 sums both (alpha) and writes
// new |s|^2 and |r|^2 partials, which the next p1 reads.
#include "phase.h"

namespace dbl {

// ------------------------------------------------------------------ init --
template <typename T, typename S>
__global__ void __launch_bounds__(NTHREADS) k_cgls_init(const Job* __restrict__ jobs,
                                                        const uint32_t* __restrict__ tiles) {
  const Job* job; int ti, tj, tix;
  decode_tile(jobs, tiles, job, ti, tj, tix);
  const int m = job->m;
  int i0, j0, TI, TJ;
  tile_geom<T>(m, ti, tj, i0, j0, TI, TJ);
  const double sg = job->scal[S_SQRTG];
  const bool shift = job->flags & F_SHIFT, sb = job->flags & F_SB, irls = job->flags & F_IRLS;
  T* x = vp<T>(job, V_X);
  S* p = vp<S>(job, V_PA);
  S* r1 = vp<S>(job, V_R1A);
  S* r2 = vp<S>(job, V_R2A);
  const T* b = vp<T>(job, V_B);
  const T* c1 = vp<T>(job, V_C1);
  const T* c2 = vp<T>(job, V_C2);
  const T* w = vp<T>(job, V_W);
  const T* x0 = vp<T>(job, V_X0);   // optional start
  const T* ax0 = vp<T>(job, V_XOLD);  // A x0 when x0 is given
  const size_t nx = (size_t)(m - 1) * m;
  for (int o = threadIdx.x; o < TI * TJ; o += NTHREADS) {
    const int gi = i0 + (o & (TI - 1)), gj = j0 + (o >> (__ffs(TI) - 1));
    const size_t g = gi + (size_t)gj * m;
    double xv = 0.0;
    if (x0) {
      xv = (double)x0[g];
      stv(r1, g, (T)((double)b[g] - (double)ax0[g]));
    } else {
      stv(r1, g, b[g]);
    }
    x[g] = (T)xv;
    stv(p, g, T(0));
    for (int dir = 0; dir < 2; ++dir) {
      if ((dir == 0 && gi >= m - 1) || (dir == 1 && gj >= m - 1)) continue;
      const size_t k = dir == 0 ? gi + (size_t)gj * (m - 1) : nx + g;
      double c = 0.0;
      if (shift) c = (double)c1[k] - (sb ? (double)c2[k] : 0.0);
      if (x0) {
        const double nb = dir == 0 ? (double)x0[g + 1] : (double)x0[g + m];
        double d = nb - xv;
        if (irls) d *= (double)w[k];
        c -= d;
      }
      stv(r2, k, (T)(sg * c));
    }
  }
}

// --------------------------------------------------------------- phase 1 --
// Outputs per item of the separable convolution in each phase kernel (the
// per-output sums do not depend on it, only register use does).
constexpr int P1_V_NARROW = 2, P1_V_WIDE = 2;
constexpr int P2_V_NARROW = 2, P2_V_WIDE = 2;
constexpr int STATS_V = 2;
// Pixels whose gradient-entry loads each thread issues together in phase 2.
constexpr int P2_GRAD_BATCH = 2;
// Launches of more tiles than this (5 resident 256-thread blocks on each of
// 256 CUs at the unconstrained register use) take the _wide phase kernels.
constexpr int P2_WIDE_TILES = 5 * 256;
template <typename T, typename S, int RB, bool SEP, int CV>
__device__ __forceinline__ void cgls_p1_body(const Job* __restrict__ jobs,
                                             const uint32_t* __restrict__ tiles) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ double red[8];
  __shared__ double bc;
  __shared__ double bc2[2];
  const Job* job; int ti, tj, tix;
  decode_tile(jobs, tiles, job, ti, tj, tix);
  const int m = job->m;
  int i0, j0, TI, TJ;
  tile_geom<T>(m, ti, tj, i0, j0, TI, TJ);
  const LevelOp& op = *job->op;
  const int H = SEP ? RB : op.R;
  T* Xs = reinterpret_cast<T*>(smem);
  void* scratch = Xs + xs_elems<SEP>(H, TI, TJ);
  const int nt = job->nti * job->ntj;
  const double sg = job->scal[S_SQRTG];
  const bool irls = job->flags & F_IRLS;
  const S* __restrict__ s = vp<S>(job, V_S);
  const S* __restrict__ pa = vp<S>(job, V_PA);
  S* __restrict__ pb = vp<S>(job, V_PB);
  S* __restrict__ q1 = vp<S>(job, V_Q1);
  S* __restrict__ q2 = vp<S>(job, V_Q2);
  const T* __restrict__ w = vp<T>(job, V_W);
  const size_t nx = (size_t)(m - 1) * m;
  // IRLS weights of the thread's pixels (o = tid + u NTHREADS; a tile has at
  // most 32 x 32 pixels), requested with the tile so that they share its
  // memory round trip
  constexpr int WPT = 32 * 32 / NTHREADS;
  T wv[2 * WPT];
  auto load_w = [&]() {
#pragma unroll
    for (int u = 0; u < WPT; ++u) {
      const int o = threadIdx.x + u * NTHREADS;
      wv[2 * u] = T(1);
      wv[2 * u + 1] = T(1);
      if (irls && o < TI * TJ) {
        const int gi = i0 + (o & (TI - 1)), gj = j0 + (o >> (__ffs(TI) - 1));
        const size_t g = gi + (size_t)gj * m;
        if (gi < m - 1) wv[2 * u] = w[gi + (size_t)gj * (m - 1)];
        if (gj < m - 1) wv[2 * u + 1] = w[nx + g];
      }
    }
  };
  if (job->flags & F_FIRST) {  // p = s
    load_w();
    load_tile<T, SEP>(Xs, xs_ld<SEP>(H, TI, TJ), i0, j0, TI, TJ, H, m,
                      [&](int g) { return rtv<S>(ldv<T>(s, g) + T(0) * ldv<T>(pa, g)); });
  } else {
    // iteration > 0: beta = |s_k|^2 / |s_{k-1}|^2 from the partials, summed
    // while the tile loads are in flight
    load_tile_overlap<T, SEP>(
        Xs, xs_ld<SEP>(H, TI, TJ), i0, j0, TI, TJ, H, m,
        [&](int g) { return ldv<T>(s, g); }, [&](int g) { return ldv<T>(pa, g); },
        [&]() {
          load_w();
          double gcur, gprev;
          sum_partials2<2, 2>(job->pr[0], 0, job->pr[1], 0, nt, red, bc2, gcur, gprev);
          const double beta = gprev > 0.0 ? gcur / gprev : 0.0;
          if ((job->flags & F_HIST) && tix == 0) {
            const double rr = sum_partials<2>(job->pr[0], nt, 1, red, &bc);
            if (threadIdx.x == 0 && job->i0 >= 1 && job->i0 <= HIST_MAX)
              job->scal[S_HIST + job->i0 - 1] = rr;
          }
          return (T)beta;
        },
        [&](T a, T b, T c) { return rtv<S>(fma(c, b, a)); });
  }
  __syncthreads();
  // FP64 norm sums as explicit fma terms (an FP64 square is inexact: the
  // tile kernels form the same sums, and the compiler must not fuse them
  // differently in one kernel than in the other)
  double acc = 0.0;
#pragma unroll
  for (int u = 0; u < WPT; ++u) {
    const int o = threadIdx.x + u * NTHREADS;
    if (o < TI * TJ) {
      const T* v = wv + 2 * u;
      const int i = (o & (TI - 1)), j = (o >> (__ffs(TI) - 1)), gi = i0 + i, gj = j0 + j;
      const size_t g = gi + (size_t)gj * m;
      const T pc = Xs[xs_at<SEP>(i, j, H, TI, TJ)];
      stv(pb, g, pc);
      if (gi < m - 1) {
        const double d = ((double)Xs[xs_at<SEP>(i + 1, j, H, TI, TJ)] - (double)pc) * (double)v[0];
        const T qv = rtv<S>((T)(sg * d));
        stv(q2, gi + (size_t)gj * (m - 1), qv);
        acc = fma((double)qv, (double)qv, acc);
      }
      if (gj < m - 1) {
        const double d = ((double)Xs[xs_at<SEP>(i, j + 1, H, TI, TJ)] - (double)pc) * (double)v[1];
        const T qv = rtv<S>((T)(sg * d));
        stv(q2, nx + g, qv);
        acc = fma((double)qv, (double)qv, acc);
      }
    }
  }
  auto epi1 = [&](int i, int j, T v) {
    const T qv = rtv<S>(v);
    stv(q1, (i0 + i) + (size_t)(j0 + j) * m, qv);
    acc = fma((double)qv, (double)qv, acc);
  };
  conv_tile<T, RB, SEP, decltype(epi1), NoHook, CV>(Xs, H, scratch, op, false, i0, j0, TI, TJ,
                                                    m, epi1);
  double vv[1] = {acc};
  put_partials<1>(job->pw, tix, vv, red);
}

// Phase 1 compiled twice, as phase 2 below: k_cgls_p1_wide (register bound
// of 6 waves per SIMD for FP32 up to radius bucket 8: 75 VGPRs, no spills)
// for launches of more than P2_WIDE_TILES tiles, k_cgls_p1 otherwise.
template <typename T, typename S, int RB, bool SEP>
__global__ void __launch_bounds__(NTHREADS, (waves_per_simd<T, RB>()))
    k_cgls_p1(const Job* __restrict__ jobs, const uint32_t* __restrict__ tiles) {
  cgls_p1_body<T, S, RB, SEP, P1_V_NARROW>(jobs, tiles);
}
template <typename T, typename S, int RB, bool SEP>
__global__ void __launch_bounds__(NTHREADS, (p2_waves<T, RB>()))
    k_cgls_p1_wide(const Job* __restrict__ jobs, const uint32_t* __restrict__ tiles) {
  cgls_p1_body<T, S, RB, SEP, P1_V_WIDE>(jobs, tiles);
}

// --------------------------------------------------------------- phase 2 --
template <typename T, typename S, int RB, bool SEP, int CV>
__device__ __forceinline__ void cgls_p2_body(const Job* __restrict__ jobs,
                                             const uint32_t* __restrict__ tiles) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ double red[8];
  __shared__ double bc;
  __shared__ double bc2[2];
  const Job* job; int ti, tj, tix;
  decode_tile(jobs, tiles, job, ti, tj, tix);
  const int m = job->m;
  int i0, j0, TI, TJ;
  tile_geom<T>(m, ti, tj, i0, j0, TI, TJ);
  const LevelOp& op = *job->op;
  const int H = SEP ? RB : op.R;
  T* Xs = reinterpret_cast<T*>(smem);
  void* scratch = Xs + xs_elems<SEP>(H, TI, TJ);
  const bool first = job->flags & F_FIRST;
  const bool irls = job->flags & F_IRLS;
  const int nt = job->nti * job->ntj;
  double alpha = 0.0;
  const double sg = job->scal[S_SQRTG];
  T* __restrict__ x = vp<T>(job, V_X);
  const S* __restrict__ p = vp<S>(job, V_PB);
  const S* __restrict__ r1a = vp<S>(job, V_R1A);
  S* __restrict__ r1b = vp<S>(job, V_R1B);
  const S* __restrict__ q1 = vp<S>(job, V_Q1);
  const S* __restrict__ r2a = vp<S>(job, V_R2A);
  S* __restrict__ r2b = vp<S>(job, V_R2B);
  const S* __restrict__ q2 = vp<S>(job, V_Q2);
  const T* __restrict__ w = vp<T>(job, V_W);
  S* __restrict__ s = vp<S>(job, V_S);
  T ta = T(0);
  if (first) {
    load_tile<T, SEP>(Xs, xs_ld<SEP>(H, TI, TJ), i0, j0, TI, TJ, H, m,
                      [&](int g) { return ldv<T>(r1a, g); });
  } else {
    // alpha = |s|^2 / |q|^2 from the partials, summed while the tile loads
    // are in flight
    load_tile_overlap<T, SEP>(
        Xs, xs_ld<SEP>(H, TI, TJ), i0, j0, TI, TJ, H, m,
        [&](int g) { return ldv<T>(r1a, g); }, [&](int g) { return ldv<T>(q1, g); },
        [&]() {
          double qq, gs;
          sum_partials2<1, 2>(job->pr[0], 0, job->pr[1], 0, nt, red, bc2, qq, gs);
          alpha = qq > 0.0 ? gs / qq : 0.0;
          ta = (T)alpha;
          return ta;
        },
        [&](T a, T b, T c) { return rtv<S>(fma(-c, b, a)); });
  }
  __syncthreads();
  double accr = 0.0, accs = 0.0;
  // r1 of the tile from LDS (no global loads: x and p are read with the
  // gradient entries below, in the same memory round trip)
  for (int o = threadIdx.x; o < TI * TJ; o += NTHREADS) {
    const int i = (o & (TI - 1)), j = (o >> (__ffs(TI) - 1));
    const size_t g = (i0 + i) + (size_t)(j0 + j) * m;
    const T rv = Xs[xs_at<SEP>(i, j, H, TI, TJ)];
    stv(r1b, g, rv);
    accr = fma((double)rv, (double)rv, accr);
  }
  const size_t nx = (size_t)(m - 1) * m;
  // Gradient part: LT[i, j] = sqrt(g) (L^T (w r2_new))[i, j] for the tile,
  // computed cooperatively (coalesced loads, all threads) into LDS, and
  // r2_new written for the tile's own gradient entries.
  T* LT = nullptr;
  auto grad_part = [&](T* buf) {
    LT = buf;
    // per pixel: entries qx(i-1,j), qx(i,j), qy(i,j-1), qy(i,j) -> (r2a, q2, w),
    // then x and p for x += alpha p
    batched_pixels<P2_GRAD_BATCH, 14, T>(
        TI * TJ,
        [&](int o, T* v) {
          const int gi = i0 + (o & (TI - 1)), gj = j0 + (o >> (__ffs(TI) - 1));
          const size_t g = gi + (size_t)gj * m;
          size_t ks[4];
          bool ok[4];
          ok[0] = gi >= 1;      ks[0] = gi - 1 + (size_t)gj * (m - 1);
          ok[1] = gi < m - 1;   ks[1] = gi + (size_t)gj * (m - 1);
          ok[2] = gj >= 1;      ks[2] = nx + g - m;
          ok[3] = gj < m - 1;   ks[3] = nx + g;
#pragma unroll
          for (int d = 0; d < 4; ++d) {
            v[3 * d] = ok[d] ? ldv<T>(r2a, ks[d]) : T(0);
            v[3 * d + 1] = (ok[d] && !first) ? ldv<T>(q2, ks[d]) : T(0);
            v[3 * d + 2] = (ok[d] && irls) ? w[ks[d]] : T(1);
          }
          if (!first) {
            v[12] = x[g];
            v[13] = ldv<T>(p, g);
          }
        },
        [&](int o, T* v) {
          const int i = (o & (TI - 1)), j = (o >> (__ffs(TI) - 1)), gi = i0 + i, gj = j0 + j;
          const size_t g = gi + (size_t)gj * m;
          T rn[4];
#pragma unroll
          for (int d = 0; d < 4; ++d)
            rn[d] = first ? v[3 * d] : rtv<S>(fma(-ta, v[3 * d + 1], v[3 * d]));
          double lt = 0.0;
          if (gi >= 1) lt += (double)v[2] * (double)rn[0];
          if (gi < m - 1) {
            stv(r2b, gi + (size_t)gj * (m - 1), rn[1]);
            accr = fma((double)rn[1], (double)rn[1], accr);
            lt -= (double)v[5] * (double)rn[1];
          }
          if (gj >= 1) lt += (double)v[8] * (double)rn[2];
          if (gj < m - 1) {
            stv(r2b, nx + g, rn[3]);
            accr = fma((double)rn[3], (double)rn[3], accr);
            lt -= (double)v[11] * (double)rn[3];
          }
          buf[i + j * TI] = (T)(sg * lt);
          if (!first) x[g] = fma(ta, v[13], v[12]);
        });
    __syncthreads();
  };
  if constexpr (SEP) {
    auto epi2 = [&](int i, int j, T v) {
      const size_t g = (i0 + i) + (size_t)(j0 + j) * m;
      const T sv = rtv<S>(v + LT[i + j * TI]);
      stv(s, g, sv);
      accs = fma((double)sv, (double)sv, accs);
    };
    auto hook = [&] { grad_part(Xs); };
    conv_tile<T, RB, SEP, decltype(epi2), decltype(hook), CV>(Xs, H, scratch, op, true, i0, j0,
                                                               TI, TJ, m, epi2, hook);
  } else {
    grad_part(reinterpret_cast<T*>(scratch) + (2 * H + 1) * (2 * H + 1) * 2);
    conv_tile<T, RB, SEP>(Xs, H, scratch, op, true, i0, j0, TI, TJ, m, [&](int i, int j, T v) {
      const size_t g = (i0 + i) + (size_t)(j0 + j) * m;
      const T sv = rtv<S>(v + LT[i + j * TI]);
      stv(s, g, sv);
      accs = fma((double)sv, (double)sv, accs);
    });
  }
  double vv[2] = {accs, accr};
  put_partials<2>(job->pw, tix, vv, red);
}

// Phase 2 compiled twice: for launches that fill the chip (more tiles than
// are resident at the unconstrained occupancy) with the register bound of
// p2_waves, so that all tiles are resident in one round; otherwise without
// it (more registers, shorter per-block latency for small launches).
template <typename T, typename S, int RB, bool SEP>
__global__ void __launch_bounds__(NTHREADS, (waves_per_simd<T, RB>()))
    k_cgls_p2(const Job* __restrict__ jobs, const uint32_t* __restrict__ tiles) {
  cgls_p2_body<T, S, RB, SEP, P2_V_NARROW>(jobs, tiles);
}
template <typename T, typename S, int RB, bool SEP>
__global__ void __launch_bounds__(NTHREADS, (p2_waves<T, RB>()))
    k_cgls_p2_wide(const Job* __restrict__ jobs, const uint32_t* __restrict__ tiles) {
  cgls_p2_body<T, S, RB, SEP, P2_V_WIDE>(jobs, tiles);
}

// Residual norm after the last CGLS iteration (one block per job): sums the
// |r|^2 partials of the final p2 into scal[S_HIST + i0].
__global__ void __launch_bounds__(NTHREADS) k_cgls_hist(const Job* __restrict__ jobs,
                                                        const uint32_t* __restrict__ tiles) {
  __shared__ double red[8];
  __shared__ double bc;
  const Job* job = jobs + (tiles[blockIdx.x] >> 16);
  const double rr = sum_partials<2>(job->pr[0], job->i1, 1, red, &bc);
  if (threadIdx.x == 0 && job->i0 >= 0 && job->i0 < HIST_MAX) job->scal[S_HIST + job->i0] = rr;
}

// ------------------------------------------------------------------- aux --
// Job::i0 = AuxMode; p0 = eps, p1 = tau.  Reads x = v[V_X] with neighbours.
template <typename T>
__global__ void __launch_bounds__(NTHREADS) k_aux(const Job* __restrict__ jobs,
                                                  const uint32_t* __restrict__ tiles) {
  const Job* job; int ti, tj, tix;
  decode_tile(jobs, tiles, job, ti, tj, tix);
  const int m = job->m;
  int i0, j0, TI, TJ;
  tile_geom<T>(m, ti, tj, i0, j0, TI, TJ);
  const int mode = job->i0;
  const double eps = job->p0, tau = job->p1;
  const T* __restrict__ x = vp<T>(job, V_X);
  T* __restrict__ w = vp<T>(job, V_W);
  T* __restrict__ c1 = vp<T>(job, V_C1);
  T* __restrict__ c2 = vp<T>(job, V_C2);
  const size_t nx = (size_t)(m - 1) * m;
  for (int o = threadIdx.x; o < TI * TJ; o += NTHREADS) {
    const int gi = i0 + (o & (TI - 1)), gj = j0 + (o >> (__ffs(TI) - 1));
    const size_t g = gi + (size_t)gj * m;
    const double xc = (double)x[g];
    for (int dir = 0; dir < 2; ++dir) {
      if ((dir == 0 && gi >= m - 1) || (dir == 1 && gj >= m - 1)) continue;
      const size_t k = dir == 0 ? gi + (size_t)gj * (m - 1) : nx + g;
      const double u = (dir == 0 ? (double)x[g + 1] : (double)x[g + m]) - xc;
      if (mode == AUX_IRLS_W) {
        const double a = fabs(u) > eps ? fabs(u) : eps;
        w[k] = (T)(1.0 / sqrt(a));
      } else if (mode == AUX_MM_W) {
        c1[k] = (T)(u * (1.0 - sqrt(eps * eps / (u * u + eps * eps))));
      } else {
        const double v = mode == AUX_SB_UPDATE ? u + (double)c2[k] : u;
        const double av = fabs(v) - tau;
        const double d = av > 0.0 ? (v > 0.0 ? av : -av) : 0.0;
        const T dt = (T)d;
        c1[k] = dt;
        c2[k] = (T)(v - (double)dt);
      }
    }
  }
}

// ----------------------------------------------------------------- stats --
// Per outer iteration: partials of |x - x_old|^2, |x_old|^2, |A x - b|^2 and
// the solver penalty; the last block writes (gamma, RC, objective) to
// job->hist[3 * i0 ...].  flags: F_IRLS / F_MM / F_SB select the penalty.
// Everything is evaluated in FP64 from the stored x, x_old and b (whatever
// their type): A x with the FP64 tap tables, so that the objective is the
// FP64 objective of the stored iterate.
template <typename T, int RB, bool SEP>
__global__ void __launch_bounds__(NTHREADS, 2) k_stats(const Job* __restrict__ jobs,
                                                      const uint32_t* __restrict__ tiles) {
  using C = double;
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ double red[16];
  const Job* job; int ti, tj, tix;
  decode_tile(jobs, tiles, job, ti, tj, tix);
  const int m = job->m;
  int i0, j0, TI, TJ;
  tile_geom<T>(m, ti, tj, i0, j0, TI, TJ);
  const LevelOp& op = *job->op;
  const int H = SEP ? RB : op.R;
  C* Xs = reinterpret_cast<C*>(smem);
  void* scratch = Xs + xs_elems<SEP>(H, TI, TJ);
  const T* __restrict__ x = vp<T>(job, V_X);
  const T* __restrict__ xo = vp<T>(job, V_XOLD);
  const T* __restrict__ b = vp<T>(job, V_B);
  const double eps = job->p0;
  const int fl = job->flags;
  load_tile<C, SEP>(Xs, xs_ld<SEP>(H, TI, TJ), i0, j0, TI, TJ, H, m,
                    [&](int g) { return (C)x[g]; });
  __syncthreads();
  double num = 0.0, den = 0.0, res = 0.0, pen = 0.0;
  for (int o = threadIdx.x; o < TI * TJ; o += NTHREADS) {
    const int i = (o & (TI - 1)), j = (o >> (__ffs(TI) - 1)), gi = i0 + i, gj = j0 + j;
    const size_t g = gi + (size_t)gj * m;
    const double xc = (double)Xs[xs_at<SEP>(i, j, H, TI, TJ)];
    const double xv = (double)xo[g];
    num += (xc - xv) * (xc - xv);
    den += xv * xv;
    for (int dir = 0; dir < 2; ++dir) {
      if ((dir == 0 && gi >= m - 1) || (dir == 1 && gj >= m - 1)) continue;
      const double t = (double)Xs[dir == 0 ? xs_at<SEP>(i + 1, j, H, TI, TJ)
                                           : xs_at<SEP>(i, j + 1, H, TI, TJ)] - xc;
      const double at = fabs(t);
      if (fl & F_IRLS) pen += at <= eps ? t * t / (2.0 * eps) : at - 0.5 * eps;
      else if (fl & F_MM) pen += sqrt(t * t + eps * eps);
      else pen += at;
    }
  }
  auto epi = [&](int i, int j, C v) {
    const double r = v - (double)b[(i0 + i) + (size_t)(j0 + j) * m];
    res += r * r;
  };
  conv_tile<C, RB, SEP, decltype(epi), NoHook, STATS_V>(Xs, H, scratch, op, false, i0, j0, TI,
                                                        TJ, m, epi);
  double vv[4] = {num, den, res, pen};
  put_partials<4>(job->pw, tix, vv, red);
}

// One block per job: total the stats partials (pr[0], i1 tiles) and write
// (gamma, RC, objective) to hist[3 * i0 ...].
__global__ void __launch_bounds__(NTHREADS) k_stats_fin(const Job* __restrict__ jobs,
                                                        const uint32_t* __restrict__ tiles) {
  __shared__ double red[8];
  __shared__ double bc;
  const Job* job = jobs + (tiles[blockIdx.x] >> 16);
  const int nt = job->i1;
  double tot[4];
  for (int c = 0; c < 4; ++c) tot[c] = sum_partials<4>(job->pr[0], nt, c, red, &bc);
  if (threadIdx.x != 0) return;
  const int fl = job->flags;
  const double gam = job->scal[S_GAMMA], eps = job->p0;
  double coef;
  if (fl & F_IRLS) coef = 2.0 * gam;
  else if (fl & F_MM) coef = 2.0 * eps * gam;
  else coef = 2.0 * job->p1 * gam;
  const double rc = tot[1] > 0.0 ? sqrt(tot[0] / tot[1]) : __builtin_nan("");
  double* h = job->hist + 3 * job->i0;
  h[0] = gam;
  h[1] = rc;
  h[2] = tot[2] + coef * tot[3];
  if (double* out = static_cast<double*>(job->v[V_RCOUT])) *out = rc;
}

// ------------------------------------------------------------- set gamma --
// One block per job: scal[S_GAMMA] = p0, scal[S_SQRTG] = p1 (fixed parameters).
__global__ void __launch_bounds__(64) k_set_gamma(const Job* __restrict__ jobs,
                                                  const uint32_t* __restrict__ tiles) {
  const Job* job = jobs + (tiles[blockIdx.x] >> 16);
  if (threadIdx.x == 0) {
    job->scal[S_GAMMA] = job->p0;
    job->scal[S_SQRTG] = job->p1;
  }
}

// ------------------------------------------------------------------ fill --
// v[0] (image space, may be null) and v[1] (gradient space, may be null) <- p0.
template <typename T>
__global__ void __launch_bounds__(NTHREADS) k_fill(const Job* __restrict__ jobs,
                                                   const uint32_t* __restrict__ tiles) {
  const Job* job; int ti, tj, tix;
  decode_tile(jobs, tiles, job, ti, tj, tix);
  const int m = job->m;
  int i0, j0, TI, TJ;
  tile_geom<T>(m, ti, tj, i0, j0, TI, TJ);
  T* a = vp<T>(job, 0);
  T* q = vp<T>(job, 1);
  const T val = (T)job->p0;
  const size_t nx = (size_t)(m - 1) * m;
  for (int o = threadIdx.x; o < TI * TJ; o += NTHREADS) {
    const int gi = i0 + (o & (TI - 1)), gj = j0 + (o >> (__ffs(TI) - 1));
    const size_t g = gi + (size_t)gj * m;
    if (a) a[g] = val;
    if (q) {
      if (gi < m - 1) q[gi + (size_t)gj * (m - 1)] = val;
      if (gj < m - 1) q[nx + g] = val;
    }
  }
}

// -------------------------------------------------------------- launchers --

template <typename T, template <typename, int, bool> class K>
struct Dummy {};

#define DISPATCH_STENCIL(KERNEL, T, la, sep, rb, H, extra_lds)                           \
  do {                                                                                 \
    const int ts_ = tile_edge((la).m_max);                                             \
    if (sep) {                                                                         \
      const size_t lds_ = sizeof(T) * sep_lds_elems(ts_, ts_, rb);                     \
      switch (rb) {                                                                    \
        case 2: hipLaunchKernelGGL((KERNEL<T, 2, true>), dim3((la).ntiles),           \
                    dim3(NTHREADS), lds_, (la).stream, (la).jobs, (la).tiles); break;  \
        case 4: hipLaunchKernelGGL((KERNEL<T, 4, true>), dim3((la).ntiles),           \
                    dim3(NTHREADS), lds_, (la).stream, (la).jobs, (la).tiles); break;  \
        case 8: hipLaunchKernelGGL((KERNEL<T, 8, true>), dim3((la).ntiles),           \
                    dim3(NTHREADS), lds_, (la).stream, (la).jobs, (la).tiles); break;  \
        case 12: hipLaunchKernelGGL((KERNEL<T, 12, true>), dim3((la).ntiles),         \
                    dim3(NTHREADS), lds_, (la).stream, (la).jobs, (la).tiles); break;  \
        case 16: hipLaunchKernelGGL((KERNEL<T, 16, true>), dim3((la).ntiles),         \
                    dim3(NTHREADS), lds_, (la).stream, (la).jobs, (la).tiles); break;  \
        default: return hipErrorInvalidValue;                                          \
      }                                                                                \
    } else {                                                                           \
      const size_t lds_ = sizeof(T) * col_lds_elems(ts_, ts_, H) +                     \
                          (2 * sizeof(T) + sizeof(short2)) * (2 * (H) + 1) * (2 * (H) + 1) + \
                          sizeof(T) * ts_ * ts_;                                      \
      hipLaunchKernelGGL((KERNEL<T, 0, false>), dim3((la).ntiles), dim3(NTHREADS),    \
                         lds_, (la).stream, (la).jobs, (la).tiles);                    \
    }                                                                                  \
  } while (0)

int cgls_wide_tiles() { return P2_WIDE_TILES; }

// The radius bucket that holds a general operator's radius H (its tile
// kernels' halo).
static int gen_halo(int H) { return H <= 2 ? 2 : H <= 4 ? 4 : H <= 8 ? 8 : H <= 12 ? 12 : 16; }

hipError_t launch_cgls_p1(const LaunchArgs& la, int precision, int sep, int rb, int H) {
  const bool wide = la.wide >= 0 ? la.wide != 0 : la.ntiles > P2_WIDE_TILES;
  if (sep && la.multi) return launch_cgls_multi(la, 1, precision, rb);
  if (sep && la.tile32) return launch_cgls_p1_sep(la, precision, rb, wide);
  if (!sep && la.tile32) return launch_cgls_p1_gen(la, precision, gen_halo(H));
  if (precision == 1) DISPATCH_STENCIL_S(k_cgls_p1, double, double, la, sep, rb, H);
  else if (wide && precision == 2)
    DISPATCH_STENCIL_S(k_cgls_p1_wide, float, bf16s, la, sep, rb, H);
  else if (precision == 2) DISPATCH_STENCIL_S(k_cgls_p1, float, bf16s, la, sep, rb, H);
  else if (wide)
    DISPATCH_STENCIL_S(k_cgls_p1_wide, float, float, la, sep, rb, H);
  else DISPATCH_STENCIL_S(k_cgls_p1, float, float, la, sep, rb, H);
  return hipGetLastError();
}

hipError_t launch_cgls_p2(const LaunchArgs& la, int precision, int sep, int rb, int H) {
  const bool wide = la.wide >= 0 ? la.wide != 0 : la.ntiles > P2_WIDE_TILES;
  if (sep && la.multi) return launch_cgls_multi(la, 2, precision, rb);
  if (sep && la.tile32) return launch_cgls_p2_sep(la, precision, rb, wide);
  if (!sep && la.tile32) return launch_cgls_p2_gen(la, precision, gen_halo(H));
  if (precision == 1) DISPATCH_STENCIL_S(k_cgls_p2, double, double, la, sep, rb, H);
  else if (wide && precision == 2)
    DISPATCH_STENCIL_S(k_cgls_p2_wide, float, bf16s, la, sep, rb, H);
  else if (precision == 2) DISPATCH_STENCIL_S(k_cgls_p2, float, bf16s, la, sep, rb, H);
  else if (wide)
    DISPATCH_STENCIL_S(k_cgls_p2_wide, float, float, la, sep, rb, H);
  else DISPATCH_STENCIL_S(k_cgls_p2, float, float, la, sep, rb, H);
  return hipGetLastError();
}

// The statistics kernel computes in FP64 whatever the storage type: its LDS
// is sized for doubles.
#define DISPATCH_STATS(T, la, sep, rb, H)                                               \
  do {                                                                                 \
    const int ts_ = tile_edge((la).m_max);                                             \
    if (sep) {                                                                         \
      const size_t lds_ = sizeof(double) * sep_lds_elems(ts_, ts_, rb);                \
      switch (rb) {                                                                    \
        case 2: hipLaunchKernelGGL((k_stats<T, 2, true>), dim3((la).ntiles),           \
                    dim3(NTHREADS), lds_, (la).stream, (la).jobs, (la).tiles); break;  \
        case 4: hipLaunchKernelGGL((k_stats<T, 4, true>), dim3((la).ntiles),           \
                    dim3(NTHREADS), lds_, (la).stream, (la).jobs, (la).tiles); break;  \
        case 8: hipLaunchKernelGGL((k_stats<T, 8, true>), dim3((la).ntiles),           \
                    dim3(NTHREADS), lds_, (la).stream, (la).jobs, (la).tiles); break;  \
        case 12: hipLaunchKernelGGL((k_stats<T, 12, true>), dim3((la).ntiles),         \
                    dim3(NTHREADS), lds_, (la).stream, (la).jobs, (la).tiles); break;  \
        case 16: hipLaunchKernelGGL((k_stats<T, 16, true>), dim3((la).ntiles),         \
                    dim3(NTHREADS), lds_, (la).stream, (la).jobs, (la).tiles); break;  \
        default: return hipErrorInvalidValue;                                          \
      }                                                                                \
    } else {                                                                           \
      const size_t lds_ = sizeof(double) * col_lds_elems(ts_, ts_, H) +                \
                          (2 * sizeof(double) + sizeof(short2)) * (2 * (H) + 1) *       \
                              (2 * (H) + 1) +                                          \
                          sizeof(double) * ts_ * ts_;                                  \
      hipLaunchKernelGGL((k_stats<T, 0, false>), dim3((la).ntiles), dim3(NTHREADS),    \
                         lds_, (la).stream, (la).jobs, (la).tiles);                    \
    }                                                                                  \
  } while (0)

hipError_t launch_stats(const LaunchArgs& la, int precision, int sep, int rb, int H) {
  if (precision == 1) DISPATCH_STATS(double, la, sep, rb, H);
  else DISPATCH_STATS(float, la, sep, rb, H);
  return hipGetLastError();
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

hipError_t launch_cgls_init(const LaunchArgs& la, int precision) {
  if (precision == 1)
    hipLaunchKernelGGL((k_cgls_init<double, double>), dim3(la.ntiles), dim3(NTHREADS), 0,
                       la.stream, la.jobs, la.tiles);
  else if (precision == 2)
    hipLaunchKernelGGL((k_cgls_init<float, bf16s>), dim3(la.ntiles), dim3(NTHREADS), 0,
                       la.stream, la.jobs, la.tiles);
  else
    hipLaunchKernelGGL((k_cgls_init<float, float>), dim3(la.ntiles), dim3(NTHREADS), 0,
                       la.stream, la.jobs, la.tiles);
  return hipGetLastError();
}

hipError_t launch_stats_fin(const LaunchArgs& la) {
  hipLaunchKernelGGL(k_stats_fin, dim3(la.ntiles), dim3(NTHREADS), 0, la.stream, la.jobs,
                     la.tiles);
  return hipGetLastError();
}

hipError_t launch_set_gamma(const LaunchArgs& la) {
  hipLaunchKernelGGL(k_set_gamma, dim3(la.ntiles), dim3(64), 0, la.stream, la.jobs, la.tiles);
  return hipGetLastError();
}

hipError_t launch_cgls_hist(const LaunchArgs& la) {
  hipLaunchKernelGGL(k_cgls_hist, dim3(la.ntiles), dim3(NTHREADS), 0, la.stream, la.jobs,
                     la.tiles);
  return hipGetLastError();
}
SIMPLE_LAUNCHER(launch_aux, k_aux)
SIMPLE_LAUNCHER(launch_fill, k_fill)

}  // namespace dbl
