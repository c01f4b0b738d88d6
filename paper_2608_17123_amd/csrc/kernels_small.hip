// One-block CGLS for the small levels of the V-cycle.
//
// The tiled CGLS phases (kernels_solve.hip) need two launches per iteration,
// and on a coarse grid (m <= 64) each launch is a handful of blocks whose
// time is dominated by the launch itself and by the memory round trips that
// carry partial sums from one launch to the next.  Here one block owns a
// whole level: p and r1 (both with a periodic halo), s, q1, r2 and the
// level's 1-D tap tables (separable operator) live in LDS, x lives in
// registers, the IRLS weights w are staged in LDS when they fit (else read
// from global memory, where they stay cache resident), and all K_in
// iterations of the CGLS recurrence on the augmented system of eq.
// (augmented) run in one launch with block-level FP64 reductions.  The
// arithmetic of every element is the tiled kernels' (same products, same
// FP32/FP64 roundings); only the order of the FP64 norm summations differs.
// A general (non-separable) operator (GEN; levels up to 32 x 32) convolves
// each pixel over its class's 2-D tap list in list order, as the tiled
// kernels do: the interior class's lists (forward and adjoint) are staged in
// LDS as (offset, value) pairs, the seam and boundary classes are read from
// the tables, where they stay cache resident.
//
// Job fields: m, op, flags (F_IRLS, F_SHIFT, F_SB, F_HIST, F_WLDS),
// scal[S_SQRTG], v[V_B] = b, v[V_W] = w, v[V_C1] / v[V_C2] = c (MM: c1;
// SB: c1 - c2), v[V_X] = result x, i0 = iterations.  x0 = 0 (the subproblem
// start).
#include "launch.h"
#include "stencil.h"

namespace dbl {

namespace {

template <typename T> __device__ __forceinline__ T* vq(const Job* j, int k) {
  return static_cast<T*>(j->v[k]);
}

}  // namespace

// M: the level size (every job of a launch has m = M); NT threads.
template <typename T, int RB, int M, bool GEN>
__global__ void __launch_bounds__(small_nt(M, sizeof(T))) k_cgls_small(const Job* __restrict__ jobs,
                                                                       const uint32_t* __restrict__ tiles) {
  constexpr int NT = small_nt(M, sizeof(T));
  constexpr int XPT = M * M / NT;  // pixels (and x values) per thread
  constexpr int m = M, H = RB, NTAP = 2 * RB + 1;
  constexpr int n = m * m, nx = (m - 1) * m, nl = 2 * nx;
  constexpr int msk = m - 1;
  constexpr int E = m + 2 * H, ld = E + 1;
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ double red[2 * (NT / 64)];
  const Job* job = jobs + (tiles[blockIdx.x] >> 16);
  const LevelOp& op = *job->op;
  const int fl = job->flags;
  const bool irls = fl & F_IRLS, shift = fl & F_SHIFT, sb = fl & F_SB;
  const bool wl = irls && (fl & F_WLDS);
  const int trows[4] = {op.f0.rows, op.f1.rows, op.a0.rows, op.a1.rows};
  const SmallLds LL =
      small_lds(m, H, (int)sizeof(T), wl, GEN ? 0 : (trows[0] + trows[1] + trows[2] + trows[3]) * NTAP,
                GEN);
  T* XP = reinterpret_cast<T*>(smem);
  T* XR = reinterpret_cast<T*>(smem + LL.halo);
  T* Z = reinterpret_cast<T*>(smem + LL.z);
  T* Sv = reinterpret_cast<T*>(smem + LL.s);
  T* Q1 = reinterpret_cast<T*>(smem + LL.q1);
  T* R2 = reinterpret_cast<T*>(smem + LL.r2);
  T* W = reinterpret_cast<T*>(smem + LL.w);
  T* TB = reinterpret_cast<T*>(smem + LL.tb);
  const int tid = threadIdx.x;
  const double sg = job->scal[S_SQRTG];
  const T* __restrict__ b = vq<T>(job, V_B);
  const T* __restrict__ w = vq<T>(job, V_W);
  const T* __restrict__ c1 = vq<T>(job, V_C1);
  const T* __restrict__ c2 = vq<T>(job, V_C2);
  const int K = job->i0;

  // the level's tap tables, copied to LDS once (separable operator), or the
  // interior class's 2-D tap lists as (offset into the halo'd buffers, value)
  Table1D tab[4] = {op.f0, op.f1, op.a0, op.a1};
  constexpr int GT = small_gen_taps(H);
  int* g_off = reinterpret_cast<int*>(Z);    // [2][GT]: forward, adjoint
  T* g_val = reinterpret_cast<T*>(g_off + 2 * GT);
  int g_cls[2] = {0, 0}, g_n[2] = {0, 0};
  if constexpr (GEN) {
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      const Table2D& tb = t ? op.a2 : op.f2;
      const T* vals = taps2<T>(tb);
      g_cls[t] = tb.St0 + tb.St1 * tb.rows0;
      const int b = tb.off[g_cls[t]];
      g_n[t] = tb.off[g_cls[t] + 1] - b;
      for (int k = tid; k < g_n[t]; k += NT) {
        const short2 e = tb.e[b + k];
        g_off[t * GT + k] = e.x * ld + e.y;  // rows = axis 0 (e.x), columns = axis 1 (e.y)
        g_val[t * GT + k] = vals[b + k];
      }
    }
  } else {
    int off = 0;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const T* src = taps1<T>(tab[t]);
      const int cnt = trows[t] * NTAP;
      for (int q = tid; q < cnt; q += NT) TB[off + q] = src[q];
      if constexpr (sizeof(T) == 4) tab[t].tf = reinterpret_cast<const float*>(TB + off);
      else tab[t].td = reinterpret_cast<const double*>(TB + off);
      off += cnt;
    }
  }

  // the thread's pixels o = tid + u * NT, u < XPT
  auto for_px = [&](auto body) {
#pragma unroll
    for (int u = 0; u < XPT; ++u) {
      const int o = tid + u * NT;
      body(u, o, o % m, o / m);
    }
  };
  // (row, column) of the halo'd buffers -> LDS index (row-major, rows = axis 0)
  auto at = [](int r, int c) { return r * ld + c; };
  // periodic halo from the interior (interior cells are only read)
  auto halo = [&](T* X) {
    constexpr int band = H * E, tot = 2 * band + 2 * H * m;
    for (int q = tid; q < tot; q += NT) {
      int r, c;
      if (q < band) {
        r = q / E;
        c = q % E;
      } else if (q < 2 * band) {
        const int u = q - band;
        r = m + H + u / E;
        c = u % E;
      } else {
        const int u = q - 2 * band, cc = u % (2 * H);
        r = H + u / (2 * H);
        c = cc < H ? cc : m + cc;
      }
      X[at(r, c)] = X[at(((r - H) & msk) + H, ((c - H) & msk) + H)];
    }
  };
  auto conv = [&](const T* X, bool adj, auto epi) {
    if constexpr (GEN) {
      // every pixel over its class's tap list, in list order: first all of
      // the thread's pixels over the interior list, taps outermost (one
      // staged offset and value per tap, the pixels' sums independent), then
      // the seam and boundary pixels again over their own lists (their
      // interior-list sums read the halo'd buffers in range and are dropped)
      const Table2D& tb = adj ? op.a2 : op.f2;
      const int t = adj ? 1 : 0;
      const T* __restrict__ vals = taps2<T>(tb);
      int base[XPT];
      T acc[XPT];
#pragma unroll
      for (int u = 0; u < XPT; ++u) {
        const int o = tid + u * NT;
        base[u] = at(o % m + H, o / m + H);
        acc[u] = T(0);
      }
      for (int k = 0; k < g_n[t]; ++k) {
        const int off = g_off[t * GT + k];
        const T v = g_val[t * GT + k];
#pragma unroll
        for (int u = 0; u < XPT; ++u) acc[u] = fma(v, X[base[u] + off], acc[u]);
      }
      // the class lists are read with global (not generic) loads, an entry
      // (e0, e1) of 16 bits each as one word (e0 in the low half); four taps
      // are requested before any is used, and summed in list order
      GlobalPtr<const T> gv = gview(vals);
      GlobalPtr<const int> te = gview(reinterpret_cast<const int*>(tb.e));
      GlobalPtr<const int> toff = gview(tb.off);
      for_px([&](int u, int, int i, int j) {
        const int cls = class_of(i, m, tb.St0, tb.Sb0) + class_of(j, m, tb.St1, tb.Sb1) * tb.rows0;
        if (cls != g_cls[t]) {
          auto px = [&](int wd) { return base[u] + (int)(short)wd * ld + (wd >> 16); };
          const int k1 = toff[cls + 1];
          int k = toff[cls];
          T a = T(0);
          for (; k + 4 <= k1; k += 4) {
            int e[4];
            T v[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              e[q] = te[k + q];
              v[q] = gv[k + q];
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) a = fma(v[q], X[px(e[q])], a);
          }
          for (; k < k1; ++k) a = fma(gv[k], X[px(te[k])], a);
          acc[u] = a;
        }
        epi(i, j, acc[u]);
      });
    } else {
      // outputs per item: enough items for every thread of the block
      constexpr int V = 2;
      sep_tile<T, RB, NT, V, false>(X, H, Z, adj ? tab[2] : tab[0], adj ? tab[3] : tab[1], 0, 0,
                                    m, m, m, epi);
    }
  };
  auto wgt = [&](int k) -> double {
    if (!irls) return 1.0;
    return wl ? (double)W[k] : (double)w[k];
  };

  // ---- start: x = 0, p = 0, r1 = b, r2 = sqrt(g) c
  for (int q = tid; q < E * ld; q += NT) XP[q] = T(0);
  for_px([&](int, int o, int i, int j) { XR[at(i + H, j + H)] = b[o]; });
  for (int k = tid; k < nl; k += NT) {
    double c = 0.0;
    if (shift) c = (double)c1[k] - (sb ? (double)c2[k] : 0.0);
    R2[k] = (T)(sg * c);
    if (wl) W[k] = w[k];
  }
  T xr[XPT];
#pragma unroll
  for (int u = 0; u < XPT; ++u) xr[u] = T(0);
  __syncthreads();
  halo(XR);
  __syncthreads();

  // ---- phase 2: r -= alpha q (skipped at the start), x += alpha p,
  //      s = A^T r1 + sqrt(g) D^T r2; returns (|s|^2, |r|^2)
  auto phase2 = [&](bool first, T ta, double& gs, double& rr) {
    double accr = 0.0, accs = 0.0;
    if (!first) {
      for_px([&](int u, int o, int i, int j) {
        const int id = at(i + H, j + H);
        const T rv = XR[id] - ta * Q1[o];
        XR[id] = rv;
        xr[u] = xr[u] + ta * XP[id];
        accr += (double)rv * (double)rv;
      });
      __syncthreads();
      halo(XR);
    } else {
      for_px([&](int, int, int i, int j) {
        const T rv = XR[at(i + H, j + H)];
        accr += (double)rv * (double)rv;
      });
    }
    // r2 -= alpha q2 with q2 = sqrt(g) D p recomputed from p (same rounding
    // as when its norm was taken)
    for_px([&](int, int o, int i, int j) {
      const T pc = XP[at(i + H, j + H)];
      if (i < m - 1) {
        const int k = i + j * (m - 1);
        T rn = R2[k];
        if (!first) {
          const double d = ((double)XP[at(i + 1 + H, j + H)] - (double)pc) * wgt(k);
          rn = (T)(rn - ta * (T)(sg * d));
          R2[k] = rn;
        }
        accr += (double)rn * (double)rn;
      }
      if (j < m - 1) {
        const int k = nx + o;
        T rn = R2[k];
        if (!first) {
          const double d = ((double)XP[at(i + H, j + 1 + H)] - (double)pc) * wgt(k);
          rn = (T)(rn - ta * (T)(sg * d));
          R2[k] = rn;
        }
        accr += (double)rn * (double)rn;
      }
    });
    __syncthreads();
    // gradient part of s into Q1 (q1 is consumed)
    for_px([&](int, int o, int i, int j) {
      double lt = 0.0;
      if (i >= 1) lt += wgt(i - 1 + j * (m - 1)) * (double)R2[i - 1 + j * (m - 1)];
      if (i < m - 1) lt -= wgt(i + j * (m - 1)) * (double)R2[i + j * (m - 1)];
      if (j >= 1) lt += wgt(nx + o - m) * (double)R2[nx + o - m];
      if (j < m - 1) lt -= wgt(nx + o) * (double)R2[nx + o];
      Q1[o] = (T)(sg * lt);
    });
    __syncthreads();
    conv(XR, true, [&](int i, int j, T v) {
      const int o = i + j * m;
      const T sv = v + Q1[o];
      Sv[o] = sv;
      accs += (double)sv * (double)sv;
    });
    double vv[2] = {accs, accr};
    block_allsum<2, NT>(vv, red);
    gs = vv[0];
    rr = vv[1];
  };

  double gs = 0.0, rr = 0.0;
  phase2(true, T(0), gs, rr);
  double gs_prev = gs;
  for (int it = 0; it < K; ++it) {
    // ---- phase 1: p = s + beta p; q1 = A p; |q|^2 = |q1|^2 + |sqrt(g) D p|^2
    const double beta = it == 0 ? 0.0 : (gs_prev > 0.0 ? gs / gs_prev : 0.0);
    const T tb = (T)beta;
    for_px([&](int, int o, int i, int j) {
      const int id = at(i + H, j + H);
      XP[id] = Sv[o] + tb * XP[id];
    });
    __syncthreads();
    halo(XP);
    __syncthreads();
    double acc = 0.0;
    for_px([&](int, int o, int i, int j) {
      const T pc = XP[at(i + H, j + H)];
      if (i < m - 1) {
        const double d = ((double)XP[at(i + 1 + H, j + H)] - (double)pc) * wgt(i + j * (m - 1));
        const T qv = (T)(sg * d);
        acc += (double)qv * (double)qv;
      }
      if (j < m - 1) {
        const double d = ((double)XP[at(i + H, j + 1 + H)] - (double)pc) * wgt(nx + o);
        const T qv = (T)(sg * d);
        acc += (double)qv * (double)qv;
      }
    });
    conv(XP, false, [&](int i, int j, T v) {
      Q1[i + j * m] = v;
      acc += (double)v * (double)v;
    });
    double vq1[1] = {acc};
    block_allsum<1, NT>(vq1, red);
    const double qq = vq1[0];
    // ---- phase 2
    const double alpha = qq > 0.0 ? gs / qq : 0.0;
    gs_prev = gs;
    phase2(false, (T)alpha, gs, rr);
    if ((fl & F_HIST) && tid == 0 && it < HIST_MAX) job->scal[S_HIST + it] = rr;
  }
  T* __restrict__ x = vq<T>(job, V_X);
  for_px([&](int u, int o, int, int) { x[o] = xr[u]; });
}

// Dynamic LDS of the one-block CGLS for a level with a separable operator
// (1-D tables of `tab_rows` rows in total, padded to radius rb) or, with
// `gen`, a general operator of radius <= rb (tab_rows unused), 0 when the
// level cannot run there.  IRLS subproblems stage their weights in LDS when
// that still fits (*wlds = 1).
size_t small_cgls_lds(int m, int precision, int rb, int tab_rows, bool irls, size_t limit,
                      int* wlds, bool gen) {
  *wlds = 0;
  if (m != 8 && m != 16 && m != 32 && !(m == 64 && precision != 1)) return 0;
  // a general operator's seam and boundary pixels read their lists from
  // memory; at 64 x 64 that made the one-block kernel slower than the tiled
  // phases (measured), up to 32 x 32 twice as fast
  if (gen && m > 32) return 0;
  const int esz = precision == 1 ? 8 : 4, te = gen ? 0 : tab_rows * (2 * rb + 1);
  const size_t base = small_lds(m, rb, esz, false, te, gen).total;
  if (base > limit) return 0;
  if (irls) {
    const size_t withw = small_lds(m, rb, esz, true, te, gen).total;
    if (withw <= limit) {
      *wlds = 1;
      return withw;
    }
  }
  return base;
}

namespace {

template <typename T, int M>
hipError_t launch_small_m(const LaunchArgs& la, int rb, size_t lds, bool gen) {
  constexpr int NT = small_nt(M, sizeof(T));
#define SMALL_CASE(R)                                                                      \
  if (gen)                                                                                 \
    hipLaunchKernelGGL((k_cgls_small<T, R, M, true>), dim3(la.ntiles), dim3(NT), lds,      \
                       la.stream, la.jobs, la.tiles);                                     \
  else                                                                                     \
    hipLaunchKernelGGL((k_cgls_small<T, R, M, false>), dim3(la.ntiles), dim3(NT), lds,     \
                       la.stream, la.jobs, la.tiles)
  switch (rb) {
    case 2: SMALL_CASE(2); break;
    case 4: SMALL_CASE(4); break;
    case 8: SMALL_CASE(8); break;
    case 12: SMALL_CASE(12); break;
    case 16: SMALL_CASE(16); break;
    default: return hipErrorInvalidValue;
  }
#undef SMALL_CASE
  return hipSuccess;
}

template <typename T>
hipError_t launch_small_t(const LaunchArgs& la, int rb, int m, size_t lds, bool gen) {
  switch (m) {
    case 8: return launch_small_m<T, 8>(la, rb, lds, gen);
    case 16: return launch_small_m<T, 16>(la, rb, lds, gen);
    case 32: return launch_small_m<T, 32>(la, rb, lds, gen);
    case 64:  // an FP64 level of 64 x 64 does not fit in LDS
      if constexpr (sizeof(T) == 4) return launch_small_m<T, 64>(la, rb, lds, gen);
      return hipErrorInvalidValue;
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

hipError_t launch_cgls_small(const LaunchArgs& la, int precision, int rb, int m, size_t lds,
                             bool gen) {
  const hipError_t e = precision == 1 ? launch_small_t<double>(la, rb, m, lds, gen)
                                      : launch_small_t<float>(la, rb, m, lds, gen);
  if (e != hipSuccess) return e;
  return hipGetLastError();
}

}  // namespace dbl
