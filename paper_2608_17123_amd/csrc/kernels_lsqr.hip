// LSQR (Golub-Kahan bidiagonalisation with Givens rotations, the inner solver
// the paper names in Sec. 3) on the augmented system of eq. (augmented),
//   [A; sqrt(g) D] x ~ [b; sqrt(g) c],   from x0 (correction form),
// fused into two tiled phases per iteration, FP64 scalars:
//
//   init : u = [b - A x0; sqrt(g) (c - D x0)], x = x0          -> |u|^2 (beta_1)
//   B_1  : v = Abar^T u / beta_1                                -> |v|^2 (alpha_1)
//   A_i  : v_i = v / alpha_i (v as stored is alpha_i v_i); the rotation of
//          iteration i-1 (rho_{i-1}, c, s, theta_i, phi_{i-1}) and
//          x += (phi_{i-1} / rho_{i-1}) w,  w = v_i - (theta_i / rho_{i-1}) w;
//          u = Abar v_i - (alpha_i / beta_i) u                  -> |u|^2 (beta_{i+1})
//   B_i+1: v = Abar^T (u / beta_{i+1}) - (beta_{i+1} / alpha_i) v  -> |v|^2
//   fin  : the rotation of iteration K and x += (phi_K / rho_K) w.
//
// u and v are stored unnormalised (scaled by beta, alpha); every phase scales
// what it reads by the reciprocal norm it sums from the previous phases'
// per-tile FP64 partials.  A_i updates u in place pointwise (its stencil reads
// v); B reads u through the stencils and updates v in place pointwise.  So
// u1, u2, v and w need one buffer each.  The rotation state (rhobar, phibar)
// lives in two scalar copies indexed by iteration parity: every block of A_i
// reads copy (i-1)&1 and recomputes the same step; the first block writes
// copy i&1.  With F_HIST the residual estimate phibar_{i}^2 = |r_{i-1}|^2 is
// recorded (A_i for i >= 2, fin for iteration K).
//
// Vector slots: V_X x (T); V_PA w; V_S v; V_R1A u1 (n); V_R2A u2 (n_L); all
// of storage type S.  Job::pr[0], pr[1] and pw are the partial arrays named
// per kernel below; Job::i0 is the iteration i.
#include "phase.h"

namespace dbl {

namespace {

__device__ __forceinline__ double rinv(double v) { return v > 0.0 ? 1.0 / v : 0.0; }

// Occupancy target of the LSQR phases (waves per SIMD): they carry more live
// values than the CGLS phases (rotation scalars, the in-place u and v updates),
// so they are held at 4 (FP32) to stay free of register spills.
// Outputs per item of the separable convolutions (as in the CGLS phases).
constexpr int LSQR_V = 2;

template <typename T, int RB>
constexpr int lsqr_waves() {
  return sizeof(T) == 4 ? (RB <= 8 ? 4 : 3) : 2;
}

// One Givens step of LSQR (Paige and Saunders): from (rhobar, phibar) of
// iteration i-1 and beta_i, alpha_i.  Returns rho_{i-1}, theta_i, phi_{i-1}
// and the new (rhobar_i, phibar_i).
struct Rot {
  double rho, theta, phi, rhobar, phibar;
};

__device__ __forceinline__ Rot rotate(double rhobar, double phibar, double beta, double alpha) {
  Rot r;
  r.rho = sqrt(rhobar * rhobar + beta * beta);
  const double c = r.rho > 0.0 ? rhobar / r.rho : 1.0;
  const double s = r.rho > 0.0 ? beta / r.rho : 0.0;
  r.theta = s * alpha;
  r.rhobar = -c * alpha;
  r.phi = c * phibar;
  r.phibar = s * phibar;
  return r;
}

}  // namespace

// ------------------------------------------------------------------ init --
// pw: |u|^2 partials (one per tile).
template <typename T, typename S>
__global__ void __launch_bounds__(NTHREADS) k_lsqr_init(const Job* __restrict__ jobs,
                                                        const uint32_t* __restrict__ tiles) {
  __shared__ double red[8];
  const Job* job; int ti, tj, tix;
  decode_tile(jobs, tiles, job, ti, tj, tix);
  const int m = job->m;
  int i0, j0, TI, TJ;
  tile_geom<T>(m, ti, tj, i0, j0, TI, TJ);
  const double sg = job->scal[S_SQRTG];
  const bool shift = job->flags & F_SHIFT, sb = job->flags & F_SB, irls = job->flags & F_IRLS;
  T* x = vp<T>(job, V_X);
  S* u1 = vp<S>(job, V_R1A);
  S* u2 = vp<S>(job, V_R2A);
  S* w = vp<S>(job, V_PA);
  const T* b = vp<T>(job, V_B);
  const T* c1 = vp<T>(job, V_C1);
  const T* c2 = vp<T>(job, V_C2);
  const T* wt = vp<T>(job, V_W);
  const T* x0 = vp<T>(job, V_X0);     // optional start
  const T* ax0 = vp<T>(job, V_XOLD);  // A x0 when x0 is given
  const size_t nx = (size_t)(m - 1) * m;
  double acc = 0.0;
  for (int o = threadIdx.x; o < TI * TJ; o += NTHREADS) {
    const int gi = i0 + (o & (TI - 1)), gj = j0 + (o >> (__ffs(TI) - 1));
    const size_t g = gi + (size_t)gj * m;
    const double xv = x0 ? (double)x0[g] : 0.0;
    const T uv = rtv<S>(x0 ? (T)((double)b[g] - (double)ax0[g]) : b[g]);
    stv(u1, g, uv);
    acc += (double)uv * (double)uv;
    x[g] = (T)xv;
    stv(w, g, T(0));
    for (int dir = 0; dir < 2; ++dir) {
      if ((dir == 0 && gi >= m - 1) || (dir == 1 && gj >= m - 1)) continue;
      const size_t k = dir == 0 ? gi + (size_t)gj * (m - 1) : nx + g;
      double c = 0.0;
      if (shift) c = (double)c1[k] - (sb ? (double)c2[k] : 0.0);
      if (x0) {
        const double nb = dir == 0 ? (double)x0[g + 1] : (double)x0[g + m];
        double d = nb - xv;
        if (irls) d *= (double)wt[k];
        c -= d;
      }
      const T qv = rtv<S>((T)(sg * c));
      stv(u2, k, qv);
      acc += (double)qv * (double)qv;
    }
  }
  double vv[1] = {acc};
  put_partials<1>(job->pw, tix, vv, red);
}

// -------------------------------------------------------------- phase A --
// pr[0]: |v|^2 partials of B_i (alpha_i); pr[1]: |u|^2 partials of A_{i-1}
// or init (beta_i); pw: |u|^2 partials (beta_{i+1}).  F_FIRST: i = 1.
template <typename T, typename S, int RB, bool SEP>
__global__ void __launch_bounds__(NTHREADS, (lsqr_waves<T, RB>()))
    k_lsqr_a(const Job* __restrict__ jobs, const uint32_t* __restrict__ tiles) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ double red[8];
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
  const bool first = job->flags & F_FIRST;
  const int it = job->i0;
  double* st = job->scal + S_LQ;
  T tx, tw, ta, cu;
  // norms, rotation and step scalars; run by every thread inside the tile
  // load, while the first batch of v is in flight
  auto scalars = [&]() {
    double aa, bb;
    sum_partials2<1, 1>(job->pr[0], 0, job->pr[1], 0, nt, red, bc2, aa, bb);
    const double alpha = sqrt(aa), beta = sqrt(bb);
    Rot r;
    if (first) {
      r.rho = r.theta = r.phi = 0.0;
      r.rhobar = alpha;
      r.phibar = beta;
    } else {
      r = rotate(st[2 * ((it - 1) & 1)], st[2 * ((it - 1) & 1) + 1], beta, alpha);
    }
    if (tix == 0 && threadIdx.x == 0) {
      st[2 * (it & 1)] = r.rhobar;
      st[2 * (it & 1) + 1] = r.phibar;
      if ((job->flags & F_HIST) && !first && it - 2 < HIST_MAX)
        job->scal[S_HIST + it - 2] = r.phibar * r.phibar;
    }
    tx = (T)(r.phi * rinv(r.rho));
    tw = (T)(r.theta * rinv(r.rho));
    ta = (T)rinv(alpha);
    cu = (T)(alpha * rinv(beta));  // u_new = Abar v_i - alpha_i u_i, u_i = u / beta_i
    return ta;
  };
  const double sg = job->scal[S_SQRTG];
  const bool irls = job->flags & F_IRLS;
  T* __restrict__ x = vp<T>(job, V_X);
  S* __restrict__ w = vp<S>(job, V_PA);
  const S* __restrict__ v = vp<S>(job, V_S);
  S* __restrict__ u1 = vp<S>(job, V_R1A);
  S* __restrict__ u2 = vp<S>(job, V_R2A);
  const T* __restrict__ wt = vp<T>(job, V_W);
  load_tile_overlap<T, SEP>(
      Xs, xs_ld<SEP>(H, TI, TJ), i0, j0, TI, TJ, H, m, [&](int g) { return ldv<T>(v, g); },
      [&](int) { return T(0); }, scalars, [&](T a, T, T c) { return a * c; });
  __syncthreads();
  double acc = 0.0;
  const size_t nx = (size_t)(m - 1) * m;
  batched_pixels<2, 6, T>(
      TI * TJ,
      [&](int o, T* q) {
        const int gi = i0 + (o & (TI - 1)), gj = j0 + (o >> (__ffs(TI) - 1));
        const size_t g = gi + (size_t)gj * m;
        const bool okx = gi < m - 1, oky = gj < m - 1;
        q[0] = (irls && okx) ? wt[gi + (size_t)gj * (m - 1)] : T(1);
        q[1] = (irls && oky) ? wt[nx + g] : T(1);
        q[2] = okx ? ldv<T>(u2, gi + (size_t)gj * (m - 1)) : T(0);
        q[3] = oky ? ldv<T>(u2, nx + g) : T(0);
        q[4] = first ? T(0) : x[g];
        q[5] = first ? T(0) : ldv<T>(w, g);
      },
      [&](int o, T* q) {
        const int i = (o & (TI - 1)), j = (o >> (__ffs(TI) - 1)), gi = i0 + i, gj = j0 + j;
        const size_t g = gi + (size_t)gj * m;
        const T vc = Xs[xs_at<SEP>(i, j, H, TI, TJ)];
        if (first) {
          stv(w, g, rtv<S>(vc));
        } else {
          x[g] = q[4] + tx * q[5];
          stv(w, g, rtv<S>(vc - tw * q[5]));
        }
        if (gi < m - 1) {
          const double d = ((double)Xs[xs_at<SEP>(i + 1, j, H, TI, TJ)] - (double)vc) * (double)q[0];
          const T un = rtv<S>((T)(sg * d - (double)(cu * q[2])));
          stv(u2, gi + (size_t)gj * (m - 1), un);
          acc += (double)un * (double)un;
        }
        if (gj < m - 1) {
          const double d = ((double)Xs[xs_at<SEP>(i, j + 1, H, TI, TJ)] - (double)vc) * (double)q[1];
          const T un = rtv<S>((T)(sg * d - (double)(cu * q[3])));
          stv(u2, nx + g, un);
          acc += (double)un * (double)un;
        }
      });
  auto epia = [&](int i, int j, T av) {
    const size_t g = (i0 + i) + (size_t)(j0 + j) * m;
    const T un = rtv<S>(av - cu * ldv<T>(u1, g));
    stv(u1, g, un);
    acc += (double)un * (double)un;
  };
  conv_tile<T, RB, SEP, decltype(epia), NoHook, LSQR_V>(Xs, H, scratch, op, false, i0, j0, TI,
                                                        TJ, m, epia);
  double vv[1] = {acc};
  put_partials<1>(job->pw, tix, vv, red);
}

// -------------------------------------------------------------- phase B --
// pr[0]: |u|^2 partials (beta); pr[1]: |v|^2 partials of the previous B
// (alpha; unused with F_FIRST); pw: |v|^2 partials.
template <typename T, typename S, int RB, bool SEP>
__global__ void __launch_bounds__(NTHREADS, (lsqr_waves<T, RB>()))
    k_lsqr_b(const Job* __restrict__ jobs, const uint32_t* __restrict__ tiles) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ double red[8];
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
  const bool first = job->flags & F_FIRST;
  const bool irls = job->flags & F_IRLS;
  T tb, cv;
  // 1 / beta and the v recurrence factor; run by every thread inside the
  // tile load, while the first batch of u1 is in flight
  auto scalars = [&]() {
    double bb, aa;
    sum_partials2<1, 1>(job->pr[0], 0, first ? job->pr[0] : job->pr[1], 0, nt, red, bc2, bb,
                        aa);
    const double beta = sqrt(bb), alpha = sqrt(aa);
    tb = (T)rinv(beta);
    cv = first ? T(0) : (T)(beta * rinv(alpha));  // v_new = ... - beta v_old / alpha
    return tb;
  };
  const double sg = job->scal[S_SQRTG];
  S* __restrict__ v = vp<S>(job, V_S);
  const S* __restrict__ u1 = vp<S>(job, V_R1A);
  const S* __restrict__ u2 = vp<S>(job, V_R2A);
  const T* __restrict__ wt = vp<T>(job, V_W);
  load_tile_overlap<T, SEP>(
      Xs, xs_ld<SEP>(H, TI, TJ), i0, j0, TI, TJ, H, m, [&](int g) { return ldv<T>(u1, g); },
      [&](int) { return T(0); }, scalars, [&](T a, T, T c) { return a * c; });
  __syncthreads();
  double acc = 0.0;
  const size_t nx = (size_t)(m - 1) * m;
  // Gradient part: LT[i, j] = sqrt(g) (D^T u2)[i, j] / beta for the tile, into
  // LDS (coalesced loads, all threads).
  T* LT = nullptr;
  auto grad_part = [&](T* buf) {
    LT = buf;
    batched_pixels<2, 8, T>(
        TI * TJ,
        [&](int o, T* q) {
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
            q[2 * d] = ok[d] ? ldv<T>(u2, ks[d]) : T(0);
            q[2 * d + 1] = (ok[d] && irls) ? wt[ks[d]] : T(1);
          }
        },
        [&](int o, T* q) {
          const int i = (o & (TI - 1)), j = (o >> (__ffs(TI) - 1)), gi = i0 + i, gj = j0 + j;
          double lt = 0.0;
          if (gi >= 1) lt += (double)q[1] * (double)q[0];
          if (gi < m - 1) lt -= (double)q[3] * (double)q[2];
          if (gj >= 1) lt += (double)q[5] * (double)q[4];
          if (gj < m - 1) lt -= (double)q[7] * (double)q[6];
          buf[i + j * TI] = (T)(sg * lt) * tb;
        });
    __syncthreads();
  };
  auto epi = [&](int i, int j, T av) {
    const size_t g = (i0 + i) + (size_t)(j0 + j) * m;
    const T old = first ? T(0) : ldv<T>(v, g);
    const T vn = rtv<S>(av + LT[i + j * TI] - cv * old);
    stv(v, g, vn);
    acc += (double)vn * (double)vn;
  };
  if constexpr (SEP) {
    auto hook = [&] { grad_part(Xs); };
    conv_tile<T, RB, SEP, decltype(epi), decltype(hook), LSQR_V>(Xs, H, scratch, op, true, i0,
                                                                 j0, TI, TJ, m, epi, hook);
  } else {
    grad_part(reinterpret_cast<T*>(scratch) + (2 * H + 1) * (2 * H + 1) * 2);
    conv_tile<T, RB, SEP>(Xs, H, scratch, op, true, i0, j0, TI, TJ, m, epi);
  }
  double vv[1] = {acc};
  put_partials<1>(job->pw, tix, vv, red);
}

// ---------------------------------------------------------------- finish --
// pr[0]: |u|^2 partials of A_K (beta_{K+1}); i0 = K.  The rotation of
// iteration K and the last update x += (phi_K / rho_K) w.
template <typename T, typename S>
__global__ void __launch_bounds__(NTHREADS) k_lsqr_fin(const Job* __restrict__ jobs,
                                                       const uint32_t* __restrict__ tiles) {
  __shared__ double red[8];
  __shared__ double bc;
  const Job* job; int ti, tj, tix;
  decode_tile(jobs, tiles, job, ti, tj, tix);
  const int m = job->m;
  int i0, j0, TI, TJ;
  tile_geom<T>(m, ti, tj, i0, j0, TI, TJ);
  const int nt = job->nti * job->ntj;
  const int K = job->i0;
  const double beta = sqrt(sum_partials<1>(job->pr[0], nt, 0, red, &bc));
  const double* st = job->scal + S_LQ + 2 * (K & 1);
  const Rot r = rotate(st[0], st[1], beta, 0.0);
  if (tix == 0 && threadIdx.x == 0 && (job->flags & F_HIST) && K - 1 < HIST_MAX)
    job->scal[S_HIST + K - 1] = r.phibar * r.phibar;
  const T tx = (T)(r.phi * rinv(r.rho));
  T* __restrict__ x = vp<T>(job, V_X);
  const S* __restrict__ w = vp<S>(job, V_PA);
  for (int o = threadIdx.x; o < TI * TJ; o += NTHREADS) {
    const size_t g = (i0 + (o & (TI - 1))) + (size_t)(j0 + (o >> (__ffs(TI) - 1))) * m;
    x[g] = x[g] + tx * ldv<T>(w, g);
  }
}

// -------------------------------------------------------------- launchers --

hipError_t launch_lsqr_init(const LaunchArgs& la, int precision) {
  if (precision == 1)
    hipLaunchKernelGGL((k_lsqr_init<double, double>), dim3(la.ntiles), dim3(NTHREADS), 0,
                       la.stream, la.jobs, la.tiles);
  else if (precision == 2)
    hipLaunchKernelGGL((k_lsqr_init<float, bf16s>), dim3(la.ntiles), dim3(NTHREADS), 0,
                       la.stream, la.jobs, la.tiles);
  else
    hipLaunchKernelGGL((k_lsqr_init<float, float>), dim3(la.ntiles), dim3(NTHREADS), 0,
                       la.stream, la.jobs, la.tiles);
  return hipGetLastError();
}

hipError_t launch_lsqr_a(const LaunchArgs& la, int precision, int sep, int rb, int H) {
  if (precision == 1) DISPATCH_STENCIL_S(k_lsqr_a, double, double, la, sep, rb, H);
  else if (precision == 2) DISPATCH_STENCIL_S(k_lsqr_a, float, bf16s, la, sep, rb, H);
  else DISPATCH_STENCIL_S(k_lsqr_a, float, float, la, sep, rb, H);
  return hipGetLastError();
}

hipError_t launch_lsqr_b(const LaunchArgs& la, int precision, int sep, int rb, int H) {
  if (precision == 1) DISPATCH_STENCIL_S(k_lsqr_b, double, double, la, sep, rb, H);
  else if (precision == 2) DISPATCH_STENCIL_S(k_lsqr_b, float, bf16s, la, sep, rb, H);
  else DISPATCH_STENCIL_S(k_lsqr_b, float, float, la, sep, rb, H);
  return hipGetLastError();
}

hipError_t launch_lsqr_fin(const LaunchArgs& la, int precision) {
  if (precision == 1)
    hipLaunchKernelGGL((k_lsqr_fin<double, double>), dim3(la.ntiles), dim3(NTHREADS), 0,
                       la.stream, la.jobs, la.tiles);
  else if (precision == 2)
    hipLaunchKernelGGL((k_lsqr_fin<float, bf16s>), dim3(la.ntiles), dim3(NTHREADS), 0,
                       la.stream, la.jobs, la.tiles);
  else
    hipLaunchKernelGGL((k_lsqr_fin<float, float>), dim3(la.ntiles), dim3(NTHREADS), 0,
                       la.stream, la.jobs, la.tiles);
  return hipGetLastError();
}

}  // namespace dbl
