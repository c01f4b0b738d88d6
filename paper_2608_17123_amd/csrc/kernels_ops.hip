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

// Streaming separable blur for large FP32 grids (m >= STREAM_MIN_M).  A block
// owns a strip of STREAM_ROWS rows (one per thread) and STREAM_COLS output
// columns, and marches along the columns: each input column of the strip
// (plus RB halo rows above and below, periodic) goes through a double-
// buffered LDS column; the thread forms its row's axis-0 sum Z[i, j] from it
// and keeps the last 2 RB + 1 of them in registers, from which the axis-1 sum
// gives the output column j - RB.  Halo re-reads are (STREAM_ROWS + 2 RB) /
// STREAM_ROWS along rows and (STREAM_COLS + 2 RB) / STREAM_COLS along
// columns.  Input columns are requested 2 RB + 1 steps before they are used
// (a register queue), so that many column loads are in flight per block.
// The two sums are formed in the same order as sep_tile's passes, so the
// result equals the tiled kernel's bit for bit.
constexpr int STREAM_ROWS = 512, STREAM_COLS = 256, STREAM_MIN_M = 512;
// class rows of an axis-1 table the streaming kernel stages in LDS
constexpr int STREAM_MAX_ROWS = 2 * (2 * MAX_R + 3) + 1;
template <int RB>
__global__ void __launch_bounds__(STREAM_ROWS) k_apply_stream(const Job* __restrict__ jobs,
                                                              const uint32_t* __restrict__ tiles) {
  using T = float;
  constexpr int NTAP = 2 * RB + 1, NT = STREAM_ROWS, JW = STREAM_COLS, K = JW + 2 * RB;
  __shared__ T col[2][NT + 2 * RB];
  // the axis-1 tap rows (interior and seam classes), read by every thread
  // with one address per column step (LDS broadcast)
  constexpr int MAX_T1 = STREAM_MAX_ROWS * NTAP;
  __shared__ T tab1[MAX_T1];
  const Job* job; int ti, tj, tix;
  decode_tile(jobs, tiles, job, ti, tj, tix);
  const int m = job->m, msk = m - 1;
  const int tid = threadIdx.x;
  const int i0 = ti * NT, j0 = tj * JW, i = i0 + tid;
  const LevelOp& op = *job->op;
  const bool adj = job->flags & F_ADJ;
  const Table1D& t0 = adj ? op.a0 : op.f0;
  const Table1D& t1 = adj ? op.a1 : op.f1;
  // global-address-space views of the caller's buffers: loads and stores
  // then wait on the vector-memory counter only, so the LDS waits of each
  // column step do not also drain the column loads queued ahead
  const GlobalPtr<const T> in = gview(static_cast<const T*>(job->v[0]));
  const GlobalPtr<T> out = gview(static_cast<T*>(job->v[1]));
  // table fields read once: a reload through the job inside the column loop
  // would be a generic-address load, whose wait also drains the queued loads
  const int St1 = t1.St, Sb1 = t1.Sb, rows1 = t1.rows;
  for (int q = tid; q < rows1 * NTAP; q += NT) tab1[q] = gview(t1.tf)[q];  // rows checked on the host
  // the interior axis-1 tap row, the one every column away from a seam uses,
  // in scalar registers (the seam columns read their rows from LDS); up to
  // radius bucket 12 (at 16 the registers would spill)
  constexpr bool SREG = RB <= 12;
  T tb1[NTAP];
#pragma unroll
  for (int e = 0; e < NTAP; ++e)
    tb1[e] = SREG ? __builtin_bit_cast(T, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(
                        int, gview(t1.tf)[St1 * NTAP + e])))
                  : T(0);
  T ta[NTAP];
  {
    const GlobalPtr<const T> row = gview(t0.tf) + class_of(i, m, t0.St, t0.Sb) * NTAP;
#pragma unroll
    for (int e = 0; e < NTAP; ++e) ta[e] = row[e];
  }
  const bool halo = tid < 2 * RB;
  const size_t ga = (size_t)((i0 - RB + tid) & msk);
  const size_t gb = (size_t)((i0 - RB + NT + tid) & msk);
  T qa[NTAP], qb[NTAP], z[NTAP];
#pragma unroll
  for (int u = 0; u < NTAP; ++u) {
    const size_t c = (size_t)((j0 - RB + u) & msk) * m;
    qa[u] = in[ga + c];
    qb[u] = halo ? in[gb + c] : T(0);
  }
#pragma unroll 1
  for (int kb = 0; kb < K; kb += NTAP) {
#pragma unroll
    for (int u = 0; u < NTAP; ++u) {
      const int k = kb + u;
      if (k >= K) break;
      T* __restrict__ buf = col[k & 1];
      buf[tid] = qa[u];
      if (halo) buf[NT + tid] = qb[u];
      const int kn = k + NTAP;
      if (kn < K) {
        const size_t c = (size_t)((j0 - RB + kn) & msk) * m;
        qa[u] = in[ga + c];
        if (halo) qb[u] = in[gb + c];
      }
      lds_barrier();
      T a = T(0);
#pragma unroll
      for (int e = 0; e < NTAP; ++e) a = fma(ta[e], buf[tid + e], a);
      z[u] = a;
      if (k >= 2 * RB) {
        const int j = j0 + k - 2 * RB;
        T y = T(0);
        if (SREG && j >= St1 && j < m - Sb1) {
#pragma unroll
          for (int e = 0; e < NTAP; ++e) y = fma(tb1[e], z[(u + 1 + e) % NTAP], y);
        } else {
          const T* row = tab1 + class_of(j, m, St1, Sb1) * NTAP;
#pragma unroll
          for (int e = 0; e < NTAP; ++e) y = fma(row[e], z[(u + 1 + e) % NTAP], y);
        }
        out[i + (size_t)j * m] = y;
      }
    }
  }
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
// Four consecutive elements of one column (16 B for FP32, 32 B for FP64): the
// address is a multiple of 4 elements in every use below (m is a multiple of
// 4 on the vector paths, and so are the row offsets).
template <typename T> struct Vec4;
template <> struct Vec4<float> {
  static __device__ __forceinline__ void ld(const float* p, float (&v)[4]) {
    const float4 a = *reinterpret_cast<const float4*>(p);
    v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
  }
  static __device__ __forceinline__ void st(float* p, const float (&v)[4]) {
    *reinterpret_cast<float4*>(p) = make_float4(v[0], v[1], v[2], v[3]);
  }
};
template <> struct Vec4<double> {
  static __device__ __forceinline__ void ld(const double* p, double (&v)[4]) {
    const double2 a = reinterpret_cast<const double2*>(p)[0];
    const double2 b = reinterpret_cast<const double2*>(p)[1];
    v[0] = a.x; v[1] = a.y; v[2] = b.x; v[3] = b.y;
  }
  static __device__ __forceinline__ void st(double* p, const double (&v)[4]) {
    reinterpret_cast<double2*>(p)[0] = make_double2(v[0], v[1]);
    reinterpret_cast<double2*>(p)[1] = make_double2(v[2], v[3]);
  }
};

// Vector paths need 16-byte aligned base pointers (every buffer the library
// allocates is; a caller's offset view may not be, and then takes the
// element-wise path).
__device__ __forceinline__ bool aligned16(const void* p) {
  return (reinterpret_cast<uintptr_t>(p) & 15u) == 0;
}

// Thread layout of the vector paths on a 32 x 32 tile: 8 threads per column,
// each owning 4 consecutive rows; a wave covers 8 columns.
__device__ __forceinline__ void quad_of(int TI, int& r4, int& jl) {
  r4 = 4 * (threadIdx.x & 7);
  jl = threadIdx.x >> 3;
  (void)TI;
}

// v[0] = x (m x m), v[1] = q (n_L): q = L x.  On 32 x 32 tiles every thread
// loads its four rows of columns j and j+1 as vectors and takes row i+4 from
// the thread below (the same column) by a lane shuffle, so each x element is
// fetched once per column it is used in.
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
  if (TI == 32) {
    // lane-row layout: a thread owns row i of four consecutive columns, so
    // every load and store instruction covers 32 consecutive elements of a
    // column; all loads are issued before any store
    const int r = threadIdx.x & 31, jb = j0 + 4 * (threadIdx.x >> 5), i = i0 + r;
    T xv[5], dn[4];
#pragma unroll
    for (int c = 0; c < 5; ++c) xv[c] = (jb + c < m) ? x[i + (size_t)(jb + c) * m] : T(0);
#pragma unroll
    for (int c = 0; c < 4; ++c)
      dn[c] = (r == 31 && i + 1 < m) ? x[i + 1 + (size_t)(jb + c) * m] : T(0);
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const T nb = __shfl_down(xv[c], 1, 32);
      if (r != 31) dn[c] = nb;
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int j = jb + c;
      if (i < m - 1) q[i + (size_t)j * (m - 1)] = dn[c] - xv[c];
      if (j < m - 1) q[nx + i + (size_t)j * m] = xv[c + 1] - xv[c];
    }
    return;
  }
  for (int o = threadIdx.x; o < TI * TJ; o += NTHREADS) {
    const int i = i0 + (o & (TI - 1)), j = j0 + (o >> (__ffs(TI) - 1));
    const T xc = x[i + (size_t)j * m];
    if (i < m - 1) q[i + (size_t)j * (m - 1)] = x[i + 1 + (size_t)j * m] - xc;
    if (j < m - 1) q[nx + i + (size_t)j * m] = x[i + (size_t)(j + 1) * m] - xc;
  }
}

// v[0] = q (n_L), v[1] = y (m x m): y = L^T q = vec(D^T Qx + Qy D).  On
// 32 x 32 tiles each thread loads its four rows of the Qy columns j-1 and j as
// vectors and its Qx entries (not 4-aligned: Qx has m-1 rows) as scalars,
// taking the entry above its first row from the thread above by a shuffle.
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
  if (TI == 32) {
    // lane-row layout as in k_grad; the Qx entry above row i comes from the
    // lane above (a load for the tile's first row)
    const int r = threadIdx.x & 31, jb = j0 + 4 * (threadIdx.x >> 5), i = i0 + r;
    T cx[4], up[4], cy[5];
#pragma unroll
    for (int c = 0; c < 4; ++c)
      cx[c] = (i < m - 1) ? q[i + (size_t)(jb + c) * (m - 1)] : T(0);
#pragma unroll
    for (int c = 0; c < 4; ++c)
      up[c] = (r == 0 && i >= 1) ? q[i - 1 + (size_t)(jb + c) * (m - 1)] : T(0);
#pragma unroll
    for (int c = 0; c < 5; ++c) {
      const int j = jb + c - 1;
      cy[c] = (j >= 0 && j < m - 1) ? qy[i + (size_t)j * m] : T(0);
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const T ab = __shfl_up(cx[c], 1, 32);
      if (r != 0) up[c] = ab;
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int j = jb + c;
      T a = T(0);
      if (i >= 1) a += up[c];
      if (i < m - 1) a -= cx[c];
      if (j >= 1) a += cy[c];
      if (j < m - 1) a -= cy[c + 1];
      y[i + (size_t)j * m] = a;
    }
    return;
  }
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
  if (!four && TI == 32 && aligned16(x) && aligned16(y)) {
    // low-pass restriction: 4 coarse rows of one coarse column per thread,
    // from fine rows 2 a0 .. 2 a0 + 7 (+ K - 2 below, wrapped) of K fine
    // columns, all loads issued before any arithmetic; the sums are those of
    // the element-wise path in the same order
    int r4, jl;
    quad_of(TI, r4, jl);
    const int a0 = i0 + r4, a1 = j0 + jl, f = 2 * a0;
    T v[4][10];
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      if (b >= K) break;
      const T* __restrict__ col = x + (size_t)((2 * a1 + b) & msk) * m;
      T lo4[4], hi4[4];
      Vec4<T>::ld(col + f, lo4);
      Vec4<T>::ld(col + f + 4, hi4);
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        v[b][u] = lo4[u];
        v[b][4 + u] = hi4[u];
      }
      // rows f + 8, f + 9 (Db4 only) are the next thread's first two rows
      // (the same column); the last thread of a column loads them (wrapped)
      const bool edge = K > 2 && (threadIdx.x & 7) == 7;
      v[b][8] = edge ? col[(f + 8) & msk] : T(0);
      v[b][9] = edge ? col[(f + 9) & msk] : T(0);
    }
    if (K > 2) {
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const T n8 = __shfl_down(v[b][0], 1, 8), n9 = __shfl_down(v[b][1], 1, 8);
        if ((threadIdx.x & 7) != 7) {
          v[b][8] = n8;
          v[b][9] = n9;
        }
      }
    }
    T out[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      double ll = 0;
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        if (b >= K) break;
        double lo = 0;
#pragma unroll
        for (int a = 0; a < 4; ++a) {
          if (a >= K) break;
          lo = fma(wl_h(wav, a), (double)v[b][2 * u + a], lo);
        }
        ll = fma(wl_h(wav, b), lo, ll);
      }
      out[u] = (T)ll;
    }
    Vec4<T>::st(y + a0 + (size_t)a1 * mc, out);
    return;
  }
  for (int o = threadIdx.x; o < TI * TJ; o += NTHREADS) {
    const int a0 = i0 + (o & (TI - 1)), a1 = j0 + (o >> (__ffs(TI) - 1));
    double ll = 0, lh = 0, hl = 0, hh = 0;
    for (int b = 0; b < K; ++b) {
      const size_t col = (size_t)((2 * a1 + b) & msk) * m;
      double lo = 0, hi = 0;
      for (int a = 0; a < K; ++a) {
        const double v = (double)x[((2 * a0 + a) & msk) + col];
        lo = fma(wl_h(wav, a), v, lo);
        hi = fma(wl_g(wav, a), v, hi);
      }
      ll = fma(wl_h(wav, b), lo, ll);
      if (four) {
        lh = fma(wl_g(wav, b), lo, lh);
        hl = fma(wl_h(wav, b), hi, hl);
        hh = fma(wl_g(wav, b), hi, hh);
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
  // low-pass prolongation onto grids of 64 and more runs on 32 x 64 fine
  // tiles (add_prolong; four 32-column parts per block measured slower than
  // two): the tile width is the job's
  TJ = m / job->ntj;
  j0 = tj * TJ;
  const int wav = job->flags, K2 = wl_len(wav) / 2;
  const bool four = job->p0 != 0.0;
  const T* __restrict__ c = static_cast<const T*>(job->v[0]);
  T* __restrict__ x = static_cast<T*>(job->v[1]);
  const size_t nc = (size_t)mc * mc;
  constexpr int PQ = 2;  // 32-column parts of the widest tile
  if (!four && TI == 32 && TJ % 32 == 0 && TJ <= 32 * PQ && aligned16(x) && aligned16(c)) {
    // low-pass prolongation: 4 fine rows f0 .. f0 + 3 of one fine column per
    // thread in each 32-column part of the tile; they need coarse rows
    // f0/2 - K2 + 1 .. f0/2 + 1 (wrapped) of K2 coarse columns.  The loads of
    // all parts are issued before any arithmetic; the sums are those of the
    // element-wise path in the same order
    int r4, jl;
    quad_of(TI, r4, jl);
    const int f0 = i0 + r4, h0 = f0 >> 1, nh = TJ / 32;
    // coarse rows h0, h0 + 1 (h0 even: one aligned pair) of each coarse
    // column; row h0 - 1 (Db4) is the pair of the thread above, or a load
    // (wrapped) for the first thread of a column
    T cv[PQ][2][3];
#pragma unroll
    for (int hh = 0; hh < PQ; ++hh) {
#pragma unroll
      for (int t1 = 0; t1 < 2; ++t1) cv[hh][t1][0] = cv[hh][t1][1] = cv[hh][t1][2] = T(0);
      if (hh >= nh) break;
      const int f1 = j0 + 32 * hh + jl;
#pragma unroll
      for (int t1 = 0; t1 < 2; ++t1) {
        if (t1 >= K2) break;
        const T* __restrict__ col = c + (size_t)(((f1 >> 1) - t1) & cm) * mc;
        cv[hh][t1][1] = col[h0];
        cv[hh][t1][2] = col[h0 + 1];
        if (K2 > 1 && (threadIdx.x & 7) == 0) cv[hh][t1][0] = col[(h0 - 1) & cm];
      }
    }
#pragma unroll
    for (int hh = 0; hh < PQ; ++hh) {
      if (hh >= nh) break;
      const int f1 = j0 + 32 * hh + jl;
      if (K2 > 1) {
#pragma unroll
        for (int t1 = 0; t1 < 2; ++t1) {
          const T a = __shfl_up(cv[hh][t1][2], 1, 8);
          if ((threadIdx.x & 7) != 0) cv[hh][t1][0] = a;
        }
      }
      T out[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int ff0 = f0 + u;
        double acc = 0;
#pragma unroll
        for (int t1 = 0; t1 < 2; ++t1) {
          if (t1 >= K2) break;
          const int k1 = (f1 & 1) + 2 * t1;
#pragma unroll
          for (int t0 = 0; t0 < 2; ++t0) {
            if (t0 >= K2) break;
            const int k0 = (ff0 & 1) + 2 * t0;
            // coarse row (ff0 >> 1) - t0 = h0 + (u >> 1) - t0 sits at d = 1 + (u >> 1) - t0
            acc = fma(wl_h(wav, k0) * wl_h(wav, k1), (double)cv[hh][t1][1 + (u >> 1) - t0], acc);
          }
        }
        out[u] = (T)acc;
      }
      Vec4<T>::st(x + f0 + (size_t)f1 * m, out);
    }
    return;
  }
  for (int o = threadIdx.x; o < TI * TJ; o += NTHREADS) {
    const int f0 = i0 + (o & (TI - 1)), f1 = j0 + (o >> (__ffs(TI) - 1));
    double acc = 0;
    for (int t1 = 0; t1 < K2; ++t1) {
      const int c1 = ((f1 >> 1) - t1) & cm, k1 = (f1 & 1) + 2 * t1;
      for (int t0 = 0; t0 < K2; ++t0) {
        const int c0 = ((f0 >> 1) - t0) & cm, k0 = (f0 & 1) + 2 * t0;
        const size_t k = c0 + (size_t)c1 * mc;
        acc = fma(wl_h(wav, k0) * wl_h(wav, k1), (double)c[k], acc);
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

bool apply_stream_ok(int m, int precision, int sep, int rows1) {
  return precision != 1 && sep && m >= STREAM_MIN_M && rows1 <= STREAM_MAX_ROWS;
}
void apply_stream_grid(int m, int* nti, int* ntj) {
  *nti = m / STREAM_ROWS;
  *ntj = m / STREAM_COLS;
}

hipError_t launch_apply_stream(const LaunchArgs& la, int rb) {
  switch (rb) {
#define CASE(R)                                                                          \
  case R:                                                                                \
    hipLaunchKernelGGL((k_apply_stream<R>), dim3(la.ntiles), dim3(STREAM_ROWS), 0,       \
                       la.stream, la.jobs, la.tiles);                                    \
    break;
    CASE(2) CASE(4) CASE(8) CASE(12) CASE(16)
#undef CASE
    default: return hipErrorInvalidValue;
  }
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

SIMPLE_LAUNCHER(launch_grad, k_grad)
SIMPLE_LAUNCHER(launch_gradT, k_gradT)
SIMPLE_LAUNCHER(launch_dwt_fwd, k_dwt_fwd)
SIMPLE_LAUNCHER(launch_dwt_inv, k_dwt_inv)
SIMPLE_LAUNCHER(launch_dtransfer, k_dtransfer)

}  // namespace dbl
