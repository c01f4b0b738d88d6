#pragma once
// Bodies of the fused CGLS phases for separable operators on 32 x 32
// output tiles (kernels_cgls_sep.hip, kernels_cgls_multi.hip).  The phases
// run the two kernels per iteration described at the top of
// kernels_solve.hip; every job of a launch has an m x m grid with m >= 32.
//
// They compute what k_cgls_p1 / k_cgls_p2 compute, with the same arithmetic
// in the same order (each thread owns the same pixels and convolution items,
// so the per-tile partial sums are the same bits), but laid out for the
// wavefront instead of for a flat pixel loop:
// * the haloed input tile is loaded one column per wave instruction (lane =
//   row; at most 64 rows), so the address of a column is a wave-uniform base
//   held in scalar registers plus a per-lane byte offset that is fixed for
//   the whole tile, with the periodic wrap folded into both;
// * the tile's own pixels are visited as lane = row i, two columns per wave
//   instruction, again a uniform column base plus fixed per-lane offsets; the
//   gradient's edge conditions are per-lane constants and one compare per
//   column, and neighbours outside the grid are read at a valid address and
//   never used, so the loads need no per-element branches;
// * every pointer is global (address space 1): loads count in vmcnt only, and
//   the barriers between the LDS passes order LDS alone, so the stores of one
//   stage stay in flight across the next.
#include "phase.h"

namespace dbl {
namespace {

constexpr int TE = 32;                  // tile edge
constexpr int NWAVE = NTHREADS / 64;    // waves per block
constexpr int PX = TE * TE / NTHREADS;  // tile pixels per thread
constexpr int CV = 2;                   // outputs per item of both convolution passes

template <int RB> struct SepTile {
  static constexpr int H = RB;              // halo
  static constexpr int NR = TE + 2 * RB;    // haloed rows (axis 0)
  static constexpr int NC = TE + 2 * RB;    // haloed columns (axis 1)
  static constexpr int LX = NC + 1;         // LDS row stride of the haloed tile
  static constexpr int LZ = TE + 1;         // LDS column stride of the pass-A result
  static constexpr int KC = NC / NWAVE;     // haloed columns loaded by each wave
  static constexpr int XS = NR * LX;        // LDS elements: haloed tile
  static constexpr int ZS = NC * LZ;        // LDS elements: pass-A result
  static constexpr int NTAP = 2 * RB + 1;
  static_assert(NC % NWAVE == 0 && NR <= 64, "a haloed column must fit one wave");
  static_assert(XS + ZS == (TE + 2 * RB) * (TE + 2 * RB + 1) + (TE + 2 * RB) * (TE + 1),
                "LDS layout of the separable tile");
};

template <typename X> using GP = GlobalPtr<X>;

// A job vector of `elems` elements of type E as a buffer resource.  Loads and
// stores take a per-lane byte offset (a vector register, fixed for the tile)
// and a wave-uniform byte offset (a scalar register: the column), so they
// need no address arithmetic; every offset the kernels form lies inside the
// vector (an offset past its end would read zero and drop the store).
constexpr int RSRC_WORD3 = 0x00020000;  // raw 32-bit buffer access on gfx9
template <typename E> struct Vec {
  __amdgpu_buffer_rsrc_t r;
  __device__ __forceinline__ Vec(const void* p, size_t elems)
      : r(__builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0,
                                            (int)(uint32_t)(elems * sizeof(E)), RSRC_WORD3)) {}
  template <typename T> __device__ __forceinline__ T ld(uint32_t lb, uint32_t ub) const {
    if constexpr (sizeof(E) == 2) {
      bf16s v;
      v.u = __builtin_amdgcn_raw_buffer_load_b16(r, lb, ub, 0);
      return (T)bf16_to_f32(v);
    } else if constexpr (sizeof(E) == 4) {
      return (T)__uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, lb, ub, 0));
    } else {
      return (T)__builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, lb, ub, 0));
    }
  }
  template <typename T> __device__ __forceinline__ void st(uint32_t lb, uint32_t ub, T v) const {
    if constexpr (sizeof(E) == 2) {
      __builtin_amdgcn_raw_buffer_store_b16(f32_to_bf16((float)v).u, r, lb, ub, 0);
    } else if constexpr (sizeof(E) == 4) {
      __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint((float)v), r, lb, ub, 0);
    } else {
      using V2 = decltype(__builtin_amdgcn_raw_buffer_load_b64(r, 0, 0, 0));
      __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(V2, (double)v), r, lb, ub, 0);
    }
  }
};

// Tap rows of a class table.
template <typename T> __device__ __forceinline__ GP<const T> gtaps(GP<const Table1D> t) {
  if constexpr (sizeof(T) == 4) return gview(t->tf);
  else return gview(t->td);
}

// Byte offsets of one thread's tile pixels, fixed for the tile: lane l owns
// row i = l % 32 of columns jp(u) + l / 32, jp(u) = 2 wave + 8 u (u < PX),
// which is the pixel set o = tid + 256 u of the generic kernels.  Offsets
// are unsigned: the axis-0 difference above a pixel, (i - 1) + jh (m - 1)
// from the column's base, is -1 for lane 0 of a tile below the first row, so
// there the -1 goes into the uniform base instead (xshift = 1) and the lane
// part is x; in the first tile row the lane part is x - 1 element (lane 0,
// which has no difference above, reads its own entry, never used).
template <typename E> struct LaneOff {
  uint32_t g;    // image grid: i + jh m
  uint32_t x;    // axis-0 differences (stride m - 1 per column): i + jh (m - 1)
  uint32_t xu;   // lane part of the axis-0 difference above
  uint32_t gu;   // lane part of the pixel above (same rule as xu)
  uint32_t r;    // i alone: the pixel's row in the column pair's first column
  __device__ __forceinline__ LaneOff(int i, int jh, int m, int row0) {
    g = (uint32_t)(i + jh * m) * (uint32_t)sizeof(E);
    x = (uint32_t)(i + jh * (m - 1)) * (uint32_t)sizeof(E);
    xu = (row0 > 0 || i == 0) ? x : x - (uint32_t)sizeof(E);
    gu = (row0 > 0 || i == 0) ? g : g - (uint32_t)sizeof(E);
    r = (uint32_t)i * (uint32_t)sizeof(E);
  }
};

// Every multiply-add of the vector updates is an explicit fma: a value such
// as p = s + beta p is formed by its tile and again by each neighbour whose
// halo holds it, and all of them must agree bit for bit (phase 2 recomputes
// q2 from the stored p), whatever the compiler would contract in each copy.
// So is every term of the FP64 norm sums (acc = fma(v, v, acc)): an FP64
// square is inexact, and a sum the compiler fused in one kernel and not in
// another would give alpha and beta a different last bit.

// ------------------------------------------- general operator (2-D taps) --
// A general (non-separable) level on the same tiles (GEN): the halo is a
// radius bucket RB >= the operator's radius, and the convolution visits the
// thread's own pixels (i, 2 wave + 8 u + lane / 32), u < PX -- the pixel set
// and order of the generic kernels' gen_tile, so every sum and every partial
// is the same.  The interior class's tap list is staged in LDS as (offset in
// the haloed tile, value) behind the tile, GT entries at most; an interior
// tile takes it taps-outermost over the thread's pixels, a tile that reaches
// a seam or the grid's edge takes each pixel's class list from the table.
template <int RB> struct GenTile {
  static constexpr int GT = (2 * RB + 1) * (2 * RB + 1);  // interior taps at most
  static constexpr int GTI = (GT + 1) & ~1;                // ints, keeping T aligned
};

template <typename T, int RB>
__device__ __forceinline__ int stage_gen(int* g_off, T* g_val, const Table2D& tb) {
  using G = SepTile<RB>;
  const T* __restrict__ vals = taps2<T>(tb);
  const int icls = tb.St0 + tb.St1 * tb.rows0;
  const int b = tb.off[icls], n = tb.off[icls + 1] - b;
  for (int k = threadIdx.x; k < n; k += NTHREADS) {
    const short2 e = tb.e[b + k];
    g_off[k] = e.x * G::LX + e.y;  // rows = axis 0 (e.x), columns = axis 1 (e.y)
    g_val[k] = vals[b + k];
  }
  return n;
}

template <typename T, int RB, class Epi>
__device__ __forceinline__ void gen_conv(const T* __restrict__ Xs, const int* __restrict__ g_off,
                                        const T* __restrict__ g_val, int n, const Table2D& tb,
                                        int row0, int col0, int m, int i, int jh, int wv,
                                        Epi epi) {
  using G = SepTile<RB>;
  const bool inter = row0 >= tb.St0 && row0 + TE - 1 < m - tb.Sb0 && col0 >= tb.St1 &&
                     col0 + TE - 1 < m - tb.Sb1;
  int xo[PX];
#pragma unroll
  for (int u = 0; u < PX; ++u) xo[u] = (i + G::H) * G::LX + (2 * wv + 8 * u + jh + G::H);
  if (inter) {
    T a[PX];
#pragma unroll
    for (int u = 0; u < PX; ++u) a[u] = T(0);
    for (int k = 0; k < n; ++k) {
      const int off = g_off[k];
      const T v = g_val[k];
#pragma unroll
      for (int u = 0; u < PX; ++u) a[u] = fma(v, Xs[xo[u] + off], a[u]);
    }
#pragma unroll
    for (int u = 0; u < PX; ++u) epi(u, a[u]);
  } else {
    // Each pixel's class list is read from global memory (global, not
    // generic, loads); four taps' entries and values are requested before
    // any of them is used, and summed in list order.
    GP<const T> vals = gview(taps2<T>(tb));
    // an entry (x, y) of 16 bits each as one word, x in the low half
    GP<const int> te = gview(reinterpret_cast<const int*>(tb.e));
    GP<const int> toff = gview(tb.off);
    auto at = [&](int w, int u) { return xo[u] + (int)(short)w * G::LX + (w >> 16); };
#pragma unroll
    for (int u = 0; u < PX; ++u) {
      const int gj = col0 + 2 * wv + 8 * u + jh;
      const int cls = class_of(row0 + i, m, tb.St0, tb.Sb0) + class_of(gj, m, tb.St1, tb.Sb1) * tb.rows0;
      const int k1 = toff[cls + 1];
      int k = toff[cls];
      T a = T(0);
      for (; k + 4 <= k1; k += 4) {
        int e[4];
        T v[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          e[q] = te[k + q];
          v[q] = vals[k + q];
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) a = fma(v[q], Xs[at(e[q], u)], a);
      }
      for (; k < k1; ++k) a = fma(vals[k], Xs[at(te[k], u)], a);
      epi(u, a);
    }
  }
}

// ------------------------------------------------------ convolution passes --
// Pass A along axis 0 for all NC haloed columns and the TE rows of the tile:
// Z[c][r] = sum_e taps[e] X[r + e][c] (class rows near a seam use their own
// tap row, read from the table).  Same sums as sep_tile's pass A.
template <typename T, int RB>
__device__ __forceinline__ void pass_a(const T* __restrict__ Xs, T* __restrict__ Zs,
                                       const T* __restrict__ taps, GP<const T> tab, int St,
                                       int Sb, int row0, int m) {
  using G = SepTile<RB>;
  constexpr int NTAP = G::NTAP, NW = CV + 2 * RB, NCH = TE / CV;
  constexpr int ITEMS = G::NC * NCH;
  T tp[NTAP];
#pragma unroll
  for (int e = 0; e < NTAP; ++e) tp[e] = taps[e];
#pragma unroll 1
  for (int item = threadIdx.x; item < ITEMS; item += NTHREADS) {
    const int c = item % G::NC, ch = item / G::NC;
    const int r0 = ch * CV;
    T win[NW];
#pragma unroll
    for (int k = 0; k < NW; ++k) win[k] = Xs[(r0 + k) * G::LX + c];
    const int ia = row0 + r0;
    if (ia >= St && ia + CV - 1 < m - Sb) {
      T out[CV];
#pragma unroll
      for (int v = 0; v < CV; ++v) {
        T a = T(0);
#pragma unroll
        for (int e = 0; e < NTAP; ++e) a = fma(tp[e], win[v + e], a);
        out[v] = a;
      }
#pragma unroll
      for (int v = 0; v < CV; ++v) Zs[c * G::LZ + r0 + v] = out[v];
    } else {
#pragma unroll 1
      for (int v = 0; v < CV; ++v) {
        const GP<const T> row = tab + class_of(ia + v, m, St, Sb) * NTAP;
        const T* __restrict__ xcol = Xs + (r0 + v) * G::LX + c;
        T a = T(0);
#pragma unroll
        for (int e = 0; e < NTAP; ++e) a = fma(row[e], xcol[e * G::LX], a);
        Zs[c * G::LZ + r0 + v] = a;
      }
    }
  }
}

// Pass B along axis 1: Y[r][c] = sum_e taps[e] Z[c + e][r] for the tile.
// Same items and sums as sep_tile's pass B: item = tid + 256 rd owns row
// r = item % 32 and the CV outputs from c0 = CV (item / 32), which is the
// wave-uniform cw = CV (2 wave + 8 rd) plus CV per half-wave.  Outputs go to
// epi(r, c, cu, value) with c = c0 + v and its uniform part cu = cw + v.
template <typename T, int RB, class Epi>
__device__ __forceinline__ void pass_b(const T* __restrict__ Zs, const T* __restrict__ taps,
                                       GP<const T> tab, int St, int Sb, int col0, int m,
                                       Epi epi) {
  using G = SepTile<RB>;
  constexpr int NTAP = G::NTAP, NW = CV + 2 * RB, ROUNDS = TE * (TE / CV) / NTHREADS;
  static_assert(TE * (TE / CV) % NTHREADS == 0, "pass B items");
  T tp[NTAP];
#pragma unroll
  for (int e = 0; e < NTAP; ++e) tp[e] = taps[e];
  const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int lane = threadIdx.x & 63;
  const int r = lane & (TE - 1), cl = (lane >> 5) * CV;
#pragma unroll
  for (int rd = 0; rd < ROUNDS; ++rd) {
    const int cw = (2 * wv + 8 * rd) * CV;
    const int c0 = cw + cl;
    T win[NW];
#pragma unroll
    for (int k = 0; k < NW; ++k) win[k] = Zs[(c0 + k) * G::LZ + r];
    const int ja = col0 + c0;
    if (ja >= St && ja + CV - 1 < m - Sb) {
#pragma unroll
      for (int v = 0; v < CV; ++v) {
        T a = T(0);
#pragma unroll
        for (int e = 0; e < NTAP; ++e) a = fma(tp[e], win[v + e], a);
        epi(r, c0 + v, cw + v, a);
      }
    } else {
#pragma unroll 1
      for (int v = 0; v < CV; ++v) {
        const GP<const T> row = tab + class_of(ja + v, m, St, Sb) * NTAP;
        const T* __restrict__ zrow = Zs + (c0 + v) * G::LZ + r;
        T a = T(0);
#pragma unroll
        for (int e = 0; e < NTAP; ++e) a = fma(row[e], zrow[e * G::LZ], a);
        epi(r, c0 + v, cw + v, a);
      }
    }
  }
}

// The interior tap rows of both axes staged in LDS (taps[0, NTAP) axis 0,
// taps[NTAP, 2 NTAP) axis 1); each pass copies its row into registers.
template <typename T, int NTAP>
__device__ __forceinline__ void stage_taps(T* taps, GP<const T> tab0, int St0, GP<const T> tab1,
                                           int St1) {
  const int t = threadIdx.x;
  if (t < NTAP) taps[t] = tab0[St0 * NTAP + t];
  else if (t < 2 * NTAP) taps[t] = tab1[St1 * NTAP + t - NTAP];
}

// Entry of q2 = sqrt(g) diag(w) L p between pixel value a and its forward
// neighbour b, as stored: both phases form it with these operations, so
// phase 2 recomputes exactly the values phase 1 summed into |q|^2.
template <typename T, typename S>
__device__ __forceinline__ T grad_entry(double sg, T a, T b, T w) {
  const double d = ((double)b - (double)a) * (double)w;
  return rtv<S>((T)(sg * d));
}

// ------------------------------------------------------------------ phase 1 --
// p = s + beta p (beta = |s_k|^2 / |s_{k-1}|^2; p = s on the first
// iteration), q1 = A p, q2 = sqrt(g) D p; |q|^2 partial per tile.
//
// Offsets: a vector's element (gi, gj) of the image grid sits at gi + gj m;
// the axis-0 differences at gi + gj (m - 1) (gi < m - 1), the axis-1
// differences at nx + gi + gj m (gj < m - 1), nx = m (m - 1).  Uniform parts
// (the column) are in elements, times the element size at the access.
template <typename T, typename S, int RB, bool GEN = false>
__device__ __forceinline__ void p1_sep_body(const Job* __restrict__ jobs,
                                            const uint32_t* __restrict__ tiles) {
  using G = SepTile<RB>;
  constexpr uint32_t ES = sizeof(S), ET = sizeof(T);
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ double red[8];
  __shared__ double bc;
  __shared__ double bc2[2];
  T* Xs = reinterpret_cast<T*>(smem);
  T* Zs = Xs + G::XS;
  T* taps = Zs + G::ZS;
  int* g_off = reinterpret_cast<int*>(Xs + G::XS);  // GEN: the interior list behind the tile
  T* g_val = reinterpret_cast<T*>(g_off + GenTile<RB>::GTI);
  const Job* job; int ti, tj, tix;
  decode_tile(jobs, tiles, job, ti, tj, tix);
  const int m = job->m;
  const int row0 = ti * TE, col0 = tj * TE;
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const GP<const LevelOp> op = gview(job->op);
  // separable tables (loaded with the tile; unused, and dropped, for GEN)
  const int St0 = op->f0.St, Sb0 = op->f0.Sb, St1 = op->f1.St, Sb1 = op->f1.Sb;
  const GP<const T> tab0 = gtaps<T>(&op->f0), tab1 = gtaps<T>(&op->f1);
  Table2D tg;
  int gn = 0;
  if constexpr (GEN) {
    tg = job->op->f2;
    gn = stage_gen<T, RB>(g_off, g_val, tg);
  } else {
    stage_taps<T, G::NTAP>(taps, tab0, St0, tab1, St1);
  }
  const int flags = job->flags;
  const bool first = flags & F_FIRST, irls = flags & F_IRLS;
  const int nt = job->nti * job->ntj;
  const double sg = job->scal[S_SQRTG];
  const unsigned msk = (unsigned)m - 1u;
  const uint32_t n = (uint32_t)m * (uint32_t)m, nx = (uint32_t)(m - 1) * (uint32_t)m;
  const Vec<S> s(job->v[V_S], n), pa(job->v[V_PA], n), pb(job->v[V_PB], n), q1(job->v[V_Q1], n);
  const Vec<T> w(job->v[V_W], 2 * nx);

  // haloed tile of s (and p): lane = row row0 - H + lane (periodic), wave wv
  // takes columns wv KC .. wv KC + KC - 1
  const bool hrow = lane < G::NR;
  const uint32_t hb = ((unsigned)(row0 - G::H + lane) & msk) * ES;
  T va[G::KC], vb[G::KC];
  if (hrow) {
#pragma unroll
    for (int k = 0; k < G::KC; ++k)
      va[k] = s.template ld<T>(hb, ((unsigned)(col0 - G::H + wv * G::KC + k) & msk) * m * ES);
    if (!first) {
#pragma unroll
      for (int k = 0; k < G::KC; ++k)
        vb[k] = pa.template ld<T>(hb, ((unsigned)(col0 - G::H + wv * G::KC + k) & msk) * m * ES);
    }
  }
  // the thread's pixels and their IRLS weights (axis-0 entry, axis-1 entry)
  const int i = lane & (TE - 1), jh = lane >> 5;
  const int gi = row0 + i;
  const bool dn = gi < m - 1;
  const LaneOff<S> oS(i, jh, m, row0);
  const LaneOff<T> oT(i, jh, m, row0);
  T wx[PX], wy[PX];
#pragma unroll
  for (int u = 0; u < PX; ++u) {
    wx[u] = T(1);
    wy[u] = T(1);
  }
  if (irls) {
#pragma unroll
    for (int u = 0; u < PX; ++u) {
      const int jp = 2 * wv + 8 * u;
      const bool rt = col0 + jp + jh < m - 1;
      const uint32_t cx = (uint32_t)(col0 + jp) * (uint32_t)(m - 1) + row0;
      const uint32_t cy = nx + (uint32_t)(col0 + jp) * (uint32_t)m + row0;
      wx[u] = w.template ld<T>(oT.x, cx * ET);  // row m - 1: a valid entry, not used
      if (rt) wy[u] = w.template ld<T>(oT.g, cy * ET);
    }
  }
  T tb = T(0);
  if (!first) {
    // beta from the |s|^2 partials of the last two phase-2 launches, summed
    // while the tile loads are in flight
    double gcur, gprev;
    sum_partials2<2, 2>(job->pr[0], 0, job->pr[1], 0, nt, red, bc2, gcur, gprev);
    tb = (T)(gprev > 0.0 ? gcur / gprev : 0.0);
    if ((flags & F_HIST) && tix == 0) {
      const double rr = sum_partials<2>(job->pr[0], nt, 1, red, &bc);
      if (threadIdx.x == 0 && job->i0 >= 1 && job->i0 <= HIST_MAX)
        job->scal[S_HIST + job->i0 - 1] = rr;
    }
  }
  if (hrow) {
#pragma unroll
    for (int k = 0; k < G::KC; ++k)
      Xs[lane * G::LX + wv * G::KC + k] = first ? va[k] : rtv<S>(fma(tb, vb[k], va[k]));
  }
  lds_barrier();

  // p of the tile; |q2|^2 of q2 = sqrt(g) D p from the LDS tile (q2 itself
  // is not stored: phase 2 forms the same values again from p)
  double acc = 0.0;
#pragma unroll
  for (int u = 0; u < PX; ++u) {
    const int jp = 2 * wv + 8 * u;
    const int j = jp + jh;
    const bool rt = col0 + j < m - 1;
    const uint32_t cg = (uint32_t)(col0 + jp) * (uint32_t)m + row0;
    const int xo = (i + G::H) * G::LX + (j + G::H);
    const T pc = Xs[xo];
    pb.st(oS.g, cg * ES, pc);
    if (dn) {
      const T qv = grad_entry<T, S>(sg, pc, Xs[xo + G::LX], wx[u]);
      acc = fma((double)qv, (double)qv, acc);
    }
    if (rt) {
      const T qv = grad_entry<T, S>(sg, pc, Xs[xo + 1], wy[u]);
      acc = fma((double)qv, (double)qv, acc);
    }
  }

  // q1 = A p
  if constexpr (GEN) {
    gen_conv<T, RB>(Xs, g_off, g_val, gn, tg, row0, col0, m, i, jh, wv, [&](int u, T v) {
      const T qv = rtv<S>(v);
      q1.st(oS.g, ((uint32_t)(col0 + 2 * wv + 8 * u) * (uint32_t)m + row0) * ES, qv);
      acc = fma((double)qv, (double)qv, acc);
    });
  } else {
    pass_a<T, RB>(Xs, Zs, taps, tab0, St0, Sb0, row0, m);
    lds_barrier();
    // pass-B outputs: lane offset i + CV (lane / 32) m of the uniform column cu
    const uint32_t ob = (uint32_t)(i + jh * CV * m) * ES;
    pass_b<T, RB>(Zs, taps + G::NTAP, tab1, St1, Sb1, col0, m, [&](int, int, int cu, T v) {
      const T qv = rtv<S>(v);
      q1.st(ob, ((uint32_t)(col0 + cu) * (uint32_t)m + row0) * ES, qv);
      acc = fma((double)qv, (double)qv, acc);
    });
  }
  double vv[1] = {acc};
  put_partials<1>(job->pw, tix, vv, red);
}

// ------------------------------------------------------------------ phase 2 --
// alpha = |s|^2 / |q|^2; x += alpha p; r -= alpha q; s = A^T r1 + sqrt(g) D^T r2;
// |s|^2 and |r|^2 partials per tile.
template <typename T, typename S, int RB, bool GEN = false>
__device__ __forceinline__ void p2_sep_body(const Job* __restrict__ jobs,
                                            const uint32_t* __restrict__ tiles) {
  using G = SepTile<RB>;
  constexpr uint32_t ES = sizeof(S), ET = sizeof(T);
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ double red[8];
  __shared__ double bc2[2];
  T* Xs = reinterpret_cast<T*>(smem);
  T* Zs = Xs + G::XS;
  T* taps = Zs + G::ZS;
  int* g_off = reinterpret_cast<int*>(Xs + G::XS);  // GEN: the interior list behind the tile
  T* g_val = reinterpret_cast<T*>(g_off + GenTile<RB>::GTI);
  // sqrt(g) D^T (w r2) of the tile, column-major
  T* LTs = GEN ? g_val + GenTile<RB>::GT : taps + 2 * G::NTAP;
  const Job* job; int ti, tj, tix;
  decode_tile(jobs, tiles, job, ti, tj, tix);
  const int m = job->m;
  const int row0 = ti * TE, col0 = tj * TE;
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const GP<const LevelOp> op = gview(job->op);
  // separable tables (loaded with the tile; unused, and dropped, for GEN)
  const int St0 = op->a0.St, Sb0 = op->a0.Sb, St1 = op->a1.St, Sb1 = op->a1.Sb;
  const GP<const T> tab0 = gtaps<T>(&op->a0), tab1 = gtaps<T>(&op->a1);
  Table2D tg;
  int gn = 0;
  if constexpr (GEN) {
    tg = job->op->a2;
    gn = stage_gen<T, RB>(g_off, g_val, tg);
  } else {
    stage_taps<T, G::NTAP>(taps, tab0, St0, tab1, St1);
  }
  const int flags = job->flags;
  const bool first = flags & F_FIRST, irls = flags & F_IRLS;
  const int nt = job->nti * job->ntj;
  const double sg = job->scal[S_SQRTG];
  const unsigned msk = (unsigned)m - 1u;
  const uint32_t n = (uint32_t)m * (uint32_t)m, nx = (uint32_t)(m - 1) * (uint32_t)m;
  const Vec<T> x(job->v[V_X], n), w(job->v[V_W], 2 * nx);
  const Vec<S> p(job->v[V_PB], n), r1a(job->v[V_R1A], n), r1b(job->v[V_R1B], n),
      q1(job->v[V_Q1], n), s(job->v[V_S], n), r2a(job->v[V_R2A], 2 * nx),
      r2b(job->v[V_R2B], 2 * nx);

  // haloed tile of r1 (and q1)
  const bool hrow = lane < G::NR;
  const uint32_t hb = ((unsigned)(row0 - G::H + lane) & msk) * ES;
  T va[G::KC], vb[G::KC];
  if (hrow) {
#pragma unroll
    for (int k = 0; k < G::KC; ++k)
      va[k] = r1a.template ld<T>(hb, ((unsigned)(col0 - G::H + wv * G::KC + k) & msk) * m * ES);
    if (!first) {
#pragma unroll
      for (int k = 0; k < G::KC; ++k)
        vb[k] = q1.template ld<T>(hb, ((unsigned)(col0 - G::H + wv * G::KC + k) & msk) * m * ES);
    }
  }
  double alpha = 0.0;
  if (!first) {
    // alpha from the |q|^2 partials of phase 1 and the |s|^2 partials of the
    // previous phase 2, summed while the tile loads are in flight
    double qq, gs;
    sum_partials2<1, 2>(job->pr[0], 0, job->pr[1], 0, nt, red, bc2, qq, gs);
    alpha = qq > 0.0 ? gs / qq : 0.0;
  }
  const T ta = (T)alpha;
  if (hrow) {
#pragma unroll
    for (int k = 0; k < G::KC; ++k)
      Xs[lane * G::LX + wv * G::KC + k] = first ? va[k] : rtv<S>(fma(-ta, vb[k], va[k]));
  }
  lds_barrier();

  const int i = lane & (TE - 1), jh = lane >> 5;
  const int gi = row0 + i;
  const bool up = gi >= 1, dn = gi < m - 1;
  const LaneOff<S> oS(i, jh, m, row0);
  const LaneOff<T> oT(i, jh, m, row0);
  const uint32_t xshift = row0 > 0 ? 1u : 0u;  // uniform part of the difference above
  double accr = 0.0, accs = 0.0;
  // r1 of the tile: stored, |r1|^2
#pragma unroll
  for (int u = 0; u < PX; ++u) {
    const int jp = 2 * wv + 8 * u;
    const T rv = Xs[(i + G::H) * G::LX + jp + jh + G::H];
    r1b.st(oS.g, ((uint32_t)(col0 + jp) * (uint32_t)m + row0) * ES, rv);
    accr = fma((double)rv, (double)rv, accr);
  }
  // gradient part, two pixels at a time: the entries qx(i-1,j), qx(i,j),
  // qy(i,j-1), qy(i,j) of r2 (and w), x, and p at the pixel and its four
  // neighbours: x += alpha p, and the q2 entries (r2 -= alpha q2) formed
  // from p as phase 1 formed them
#pragma unroll
  for (int u0 = 0; u0 < PX; u0 += 2) {
    T a[2][4], wg[2][4], xv[2], pv[2], pn[2][4];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int jp = 2 * wv + 8 * (u0 + h);
      const bool rt = col0 + jp + jh < m - 1;
      const uint32_t cx = (uint32_t)(col0 + jp) * (uint32_t)(m - 1) + row0;
      const uint32_t cg = (uint32_t)(col0 + jp) * (uint32_t)m + row0;
      const uint32_t cy = nx + cg;
      const uint32_t cu = cx - xshift;  // >= 0: cx >= row0 >= 1 when shifted
      // grid row 0: xu is a valid stand-in; column 0: cy - m lies in the
      // axis-0 block (m >= 32); row m - 1: (m - 1)(j + 1) <= nx; none is used
      a[h][0] = r2a.template ld<T>(oS.xu, cu * ES);
      a[h][1] = r2a.template ld<T>(oS.x, cx * ES);
      a[h][2] = r2a.template ld<T>(oS.g, (cy - m) * ES);
      a[h][3] = rt ? r2a.template ld<T>(oS.g, cy * ES) : T(0);
#pragma unroll
      for (int d = 0; d < 4; ++d) {
        pn[h][d] = T(0);
        wg[h][d] = T(1);
      }
      if (!first) {
        // p above (grid row 0: own value, not used), left (grid column 0:
        // the first column of the pair, not used), below, right
        const bool c0 = col0 + jp == 0;
        xv[h] = x.template ld<T>(oT.g, cg * ET);
        pv[h] = p.template ld<T>(oS.g, cg * ES);
        pn[h][0] = p.template ld<T>(oS.gu, (cg - xshift) * ES);
        pn[h][2] = p.template ld<T>(c0 ? oS.r : oS.g, (c0 ? cg : cg - m) * ES);
        if (dn) pn[h][1] = p.template ld<T>(oS.g + ES, cg * ES);
        if (rt) pn[h][3] = p.template ld<T>(oS.g, (cg + m) * ES);
      }
      if (irls) {
        wg[h][0] = w.template ld<T>(oT.xu, cu * ET);
        wg[h][1] = w.template ld<T>(oT.x, cx * ET);
        wg[h][2] = w.template ld<T>(oT.g, (cy - m) * ET);
        if (rt) wg[h][3] = w.template ld<T>(oT.g, cy * ET);
      }
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int jp = 2 * wv + 8 * (u0 + h);
      const int gj = col0 + jp + jh;
      const uint32_t cx = (uint32_t)(col0 + jp) * (uint32_t)(m - 1) + row0;
      const uint32_t cg = (uint32_t)(col0 + jp) * (uint32_t)m + row0;
      T q[4];
      if (!first) {
        q[0] = grad_entry<T, S>(sg, pn[h][0], pv[h], wg[h][0]);
        q[1] = grad_entry<T, S>(sg, pv[h], pn[h][1], wg[h][1]);
        q[2] = grad_entry<T, S>(sg, pn[h][2], pv[h], wg[h][2]);
        q[3] = grad_entry<T, S>(sg, pv[h], pn[h][3], wg[h][3]);
      }
      T rn[4];
#pragma unroll
      for (int d = 0; d < 4; ++d) rn[d] = first ? a[h][d] : rtv<S>(fma(-ta, q[d], a[h][d]));
      double lt = 0.0;
      if (up) lt += (double)wg[h][0] * (double)rn[0];
      if (dn) {
        r2b.st(oS.x, cx * ES, rn[1]);
        accr = fma((double)rn[1], (double)rn[1], accr);
        lt -= (double)wg[h][1] * (double)rn[1];
      }
      if (gj >= 1) lt += (double)wg[h][2] * (double)rn[2];
      if (gj < m - 1) {
        r2b.st(oS.g, (nx + cg) * ES, rn[3]);
        accr = fma((double)rn[3], (double)rn[3], accr);
        lt -= (double)wg[h][3] * (double)rn[3];
      }
      LTs[i + (jp + jh) * TE] = (T)(sg * lt);
      if (!first) x.st(oT.g, cg * ET, fma(ta, pv[h], xv[h]));
    }
  }
  lds_barrier();  // LT complete (the haloed tile was complete before)

  // s = A^T r1 + LT
  if constexpr (GEN) {
    gen_conv<T, RB>(Xs, g_off, g_val, gn, tg, row0, col0, m, i, jh, wv, [&](int u, T v) {
      const int jp = 2 * wv + 8 * u;
      const T sv = rtv<S>(v + LTs[i + (jp + jh) * TE]);
      s.st(oS.g, ((uint32_t)(col0 + jp) * (uint32_t)m + row0) * ES, sv);
      accs = fma((double)sv, (double)sv, accs);
    });
  } else {
    pass_a<T, RB>(Xs, Zs, taps, tab0, St0, Sb0, row0, m);
    lds_barrier();
    const uint32_t ob = (uint32_t)(i + jh * CV * m) * ES;
    pass_b<T, RB>(Zs, taps + G::NTAP, tab1, St1, Sb1, col0, m, [&](int r, int c, int cu, T v) {
      const T sv = rtv<S>(v + LTs[r + c * TE]);
      s.st(ob, ((uint32_t)(col0 + cu) * (uint32_t)m + row0) * ES, sv);
      accs = fma((double)sv, (double)sv, accs);
    });
  }
  double vv[2] = {accs, accr};
  put_partials<2>(job->pw, tix, vv, red);
}

}  // namespace

// Minimum waves per SIMD of the register-bounded (wide) variant: FP32 up to
// radius bucket 8 in 64 VGPRs (8 waves: as many as the LDS admits), bucket 12
// in 80, bucket 16 in 128, all without spills; FP64 as the generic kernels.
template <typename T, int RB>
constexpr int sep_wide_waves() {
  return sizeof(T) == 4 ? (RB <= 8 ? 8 : RB <= 12 ? 6 : 4) : 2;
}

}  // namespace dbl
