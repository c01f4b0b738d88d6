// Tile-level stencil building blocks for the blur operators A^(i), A^(i)^T.
//
// A tile of TI x TJ outputs is computed from an LDS copy of the input with a
// halo of H pixels on every side, loaded with periodic indexing (the class
// tables hold zeros wherever a level has no coupling, so wrapped halo values
// only matter where the periodic wavelet seam really couples the two ends).
//
// Separable operators (A^(i) = C1 (x) C0) run two register-blocked passes:
//   pass A: Z = C0 X along axis 0 for every column of the tile plus halo; a
//           thread owns one column and V consecutive rows, so each LDS value
//           is read once per V outputs and the interior taps sit in registers;
//   pass B: Y = Z C1^T along axis 1; a thread owns one row and V columns.
// Rows near the seam use their own tap row (wave-uniform address).
//
// General (non-separable) operators use per class-pair tap lists; tiles that
// lie entirely in the interior read the interior list from LDS.
#pragma once
#include "common.h"

namespace dbl {

template <typename T> __device__ __forceinline__ const T* taps1(const Table1D& t);
template <> __device__ __forceinline__ const float* taps1<float>(const Table1D& t) { return t.tf; }
template <> __device__ __forceinline__ const double* taps1<double>(const Table1D& t) { return t.td; }
template <typename T> __device__ __forceinline__ const T* taps2(const Table2D& t);
template <> __device__ __forceinline__ const float* taps2<float>(const Table2D& t) { return t.vf; }
template <> __device__ __forceinline__ const double* taps2<double>(const Table2D& t) { return t.vd; }

template <typename T> struct TileCfg;
template <> struct TileCfg<float> { static constexpr int V = 8; };
template <> struct TileCfg<double> { static constexpr int V = 8; };

// Row-major LDS tile (separable kernels): Xs[r * LX + c], r indexes axis 0
// (rows, i) and c axis 1 (columns, j), both offset by the halo H.
__host__ __device__ inline int sep_lx(int TJ, int H) { return TJ + 2 * H + 1; }
__host__ __device__ inline int sep_lz(int TI) { return TI + 1; }
// LDS elements needed by the separable path.
__host__ __device__ inline int sep_lds_elems(int TI, int TJ, int H) {
  return (TI + 2 * H) * sep_lx(TJ, H) + (TJ + 2 * H) * sep_lz(TI);
}
// Column-major LDS tile (general 2-D kernels): Xs[c * LXC + r].
__host__ __device__ inline int col_lx(int TI, int H) { return TI + 2 * H + 1; }
__host__ __device__ inline int col_lds_elems(int TI, int TJ, int H) {
  return (TJ + 2 * H) * col_lx(TI, H);
}

// q = n / d and r = n % d for 0 <= n <= 4096 and 1 <= d <= 128 without an
// integer division: (n + 1/2) / d lies at least 1/(2d) >= 1/256 from an
// integer, and its FP32 evaluation with the hardware reciprocal (1 ulp) errs
// by less than 1e-3 at these sizes, so the truncation is exact.  A divisor
// known at compile time (after inlining, as in the one-block kernels) keeps
// the compiler's multiply-shift sequence, which is shorter.
__device__ __forceinline__ void divmod_small(int n, int d, float rd, int& q, int& r) {
  if (__builtin_constant_p(d)) {
    q = (int)((unsigned)n / (unsigned)d);
  } else {
    q = (int)(((float)n + 0.5f) * rd);
  }
  r = n - q * d;
}
__device__ __forceinline__ float rcp_small(int d) { return __builtin_amdgcn_rcpf((float)d); }

// Row and column of pixel o in a tile of TI rows (TI a power of two).
__device__ __forceinline__ void tile_ij(int o, int TI, int& i, int& j) {
  i = o & (TI - 1);
  j = o >> (__ffs(TI) - 1);
}

// Load the (TI+2H) x (TJ+2H) region starting at global (i0-H, j0-H) with
// periodic wrap.  f(gi) returns the value at flat global index gi.  Loads are
// issued in groups of U per thread before the LDS stores, so the whole tile
// is requested in one or two memory round trips.  Elements before `start`
// (in the thread-strided order) are left to the caller.
template <typename T, bool ROWMAJOR, int NT = NTHREADS, class F>
__device__ __forceinline__ void load_tile(T* Xs, int ld, int i0, int j0, int TI, int TJ, int H,
                                          int m, F f, int start = 0) {
  constexpr int U = sizeof(T) == 4 ? 16 : 8;
  const int NR = TI + 2 * H, NC = TJ + 2 * H, tot = NR * NC;  // <= 64 x 64
  const int msk = m - 1;
  const float rNR = rcp_small(NR);
#pragma unroll 1
  for (int base = start + threadIdx.x; base < tot; base += NT * U) {
    T v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int idx = base + u * NT;
      if (idx < tot) {
        int c, r;
        divmod_small(idx, NR, rNR, c, r);
        const int gi = (i0 - H + r) & msk, gj = (j0 - H + c) & msk;
        v[u] = f(gi + gj * m);
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int idx = base + u * NT;
      if (idx < tot) {
        int c, r;
        divmod_small(idx, NR, rNR, c, r);
        if (ROWMAJOR) Xs[r * ld + c] = v[u]; else Xs[c * ld + r] = v[u];
      }
    }
  }
}

// load_tile for values comb(a[g], b[g], c) whose scalar c comes from a block
// reduction (the CGLS step lengths): the first batch of a and b is requested
// before scalar() runs, so those loads and the reduction's reads of the
// previous launch's partials are in flight together.  scalar() holds
// barriers: every thread calls it exactly once, outside any branch.  The
// first batch holds U elements per thread (a whole 48 x 48 FP32 tile), few
// enough that the held values do not raise the phases' register peak.
template <typename T, bool ROWMAJOR, int NT = NTHREADS, class FA, class FB, class FS, class FC>
__device__ __forceinline__ void load_tile_overlap(T* Xs, int ld, int i0, int j0, int TI, int TJ,
                                                  int H, int m, FA fa, FB fb, FS scalar,
                                                  FC comb) {
  constexpr int U = sizeof(T) == 4 ? 10 : 5;
  const int NR = TI + 2 * H, NC = TJ + 2 * H, tot = NR * NC;  // <= 64 x 64
  const int msk = m - 1;
  const float rNR = rcp_small(NR);
  T va[U], vb[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int idx = threadIdx.x + u * NT;
    if (idx < tot) {
      int c, r;
      divmod_small(idx, NR, rNR, c, r);
      const int g = ((i0 - H + r) & msk) + ((j0 - H + c) & msk) * m;
      va[u] = fa(g);
      vb[u] = fb(g);
    }
  }
  const T cv = scalar();
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int idx = threadIdx.x + u * NT;
    if (idx < tot) {
      int c, r;
      divmod_small(idx, NR, rNR, c, r);
      const T v = comb(va[u], vb[u], cv);
      if (ROWMAJOR) Xs[r * ld + c] = v; else Xs[c * ld + r] = v;
    }
  }
  // tiles beyond one batch per thread (FP64 with the widest halos)
  load_tile<T, ROWMAJOR, NT>(Xs, ld, i0, j0, TI, TJ, H, m, [&](int g) {
    return comb(fa(g), fb(g), cv);
  }, NT * U);
}

// Separable two-pass tile convolution.  Tables padded to radius RB (2RB+1
// taps per row), RB <= H; each thread computes V consecutive outputs per
// item (register blocking).  epi(i_local, j_local, value) consumes outputs;
// every thread calls it for the outputs it owns (rows i, columns j..j+V-1).
struct NoHook {
  __device__ __forceinline__ void operator()() const {}
};

// ROLLED: seam rows computed one output at a time straight from LDS (small
// register footprint; right for tiles, where seam rows are rare) or, when
// false, register-blocked like the interior (for whole small levels, where
// a large share of the rows are seam rows).
template <typename T, int RB, int NTH = NTHREADS, int V = TileCfg<T>::V, bool ROLLED = true,
          class Epi, class Hook = NoHook>
__device__ __forceinline__ void sep_tile(const T* __restrict__ Xs, int H, T* __restrict__ Zs,
                                         const Table1D& t0, const Table1D& t1, int i0, int j0,
                                         int TI, int TJ, int m, Epi epi, Hook hook = Hook()) {
  constexpr int NTAP = 2 * RB + 1;
  constexpr int NW = V + 2 * RB;
  const int LX = sep_lx(TJ, H), LZ = sep_lz(TI);
  const T* __restrict__ T0 = taps1<T>(t0);
  const T* __restrict__ T1 = taps1<T>(t1);
  const int NRX = TI + 2 * H;

  // ---- pass A: along axis 0, for the TJ + 2RB columns pass B needs
  {
    T tp[NTAP];
#pragma unroll
    for (int e = 0; e < NTAP; ++e) tp[e] = T0[t0.St * NTAP + e];
    const int NC = TJ + 2 * RB;  // <= 128; NC * nch <= 4096
    const int nch = (TI + V - 1) / V;
    const float rNC = rcp_small(NC);
#pragma unroll 1
    for (int item = threadIdx.x; item < NC * nch; item += NTH) {
      int c, ch;
      divmod_small(item, NC, rNC, ch, c);
      const int r0 = ch * V;
      const int xc = c + (H - RB);
      T win[NW];
#pragma unroll
      for (int k = 0; k < NW; ++k) {
        const int rr = r0 + k + (H - RB);
        win[k] = (rr < NRX) ? Xs[rr * LX + xc] : T(0);
      }
      const int ia = i0 + r0;
      const bool inter = (ia >= t0.St) && (ia + V - 1 < m - t0.Sb);
      if (inter) {
        T out[V];
#pragma unroll
        for (int v = 0; v < V; ++v) {
          T a = T(0);
#pragma unroll
          for (int e = 0; e < NTAP; ++e) a = fma(tp[e], win[v + e], a);
          out[v] = a;
        }
#pragma unroll
        for (int v = 0; v < V; ++v)
          if (r0 + v < TI) Zs[c * LZ + r0 + v] = out[v];
      } else if constexpr (ROLLED) {
        // rows near a seam: own tap row, operands straight from LDS, one
        // output at a time
#pragma unroll 1
        for (int v = 0; v < V; ++v) {
          const int i = ia + v;
          if (r0 + v >= TI) break;
          const int cls = (i < m) ? class_of(i, m, t0.St, t0.Sb) : t0.St;
          const T* __restrict__ row = T0 + cls * NTAP;
          const T* __restrict__ xcol = Xs + (r0 + v + (H - RB)) * LX + xc;
          T a = T(0);
#pragma unroll
          for (int e = 0; e < NTAP; ++e) a = fma(row[e], xcol[e * LX], a);
          Zs[c * LZ + r0 + v] = a;
        }
      } else {
        T out[V];
#pragma unroll
        for (int v = 0; v < V; ++v) {
          const int i = ia + v;
          const int cls = (i < m) ? class_of(i, m, t0.St, t0.Sb) : t0.St;
          const T* __restrict__ row = T0 + cls * NTAP;
          T a = T(0);
#pragma unroll
          for (int e = 0; e < NTAP; ++e) a = fma(row[e], win[v + e], a);
          out[v] = a;
        }
#pragma unroll
        for (int v = 0; v < V; ++v)
          if (r0 + v < TI) Zs[c * LZ + r0 + v] = out[v];
      }
    }
  }
  __syncthreads();
  hook();  // Xs is no longer read: the hook may reuse it (and must sync)
  // ---- pass B: along axis 1
  {
    T tp[NTAP];
#pragma unroll
    for (int e = 0; e < NTAP; ++e) tp[e] = T1[t1.St * NTAP + e];
    const int NC = TJ + 2 * RB;
    const int nch = (TJ + V - 1) / V;
#pragma unroll 1
    for (int item = threadIdx.x; item < TI * nch; item += NTH) {
      int r, ch;
      tile_ij(item, TI, r, ch);
      const int c0 = ch * V;
      T win[NW];
#pragma unroll
      for (int k = 0; k < NW; ++k) win[k] = (c0 + k < NC) ? Zs[(c0 + k) * LZ + r] : T(0);
      const int ja = j0 + c0;
      const bool inter = (ja >= t1.St) && (ja + V - 1 < m - t1.Sb);
      if (inter) {
#pragma unroll
        for (int v = 0; v < V; ++v) {
          T a = T(0);
#pragma unroll
          for (int e = 0; e < NTAP; ++e) a = fma(tp[e], win[v + e], a);
          if (c0 + v < TJ) epi(r, c0 + v, a);
        }
      } else if constexpr (ROLLED) {
#pragma unroll 1
        for (int v = 0; v < V; ++v) {
          const int j = ja + v;
          if (c0 + v >= TJ) break;
          const int cls = (j < m) ? class_of(j, m, t1.St, t1.Sb) : t1.St;
          const T* __restrict__ row = T1 + cls * NTAP;
          const T* __restrict__ zrow = Zs + (c0 + v) * LZ + r;
          T a = T(0);
#pragma unroll
          for (int e = 0; e < NTAP; ++e) a = fma(row[e], zrow[e * LZ], a);
          epi(r, c0 + v, a);
        }
      } else {
#pragma unroll
        for (int v = 0; v < V; ++v) {
          const int j = ja + v;
          const int cls = (j < m) ? class_of(j, m, t1.St, t1.Sb) : t1.St;
          const T* __restrict__ row = T1 + cls * NTAP;
          T a = T(0);
#pragma unroll
          for (int e = 0; e < NTAP; ++e) a = fma(row[e], win[v + e], a);
          if (c0 + v < TJ) epi(r, c0 + v, a);
        }
      }
    }
  }
}

// General 2-D tile convolution over class-pair tap lists.  Xs is the
// column-major tile (halo H >= max(R0, R1)); `itaps` is LDS scratch for up
// to (2H+1)^2 interior taps.  epi(i_local, j_local, value).
template <typename T, int NT = NTHREADS, class Epi>
__device__ __forceinline__ void gen_tile(const T* __restrict__ Xs, int H, const Table2D& tb,
                                         short2* s_e, T* s_v, int i0, int j0, int TI, int TJ,
                                         int m, Epi epi) {
  const int LXC = col_lx(TI, H);
  const T* __restrict__ vals = taps2<T>(tb);
  const bool inter = (i0 >= tb.St0) && (i0 + TI - 1 < m - tb.Sb0) && (j0 >= tb.St1) &&
                     (j0 + TJ - 1 < m - tb.Sb1);
  if (inter) {
    // Interior tile: one tap list for every pixel.  Each tap is staged as its
    // tile offset e1 LXC + e0 and value, and one pass over the taps updates
    // all of the thread's pixels (each pixel's sum keeps the tap order): per
    // tap and pixel, one LDS read of the tile and one fma.
    const int cls = tb.St0 + tb.St1 * tb.rows0;
    const int b = tb.off[cls], n = tb.off[cls + 1] - b;
    int* s_off = reinterpret_cast<int*>(s_e);
    for (int k = threadIdx.x; k < n; k += NT) {
      const short2 e = tb.e[b + k];
      s_off[k] = e.y * LXC + e.x;
      s_v[k] = vals[b + k];
    }
    __syncthreads();
    constexpr int UMAX = (32 * 32 + NT - 1) / NT;  // pixels per thread (tiles <= 32 x 32)
    const int np = TI * TJ;
    int base[UMAX];
    T acc[UMAX];
#pragma unroll
    for (int u = 0; u < UMAX; ++u) {
      const int o = threadIdx.x + u * NT;
      int i, j;
      tile_ij(o, TI, i, j);
      // a slot past the tile reads around (H, H): every tap offset stays inside
      base[u] = o < np ? (j + H) * LXC + (i + H) : H * LXC + H;
      acc[u] = T(0);
    }
    for (int k = 0; k < n; ++k) {
      const int off = s_off[k];
      const T v = s_v[k];
#pragma unroll
      for (int u = 0; u < UMAX; ++u) acc[u] = fma(v, Xs[base[u] + off], acc[u]);
    }
#pragma unroll
    for (int u = 0; u < UMAX; ++u) {
      const int o = threadIdx.x + u * NT;
      if (o < np) {
        int i, j;
        tile_ij(o, TI, i, j);
        epi(i, j, acc[u]);
      }
    }
  } else {
    // Each pixel's class list is read from global memory (global, not
    // generic, loads; an entry (e0, e1) of 16 bits each as one word, e0 in
    // the low half); four taps are requested before any is used, and summed
    // in list order.
    GlobalPtr<const T> gv = gview(vals);
    GlobalPtr<const int> te = gview(reinterpret_cast<const int*>(tb.e));
    GlobalPtr<const int> toff = gview(tb.off);
    for (int o = threadIdx.x; o < TI * TJ; o += NT) {
      int i, j;
      tile_ij(o, TI, i, j);
      const int c0 = class_of(i0 + i, m, tb.St0, tb.Sb0);
      const int c1 = class_of(j0 + j, m, tb.St1, tb.Sb1);
      const int cls = c0 + c1 * tb.rows0;
      const int e_ = toff[cls + 1], p0 = (j + H) * LXC + (i + H);
      auto at = [&](int w) { return p0 + (w >> 16) * LXC + (int)(short)w; };
      int k = toff[cls];
      T a = T(0);
      for (; k + 4 <= e_; k += 4) {
        int e[4];
        T v[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          e[q] = te[k + q];
          v[q] = gv[k + q];
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) a = fma(v[q], Xs[at(e[q])], a);
      }
      for (; k < e_; ++k) a = fma(gv[k], Xs[at(te[k])], a);
      epi(i, j, a);
    }
  }
}

// Apply `body(o, vals)` to the thread's pixels o = tid, tid + NT, ...
// of a tile with N pixels, U pixels at a time: `ld(o, vals)` first issues
// every load of the group (into registers), then `body` consumes them.
template <int U, int NV, typename T, int NT = NTHREADS, class LD, class BODY>
__device__ __forceinline__ void batched_pixels(int N, LD ld, BODY body) {
#pragma unroll 1
  for (int base = threadIdx.x; base < N; base += NT * U) {
    T vals[U][NV];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int o = base + u * NT;
      if (o < N) ld(o, vals[u]);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int o = base + u * NT;
      if (o < N) body(o, vals[u]);
    }
  }
}

// Tile geometry of a job: tile (ti, tj) covers rows [i0, i0+TI), cols [j0, j0+TJ).
template <typename T>
__device__ __forceinline__ void tile_geom(int m, int ti, int tj, int& i0, int& j0, int& TI,
                                          int& TJ) {
  TI = TJ = tile_edge(m);
  i0 = ti * TI;
  j0 = tj * TJ;
}

}  // namespace dbl
