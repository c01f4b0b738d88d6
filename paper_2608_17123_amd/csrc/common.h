// Shared host/device definitions of the deblurring library (gfx950).
//
// Device data model
// -----------------
// * Every kernel launch covers a list of jobs (one job = one image at one
//   level) cut into square output tiles (tile_edge(m) pixels a side; the
//   FP64 DCT products use 64 x 64).  Block b of a launch handles tile
//   table entry b: job index in the upper 16 bits, tile index within the job in
//   the lower 16 bits.  A single solve is a launch with one job; a batch or a
//   server step is the same launch with many jobs.
// * Each job owns an FP64 scalar block (gamma, GCV state, histories) and
//   partial-sum arrays indexed by tile.  Reductions never synchronise blocks
//   inside a launch: a producer launch stores one FP64 partial per tile, and
//   the consumer launch that needs the total has every block sum the job's
//   partials in the same fixed order (no atomics, no fences).  Every block
//   therefore sees bit-identical scalars, and a job's results do not depend
//   on which other jobs share the launch.
// * Coarse operators are stored as "class tables": along one axis, rows near
//   the periodic wavelet seam (top St rows, bottom Sb rows) have their own tap
//   rows, every other row uses the interior Toeplitz row; taps are indexed by
//   circular offset e in [-R, R] and applied with periodic indexing.  The
//   finest level (zero boundary) is the same structure with truncated rows.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dbl {

constexpr int NTHREADS = 256;
// Edge of the output tiles of the image and gradient kernels on an m x m
// grid: the whole grid below 32, else 32.  (16 x 16 tiles on grids of 64 and
// 128 quadruple the blocks but measured slower in batched launches: 4x halo
// reads per output against 2.25x, and idle threads in the convolution
// passes.)  Non-decreasing in m, so the largest grid of a launch sizes its LDS.
__host__ __device__ constexpr int tile_edge(int m) { return m < 32 ? m : 32; }
// XCDs of the device: the dispatcher hands workgroup ids to them round-robin.
constexpr int XCDS = 8;
constexpr int MAX_R = 16;
constexpr int NSCAL = 512;  // doubles per job scalar block

// Scalar block layout (FP64, device).
enum Scal : int {
  S_GAMMA = 0, S_SQRTG, S_GS, S_ALPHA, S_BETA, S_QQ, S_RR, S_GS0,
  S_RCNUM, S_RCDEN, S_RES2, S_PEN, S_EPS, S_TAU, S_WSQ, S_ITER,
  S_LQ = 16,     // LSQR rotation state (rhobar, phibar), two copies by parity
  // GCV state
  S_G_TLO = 32, S_G_THI, S_G_A, S_G_B, S_G_X, S_G_W, S_G_V, S_G_FX, S_G_FW,
  S_G_FV, S_G_D, S_G_E, S_G_U, S_G_DONE, S_G_NEV, S_G_XTOL, S_G_IT, S_G_RMIN,
  S_G_RMAX, S_G_NPTS, S_G_WBAR, S_G_RES, S_G_TR, S_G_FBEST, S_G_BB,
  S_GRID = 64,   // up to 64 grid values
  S_HIST = 128,  // CGLS residual history (up to 128 iterations)
  S_BR = 256     // Brent state, two copies of BR_SIZE (read one, write the other)
};
constexpr int HIST_MAX = 128;

// Brent state layout (offsets inside one copy)
enum Brent : int {
  BR_A = 0, BR_B, BR_X, BR_W, BR_V, BR_FX, BR_FW, BR_FV, BR_D, BR_E, BR_U, BR_IT, BR_PHASE,
  BR_DONE, BR_SIZE = 16
};

struct Table1D {
  int R;            // radius (taps per row = 2R + 1)
  int St, Sb;       // seam rows at top / bottom
  int rows;         // St + 1 + Sb
  const float* tf;  // rows * (2R+1), row-major
  const double* td;
};

struct Table2D {
  int R0, R1;
  int St0, Sb0, St1, Sb1;
  int rows0, rows1;
  const int* off;     // rows0 * rows1 + 1 offsets into taps
  const short2* e;    // (e0, e1) per tap
  const float* vf;
  const double* vd;
};

struct LevelOp {
  int m;
  int sep;   // 1: separable (two 1-D passes), 0: general 2-D tap lists
  int rb;    // radius bucket used by the separable kernels (tables padded to rb)
  int R;     // halo radius (max over both axes)
  Table1D f0, f1, a0, a1;  // forward / adjoint tables, axis 0 (rows) and 1 (cols)
  Table2D f2, a2;
};

// One-block CGLS for small levels (kernels_small.hip): a block of
// small_nt(m, esz) threads keeps a whole level in LDS for all iterations.
// Byte layout of its dynamic LDS, shared by the host (launch size,
// eligibility) and the kernel:
//   XP, XR : p and r1 with a periodic halo of H, (m+2H) x (m+2H+1) each
//   Z      : pass-A scratch (m+2H) x (m+1) (separable operator), or the
//            staged interior taps (general operator)
//   S, Q1  : n each (s, then q1 = A p or the gradient part of s)
//   R2     : n_L (gradient-space residual)
//   W      : n_L IRLS weights, when they fit (else read from global memory)
//   TB     : the level's four 1-D tap tables (tab_elems values; none for a
//            general operator, whose class lists are read from its tables)
constexpr int SMALL_MAX_M = 64;
// threads of the one-block CGLS for an m x m level with esz-byte elements:
// one pixel per thread up to m = 16, then 512 threads (at 1024 the kernel's
// registers would spill)
__host__ __device__ constexpr int small_nt(int m, int esz) {
  return (m >= 32 || esz == 0) ? 512 : m * m;
}
struct SmallLds {
  int E, ld;
  size_t halo, z, s, q1, r2, w, tb, total;  // byte offsets of the regions and the total
};
__host__ __device__ inline size_t align16(size_t b) { return (b + 15) & ~size_t(15); }
// gen: a general (2-D tap list) operator: no pass-A scratch; Z holds the
// interior class's taps of the forward and the adjoint table, staged as
// (tile offset, value) pairs, at most (2H + 1)^2 each (small_gen_taps).
__host__ __device__ constexpr int small_gen_taps(int H) { return (2 * H + 1) * (2 * H + 1); }
__host__ __device__ inline SmallLds small_lds(int m, int H, int esz, bool wlds, int tab_elems,
                                              bool gen = false) {
  SmallLds L;
  L.E = m + 2 * H;
  L.ld = L.E + 1;
  L.halo = align16((size_t)L.E * L.ld * esz);
  L.z = 2 * L.halo;
  L.s = L.z + (gen ? align16((size_t)2 * small_gen_taps(H) * (4 + esz))
                   : align16((size_t)L.E * (m + 1) * esz));
  L.q1 = L.s + align16((size_t)m * m * esz);
  L.r2 = L.q1 + align16((size_t)m * m * esz);
  L.w = L.r2 + align16((size_t)2 * m * (m - 1) * esz);
  L.tb = L.w + (wlds ? align16((size_t)2 * m * (m - 1) * esz) : 0);
  L.total = L.tb + align16((size_t)tab_elems * esz);
  return L;
}

__host__ __device__ inline int class_of(int i, int m, int St, int Sb) {
  if (i < St) return i;
  if (i >= m - Sb) return St + 1 + (i - (m - Sb));
  return St;
}

struct Job {
  int m;
  int nti, ntj;     // tiles along axis 0 and axis 1
  int flags;        // kernel specific
  const LevelOp* op;
  void* v[16];      // vectors (meaning set by each kernel)
  double* scal;     // FP64 scalar block
  double* part;     // FP64 partials, >= 4 per tile
  double p0, p1;    // extra scalars passed by value
  int i0, i1;       // extra integers passed by value
  double* hist;     // per-solve history (gamma, rc, objective) for stats kernels
  double* pw;       // partials written by this launch: pw[tile * K + k]
  const double* pr[3];  // partials of earlier launches summed by this launch
};

// Job flags
enum : int {
  F_IRLS = 1,       // D = diag(w) L
  F_SHIFT = 2,      // c != 0 (MM, SB)
  F_SB = 4,
  F_MM = 8,
  F_ADJ = 16,       // transpose
  F_HIST = 32,      // record CGLS residual history
  F_FIRST = 64,     // first phase after init (alpha = 0)
  F_WLDS = 128,     // one-block CGLS: IRLS weights staged in LDS
  F_EXACT = 256,    // GCV job on exact pencil data (nu, f, g, ||b||^2)
};

__device__ __forceinline__ void decode_tile(const Job* __restrict__ jobs,
                                            const uint32_t* __restrict__ tiles,
                                            const Job*& job, int& ti, int& tj, int& tix) {
  uint32_t t = tiles[blockIdx.x];
  job = jobs + (t >> 16);
  tix = int(t & 0xffffu);
  ti = tix % job->nti;
  tj = tix / job->nti;
}

// A pointer the kernel may only use for device (global) memory: every vector
// a job names is a device allocation (the library's or the caller's), whose
// generic address is its global address.  Loads through it are global loads,
// which count in vmcnt alone (a generic load also counts in lgkmcnt, so every
// later wait for LDS would wait for it too).
template <typename T> using GlobalPtr = __attribute__((address_space(1))) T*;
template <typename T> __device__ __forceinline__ GlobalPtr<T> gview(T* p) {
  return (GlobalPtr<T>)p;
}

// ------------------------------------------------------------ storage --
// Storage types of the CGLS state vectors.  With DBL_BF16 the vectors p, s,
// r1, r2, q1, q2 are stored as bfloat16 (round to nearest even from FP32)
// and every operation on them runs in FP32; otherwise storage = compute type.
struct bf16s {
  uint16_t u;
};

__device__ __forceinline__ float bf16_to_f32(bf16s v) {
  return __uint_as_float((uint32_t)v.u << 16);
}
__device__ __forceinline__ bf16s f32_to_bf16(float f) {
  const uint32_t b = __float_as_uint(f);
  bf16s r;
  if ((b & 0x7f800000u) == 0x7f800000u && (b & 0x007fffffu))
    r.u = (uint16_t)((b >> 16) | 0x40u);  // NaN stays a (quiet) NaN
  else
    r.u = (uint16_t)((b + 0x7fffu + ((b >> 16) & 1u)) >> 16);
  return r;
}

// load element i of a storage-S vector as compute type T
template <typename T, typename S>
__device__ __forceinline__ T ldv(const S* p, size_t i) {
  if constexpr (sizeof(S) == 2) return (T)bf16_to_f32(p[i]);
  else return (T)p[i];
}
// value of v after a round trip through storage S
template <typename S, typename T>
__device__ __forceinline__ T rtv(T v) {
  if constexpr (sizeof(S) == 2) return (T)bf16_to_f32(f32_to_bf16((float)v));
  else return v;
}
// store v (already representable in S when it came from rtv) at element i
template <typename S, typename T>
__device__ __forceinline__ void stv(S* p, size_t i, T v) {
  if constexpr (sizeof(S) == 2) p[i] = f32_to_bf16((float)v);
  else p[i] = (S)v;
}

// ---------------------------------------------------------------- reduce --

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Sum over the block (NT threads), result valid in thread 0.  `red` must
// hold NT/64 doubles per value.  Order is fixed.
template <int K, int NT = NTHREADS>
__device__ __forceinline__ void block_sum(double (&v)[K], double* red) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] = wave_sum(v[k]);
  __syncthreads();
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < K; ++k) red[k * (NT / 64) + wid] = v[k];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < K; ++k) {
      double s = 0.0;
      for (int w = 0; w < NT / 64; ++w) s += red[k * (NT / 64) + w];
      v[k] = s;
    }
  }
}

// Block sum with the totals returned in every thread: every thread adds the
// per-wave sums in the same fixed order, so all of them hold the same bits.
// `red` holds K * NT/64 doubles.
template <int K, int NT = NTHREADS>
__device__ __forceinline__ void block_allsum(double (&v)[K], double* red) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] = wave_sum(v[k]);
  __syncthreads();  // earlier readers of red are done
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < K; ++k) red[k * (NT / 64) + wid] = v[k];
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < K; ++k) {
    double s = 0.0;
    for (int w = 0; w < NT / 64; ++w) s += red[k * (NT / 64) + w];
    v[k] = s;
  }
}

// Store this block's K partial sums at p[tix * K + k] (fixed-order block sum).
template <int K>
__device__ __forceinline__ void put_partials(double* p, int tix, double (&v)[K], double* red) {
  block_sum<K>(v, red);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < K; ++k) p[tix * K + k] = v[k];
  }
}

// Sum component `comp` of K-component partials over the nt tiles of a job in
// a fixed order (thread t takes tiles t, t + NTHREADS, ...; then the block
// tree); the total is returned in every thread.  `red` holds 4 doubles.
template <int K>
__device__ __forceinline__ double sum_partials(const double* p, int nt, int comp, double* red,
                                               double* bcast) {
  double a = 0.0;
  for (int t = threadIdx.x; t < nt; t += NTHREADS) a += p[t * K + comp];
  double v[1] = {a};
  block_sum<1>(v, red);
  if (threadIdx.x == 0) *bcast = v[0];
  __syncthreads();
  const double r = *bcast;
  __syncthreads();
  return r;
}

// Two partial sums at once (components c0 of K0-component partials p0 and c1
// of K1-component partials p1, nt tiles each), with one block reduction; each
// total is bitwise what sum_partials returns for it.  bcast holds 2 doubles.
template <int K0, int K1>
__device__ __forceinline__ void sum_partials2(const double* p0, int c0, const double* p1, int c1,
                                              int nt, double* red, double* bcast, double& s0,
                                              double& s1) {
  double v[2] = {0.0, 0.0};
  for (int t = threadIdx.x; t < nt; t += NTHREADS) {
    v[0] += p0[t * K0 + c0];
    v[1] += p1[t * K1 + c1];
  }
  block_sum<2>(v, red);
  if (threadIdx.x == 0) {
    bcast[0] = v[0];
    bcast[1] = v[1];
  }
  __syncthreads();
  s0 = bcast[0];
  s1 = bcast[1];
  __syncthreads();
}

// Workgroup barrier that orders LDS accesses only.  A thread's global loads
// stay in flight across it (__syncthreads also waits for them), so a kernel
// that keeps loads queued ahead in registers uses this where its threads
// exchange data through LDS alone.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Publish a scalar written by the finalising thread so later kernels and
// other XCDs read it from memory.
__device__ __forceinline__ void put_scal(double* s, int k, double v) {
  __hip_atomic_store(s + k, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

}  // namespace dbl
