// Helpers shared by the fused Krylov phase kernels (CGLS in kernels_solve.hip,
// LSQR in kernels_lsqr.hip): the LDS input tile of the stencils, the tile
// convolution with its between-pass hook, the occupancy target and the
// launch dispatch over radius buckets.
#pragma once
#include "launch.h"
#include "stencil.h"

namespace dbl {

template <bool SEP>
__device__ __forceinline__ int xs_at(int i, int j, int H, int TI, int TJ) {
  return SEP ? (i + H) * sep_lx(TJ, H) + (j + H) : (j + H) * col_lx(TI, H) + (i + H);
}

template <bool SEP>
__device__ __forceinline__ int xs_ld(int H, int TI, int TJ) {
  return SEP ? sep_lx(TJ, H) : col_lx(TI, H);
}

template <bool SEP>
__device__ __forceinline__ int xs_elems(int H, int TI, int TJ) {
  return SEP ? (TI + 2 * H) * sep_lx(TJ, H) : col_lds_elems(TI, TJ, H);
}

// Tile convolution.  `hook` runs once all threads are done reading the input
// tile Xs (separable: between the two passes; general: after an extra sync,
// which requires a copy of the input -- the general path instead runs the
// hook before the convolution, so it must not overwrite Xs there).
template <typename T, int RB, bool SEP, class Epi, class Hook = NoHook,
          int V = TileCfg<T>::V>
__device__ __forceinline__ void conv_tile(const T* Xs, int H, void* scratch, const LevelOp& op,
                                          bool adj, int i0, int j0, int TI, int TJ, int m,
                                          Epi epi, Hook hook = Hook()) {
  if constexpr (SEP) {
    sep_tile<T, RB, NTHREADS, V>(Xs, H, static_cast<T*>(scratch), adj ? op.a0 : op.f0,
                                 adj ? op.a1 : op.f1, i0, j0, TI, TJ, m, epi, hook);
  } else {
    T* s_v = static_cast<T*>(scratch);
    short2* s_e = reinterpret_cast<short2*>(s_v + (2 * H + 1) * (2 * H + 1));
    gen_tile<T>(Xs, H, adj ? op.a2 : op.f2, s_e, s_v, i0, j0, TI, TJ, m, epi);
  }
}

// Minimum waves per SIMD the CGLS phase kernels are compiled for (one wave
// per SIMD per 256-thread block).  Phase 1: 3 (FP32) or 2 (FP64); a tighter
// bound costs it latency where launches are small.  Phase 2: 6 for FP32 up
// to radius bucket 8 (77 VGPRs with its 4-output convolution window, no
// spills), so the 1536 tiles of a 24-image 256 x 256 launch are resident in
// one round; else as phase 1.
template <typename T, int RB>
constexpr int waves_per_simd() {
  return sizeof(T) == 4 ? 3 : 2;
}
template <typename T, int RB>
constexpr int p2_waves() {
  return sizeof(T) == 4 ? (RB <= 8 ? 6 : 3) : 2;
}

template <typename T> __device__ __forceinline__ T* vp(const Job* j, int k) {
  return static_cast<T*>(j->v[k]);
}

}  // namespace dbl

// Same, for kernels that also take the storage type S of the state vectors.
#define DISPATCH_STENCIL_S(KERNEL, T, S, la, sep, rb, H)                           \
  do {                                                                                 \
    const int ts_ = tile_edge((la).m_max);                                             \
    if (sep) {                                                                         \
      const size_t lds_ = sizeof(T) * sep_lds_elems(ts_, ts_, rb);                     \
      switch (rb) {                                                                    \
        case 2: hipLaunchKernelGGL((KERNEL<T, S, 2, true>), dim3((la).ntiles),           \
                    dim3(NTHREADS), lds_, (la).stream, (la).jobs, (la).tiles); break;  \
        case 4: hipLaunchKernelGGL((KERNEL<T, S, 4, true>), dim3((la).ntiles),           \
                    dim3(NTHREADS), lds_, (la).stream, (la).jobs, (la).tiles); break;  \
        case 8: hipLaunchKernelGGL((KERNEL<T, S, 8, true>), dim3((la).ntiles),           \
                    dim3(NTHREADS), lds_, (la).stream, (la).jobs, (la).tiles); break;  \
        case 12: hipLaunchKernelGGL((KERNEL<T, S, 12, true>), dim3((la).ntiles),         \
                    dim3(NTHREADS), lds_, (la).stream, (la).jobs, (la).tiles); break;  \
        case 16: hipLaunchKernelGGL((KERNEL<T, S, 16, true>), dim3((la).ntiles),         \
                    dim3(NTHREADS), lds_, (la).stream, (la).jobs, (la).tiles); break;  \
        default: return hipErrorInvalidValue;                                          \
      }                                                                                \
    } else {                                                                           \
      const size_t lds_ = sizeof(T) * col_lds_elems(ts_, ts_, H) +                     \
                          (2 * sizeof(T) + sizeof(short2)) * (2 * (H) + 1) * (2 * (H) + 1) + \
                          sizeof(T) * ts_ * ts_;                                      \
      hipLaunchKernelGGL((KERNEL<T, S, 0, false>), dim3((la).ntiles), dim3(NTHREADS),    \
                         lds_, (la).stream, (la).jobs, (la).tiles);                    \
    }                                                                                  \
  } while (0)

