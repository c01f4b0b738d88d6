// Host-side launch interface of the device kernels.
#pragma once
#include <hip/hip_runtime.h>
#include "common.h"

namespace dbl {

struct LaunchArgs {
  const Job* jobs;       // device array of jobs
  const uint32_t* tiles; // device tile table
  int ntiles;            // blocks in the launch
  int m_max;             // largest grid among the jobs (sizes LDS)
  hipStream_t stream;
  // every job has m >= 32 and the 32 x 32 tile kernels are enabled: the CGLS
  // phases take k_cgls_p1_sep / k_cgls_p2_sep (separable operators) or
  // k_cgls_p1_gen / k_cgls_p2_gen (general ones)
  bool tile32 = false;
  // CGLS phases: 1 / 0 forces the register-bounded / unbounded variant; -1
  // takes the bounded one for launches of more than cgls_wide_tiles() tiles
  int wide = -1;
  // CGLS phases: the jobs' tables are padded to their own radius buckets,
  // which differ, up to the bucket the launch names (kernels_cgls_multi.hip;
  // implies the 32 x 32 tile kernels)
  bool multi = false;
};
int cgls_wide_tiles();

// Vector slots of CGLS / solver jobs (Job::v indices).
enum VSlot : int {
  V_X = 0,   // CGLS iterate
  V_PA,      // search direction, read buffer
  V_PB,      // search direction, write buffer
  V_S,       // A^ T r
  V_R1A, V_R1B,  // image-space residual, read / write buffers
  V_Q1,      // A p
  V_R2A, V_R2B,  // gradient-space residual, read / write buffers
  V_Q2,      // sqrt(gamma) D p
  V_W,       // IRLS weights (n_L)
  V_B,       // right-hand side b (n)
  V_C1, V_C2,// shift c = C1 - C2 (SB: d - g), c = C1 (MM)
  V_XOLD,    // previous outer iterate (CGLS start: A x0)
  V_X0,      // optional CGLS start
  // statistics finish jobs: optional FP64 destination of the step's RC
  V_RCOUT = V_X0
};

hipError_t launch_apply_A(const LaunchArgs& la, int precision, int sep, int rb, int H);
// Streaming separable blur for large FP32 grids: eligibility, its strip grid
// (tiles per axis of a job: row strips x column blocks) and the launch.
bool apply_stream_ok(int m, int precision, int sep, int rows1);
void apply_stream_grid(int m, int* nti, int* ntj);
hipError_t launch_apply_stream(const LaunchArgs& la, int rb);
hipError_t launch_grad(const LaunchArgs& la, int precision);
hipError_t launch_gradT(const LaunchArgs& la, int precision);
hipError_t launch_dwt_fwd(const LaunchArgs& la, int precision);
hipError_t launch_dwt_inv(const LaunchArgs& la, int precision);
hipError_t launch_dtransfer(const LaunchArgs& la, int precision);

// CGLS phases (kernels_solve.hip)
hipError_t launch_cgls_init(const LaunchArgs& la, int precision);
hipError_t launch_cgls_p1(const LaunchArgs& la, int precision, int sep, int rb, int H);
hipError_t launch_cgls_p2(const LaunchArgs& la, int precision, int sep, int rb, int H);
// CGLS phases for separable operators on 32 x 32 tiles (kernels_cgls_sep.hip);
// `wide` selects the register-bounded variant for launches that fill the chip.
hipError_t launch_cgls_p1_sep(const LaunchArgs& la, int precision, int rb, bool wide);
hipError_t launch_cgls_p2_sep(const LaunchArgs& la, int precision, int rb, bool wide);
size_t cgls_sep_lds(int phase, int precision, int rb);
// The same for general operators of radius <= rb (kernels_cgls_gen.hip).
hipError_t launch_cgls_p1_gen(const LaunchArgs& la, int precision, int rb);
hipError_t launch_cgls_p2_gen(const LaunchArgs& la, int precision, int rb);
size_t cgls_gen_lds(int phase, int precision, int rb);
// CGLS phase `phase` (1 or 2) over jobs of several radius buckets up to rbmax
// (kernels_cgls_multi.hip, register-bounded kernels only: a mixed launch
// gathers enough tiles to fill the chip); cgls_multi_bucket(rbmax): a launch
// can cover them.
hipError_t launch_cgls_multi(const LaunchArgs& la, int phase, int precision, int rbmax);
bool cgls_multi_bucket(int rbmax);
hipError_t launch_aux(const LaunchArgs& la, int precision);
hipError_t launch_stats(const LaunchArgs& la, int precision, int sep, int rb, int H);
hipError_t launch_fill(const LaunchArgs& la, int precision);
hipError_t launch_stats_fin(const LaunchArgs& la);
hipError_t launch_cgls_hist(const LaunchArgs& la);
hipError_t launch_set_gamma(const LaunchArgs& la);
// LSQR phases (kernels_lsqr.hip)
hipError_t launch_lsqr_init(const LaunchArgs& la, int precision);
hipError_t launch_lsqr_a(const LaunchArgs& la, int precision, int sep, int rb, int H);
hipError_t launch_lsqr_b(const LaunchArgs& la, int precision, int sep, int rb, int H);
hipError_t launch_lsqr_fin(const LaunchArgs& la, int precision);
// One-block CGLS (kernels_small.hip): one block per job, all iterations.
// Every job of a launch has m x m grids, m in {8, 16, 32, 64}, and operators
// of one kind: separable with tables padded to bucket rb, or (gen) general
// with radius <= rb (rb then only sets the halo).
size_t small_cgls_lds(int m, int precision, int rb, int tab_rows, bool irls, size_t limit,
                      int* wlds, bool gen = false);
hipError_t launch_cgls_small(const LaunchArgs& la, int precision, int rb, int m, size_t lds,
                             bool gen);

// aux modes (Job::i0)
enum AuxMode : int {
  AUX_IRLS_W = 0,   // v[V_W] = max(|Lx|, eps)^(-1/2)      from v[V_X]
  AUX_MM_W = 1,     // v[V_C1] = u (1 - (eps^2/(u^2+eps^2))^(1/2)), u = L x
  AUX_SB_INIT = 2,  // d = shrink(Lx, tau), g = Lx - d      (v[V_C1] = d, v[V_C2] = g)
  AUX_SB_UPDATE = 3 // d = shrink(Lx + g, tau), g += Lx - d
};

// GCV (kernels_gcv.hip)
hipError_t launch_gcv_prep(const LaunchArgs& la, int precision);
hipError_t launch_gcv_complete(const LaunchArgs& la);
hipError_t launch_gemm64(const LaunchArgs& la);
hipError_t launch_gcv_symbol(const LaunchArgs& la);
hipError_t launch_gcv_data(const LaunchArgs& la);
hipError_t launch_gcv_grid(const LaunchArgs& la, int ngroups);
hipError_t launch_gcv_brent(const LaunchArgs& la);
hipError_t launch_gcv_gridfin(const LaunchArgs& la);
// levels of at most 64 x 64: grid and all Brent steps in one block per job
hipError_t launch_gcv_solo(const LaunchArgs& la);
// EXACT tier: n x n identity; M += D^T D (D = diag(w) L, w of `precision`, or L)
hipError_t launch_gcv_eye(double* I, int n, hipStream_t stream);
hipError_t launch_gcv_add_dtd(double* M, const void* w, int precision, int m,
                              hipStream_t stream);

}  // namespace dbl
