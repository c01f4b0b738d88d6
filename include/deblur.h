/*
 * deblur.h -- C ABI of the MI355X (gfx950) wavelet multilevel l1 deblurring
 * library.
 *
 * The library solves, for an m x m image (m a power of two),
 *
 *     min_x ||A x - b||_2^2 + mu ||L x||_1                  (paper eq. (l1b))
 *
 * with A a zero-boundary blur and L the discrete gradient, by a wavelet
 * V-cycle (Alg. 4) whose levels run IRLS (Alg. 1), MM (Alg. 2) or Split
 * Bregman (Alg. 3).  Each outer iteration solves the l2 subproblem of eq.
 * (generic_sub) by CGLS on the augmented system of eq. (augmented), with the
 * parameter chosen by GCV (eqs. (xgamma), (GCV)).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Images: device pointers to m x m arrays stored column-major (x = vec(X),
 *   Sec. 4.1 and Sec. 5), contiguous, element type given by the precision
 *   (DBL_F32: float, DBL_F64: double).
 * Gradient-space vectors (length n_L = 2 m (m-1)): [vec(D X); vec(X D^T)],
 *   i.e. the (m-1) x m block of row differences followed by the m x (m-1)
 *   block of column differences, both column-major (Sec. 4.2).
 * Kernels (PSFs): host float64 arrays of odd shape ph x pw, column-major,
 *   centred: entry (a + ph/2) + (b + pw/2) * ph weighs offset (a, b), a along
 *   the row index.  (A X)[i,j] = sum_{a,b} P[a,b] X[i-a, j-b], X = 0 outside.
 * Ownership: the caller owns every buffer it passes; the library keeps no
 *   pointer to them after a call returns.  The library owns dbl_ctx, dbl_op
 *   and dbl_server objects and their device workspaces.
 * Streams: all device work of a context is issued on the stream given to
 *   dbl_create (NULL = the null stream).  Entry points that return results
 *   to host memory (reports, gamma) synchronise that stream; the others are
 *   asynchronous with respect to the host -- call dbl_sync before reading.
 * Errors: every function returns 0 (DBL_OK) or a negative dbl_status.
 *   Argument validation happens before any device work is issued, so a
 *   rejected call has no side effects.  dbl_last_error(ctx) describes the
 *   last failure on that context.
 * Threads: a context must not be used by two host threads at once.
 */
#ifndef DEBLUR_H
#define DEBLUR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DBL_MAX_LEVELS 8
#define DBL_MAX_KOUT 64
#define DBL_MAX_PSF_RADIUS 16   /* largest supported kernel half-width   */
#define DBL_GCV_GRID_MAX 64

typedef enum {
  DBL_OK = 0,
  DBL_EINVAL = -1,    /* bad argument (null pointer, size, enum, range)     */
  DBL_ENOMEM = -2,    /* workspace budget or device allocation exhausted    */
  DBL_EDEVICE = -3,   /* HIP runtime error                                  */
  DBL_ENOTSUP = -4,   /* valid request this build does not support          */
  DBL_ENUMERIC = -5,  /* NaN or Inf detected in a result                    */
  DBL_ENOTFOUND = -6  /* unknown server ticket                              */
} dbl_status;

typedef enum { DBL_IRLS = 0, DBL_MM = 1, DBL_SB = 2 } dbl_solver;
/* Low-pass filters of Sec. 4: the two-tap Haar filter and the four-tap
 * Daubechies filter (1+sqrt3, 3+sqrt3, 3-sqrt3, 1-sqrt3) / (4 sqrt2). */
typedef enum { DBL_HAAR = 0, DBL_DB4 = 1 } dbl_wavelet;
/* Information transfer of Sec. 4.1: X = coarse solution, D = auxiliaries.
 * With levels == 1 the transfer is unused (Approach I). */
typedef enum { DBL_XFER_X = 0, DBL_XFER_D = 1 } dbl_transfer;
/* Element types.  DBL_F32 / DBL_F64: every device vector in float / double.
 * DBL_BF16: every vector a caller passes (b, x, weights, shifts, operator
 * inputs and outputs) is float; inside CGLS the state vectors p, s, r1, r2,
 * q1, q2 are stored as bfloat16 (rounded to nearest even from FP32) and
 * every operation on them is FP32, with FP64 scalars (alpha, beta, norms);
 * each outer iteration restarts CGLS from the FP32 data (r1 = b) and its
 * residual and objective are recomputed in FP32 from x.  Levels that run
 * the one-block CGLS keep their state in LDS in FP32. */
typedef enum { DBL_F32 = 0, DBL_F64 = 1, DBL_BF16 = 2 } dbl_precision;
typedef enum { DBL_INNER_CGLS = 0, DBL_INNER_LSQR = 1 } dbl_inner;
/* GCV tiers: SPECTRAL evaluates the GCV function of eq. (GCV) on the DCT
 * surrogate (reflexive-boundary blur, exact Neumann gradient); EXACT uses the
 * generalised eigendecomposition of the pair {A, D} (the paper's GSVD route,
 * Sec. 3): the dense level operator is formed on the device, A^T A v =
 * nu (A^T A + D^T D) v is solved in FP64 (rocSOLVER sygvd), and the GCV
 * function is evaluated from (nu, V^T A^T b, V^T D^T c, ||b||^2).  EXACT is
 * limited to n <= DBL_GCV_EXACT_MAX_N (a 128 x 128 level; DBL_ENOTSUP above)
 * and needs about 3 n^2 doubles of workspace (384 MB at n = 4096, 6.4 GB at
 * n = 16384) besides the eigensolver's own; AUTO picks EXACT when
 * n <= DBL_GCV_AUTO_EXACT_N. */
#define DBL_GCV_EXACT_MAX_N 16384
#define DBL_GCV_AUTO_EXACT_N 4096
typedef enum { DBL_GCV_AUTO = 0, DBL_GCV_EXACT = 1, DBL_GCV_SPECTRAL = 2 } dbl_gcv_mode;

typedef struct dbl_ctx dbl_ctx;
typedef struct dbl_op dbl_op;
typedef struct dbl_server dbl_server;

/* Solver options.  dbl_opts_default() fills the paper's values: eps = 0.03,
 * tau = 0.005 (Sec. 5), 50 GCV grid points (Sec. 3), 10 outer x 30 CGLS
 * iterations, GCV on, AUTO tier, FP32. */
typedef struct dbl_opts {
  double eps;            /* IRLS / MM stabilisation (Algs. 1, 2)              */
  double tau;            /* SB shrink threshold (Alg. 3)                      */
  int k_out;             /* outer iterations per level, 1..DBL_MAX_KOUT      */
  int k_in;              /* CGLS iterations per subproblem, >= 1              */
  double mu_fixed;       /* > 0: use this parameter everywhere (no GCV)       */
  const double* mu_schedule; /* optional host array levels*k_out, finest level
                                first; overrides mu_fixed and GCV             */
  int gcv_mode;          /* dbl_gcv_mode                                      */
  int gcv_grid;          /* grid points, 3..DBL_GCV_GRID_MAX                  */
  int precision;         /* dbl_precision for vectors on the device           */
  void* x_hist;          /* optional device array of k_out * m * m elements of
                            x's type, owned by the caller and kept valid until
                            the solve completes: slice k receives the finest
                            level's iterate after outer iteration k, so that
                            convergence curves (RRE per iteration, Sec. 5) can
                            be drawn from one solve.  NULL: no history.
                            Slices past an early stop are left untouched.    */
  double tol_fine;       /* RC tolerance of eq. (stop) on the finest grid (and
                            the single grid of Approach I): the grid stops
                            after the first outer iteration with
                            ||x_k+1 - x_k|| / ||x_k|| < tol, else after k_out.
                            Sec. 5 uses 1e-3.  0: always run k_out.         */
  double tol_coarse;     /* the same on every coarser grid; Sec. 5: 1e-6     */
  int inner_solver;      /* dbl_inner: the Krylov solver of every subproblem,
                            k_in iterations from x = 0.  CGLS (default) and
                            LSQR (the paper's, Sec. 3) give the same iterates
                            in exact arithmetic; LSQR always runs the tiled
                            phase kernels.                                   */
} dbl_opts;

/* Per-solve report.  Level 0 is the finest grid.  Arrays are filled for
 * levels < levels and k < k_out.  rc[l][0] is NaN when the level starts
 * from x = 0 (Approaches I and D). */
typedef struct dbl_report {
  int levels;
  int k_out;
  int sizes[DBL_MAX_LEVELS];
  double gamma[DBL_MAX_LEVELS][DBL_MAX_KOUT];     /* mu (IRLS, MM) or lambda (SB) */
  double rc[DBL_MAX_LEVELS][DBL_MAX_KOUT];        /* eq. (stop)                    */
  double objective[DBL_MAX_LEVELS][DBL_MAX_KOUT]; /* solver objective, FP64        */
  double seconds;        /* device time of the solve (plain path), or latency */
  int status;            /* dbl_status of this solve                          */
  int iters[DBL_MAX_LEVELS]; /* outer iterations run per level (k_out unless a
                                tolerance stopped the level earlier); entries
                                past iters[l] are NaN                        */
} dbl_report;

/* A deblurring request for the batched and serving entry points.  b and x
 * are device pointers (m x m, element type per opts->precision); psf is a
 * host array that is copied during the call that takes the request. */
typedef struct dbl_request {
  const void* b;
  void* x;
  const double* psf;
  int ph, pw;
  int m;
  int solver, wavelet, levels, transfer;
  dbl_opts opts;
} dbl_request;

/* CGLS subproblem description (eq. (generic_sub)).  d_kind 0: D = L;
 * 1: D = diag(w) L.  w (n_L, device, same element type) is required for
 * d_kind 1; c (n_L, device) may be NULL for c = 0. */
typedef struct dbl_sub {
  int d_kind;
  const void* w;
  double gamma;
  const void* c;
} dbl_sub;

/* ---------------------------------------------------------------- context */

/* Create a context on HIP device `device`, issuing work on `hip_stream`
 * (a hipStream_t, or NULL for the null stream).  hbm_budget_bytes caps the
 * device workspace the context may allocate (0 = no cap).  device = -1
 * creates an argument-checking context with no device: every entry point
 * validates its arguments as usual and then returns DBL_EDEVICE. */
int dbl_create(dbl_ctx** out, int device, void* hip_stream, size_t hbm_budget_bytes);
int dbl_destroy(dbl_ctx* ctx);
/* Autotuner (for callers that want the fastest kernel variant per workload;
 * no paper passage: it never changes a result).  The CGLS phase launches of
 * separable operators have four compiled variants that form every sum in the
 * same order: the generic tile kernels and the 32 x 32 tile kernels, each
 * with and without a register bound.  dbl_autotune times all four on
 * synthetic jobs (zero data, on the context's stream) for every
 * (phase, radius bucket, grid size, launch size) of a sweep -- radius
 * buckets 2..16, grids 32..1024, 1 to 64 jobs per launch, at most 2^22
 * pixels per launch -- in `precision`, and keeps the fastest per key; every
 * later phase launch of that precision on `ctx` takes the entry nearest its
 * own key (same phase and bucket; grid size first, then tile count).
 * cache_path (optional): a JSON file of the results; when it exists, was
 * written on the same device kind for the same precision and flags lacks
 * DBL_TUNE_REMEASURE, it is loaded instead of measuring; otherwise the
 * measurement is written there.  DBL_TUNE_QUICK measures a reduced sweep
 * (buckets 4 and 8, grids 64 and 256, 1 and 16 jobs).  *n_entries
 * (optional) receives the number of entries installed.  DBL_EINVAL for an
 * unknown precision or flag, or an unwritable cache path; DBL_ENOMEM when
 * the synthetic jobs do not fit the context's budget.  Synchronises the
 * context's stream. */
#define DBL_TUNE_REMEASURE 1
#define DBL_TUNE_QUICK 2
int dbl_autotune(dbl_ctx* ctx, int precision, const char* cache_path, int flags,
                 int* n_entries);
/* The variant (0 generic, 1 generic register-bounded, 2 32 x 32 tile, 3 tile
 * register-bounded) a CGLS phase launch (phase 1 or 2) of `precision` with
 * radius bucket rb, largest grid m and ntiles tiles would take on ctx now.
 * DBL_EINVAL for a bad phase, size or null pointer. */
int dbl_tune_choice(const dbl_ctx* ctx, int phase, int precision, int rb, int m, int ntiles,
                    int* variant);
/* Context options (dbl_set_option). */
typedef enum dbl_option {
  /* 1 (default): a level with m <= 64 whose CGLS state fits in one block's
   * LDS runs all K_in iterations of a subproblem in one launch (one block per
   * subproblem); 0: every level uses the tiled two-phase launches.  Both
   * compute the CGLS recurrence of eq. (augmented) with the same element
   * arithmetic; the FP64 norm sums are ordered differently. */
  DBL_OPT_SMALL_CGLS = 1,
  /* 1 (default): dbl_apply_A / dbl_apply_A_batch on a separable FP32 level of
   * at least 512 x 512 run the streaming column kernel (a block marches
   * along the columns of a 512-row strip); 0: the tiled kernel.  Both form
   * the same sums in the same order, so results are identical. */
  DBL_OPT_STREAM_A = 2,
  /* 1 (default): the tiled CGLS phases of a level with a separable operator
   * and m >= 32 run the 32 x 32 tile kernels laid out for the wavefront; 0:
   * the generic tile kernels.  Both form every sum, including the per-tile
   * FP64 norm partials, in the same order. */
  DBL_OPT_TILE32 = 3,
  /* Mixed-bucket CGLS launches in batched solves (dbl_deblur_batch, the
   * server).  Jobs whose operators are padded to different radius buckets
   * normally launch apart, one launch per bucket; with this option the
   * levels of at least 32 x 32 on the tile kernels (DBL_OPT_TILE32) share
   * launches in which every job keeps its own bucket, so results are
   * identical (separable and general operators in launches of their own;
   * a general operator's bucket is the one above its radius).  Value < 0:
   * off.  Value >= 0 (default 3072): buckets up to 8 always share one
   * launch, and bucket 12 joins it in a CGLS stage where it has fewer tiles
   * (32 x 32 each) than the value. */
  DBL_OPT_MULTI_BUCKET = 4
} dbl_option;
/* Set a context option.  Returns DBL_EINVAL for an unknown option or value.
 * Takes effect for work issued afterwards. */
int dbl_set_option(dbl_ctx* ctx, int option, long long value);
/* Message describing the last error on ctx (never NULL). */
const char* dbl_last_error(const dbl_ctx* ctx);
/* Wait for all work issued by ctx. */
int dbl_sync(dbl_ctx* ctx);
/* Bytes of device workspace currently held by ctx. */
size_t dbl_workspace_bytes(const dbl_ctx* ctx);
void dbl_opts_default(dbl_opts* opts);

/* Per-kernel timing.  dbl_profile(ctx, 1) clears the counters and starts
 * bracketing every kernel launch of ctx with HIP events on its stream;
 * dbl_profile(ctx, 0) stops.  dbl_profile_read returns, for kernel family
 * `index` (0, 1, ...; DBL_ENOTFOUND past the last), its name, the number of
 * launches, their summed device time in milliseconds and the algorithmic
 * bytes they moved (each operand read or written once; 0 where not
 * counted).  Reading synchronises the stream. */
int dbl_profile(dbl_ctx* ctx, int enable);
int dbl_profile_read(dbl_ctx* ctx, int index, char* name, size_t name_cap, int64_t* launches,
                     double* ms, double* bytes);
/* Restrict the bracketing of dbl_profile to the launches of one kernel
 * family (`name` as dbl_profile_read reports it; NULL or "" = every
 * family), so that one family can be timed inside a run without events
 * around the others.  Takes effect for work issued afterwards. */
int dbl_profile_only(dbl_ctx* ctx, const char* name);

/* -------------------------------------------------------------- operators */

/* Build the level hierarchy A^(i+1) = W^T A^(i) W, b^(i+1) = W^T b^(i)
 * (Sec. 4, Alg. 4) for kernel psf on an m x m grid with `levels` grids.
 * The coarse operators are exact (Galerkin, periodic wavelet seam included)
 * and are stored as small per-level stencil tables.  Requires m a power of
 * two, odd ph, pw with half-widths <= DBL_MAX_PSF_RADIUS, and a coarsest
 * grid of at least 8 pixels per side. */
int dbl_op_create(dbl_ctx* ctx, const double* psf, int ph, int pw, int m, int levels,
                  int wavelet, int precision, dbl_op** out);
/* Release an operator.  Operators (and servers) must be destroyed before the
 * context they were made on; dbl_destroy releases their device memory. */
int dbl_op_destroy(dbl_op* op);

/* out = A^(level) in (transpose = 0) or A^(level)^T in (transpose = 1).
 * in and out are (m/2^level)^2 device arrays of the op's precision. */
int dbl_apply_A(dbl_ctx* ctx, const dbl_op* op, int level, int transpose,
                const void* in, void* out);

/* The same for `count` images at once (one launch; all share op and level):
 * in[q] and out[q] are device pointers, 0 <= count <= 65536.  in and out
 * are host arrays of count pointers, read during the call. */
int dbl_apply_A_batch(dbl_ctx* ctx, const dbl_op* op, int level, int transpose, int count,
                      const void* const* in, void* const* out);

/* Gradient L of Sec. 4.2 on an m x m grid: transpose = 0 maps n -> n_L,
 * transpose = 1 maps n_L -> n (the negative divergence). */
int dbl_apply_L(dbl_ctx* ctx, int m, int precision, int transpose, const void* in, void* out);
/* The same for `count` vectors in one launch (pointer arrays as for
 * dbl_apply_A_batch). */
int dbl_apply_L_batch(dbl_ctx* ctx, int m, int precision, int transpose, int count,
                      const void* const* in, void* const* out);

/* One level of the periodic DWT with the filters of Sec. 4.
 * inverse = 0: in m x m -> out; lowpass_only = 1 writes only the (m/2)^2
 * low-pass band (restriction W^T), else the four bands [LL, LH, HL, HH]
 * (first letter: filter along rows) as 4 consecutive (m/2)^2 blocks; the
 * high-pass filter is g_k = (-1)^k h_{kappa-1-k}.
 * inverse = 1: lowpass_only = 1 maps (m/2)^2 -> m x m by the adjoint of the
 * restriction (prolongation W, Approach X); else the four bands back to the
 * image (perfect reconstruction).  m is the fine size. */
int dbl_dwt(dbl_ctx* ctx, int wavelet, int m, int precision, int inverse, int lowpass_only,
            const void* in, void* out);
/* The same for `count` images in one launch (pointer arrays as for
 * dbl_apply_A_batch). */
int dbl_dwt_batch(dbl_ctx* ctx, int wavelet, int m, int precision, int inverse,
                  int lowpass_only, int count, const void* const* in, void* const* out);

/* Approach D block transfer (Sec. 4.2): a coarse gradient-space vector
 * (m_coarse) -> the fine one (2 m_coarse):  Q_x <- W~1 Q_x W1^T,
 * Q_y <- W1 Q_y W~1^T, W~1 = first m_f - 1 rows and m_c - 1 columns of W1. */
int dbl_dtransfer(dbl_ctx* ctx, int wavelet, int m_coarse, int precision,
                  const void* in, void* out);

/* Run exactly `iters` CGLS iterations on min ||A^ x - b^|| with
 * A^ = [A^(level); sqrt(gamma) D] and b^ = [b; sqrt(gamma) c] (eq.
 * (augmented)), from x0 (NULL = 0).  resid_hist (host, may be NULL) receives
 * ||b^ - A^ x_k||^2 after each iteration, in FP64.  CGLS is the default
 * inner solver: it produces the same iterates as the paper's LSQR in exact
 * arithmetic, with fewer vectors per iteration.  iters in [0, 128]. */
int dbl_cgls(dbl_ctx* ctx, const dbl_op* op, int level, const dbl_sub* sub, const void* b,
             const void* x0, int iters, void* x, double* resid_hist);

/* dbl_cgls for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same kernels and launches, with every buffer beyond the caller's (CGLS
 * state vectors, scalars, partial sums, job and tile tables) in one static
 * device array of 64 MiB that each GPU the library runs on holds until the
 * process ends.  The call itself allocates nothing (no hipMalloc / hipFree).
 * A subproblem whose workspace exceeds the array (about 52 n + 64 KiB bytes
 * in FP32 and BF16, 104 n in FP64: up to m = 1024 FP32, 512 FP64) returns
 * DBL_ENOMEM before any device work.  Results equal dbl_cgls's.  All calls on
 * one GPU share the array: calls that overlap on one GPU race. */
int dbl_cgls_noalloc(dbl_ctx* ctx, const dbl_op* op, int level, const dbl_sub* sub,
                     const void* b, const void* x0, int iters, void* x, double* resid_hist);

/* The same subproblem and arguments solved by LSQR (Golub-Kahan
 * bidiagonalisation with Givens rotations; the inner solver of Sec. 3), for
 * exactly `iters` iterations from x0 (correction form: LSQR runs on the
 * residual b^ - A^ x0).  resid_hist receives LSQR's residual estimate
 * phibar_{k+1}^2 = ||b^ - A^ x_k||^2 (exact in exact arithmetic), FP64.
 * Always runs the tiled phase kernels (no one-block variant).  Errors as
 * dbl_cgls. */
int dbl_lsqr(dbl_ctx* ctx, const dbl_op* op, int level, const dbl_sub* sub, const void* b,
             const void* x0, int iters, void* x, double* resid_hist);

/* GCV choice of gamma for the subproblem {A^(level), D, c} and data b
 * (Sec. 3): a grid of opts.gcv_grid log-spaced values followed by Brent's
 * minimisation on the neighbouring interval.  Writes gamma and GCV(gamma)
 * to host doubles.  sub->gamma is ignored.  mode: dbl_gcv_mode. */
int dbl_gcv(dbl_ctx* ctx, const dbl_op* op, int level, const dbl_sub* sub, const void* b,
            int mode, int grid, double* gamma_out, double* gcv_out);

/* ------------------------------------------------------------------ solve */

/* Full V-cycle solve (Alg. 4).  b, x: device m x m arrays of
 * opts->precision.  levels = 1 runs Approach I.  rep may be NULL. */
int dbl_deblur(dbl_ctx* ctx, const void* b, const double* psf, int ph, int pw, int m,
               int solver, int wavelet, int levels, int transfer, const dbl_opts* opts,
               void* x, dbl_report* rep);

/* Solve `count` independent requests together: their V-cycles advance in
 * lock step, one fused launch per CGLS phase covering every image.  Each
 * result equals the plain dbl_deblur result of the same request.  reps may
 * be NULL, else `count` reports. */
int dbl_deblur_batch(dbl_ctx* ctx, int count, const dbl_request* reqs, dbl_report* reps);

/* ---------------------------------------------------------------- serving */

/* Continuous-batching server on ctx: up to max_slots solves are resident at
 * once and share every launch; new requests are admitted at outer-iteration
 * boundaries while slots and the HBM budget allow. */
int dbl_server_create(dbl_ctx* ctx, int max_slots, size_t hbm_budget_bytes, dbl_server** out);
int dbl_server_destroy(dbl_server* srv);
/* Device workspace bytes one resident solve of `req` needs (what admission
 * by budget charges); 0 for an invalid request. */
size_t dbl_request_bytes(const dbl_request* req);
/* Queue a request; returns a ticket.  The psf is copied; b and x must stay
 * valid until the ticket completes. */
int dbl_server_submit(dbl_server* srv, const dbl_request* req, int64_t* ticket);
/* Advance the server by one outer-iteration step (admits, computes,
 * retires).  *active receives the number of resident solves afterwards.
 * A request whose workspace or hierarchy cannot be set up completes at
 * once: its ticket's report carries the error in `status` (DBL_ENOMEM when
 * it does not fit even with no other solve resident) and admission goes on
 * with the next request.  Out of memory while other solves are resident
 * only defers the request until they retire. */
int dbl_server_step(dbl_server* srv, int* active);
/* *done = 1 when the ticket has completed; then rep (may be NULL) receives
 * its report and the ticket is released. */
int dbl_server_poll(dbl_server* srv, int64_t ticket, int* done, dbl_report* rep);

/* ---------------------------------------------------------------- quality */

#define DBL_SSIM_MAX_M 8192
#define DBL_SSIM_MAX_RADIUS 16
/* Mean structural similarity (SSIM), the second quality measure of Sec. 5,
 * of `count` m x m images x[q] against one reference image ref.  Per pixel,
 * the local means mu, variances s^2 and covariance s_ab of the two images
 * under the Gaussian window w(k) w(l), w(k) = exp(-k^2 / (2 sigma^2)) for
 * |k| <= radius normalised to unit mass, with pixels outside the image
 * replaced by the nearest edge pixel, give
 *   (2 mu_a mu_b + c1)(2 s_ab + c2) / ((mu_a^2 + mu_b^2 + c1)(s_a^2 + s_b^2 + c2)),
 * c1 = (0.01 L)^2, c2 = (0.03 L)^2 with L = dyn_range; out[q] is its mean
 * over the m^2 pixels.  (sigma = 1.5, radius = 5, L = 1 is the window of the
 * SSIM reference the paper cites, for images in [0, 1].)
 * ref: device m x m FP64 array, column-major.  x: host array of count device
 * pointers, each an m x m column-major array of `precision` (DBL_F32 or
 * DBL_F64), read during the call.  out: device array of count doubles.
 * All statistics are formed in FP64.  1 <= m <= DBL_SSIM_MAX_M,
 * 0 <= count <= 65536 with count * ceil(m/32)^2 <= 2^24 (one block per
 * 32 x 32 tile), 0 <= radius <= DBL_SSIM_MAX_RADIUS, sigma and dyn_range
 * finite and > 0; anything else is DBL_EINVAL.  Asynchronous: out is
 * written on the context stream. */
int dbl_ssim(dbl_ctx* ctx, int m, int precision, int count, const double* ref,
             const void* const* x, double sigma, int radius, double dyn_range, double* out);

#ifdef __cplusplus
}
#endif
#endif /* DEBLUR_H */
