// Runtime objects behind the C ABI: context, operator hierarchy, solve slots.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <deque>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "host.h"

// One autotuner choice: the fastest CGLS phase variant (0 generic, 1 generic
// register-bounded, 2 32 x 32 tile, 3 tile register-bounded) measured for a
// phase (1 or 2), precision, radius bucket, grid size 2^mlog and launch of
// 2^tlog tiles, with the four timings (microseconds per launch).
struct TuneEntry {
  int phase, prec, rb, mlog, tlog, variant;
  double us[4];
};

struct dbl_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  size_t budget = 0;
  size_t used = 0;
  std::string err = "no error";
  std::map<void*, size_t> allocs;
  // job-table staging ring: pinned host memory mirrored to device memory
  char* h_stage = nullptr;
  char* d_stage = nullptr;
  size_t stage_cap = 0;
  size_t stage_off = 0;
  std::vector<std::pair<char*, char*>> retired;  // (pinned host, device) awaiting release
  // cached orthonormal DCT-II matrices (FP64, column-major) per grid size
  std::map<int, double*> dct;
  // scratch block for single-operator entry points
  void* scratch = nullptr;
  size_t scratch_bytes = 0;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  // optional per-kernel timing (dbl_profile): event pairs around launches
  bool prof_on = false;
  std::string prof_only;  // non-empty: time only this kernel family (dbl_profile_only)
  struct ProfPending { int id; hipEvent_t a, b; double bytes; };
  std::vector<ProfPending> prof_pending;
  std::vector<hipEvent_t> prof_pool;
  std::vector<std::string> prof_names;
  std::vector<long long> prof_launches;
  std::vector<double> prof_ms, prof_bytes;
  // operator hierarchies shared by solves with identical (kernel, m, levels,
  // wavelet, precision); entries without users are evicted beyond a bound
  // released solve workspaces kept for reuse (size -> block)
  std::multimap<size_t, void*> pool;
  size_t pool_bytes = 0;
  struct OpEntry { dbl_op* op; int refs; unsigned long long last; };
  std::map<std::string, OpEntry> op_cache;
  unsigned long long op_clock = 0;
  // one-block CGLS for small levels (DBL_OPT_SMALL_CGLS) and the device's
  // dynamic LDS limit per block
  int small_cgls = 1;
  // streaming separable blur for large FP32 grids in the operator entry points
  int stream_a = 1;
  int tile32 = 1;  // 32 x 32 tile CGLS kernels for separable operators (DBL_OPT_TILE32)
  // CGLS stage launches that mix radius buckets (DBL_OPT_MULTI_BUCKET): < 0
  // off; else buckets up to 8 share a launch, and bucket 12 joins them when
  // it has fewer tiles than this (3072: two rounds of the chip at 6 blocks
  // per CU)
  long long multi_tiles = 3072;
  // autotuned CGLS phase variants (dbl_autotune); empty: the built-in rule
  std::vector<TuneEntry> tune;
  size_t lds_limit = 65536;
  // EXACT-tier GCV: rocBLAS handle (rocblas_handle) and dense FP64 workspace
  void* blas = nullptr;
  void* gx = nullptr;
  size_t gx_bytes = 0;
  // RC of the solves that stop on a tolerance, gathered once per engine step
  // (device array written by the statistics kernel, pinned host copy)
  double* d_rc = nullptr;
  double* h_rc = nullptr;
  int rc_cap = 0;
  // done flags of the multi-launch Brent minimisations of one GCV batch
  double* d_gflag = nullptr;
  double* h_gflag = nullptr;
  int gflag_cap = 0;
};

struct dbl_op {
  dbl_ctx* ctx = nullptr;
  int m = 0, levels = 0, wavelet = 0, precision = 0;
  bool sep = true;
  dbl::HierHost host;
  dbl::LevelOp* d_ops = nullptr;     // device array [levels]
  // separable levels: the same operators with tables padded to every radius
  // bucket >= the level's own ([levels * NBUCKETS]; smaller buckets unset),
  // so jobs of different radii can share one launch
  dbl::LevelOp* d_pad = nullptr;
  // every table of the hierarchy, d_ops, d_pad and the GCV symbol inputs in
  // one device allocation, uploaded with one copy
  void* blob = nullptr;
  std::vector<double*> lam;          // per level: l(k) (m) then the interior kernel (FP64)
  // per level GCV symbol a_k (FP64, n_i each), in one allocation made and
  // filled (one launch for every level that needs it) on first use
  double* sym_blk = nullptr;
  std::vector<double*> sym;
  std::vector<char> sym_ready;
};

namespace dbl {

int set_err(dbl_ctx* ctx, int code, const std::string& msg);
int hip_check(dbl_ctx* ctx, hipError_t e, const char* what);
int dmalloc(dbl_ctx* ctx, size_t bytes, void** p);
void dfree(dbl_ctx* ctx, void* p);
// Workspace blocks recycled through the context pool (no hipMalloc/hipFree
// on the steady-state path).
int pool_get(dbl_ctx* ctx, size_t bytes, void** p);
void pool_put(dbl_ctx* ctx, void* p, size_t bytes);
void pool_trim(dbl_ctx* ctx, size_t keep_bytes);
int stage(dbl_ctx* ctx, const void* src, size_t bytes, void** dptr);
int stage_checkpoint(dbl_ctx* ctx);

// CGLS phase launches of general operators that mix radius buckets up to
// rbmax in {4, 8, 12} (kernels_cgls_gen.hip).
hipError_t launch_cgls_gen_multi(const LaunchArgs& la, int phase, int precision, int rbmax);
bool cgls_gen_multi_bucket(int rbmax);

// Per-kernel timing: when profiling is on, `launch` runs between two events on
// the context stream and the launch is charged `bytes` algorithmic bytes.
template <class F>
hipError_t timed(dbl_ctx* ctx, const char* name, double bytes, F&& launch);
int prof_collect(dbl_ctx* ctx);
hipEvent_t prof_event(dbl_ctx* ctx);
int prof_id(dbl_ctx* ctx, const char* name);

template <class F>
hipError_t timed(dbl_ctx* ctx, const char* name, double bytes, F&& launch) {
  if (!ctx->prof_on || (!ctx->prof_only.empty() && ctx->prof_only != name)) return launch();
  dbl_ctx::ProfPending p;
  p.id = prof_id(ctx, name);
  p.a = prof_event(ctx);
  p.b = prof_event(ctx);
  p.bytes = bytes;
  hipError_t e = hipEventRecord(p.a, ctx->stream);
  if (e != hipSuccess) return e;
  e = launch();
  if (e != hipSuccess) return e;
  e = hipEventRecord(p.b, ctx->stream);
  ctx->prof_pending.push_back(p);
  return e;
}

// Variant of a CGLS phase launch (phase 1 or 2) from the autotuner's table:
// sets la.tile32 (kept off where the launch cannot take the tile kernels) and
// la.wide.  No table, or a non-separable operator: la is left as it is.
void tune_cgls_launch(const dbl_ctx* ctx, int phase, int prec, int sep, int rb, LaunchArgs& la);

// Device operator of `level` with tables padded to radius bucket rb (the
// level's own bucket, or a larger one for a separable level).
const LevelOp* op_dev(const dbl_op* op, int level, int rb);

// Dynamic LDS of the one-block CGLS at `level` when this context runs that
// level with it, else 0; *wlds = 1 when IRLS weights are staged in LDS.
size_t small_lds_bytes(const dbl_ctx* ctx, const dbl_op* op, int level, bool irls, int* wlds);
// Halo (radius bucket) of the one-block CGLS on a level: the separable
// tables' bucket, or the smallest bucket above a general operator's radius.
int small_halo(const LevelHost& L);

// Algorithmic bytes of one job (each operand read or written once).
double job_bytes(const char* kernel, const Job& j, int precision);

// Tile table of one launch.  Jobs are added in order; `group` separates jobs
// that a prefix launch (tiles_upto) may cut between (the CGLS and LSQR
// phases launch the prefix of jobs with the most iterations left).  At
// upload the table is reordered within each run of equal group so that the
// blocks that the dispatcher sends to one XCD (block ids equal mod 8) take a
// contiguous run of tiles: neighbouring tiles then share that XCD's L2 for
// their halos.  Every block still finds its job and tile in the table, so
// results do not depend on the order.
struct Launch {
  std::vector<Job> jobs;
  std::vector<uint32_t> tiles;
  std::vector<int> tiles_upto;  // tiles after each job (prefix launches)
  std::vector<int> seg_start;   // first tile of each run of equal group
  int last_group = 0;
  int m_max = 0;
  int m_min = 1 << 30;
  void add(const Job& j, int grid_m, int esz, int group = 0);
  // a job cut into nti x ntj tiles of a kernel's own geometry
  void add_grid(const Job& j, int nti, int ntj, int group = 0);
  int upload(dbl_ctx* ctx, LaunchArgs& la);
  bool empty() const { return jobs.empty(); }
  // Host image of the launch's tables appended to buf at a 256-byte
  // boundary: the job table, then the tile table (XCD-ordered) at the next
  // boundary.  Returns the offset of the job table.
  size_t pack(std::vector<char>& buf) const;
  // la for the tables packed at `off` of a staged copy at device address d.
  void bind(const dbl_ctx* ctx, char* d, size_t off, LaunchArgs& la) const;
};
// The tables of several launches staged with one copy (each LaunchArgs gets
// the same fields as from Launch::upload).
int upload_all(dbl_ctx* ctx, const std::vector<std::pair<const Launch*, LaunchArgs*>>& ls);

// A low-pass prolongation job onto its m x m grid: 32 x 64 fine tiles from
// m = 64 on (k_dwt_inv takes the tile width from the job, two 32-column
// halves per block), the usual tiles below.
void add_prolong(Launch& L, const Job& j, int esz);

// Reorder tiles[s0, s1) so that positions p with p % nxcd == x hold the x-th
// contiguous chunk of the run (chunk x has as many tiles as there are such
// positions).  Exposed for the host tests.
void xcd_order(std::vector<uint32_t>& tiles, size_t s0, size_t s1, int nxcd);

int tiles_per_axis(int grid_m, int esz);
// FP64 partial-sum slots a job on an m x m grid may need (CGLS, GCV grid).
size_t part_doubles(int m);

// Partial-sum regions carved from one FP64 block for a grid of size m.
struct PartLayout {
  double *q, *s[2], *st;                  // CGLS |q|^2, |s|^2 & |r|^2 (x2), stats
  double *gw, *gmm, *ggrid, *gb[2];       // GCV weights, bounds, grid, Brent (x2)
};
PartLayout part_layout(double* base, int m);

// Build the hierarchy and upload its tables.
int op_build(dbl_ctx* ctx, const double* psf, int ph, int pw, int m, int levels, int wavelet,
             int precision, dbl_op** out);
void op_free(dbl_op* op);
// Shared hierarchy from the context cache (reference counted).
int op_acquire(dbl_ctx* ctx, const double* psf, int ph, int pw, int m, int levels, int wavelet,
               int precision, dbl_op** out);
void op_release(dbl_ctx* ctx, dbl_op* op);
void op_cache_clear(dbl_ctx* ctx);

// One V-cycle solve in flight.
struct Slot {
  dbl_request req{};
  dbl_opts opts{};
  dbl_op* op = nullptr;
  int prec = 0;
  size_t esz = 4;
  int m = 0, levels = 1, solver = 0, wavelet = 0, transfer = 0;
  int n0 = 0, nl0 = 0;
  void* block = nullptr;  // single device allocation carved below
  void* X[2]{};
  void* P[2]{};
  void* S = nullptr;
  void* R1[2]{};
  void* Q1 = nullptr;
  void* R2[2]{};
  void* Q2 = nullptr;
  void* W = nullptr;
  void* C1 = nullptr;
  void* C2 = nullptr;
  std::vector<const void*> B;  // b per level (B[0] = caller's b)
  double* scal = nullptr;
  double* part = nullptr;
  double* hist = nullptr;  // levels * k_out * 3 (gamma, rc, objective)
  double* g_bh = nullptr;  // GCV: DCT of b (per level, recomputed on entry)
  double* g_e = nullptr;   // GCV: per-frequency residual numerator
  double* g_tmp = nullptr; // GCV: GEMM / input staging
  double* g_in = nullptr;  // GCV: FP64 input staging
  bool gcv = false;
  std::vector<double> mu;  // levels * k_out fixed parameters (when !gcv)
  // progress
  int level = 0, k = 0, cur = 0;
  int iters[DBL_MAX_LEVELS]{};  // outer iterations run per level
  int rc_idx = -1;              // this step's entry of ctx->d_rc (tolerance stop)
  bool started = false, done = false, bh_valid = false;
  int status = 0;
  double t_submit = 0.0, t_done = 0.0;
  int64_t ticket = -1;
};

int slot_init(dbl_ctx* ctx, const dbl_request& req, Slot* s);
void slot_free(dbl_ctx* ctx, Slot* s);
size_t slot_bytes(const dbl_request& req);
// Advance every slot by one outer iteration (level entry, aux, gamma, CGLS,
// post-update, statistics).  Slots that finish copy their result out.
int engine_step(dbl_ctx* ctx, std::vector<Slot*>& slots);
int slot_report(dbl_ctx* ctx, Slot* s, dbl_report* rep);

// GCV for a set of (slot-like) requests, writes S_GAMMA / S_SQRTG in scal.
struct GcvReq {
  const dbl_op* op;
  int level;
  int prec;
  const void* b;     // level data (device, prec)
  const void* w;     // IRLS weights or null
  const void* c1;    // shift part 1 or null
  const void* c2;    // shift part 2 (SB: c = c1 - c2) or null
  double* scal;
  double* part;
  double* bh;        // FP64 n: DCT(b) (computed when !bh_valid)
  double* e;         // FP64 n
  double* tmp;       // FP64 n
  double* in;        // FP64 n
  bool bh_valid;
  int grid;
  int mode;          // resolved: DBL_GCV_SPECTRAL / DBL_GCV_EXACT
};
int gcv_run(dbl_ctx* ctx, std::vector<GcvReq>& reqs);

}  // namespace dbl
