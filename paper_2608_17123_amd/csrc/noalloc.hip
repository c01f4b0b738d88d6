// dbl_cgls_noalloc: the CGLS entry point for callers that cannot allocate
// device memory.  Every buffer the CGLS phases need beyond the caller's own
// (the state vectors p, s, r1, r2, q1, q2, A x0, the FP64 scalar block, the
// per-tile partial sums and the job and tile tables the kernels read) lives
// in one file-scope device array of NOALLOC_BYTES, `scratch`.  The array is
// created with the code object on each device the library runs on and is
// held until the process ends.  Host code never uses the array's name as an
// address: its device address is looked up once per device with
// hipGetSymbolAddress and kept in dev_scratch[].
//
// The kernels and the launch sequence are those of dbl_cgls (same jobs, same
// arithmetic), so the results are identical; only where the workspace and
// the tables live differs.  Calls on one device share the array and keep the
// previous call's contents: everything a call reads is written by that call
// first (tables and scalars by host copies and the set-gamma kernel, the
// vectors by the CGLS start), and calls that overlap on one device race.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>

#include "runtime.h"

namespace dbl {
namespace {

constexpr size_t NOALLOC_BYTES = size_t(64) << 20;
constexpr int NOALLOC_MAX_DEVICES = 64;

__device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];

char* dev_scratch[NOALLOC_MAX_DEVICES] = {};
std::mutex dev_scratch_mu;

// Device address of `scratch` on the current device (set up once per device).
int scratch_base(dbl_ctx* ctx, char** out) {
  if (ctx->device < 0 || ctx->device >= NOALLOC_MAX_DEVICES)
    return set_err(ctx, DBL_ENOTSUP, "device index beyond the no-allocation table");
  std::lock_guard<std::mutex> lock(dev_scratch_mu);
  if (!dev_scratch[ctx->device]) {
    void* p = nullptr;
    const int rc = hip_check(ctx, hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)),
                             "hipGetSymbolAddress(scratch)");
    if (rc) return rc;
    dev_scratch[ctx->device] = static_cast<char*>(p);
  }
  *out = dev_scratch[ctx->device];
  return DBL_OK;
}

size_t al256(size_t b) { return (b + 255) & ~size_t(255); }

// Host copy of the tables of one call, written to the array in one copy.
// Fixed size: no host allocation on the call path either.
constexpr int MAX_JOBS = HIST_MAX + 8;
constexpr int MAX_TILES = 64 * 64;  // tiles of an m <= 2048 grid
struct Tables {
  Job jobs[MAX_JOBS];
  uint32_t tiles[MAX_TILES];
};
Tables host_tables[NOALLOC_MAX_DEVICES];

}  // namespace
}  // namespace dbl

using namespace dbl;

extern "C" int dbl_cgls_noalloc(dbl_ctx* ctx, const dbl_op* op, int level, const dbl_sub* sub,
                                const void* b, const void* x0, int iters, void* x,
                                double* resid_hist) {
  if (!ctx || !op) return DBL_EINVAL;
  if (!sub || !b || !x) return set_err(ctx, DBL_EINVAL, "sub, b or x is NULL");
  if (level < 0 || level >= op->levels) return set_err(ctx, DBL_EINVAL, "level out of range");
  if (iters < 0 || iters > HIST_MAX) return set_err(ctx, DBL_EINVAL, "iters out of range [0, 128]");
  if (sub->d_kind != 0 && sub->d_kind != 1) return set_err(ctx, DBL_EINVAL, "bad d_kind");
  if (sub->d_kind == 1 && !sub->w) return set_err(ctx, DBL_EINVAL, "weights required for d_kind 1");
  if (!(sub->gamma >= 0.0) || !std::isfinite(sub->gamma))
    return set_err(ctx, DBL_EINVAL, "gamma must be finite and >= 0");
  if (ctx->device < 0) return set_err(ctx, DBL_EDEVICE, "context has no device");
  const LevelHost& L = op->host.levels[level];
  const int m = L.m, prec = op->precision;
  const size_t esz = prec == DBL_F64 ? 8 : 4;
  const size_t ssz = prec == DBL_BF16 ? 2 : esz;
  const size_t n = (size_t)m * m, nl = 2 * (size_t)m * (m - 1);
  const int tpa = tiles_per_axis(m, (int)esz), ntiles = tpa * tpa;
  const size_t table_bytes = al256(sizeof(Job) * MAX_JOBS) + al256(sizeof(uint32_t) * ntiles);
  const size_t need = table_bytes + 6 * al256(n * ssz) + 3 * al256(nl * ssz) + al256(n * esz) +
                      al256(NSCAL * 8) + al256(part_doubles(m) * 8);
  if (need > NOALLOC_BYTES || ntiles > MAX_TILES)
    return set_err(ctx, DBL_ENOMEM,
                   "subproblem needs " + std::to_string(need) + " bytes of the no-allocation "
                   "workspace, which holds " + std::to_string(NOALLOC_BYTES));
  (void)hipSetDevice(ctx->device);
  char* base = nullptr;
  int rc = scratch_base(ctx, &base);
  if (rc) return rc;

  // workspace layout: tables, then the vectors, the scalar block, partials
  char* p = base;
  auto take = [&](size_t bytes) { char* r = p; p += al256(bytes); return r; };
  Job* d_jobs = reinterpret_cast<Job*>(take(sizeof(Job) * MAX_JOBS));
  uint32_t* d_tiles = reinterpret_cast<uint32_t*>(take(sizeof(uint32_t) * ntiles));
  void* P[2] = {take(n * ssz), take(n * ssz)};
  void* S = take(n * ssz);
  void* R1[2] = {take(n * ssz), take(n * ssz)};
  void* Q1 = take(n * ssz);
  void* R2[2] = {take(nl * ssz), take(nl * ssz)};
  void* Q2 = take(nl * ssz);
  void* AX0 = take(n * esz);
  double* scal = reinterpret_cast<double*>(take(NSCAL * 8));
  double* part = reinterpret_cast<double*>(take(part_doubles(m) * 8));

  Tables& T = host_tables[ctx->device];
  int nj = 0;
  auto add = [&](const Job& j) {
    T.jobs[nj] = j;
    T.jobs[nj].nti = T.jobs[nj].ntj = tpa;
    return nj++;
  };
  // one job per launch; every launch of the call shares the tile table
  // (tile t of job 0, in the dispatcher's XCD order)
  for (int t = 0; t < ntiles; ++t) T.tiles[t] = (uint32_t)t;
  {
    // XCD-aware order of the tiled launches (results do not depend on it)
    uint32_t tmp[MAX_TILES];
    int cnt[XCDS] = {0}, next[XCDS] = {0};
    for (int q = 0; q < ntiles; ++q) ++cnt[q % XCDS];
    for (int x = 0, acc = 0; x < XCDS; ++x) { next[x] = acc; acc += cnt[x]; }
    for (int q = 0; q < ntiles; ++q) tmp[q] = T.tiles[next[q % XCDS]++];
    std::memcpy(T.tiles, tmp, sizeof(uint32_t) * ntiles);
  }

  Job j;
  std::memset(&j, 0, sizeof(j));
  j.m = m;
  j.op = op->d_ops + level;
  j.scal = scal;
  j.part = part;
  j.flags = (sub->d_kind == 1 ? F_IRLS : 0) | (sub->c ? F_SHIFT : 0) | F_HIST;
  j.v[V_X] = x;
  j.v[V_S] = S;
  j.v[V_Q1] = Q1;
  j.v[V_Q2] = Q2;
  j.v[V_W] = const_cast<void*>(sub->w);
  j.v[V_B] = const_cast<void*>(b);
  j.v[V_C1] = const_cast<void*>(sub->c);
  const int sep = L.sep ? 1 : 0, rb = L.rb, H = L.sep ? L.rb : L.R;

  Job jg = j;  // scal[S_GAMMA], scal[S_SQRTG] <- gamma, sqrt(gamma)
  jg.p0 = sub->gamma;
  jg.p1 = std::sqrt(sub->gamma);
  const int k_gamma = add(jg);
  int wl = 0;
  const size_t small = x0 ? 0 : small_lds_bytes(ctx, op, level, sub->d_kind == 1, &wl);
  int k_small = -1, k_ax0 = -1, k_init = -1, k_first = -1, k_hist = -1;
  int k_p1[HIST_MAX], k_p2[2];
  const PartLayout PL = part_layout(part, m);
  if (small && iters > 0) {
    Job js = j;
    if (wl) js.flags |= F_WLDS;
    js.i0 = iters;
    k_small = add(js);
  } else {
    if (x0) {
      Job ja = j;
      ja.v[0] = const_cast<void*>(x0);
      ja.v[1] = AX0;
      ja.flags = 0;
      k_ax0 = add(ja);
    }
    Job ji = j;
    ji.v[V_PA] = P[0];
    ji.v[V_R1A] = R1[0];
    ji.v[V_R2A] = R2[0];
    ji.v[V_X0] = const_cast<void*>(x0);
    ji.v[V_XOLD] = AX0;
    k_init = add(ji);
    Job jf = j;
    jf.flags |= F_FIRST;
    jf.v[V_R1A] = R1[0];
    jf.v[V_R1B] = R1[1];
    jf.v[V_R2A] = R2[0];
    jf.v[V_R2B] = R2[1];
    jf.pw = PL.s[0];
    k_first = add(jf);
    for (int par = 0; par < 2; ++par) {
      Job bb = j;
      bb.v[V_PB] = P[1 - par];
      bb.v[V_R1A] = R1[1 - par];
      bb.v[V_R1B] = R1[par];
      bb.v[V_R2A] = R2[1 - par];
      bb.v[V_R2B] = R2[par];
      bb.pr[0] = PL.q;
      bb.pr[1] = PL.s[par];
      bb.pw = PL.s[1 - par];
      k_p2[par] = add(bb);
    }
    for (int it = 0; it < iters; ++it) {
      const int par = it & 1;
      Job a = j;
      a.v[V_PA] = P[par];
      a.v[V_PB] = P[1 - par];
      a.pw = PL.q;
      a.pr[0] = PL.s[par];
      a.pr[1] = PL.s[1 - par];
      a.i0 = it;
      if (it == 0) a.flags |= F_FIRST;
      k_p1[it] = add(a);
    }
    if (iters > 0) {
      Job h = j;
      h.pr[0] = PL.s[iters & 1];
      h.i0 = iters - 1;
      h.i1 = ntiles;
      k_hist = add(h);
    }
  }
  // the one-block launches (gamma, one-block CGLS, history) read only the
  // job index of their tile entry, which is 0 in every entry
  const uint32_t* d_one = d_tiles;

  rc = hip_check(ctx, hipMemcpyAsync(d_jobs, T.jobs, sizeof(Job) * nj, hipMemcpyHostToDevice,
                                     ctx->stream), "copy job table");
  if (!rc)
    rc = hip_check(ctx, hipMemcpyAsync(d_tiles, T.tiles, sizeof(uint32_t) * ntiles,
                                       hipMemcpyHostToDevice, ctx->stream), "copy tile table");
  if (rc) return rc;
  auto la_for = [&](int k, int tiles_n, const uint32_t* tl) {
    LaunchArgs la;
    la.jobs = d_jobs + k;
    la.tiles = tl;
    la.ntiles = tiles_n;
    la.m_max = m;
    la.stream = ctx->stream;
    la.tile32 = ctx->tile32 && m >= 32;
    return la;
  };
  // a CGLS phase launch with the autotuner's variant (host table lookup only)
  auto la_phase = [&](int phase, int k) {
    LaunchArgs la = la_for(k, ntiles, d_tiles);
    tune_cgls_launch(ctx, phase, prec, sep, rb, la);
    return la;
  };
  if ((rc = hip_check(ctx, launch_set_gamma(la_for(k_gamma, 1, d_one)), "set gamma"))) return rc;
  if (k_small >= 0) {
    if ((rc = hip_check(ctx, launch_cgls_small(la_for(k_small, 1, d_one), prec, small_halo(L), m,
                                               small, !L.sep),
                        "cgls small")))
      return rc;
  } else {
    if (k_ax0 >= 0 &&
        (rc = hip_check(ctx, launch_apply_A(la_for(k_ax0, ntiles, d_tiles), prec, sep, rb, H),
                        "A x0")))
      return rc;
    if ((rc = hip_check(ctx, launch_cgls_init(la_for(k_init, ntiles, d_tiles), prec),
                        "cgls init")))
      return rc;
    if ((rc = hip_check(ctx, launch_cgls_p2(la_phase(2, k_first), prec, sep, rb, H),
                        "cgls p2")))
      return rc;
    for (int it = 0; it < iters; ++it) {
      if ((rc = hip_check(ctx, launch_cgls_p1(la_phase(1, k_p1[it]), prec, sep, rb, H),
                          "cgls p1")))
        return rc;
      if ((rc = hip_check(ctx, launch_cgls_p2(la_phase(2, k_p2[it & 1]), prec, sep, rb, H),
                          "cgls p2")))
        return rc;
    }
    if (k_hist >= 0 &&
        (rc = hip_check(ctx, launch_cgls_hist(la_for(k_hist, 1, d_one)), "cgls history")))
      return rc;
  }
  if (resid_hist && iters > 0) {
    if ((rc = hip_check(ctx, hipMemcpyAsync(resid_hist, scal + S_HIST, iters * sizeof(double),
                                            hipMemcpyDeviceToHost, ctx->stream),
                        "read history")))
      return rc;
    if ((rc = hip_check(ctx, hipStreamSynchronize(ctx->stream), "sync"))) return rc;
  }
  return DBL_OK;
}
