// extern "C" entry points (include/deblur.h): argument validation first, then
// the runtime.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <limits>
#include <new>

#include <rocblas/rocblas.h>

#include "metrics.h"
#include "runtime.h"

using namespace dbl;

namespace {

bool pow2(int m) { return m > 0 && (m & (m - 1)) == 0; }

int check_prec(dbl_ctx* ctx, int p) {
  if (p != DBL_F32 && p != DBL_F64 && p != DBL_BF16)
    return set_err(ctx, DBL_EINVAL, "precision must be F32, F64 or BF16");
  return DBL_OK;
}

int check_psf(dbl_ctx* ctx, const double* psf, int ph, int pw) {
  if (!psf) return set_err(ctx, DBL_EINVAL, "psf is NULL");
  if (ph <= 0 || pw <= 0 || ph % 2 == 0 || pw % 2 == 0)
    return set_err(ctx, DBL_EINVAL, "psf dimensions must be odd and positive");
  if (ph / 2 > DBL_MAX_PSF_RADIUS || pw / 2 > DBL_MAX_PSF_RADIUS)
    return set_err(ctx, DBL_ENOTSUP, "psf half-width exceeds DBL_MAX_PSF_RADIUS");
  double s = 0.0;
  for (int k = 0; k < ph * pw; ++k) {
    if (!std::isfinite(psf[k])) return set_err(ctx, DBL_EINVAL, "psf has non-finite entries");
    s += std::fabs(psf[k]);
  }
  if (s == 0.0) return set_err(ctx, DBL_EINVAL, "psf is zero");
  return DBL_OK;
}

int check_grid(dbl_ctx* ctx, int m, int levels, int wavelet) {
  if (!pow2(m) || m < 8 || m > 8192) return set_err(ctx, DBL_EINVAL, "m must be a power of two in [8, 8192]");
  if (wavelet != DBL_HAAR && wavelet != DBL_DB4) return set_err(ctx, DBL_EINVAL, "bad wavelet");
  if (levels < 1 || levels > DBL_MAX_LEVELS) return set_err(ctx, DBL_EINVAL, "bad level count");
  if ((m >> (levels - 1)) < 8) return set_err(ctx, DBL_EINVAL, "coarsest grid smaller than 8");
  return DBL_OK;
}

int check_opts(dbl_ctx* ctx, const dbl_opts& o) {
  if (!(o.eps > 0.0) || !(o.tau >= 0.0)) return set_err(ctx, DBL_EINVAL, "eps must be > 0, tau >= 0");
  if (o.k_out < 1 || o.k_out > DBL_MAX_KOUT) return set_err(ctx, DBL_EINVAL, "k_out out of range");
  if (o.k_in < 1 || o.k_in > 100000) return set_err(ctx, DBL_EINVAL, "k_in out of range");
  if (o.gcv_mode < 0 || o.gcv_mode > 2) return set_err(ctx, DBL_EINVAL, "bad gcv_mode");
  if (o.gcv_grid < 3 || o.gcv_grid > DBL_GCV_GRID_MAX) return set_err(ctx, DBL_EINVAL, "bad gcv_grid");
  if (!(o.tol_fine >= 0.0) || !(o.tol_coarse >= 0.0) || !std::isfinite(o.tol_fine) ||
      !std::isfinite(o.tol_coarse))
    return set_err(ctx, DBL_EINVAL, "tolerances must be finite and >= 0");
  if (o.inner_solver != DBL_INNER_CGLS && o.inner_solver != DBL_INNER_LSQR)
    return set_err(ctx, DBL_EINVAL, "bad inner_solver");
  return check_prec(ctx, o.precision);
}

int check_request(dbl_ctx* ctx, const dbl_request& r) {
  if (!r.b || !r.x) return set_err(ctx, DBL_EINVAL, "b or x is NULL");
  int rc = check_psf(ctx, r.psf, r.ph, r.pw);
  if (!rc) rc = check_grid(ctx, r.m, r.levels, r.wavelet);
  if (!rc && (r.solver < 0 || r.solver > 2)) rc = set_err(ctx, DBL_EINVAL, "bad solver");
  if (!rc && (r.transfer < 0 || r.transfer > 1)) rc = set_err(ctx, DBL_EINVAL, "bad transfer");
  if (!rc) rc = check_opts(ctx, r.opts);
  if (!rc && r.opts.mu_schedule) {
    for (int k = 0; k < r.levels * r.opts.k_out; ++k)
      if (!(r.opts.mu_schedule[k] > 0.0) || !std::isfinite(r.opts.mu_schedule[k]))
        return set_err(ctx, DBL_EINVAL, "mu_schedule entries must be positive and finite");
  }
  return rc;
}

}  // namespace

namespace dbl {
int validate_request(dbl_ctx* ctx, const dbl_request& r) { return check_request(ctx, r); }
}  // namespace dbl

extern "C" {

void dbl_opts_default(dbl_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->eps = 0.03;
  o->tau = 0.005;
  o->k_out = 10;
  o->k_in = 30;
  o->mu_fixed = 0.0;
  o->mu_schedule = nullptr;
  o->gcv_mode = DBL_GCV_AUTO;
  o->gcv_grid = 50;
  o->precision = DBL_F32;
  o->x_hist = nullptr;
  o->tol_fine = 0.0;
  o->tol_coarse = 0.0;
  o->inner_solver = DBL_INNER_CGLS;
}

int dbl_create(dbl_ctx** out, int device, void* hip_stream, size_t budget) {
  if (!out) return DBL_EINVAL;
  *out = nullptr;
  if (device == -1) {  // argument-checking context: no device, no work
    dbl_ctx* ctx = new (std::nothrow) dbl_ctx();
    if (!ctx) return DBL_ENOMEM;
    ctx->device = -1;
    *out = ctx;
    return DBL_OK;
  }
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) {
    (void)hipGetLastError();
    return DBL_EDEVICE;
  }
  if (device < 0 || device >= ndev) return DBL_EINVAL;
  if (hipSetDevice(device) != hipSuccess) return DBL_EDEVICE;
  dbl_ctx* ctx = new (std::nothrow) dbl_ctx();
  if (!ctx) return DBL_ENOMEM;
  ctx->device = device;
  ctx->stream = static_cast<hipStream_t>(hip_stream);
  ctx->budget = budget;
  int lds = 0;
  if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, device) ==
          hipSuccess &&
      lds > 0)
    ctx->lds_limit = (size_t)lds;
  else
    (void)hipGetLastError();
  if (hipEventCreate(&ctx->ev0) != hipSuccess || hipEventCreate(&ctx->ev1) != hipSuccess) {
    delete ctx;
    return DBL_EDEVICE;
  }
  *out = ctx;
  return DBL_OK;
}

int dbl_set_option(dbl_ctx* ctx, int option, long long value) {
  if (!ctx) return DBL_EINVAL;
  switch (option) {
    case DBL_OPT_SMALL_CGLS:
      if (value != 0 && value != 1) return set_err(ctx, DBL_EINVAL, "DBL_OPT_SMALL_CGLS takes 0 or 1");
      ctx->small_cgls = (int)value;
      return DBL_OK;
    case DBL_OPT_TILE32:
      if (value != 0 && value != 1) return set_err(ctx, DBL_EINVAL, "DBL_OPT_TILE32 takes 0 or 1");
      ctx->tile32 = (int)value;
      return DBL_OK;
    case DBL_OPT_MULTI_BUCKET:
      ctx->multi_tiles = value < 0 ? -1 : value;
      return DBL_OK;
    case DBL_OPT_STREAM_A:
      if (value != 0 && value != 1) return set_err(ctx, DBL_EINVAL, "DBL_OPT_STREAM_A takes 0 or 1");
      ctx->stream_a = (int)value;
      return DBL_OK;
    default:
      return set_err(ctx, DBL_EINVAL, "unknown option");
  }
}

int dbl_destroy(dbl_ctx* ctx) {
  if (!ctx) return DBL_EINVAL;
  if (ctx->device < 0) {
    delete ctx;
    return DBL_OK;
  }
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  (void)prof_collect(ctx);
  if (ctx->blas) (void)rocblas_destroy_handle(static_cast<rocblas_handle>(ctx->blas));
  // Cached operators free their own buffers (and untrack them) first; every
  // allocation still tracked after that is freed exactly once below.  A
  // second hipFree of a pointer would leave hipErrorInvalidValue as the
  // thread's last error, where the caller's next launch check would find it.
  op_cache_clear(ctx);
  ctx->pool.clear();
  ctx->pool_bytes = 0;
  for (auto& kv : ctx->dct) (void)hipFree(kv.second);
  for (auto& kv : ctx->allocs) (void)hipFree(kv.first);
  ctx->allocs.clear();
  if (ctx->h_stage) (void)hipHostFree(ctx->h_stage);
  for (auto& b : ctx->retired) (void)hipHostFree(b.first);
  if (ctx->h_rc) (void)hipHostFree(ctx->h_rc);
  if (ctx->h_gflag) (void)hipHostFree(ctx->h_gflag);
  for (hipEvent_t e : ctx->prof_pool) (void)hipEventDestroy(e);
  if (ctx->ev0) (void)hipEventDestroy(ctx->ev0);
  if (ctx->ev1) (void)hipEventDestroy(ctx->ev1);
  delete ctx;
  return DBL_OK;
}

const char* dbl_last_error(const dbl_ctx* ctx) {
  return ctx ? ctx->err.c_str() : "null context";
}

int dbl_sync(dbl_ctx* ctx) {
  if (!ctx) return DBL_EINVAL;
  if (ctx->device < 0) return DBL_OK;
  return hip_check(ctx, hipStreamSynchronize(ctx->stream), "hipStreamSynchronize");
}

size_t dbl_workspace_bytes(const dbl_ctx* ctx) { return ctx ? ctx->used : 0; }

int dbl_profile(dbl_ctx* ctx, int enable) {
  if (!ctx) return DBL_EINVAL;
  if (enable != 0 && enable != 1) return set_err(ctx, DBL_EINVAL, "enable must be 0 or 1");
  if (ctx->device < 0) return set_err(ctx, DBL_EDEVICE, "context has no device");
  int rc = prof_collect(ctx);
  if (rc) return rc;
  if (enable) {
    ctx->prof_names.clear();
    ctx->prof_launches.clear();
    ctx->prof_ms.clear();
    ctx->prof_bytes.clear();
  }
  ctx->prof_on = enable != 0;
  return DBL_OK;
}

int dbl_profile_only(dbl_ctx* ctx, const char* name) {
  if (!ctx) return DBL_EINVAL;
  if (name && std::strlen(name) >= 64) return set_err(ctx, DBL_EINVAL, "family name too long");
  ctx->prof_only = name ? name : "";
  return DBL_OK;
}

int dbl_profile_read(dbl_ctx* ctx, int index, char* name, size_t name_cap, int64_t* launches,
                     double* ms, double* bytes) {
  if (!ctx || !name || name_cap == 0 || !launches || !ms || !bytes) return DBL_EINVAL;
  if (ctx->device < 0) return set_err(ctx, DBL_EDEVICE, "context has no device");
  int rc = prof_collect(ctx);
  if (rc) return rc;
  if (index < 0 || index >= (int)ctx->prof_names.size()) return DBL_ENOTFOUND;
  std::strncpy(name, ctx->prof_names[index].c_str(), name_cap - 1);
  name[name_cap - 1] = 0;
  *launches = ctx->prof_launches[index];
  *ms = ctx->prof_ms[index];
  *bytes = ctx->prof_bytes[index];
  return DBL_OK;
}

int dbl_op_create(dbl_ctx* ctx, const double* psf, int ph, int pw, int m, int levels,
                  int wavelet, int precision, dbl_op** out) {
  if (!ctx || !out) return DBL_EINVAL;
  *out = nullptr;
  int rc = check_psf(ctx, psf, ph, pw);
  if (!rc) rc = check_grid(ctx, m, levels, wavelet);
  if (!rc) rc = check_prec(ctx, precision);
  if (rc) return rc;
  if (ctx->device < 0) return set_err(ctx, DBL_EDEVICE, "context has no device");
  (void)hipSetDevice(ctx->device);
  if (int rc0 = stage_checkpoint(ctx)) return rc0;
  return op_build(ctx, psf, ph, pw, m, levels, wavelet, precision, out);
}

int dbl_op_destroy(dbl_op* op) {
  if (!op) return DBL_EINVAL;
  (void)hipStreamSynchronize(op->ctx->stream);
  op_free(op);
  return DBL_OK;
}

int dbl_apply_A_batch(dbl_ctx* ctx, const dbl_op* op, int level, int transpose, int count,
                      const void* const* in, void* const* out) {
  if (!ctx || !op) return DBL_EINVAL;
  if (count < 0 || count > 65536) return set_err(ctx, DBL_EINVAL, "count out of range");
  if (count > 0 && (!in || !out)) return set_err(ctx, DBL_EINVAL, "in or out array is NULL");
  for (int q = 0; q < count; ++q)
    if (!in[q] || !out[q]) return set_err(ctx, DBL_EINVAL, "in or out is NULL");
  if (level < 0 || level >= op->levels) return set_err(ctx, DBL_EINVAL, "level out of range");
  if (transpose != 0 && transpose != 1) return set_err(ctx, DBL_EINVAL, "bad transpose flag");
  if (ctx->device < 0) return set_err(ctx, DBL_EDEVICE, "context has no device");
  if (count == 0) return DBL_OK;
  (void)hipSetDevice(ctx->device);
  if (int rc0 = stage_checkpoint(ctx)) return rc0;
  const LevelHost& L = op->host.levels[level];
  const int esz = op->precision == DBL_F64 ? 8 : 4;
  const bool stream = ctx->stream_a && L.sep &&
                      apply_stream_ok(L.m, op->precision, 1, std::max(L.f1.rows, L.a1.rows));
  int snti = 0, sntj = 0;
  if (stream) apply_stream_grid(L.m, &snti, &sntj);
  Launch Lc;
  double bytes = 0.0;
  for (int q = 0; q < count; ++q) {
    Job j;
    std::memset(&j, 0, sizeof(j));
    j.m = L.m;
    j.op = op->d_ops + level;
    j.flags = transpose ? F_ADJ : 0;
    j.v[0] = const_cast<void*>(in[q]);
    j.v[1] = out[q];
    if (stream) Lc.add_grid(j, snti, sntj);
    else Lc.add(j, j.m, esz);
    bytes += job_bytes("apply_A", j, op->precision);
  }
  LaunchArgs la;
  int rc = Lc.upload(ctx, la);
  if (rc) return rc;
  return hip_check(ctx, timed(ctx, "apply_A", bytes, [&] {
                     return stream ? launch_apply_stream(la, L.rb)
                                   : launch_apply_A(la, op->precision, L.sep ? 1 : 0, L.rb,
                                                    L.sep ? L.rb : L.R);
                   }),
                   "apply A");
}

int dbl_apply_A(dbl_ctx* ctx, const dbl_op* op, int level, int transpose, const void* in,
                void* out) {
  return dbl_apply_A_batch(ctx, op, level, transpose, 1, &in, &out);
}

int dbl_apply_L_batch(dbl_ctx* ctx, int m, int precision, int transpose, int count,
                      const void* const* in, void* const* out) {
  if (!ctx) return DBL_EINVAL;
  if (count < 0 || count > 65536) return set_err(ctx, DBL_EINVAL, "count out of range");
  if (count > 0 && (!in || !out)) return set_err(ctx, DBL_EINVAL, "in or out array is NULL");
  for (int q = 0; q < count; ++q)
    if (!in[q] || !out[q]) return set_err(ctx, DBL_EINVAL, "in or out is NULL");
  if (!pow2(m) || m < 2) return set_err(ctx, DBL_EINVAL, "m must be a power of two >= 2");
  if (transpose != 0 && transpose != 1) return set_err(ctx, DBL_EINVAL, "bad transpose flag");
  int rc = check_prec(ctx, precision);
  if (rc) return rc;
  if (ctx->device < 0) return set_err(ctx, DBL_EDEVICE, "context has no device");
  if (count == 0) return DBL_OK;
  (void)hipSetDevice(ctx->device);
  if (int rc0 = stage_checkpoint(ctx)) return rc0;
  Launch Lc;
  double bytes = 0.0;
  for (int q = 0; q < count; ++q) {
    Job j;
    std::memset(&j, 0, sizeof(j));
    j.m = m;
    j.v[0] = const_cast<void*>(in[q]);
    j.v[1] = out[q];
    Lc.add(j, m, precision == DBL_F64 ? 8 : 4);
    bytes += job_bytes("apply_L", j, precision);
  }
  LaunchArgs la;
  if ((rc = Lc.upload(ctx, la))) return rc;
  const char* name = transpose ? "apply_LT" : "apply_L";
  return hip_check(ctx, timed(ctx, name, bytes, [&] {
                     return transpose ? launch_gradT(la, precision) : launch_grad(la, precision);
                   }),
                   "apply L");
}

int dbl_apply_L(dbl_ctx* ctx, int m, int precision, int transpose, const void* in, void* out) {
  return dbl_apply_L_batch(ctx, m, precision, transpose, 1, &in, &out);
}

int dbl_dwt_batch(dbl_ctx* ctx, int wavelet, int m, int precision, int inverse,
                  int lowpass_only, int count, const void* const* in, void* const* out) {
  if (!ctx) return DBL_EINVAL;
  if (count < 0 || count > 65536) return set_err(ctx, DBL_EINVAL, "count out of range");
  if (count > 0 && (!in || !out)) return set_err(ctx, DBL_EINVAL, "in or out array is NULL");
  for (int q = 0; q < count; ++q)
    if (!in[q] || !out[q]) return set_err(ctx, DBL_EINVAL, "in or out is NULL");
  if (!pow2(m) || m < 4) return set_err(ctx, DBL_EINVAL, "m must be a power of two >= 4");
  if (wavelet != DBL_HAAR && wavelet != DBL_DB4) return set_err(ctx, DBL_EINVAL, "bad wavelet");
  if ((inverse != 0 && inverse != 1) || (lowpass_only != 0 && lowpass_only != 1))
    return set_err(ctx, DBL_EINVAL, "bad flag");
  int rc = check_prec(ctx, precision);
  if (rc) return rc;
  if (ctx->device < 0) return set_err(ctx, DBL_EDEVICE, "context has no device");
  if (count == 0) return DBL_OK;
  (void)hipSetDevice(ctx->device);
  if (int rc0 = stage_checkpoint(ctx)) return rc0;
  Launch Lc;
  double bytes = 0.0;
  const char* name = inverse ? (lowpass_only ? "prolong" : "dwt_inv4")
                             : (lowpass_only ? "restrict" : "dwt_fwd4");
  for (int q = 0; q < count; ++q) {
    Job j;
    std::memset(&j, 0, sizeof(j));
    j.m = m;
    j.flags = wavelet;
    j.p0 = lowpass_only ? 0.0 : 1.0;
    j.v[0] = const_cast<void*>(in[q]);
    j.v[1] = out[q];
    if (inverse && lowpass_only)
      add_prolong(Lc, j, precision == DBL_F64 ? 8 : 4);
    else
      Lc.add(j, inverse ? m : m / 2, precision == DBL_F64 ? 8 : 4);
    bytes += job_bytes(name, j, precision);
  }
  LaunchArgs la;
  if ((rc = Lc.upload(ctx, la))) return rc;
  return hip_check(ctx, timed(ctx, name, bytes, [&] {
                     return inverse ? launch_dwt_inv(la, precision) : launch_dwt_fwd(la, precision);
                   }),
                   "dwt");
}

int dbl_dwt(dbl_ctx* ctx, int wavelet, int m, int precision, int inverse, int lowpass_only,
            const void* in, void* out) {
  return dbl_dwt_batch(ctx, wavelet, m, precision, inverse, lowpass_only, 1, &in, &out);
}

int dbl_dtransfer(dbl_ctx* ctx, int wavelet, int m_coarse, int precision, const void* in,
                  void* out) {
  if (!ctx) return DBL_EINVAL;
  if (!in || !out) return set_err(ctx, DBL_EINVAL, "in or out is NULL");
  if (!pow2(m_coarse) || m_coarse < 2) return set_err(ctx, DBL_EINVAL, "m_coarse must be a power of two >= 2");
  if (wavelet != DBL_HAAR && wavelet != DBL_DB4) return set_err(ctx, DBL_EINVAL, "bad wavelet");
  int rc = check_prec(ctx, precision);
  if (rc) return rc;
  if (ctx->device < 0) return set_err(ctx, DBL_EDEVICE, "context has no device");
  (void)hipSetDevice(ctx->device);
  if (int rc0 = stage_checkpoint(ctx)) return rc0;
  Job j;
  std::memset(&j, 0, sizeof(j));
  j.m = 2 * m_coarse;
  j.flags = wavelet;
  j.v[0] = const_cast<void*>(in);
  j.v[1] = out;
  Launch Lc;
  Lc.add(j, j.m, precision == DBL_F64 ? 8 : 4);
  LaunchArgs la;
  if ((rc = Lc.upload(ctx, la))) return rc;
  return hip_check(ctx, launch_dtransfer(la, precision), "dtransfer");
}

int dbl_ssim(dbl_ctx* ctx, int m, int precision, int count, const double* ref,
             const void* const* x, double sigma, int radius, double dyn_range, double* out) {
  if (!ctx) return DBL_EINVAL;
  if (m < 1 || m > DBL_SSIM_MAX_M) return set_err(ctx, DBL_EINVAL, "m out of range [1, 8192]");
  if (count < 0 || count > 65536) return set_err(ctx, DBL_EINVAL, "count out of range");
  if (count > 0 && (!ref || !x || !out)) return set_err(ctx, DBL_EINVAL, "ref, x or out is NULL");
  for (int q = 0; q < count; ++q)
    if (!x[q]) return set_err(ctx, DBL_EINVAL, "x is NULL");
  if (precision != DBL_F32 && precision != DBL_F64)
    return set_err(ctx, DBL_EINVAL, "precision must be DBL_F32 or DBL_F64");
  if (radius < 0 || radius > DBL_SSIM_MAX_RADIUS)
    return set_err(ctx, DBL_EINVAL, "radius out of range [0, 16]");
  if (!(sigma > 0.0) || !std::isfinite(sigma)) return set_err(ctx, DBL_EINVAL, "sigma must be finite and > 0");
  if (!(dyn_range > 0.0) || !std::isfinite(dyn_range))
    return set_err(ctx, DBL_EINVAL, "dyn_range must be finite and > 0");
  if (ctx->device < 0) return set_err(ctx, DBL_EDEVICE, "context has no device");
  if (ssim_lds(radius) + 512 > ctx->lds_limit)
    return set_err(ctx, DBL_ENOTSUP, "SSIM tile does not fit the device's LDS");
  if (count == 0) return DBL_OK;
  (void)hipSetDevice(ctx->device);
  if (int rc0 = stage_checkpoint(ctx)) return rc0;
  // the window taps, normalised to unit mass
  double taps[2 * DBL_SSIM_MAX_RADIUS + 1];
  double tsum = 0.0;
  for (int k = -radius; k <= radius; ++k) {
    taps[k + radius] = std::exp(-(double)k * k / (2.0 * sigma * sigma));
    tsum += taps[k + radius];
  }
  for (int k = 0; k <= 2 * radius; ++k) taps[k] /= tsum;
  void* dtaps = nullptr;
  int rc = stage(ctx, taps, sizeof(double) * (2 * radius + 1), &dtaps);
  if (rc) return rc;
  // one FP64 partial per 32 x 32 tile of every image
  const int nt1 = (m + 31) / 32, nt = nt1 * nt1;
  if ((size_t)count * nt > (size_t(1) << 24))
    return set_err(ctx, DBL_EINVAL, "count x tiles above 2^24");
  const size_t need = ((size_t)count * nt * sizeof(double) + 255) & ~size_t(255);
  if (ctx->scratch_bytes < need) {
    if ((rc = hip_check(ctx, hipStreamSynchronize(ctx->stream), "sync"))) return rc;
    dfree(ctx, ctx->scratch);
    ctx->scratch = nullptr;
    ctx->scratch_bytes = 0;
    if ((rc = dmalloc(ctx, need, &ctx->scratch))) return rc;
    ctx->scratch_bytes = need;
  }
  double* part = static_cast<double*>(ctx->scratch);
  Launch Lt, Lf;
  for (int q = 0; q < count; ++q) {
    Job j;
    std::memset(&j, 0, sizeof(j));
    j.m = m;
    j.v[0] = const_cast<double*>(ref);
    j.v[1] = const_cast<void*>(x[q]);
    j.v[2] = dtaps;
    j.v[3] = out + q;
    j.i0 = radius;
    j.p0 = (0.01 * dyn_range) * (0.01 * dyn_range);
    j.p1 = (0.03 * dyn_range) * (0.03 * dyn_range);
    j.pw = part + (size_t)q * nt;
    j.pr[0] = j.pw;
    j.i1 = nt;
    Lt.add_grid(j, nt1, nt1);
    Lf.add_grid(j, 1, 1);
  }
  LaunchArgs lt, lf;
  if ((rc = upload_all(ctx, {{&Lt, &lt}, {&Lf, &lf}}))) return rc;
  // algorithmic bytes: both images read once, one partial per tile
  const double bytes = (double)count * ((double)m * m * (8.0 + (precision == DBL_F64 ? 8 : 4)) +
                                        8.0 * nt);
  if ((rc = hip_check(ctx, timed(ctx, "ssim", bytes,
                                 [&] { return launch_ssim(lt, precision, radius); }),
                      "ssim")))
    return rc;
  return hip_check(ctx, timed(ctx, "ssim_fin", 8.0 * count * (nt + 1),
                              [&] { return launch_ssim_fin(lf); }),
                   "ssim finish");
}

}  // extern "C"

namespace {

// LSQR phase sequence of one subproblem (the scratch layout of krylov_entry):
// init, B_1, then A_i and B_{i+1} for i < iters, A_iters, finish.
int lsqr_sequence(dbl_ctx* ctx, const Job& j, int m, int esz, int prec, int sep, int rb, int H,
                  int iters, void* W, void* V, void* U1, void* U2, const void* x0, void* AX0) {
  const PartLayout PL = part_layout(j.part, m);
  const int t = tiles_per_axis(m, esz);
  double* PA[2] = {PL.s[0], PL.s[0] + (size_t)t * t};  // |u|^2 partials by parity
  double* PB[2] = {PL.s[1], PL.s[1] + (size_t)t * t};  // |v|^2 partials by parity
  Job jl = j;
  jl.v[V_PA] = W;
  jl.v[V_S] = V;
  jl.v[V_R1A] = U1;
  jl.v[V_R2A] = U2;
  int rc = DBL_OK;
  auto run = [&](Job jj, const char* what, auto launcher) {
    Launch L;
    L.add(jj, m, esz);
    LaunchArgs la;
    if ((rc = L.upload(ctx, la))) return rc;
    return rc = hip_check(ctx, launcher(la), what);
  };
  Job ji = jl;
  ji.v[V_X0] = const_cast<void*>(x0);
  ji.v[V_XOLD] = AX0;
  ji.pw = PA[0];
  if (run(ji, "lsqr init", [&](const LaunchArgs& la) { return launch_lsqr_init(la, prec); }))
    return rc;
  if (iters == 0) return DBL_OK;
  for (int i = 1; i <= iters; ++i) {
    Job jb = jl;
    jb.i0 = i;
    if (i == 1) jb.flags |= F_FIRST;
    jb.pr[0] = PA[(i - 1) & 1];
    jb.pr[1] = PB[(i - 1) & 1];
    jb.pw = PB[i & 1];
    if (run(jb, "lsqr B", [&](const LaunchArgs& la) {
          return launch_lsqr_b(la, prec, sep, rb, H);
        }))
      return rc;
    Job ja = jl;
    ja.i0 = i;
    if (i == 1) ja.flags |= F_FIRST;
    ja.pr[0] = PB[i & 1];
    ja.pr[1] = PA[(i - 1) & 1];
    ja.pw = PA[i & 1];
    if (run(ja, "lsqr A", [&](const LaunchArgs& la) {
          return launch_lsqr_a(la, prec, sep, rb, H);
        }))
      return rc;
  }
  Job jf = jl;
  jf.i0 = iters;
  jf.pr[0] = PA[iters & 1];
  return run(jf, "lsqr finish", [&](const LaunchArgs& la) { return launch_lsqr_fin(la, prec); });
}

int krylov_entry(dbl_ctx* ctx, const dbl_op* op, int level, const dbl_sub* sub, const void* b,
                 const void* x0, int iters, void* x, double* resid_hist, bool lsqr) {
  if (!ctx || !op) return DBL_EINVAL;
  if (!sub || !b || !x) return set_err(ctx, DBL_EINVAL, "sub, b or x is NULL");
  if (level < 0 || level >= op->levels) return set_err(ctx, DBL_EINVAL, "level out of range");
  if (iters < 0 || iters > HIST_MAX) return set_err(ctx, DBL_EINVAL, "iters out of range [0, 128]");
  if (sub->d_kind != 0 && sub->d_kind != 1) return set_err(ctx, DBL_EINVAL, "bad d_kind");
  if (sub->d_kind == 1 && !sub->w) return set_err(ctx, DBL_EINVAL, "weights required for d_kind 1");
  if (!(sub->gamma >= 0.0) || !std::isfinite(sub->gamma)) return set_err(ctx, DBL_EINVAL, "gamma must be finite and >= 0");
  if (ctx->device < 0) return set_err(ctx, DBL_EDEVICE, "context has no device");
  (void)hipSetDevice(ctx->device);
  if (int rc0 = stage_checkpoint(ctx)) return rc0;
  const LevelHost& L = op->host.levels[level];
  const int m = L.m, prec = op->precision;
  const size_t esz = prec == DBL_F64 ? 8 : 4;
  const size_t ssz = prec == DBL_BF16 ? 2 : esz;  // CGLS state vectors
  const size_t n = (size_t)m * m, nl = 2 * (size_t)m * (m - 1);
  auto al = [](size_t b) { return (b + 255) & ~size_t(255); };
  const size_t need = 6 * al(n * ssz) + 3 * al(nl * ssz) + al(n * esz) + al(NSCAL * 8) +
                      al(part_doubles(m) * 8);
  int rc = DBL_OK;
  if (ctx->scratch_bytes < need) {
    if ((rc = hip_check(ctx, hipStreamSynchronize(ctx->stream), "sync"))) return rc;
    dfree(ctx, ctx->scratch);
    ctx->scratch = nullptr;
    ctx->scratch_bytes = 0;
    if ((rc = dmalloc(ctx, need, &ctx->scratch))) return rc;
    ctx->scratch_bytes = need;
  }
  char* p = static_cast<char*>(ctx->scratch);
  auto take = [&](size_t b) { void* r = p; p += al(b); return r; };
  void* P[2] = {take(n * ssz), take(n * ssz)};
  void* S = take(n * ssz);
  void* R1[2] = {take(n * ssz), take(n * ssz)};
  void* Q1 = take(n * ssz);
  void* R2[2] = {take(nl * ssz), take(nl * ssz)};
  void* Q2 = take(nl * ssz);
  void* AX0 = take(n * esz);  // A x0 (compute type)
  double* scal = static_cast<double*>(take(NSCAL * 8));
  double* part = static_cast<double*>(take(part_doubles(m) * 8));
  const double gv[2] = {sub->gamma, std::sqrt(sub->gamma)};
  void* dg = nullptr;
  if ((rc = stage(ctx, gv, sizeof(gv), &dg))) return rc;
  if ((rc = hip_check(ctx, hipMemcpyAsync(scal + S_GAMMA, dg, sizeof(gv), hipMemcpyDeviceToDevice,
                                          ctx->stream), "set gamma")))
    return rc;
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
  int wl = 0;
  const size_t small = (x0 || lsqr) ? 0 : small_lds_bytes(ctx, op, level, sub->d_kind == 1, &wl);
  if (small && iters > 0) {
    Job js = j;
    if (wl) js.flags |= F_WLDS;
    js.v[V_C1] = const_cast<void*>(sub->c);
    js.i0 = iters;
    Launch Ls;
    Ls.add(js, 1, 4);
    LaunchArgs la;
    if ((rc = Ls.upload(ctx, la))) return rc;
    const double bytes = job_bytes("cgls_small", js, prec);
    if ((rc = hip_check(ctx, timed(ctx, "cgls_small", bytes, [&] {
                          return launch_cgls_small(la, prec, small_halo(L), m, small, !L.sep);
                        }),
                        "cgls small")))
      return rc;
    if (resid_hist) {
      if ((rc = hip_check(ctx, hipMemcpyAsync(resid_hist, scal + S_HIST, iters * sizeof(double),
                                              hipMemcpyDeviceToHost, ctx->stream),
                          "read history")))
        return rc;
      if ((rc = hip_check(ctx, hipStreamSynchronize(ctx->stream), "sync"))) return rc;
    }
    return DBL_OK;
  }
  if (x0) {
    Job ja = j;
    ja.v[0] = const_cast<void*>(x0);
    ja.v[1] = AX0;
    ja.flags = 0;
    Launch La;
    La.add(ja, m, (int)esz);
    LaunchArgs la;
    if ((rc = La.upload(ctx, la))) return rc;
    if ((rc = hip_check(ctx, launch_apply_A(la, prec, sep, rb, H), "A x0"))) return rc;
  }
  if (lsqr) {
    if ((rc = lsqr_sequence(ctx, j, m, (int)esz, prec, sep, rb, H, iters, P[0], S, R1[0], R2[0],
                            x0, AX0)))
      return rc;
    if (resid_hist && iters > 0) {
      if ((rc = hip_check(ctx, hipMemcpyAsync(resid_hist, scal + S_HIST, iters * sizeof(double),
                                              hipMemcpyDeviceToHost, ctx->stream),
                          "read history")))
        return rc;
      if ((rc = hip_check(ctx, hipStreamSynchronize(ctx->stream), "sync"))) return rc;
    }
    return DBL_OK;
  }
  Job ji = j;
  ji.v[V_PA] = P[0];
  ji.v[V_R1A] = R1[0];
  ji.v[V_R2A] = R2[0];
  ji.v[V_X0] = const_cast<void*>(x0);
  ji.v[V_XOLD] = AX0;
  Launch Li;
  Li.add(ji, m, (int)esz);
  LaunchArgs la;
  if ((rc = Li.upload(ctx, la))) return rc;
  if ((rc = hip_check(ctx, launch_cgls_init(la, prec), "cgls init"))) return rc;
  const PartLayout PL = part_layout(part, m);
  Job jf = j;
  jf.flags |= F_FIRST;
  jf.v[V_R1A] = R1[0];
  jf.v[V_R1B] = R1[1];
  jf.v[V_R2A] = R2[0];
  jf.v[V_R2B] = R2[1];
  jf.pw = PL.s[0];
  Launch Lf;
  Lf.add(jf, m, (int)esz);
  if ((rc = Lf.upload(ctx, la))) return rc;
  tune_cgls_launch(ctx, 2, prec, sep, rb, la);
  if ((rc = hip_check(ctx, launch_cgls_p2(la, prec, sep, rb, H), "cgls p2"))) return rc;
  LaunchArgs a2[2];
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
    Launch L2;
    L2.add(bb, m, (int)esz);
    if ((rc = L2.upload(ctx, a2[par]))) return rc;
    tune_cgls_launch(ctx, 2, prec, sep, rb, a2[par]);
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
    Launch L1;
    L1.add(a, m, (int)esz);
    LaunchArgs a1;
    if ((rc = L1.upload(ctx, a1))) return rc;
    tune_cgls_launch(ctx, 1, prec, sep, rb, a1);
    if ((rc = hip_check(ctx, launch_cgls_p1(a1, prec, sep, rb, H), "cgls p1"))) return rc;
    if ((rc = hip_check(ctx, launch_cgls_p2(a2[par], prec, sep, rb, H), "cgls p2"))) return rc;
  }
  if (iters > 0) {
    Job h = j;
    h.pr[0] = PL.s[iters & 1];
    h.i0 = iters - 1;
    const int t = tiles_per_axis(m, (int)esz);
    h.i1 = t * t;
    Launch Lh;
    Lh.add(h, 1, 4);
    LaunchArgs lh;
    if ((rc = Lh.upload(ctx, lh))) return rc;
    if ((rc = hip_check(ctx, launch_cgls_hist(lh), "cgls history"))) return rc;
  }
  if (resid_hist && iters > 0) {
    if ((rc = hip_check(ctx, hipMemcpyAsync(resid_hist, scal + S_HIST, iters * sizeof(double),
                                            hipMemcpyDeviceToHost, ctx->stream), "read history")))
      return rc;
    if ((rc = hip_check(ctx, hipStreamSynchronize(ctx->stream), "sync"))) return rc;
  }
  return DBL_OK;
}

}  // namespace

extern "C" {

int dbl_cgls(dbl_ctx* ctx, const dbl_op* op, int level, const dbl_sub* sub, const void* b,
             const void* x0, int iters, void* x, double* resid_hist) {
  return krylov_entry(ctx, op, level, sub, b, x0, iters, x, resid_hist, false);
}

int dbl_lsqr(dbl_ctx* ctx, const dbl_op* op, int level, const dbl_sub* sub, const void* b,
             const void* x0, int iters, void* x, double* resid_hist) {
  return krylov_entry(ctx, op, level, sub, b, x0, iters, x, resid_hist, true);
}

int dbl_gcv(dbl_ctx* ctx, const dbl_op* op, int level, const dbl_sub* sub, const void* b,
            int mode, int grid, double* gamma_out, double* gcv_out) {
  if (!ctx || !op) return DBL_EINVAL;
  if (!sub || !b || !gamma_out) return set_err(ctx, DBL_EINVAL, "sub, b or gamma_out is NULL");
  if (level < 0 || level >= op->levels) return set_err(ctx, DBL_EINVAL, "level out of range");
  if (sub->d_kind != 0 && sub->d_kind != 1) return set_err(ctx, DBL_EINVAL, "bad d_kind");
  if (sub->d_kind == 1 && !sub->w) return set_err(ctx, DBL_EINVAL, "weights required for d_kind 1");
  if (sub->d_kind == 1 && sub->c) return set_err(ctx, DBL_EINVAL, "weighted pair takes no shift");
  if (mode < 0 || mode > 2) return set_err(ctx, DBL_EINVAL, "bad mode");
  if (grid < 3 || grid > DBL_GCV_GRID_MAX) return set_err(ctx, DBL_EINVAL, "bad grid size");
  const int m = op->host.levels[level].m;
  const size_t n = (size_t)m * m;
  if (mode == DBL_GCV_AUTO) mode = n <= DBL_GCV_AUTO_EXACT_N ? DBL_GCV_EXACT : DBL_GCV_SPECTRAL;
  if (mode == DBL_GCV_EXACT && n > DBL_GCV_EXACT_MAX_N)
    return set_err(ctx, DBL_ENOTSUP, "EXACT GCV is limited to n <= 16384");
  if (ctx->device < 0) return set_err(ctx, DBL_EDEVICE, "context has no device");
  (void)hipSetDevice(ctx->device);
  if (int rc0 = stage_checkpoint(ctx)) return rc0;
  void* blk = nullptr;
  const size_t bytes = 4 * ((n * 8 + 255) & ~size_t(255)) + NSCAL * 8 + 256 + 256 +
                       part_doubles(m) * 8;
  int rc = dmalloc(ctx, bytes, &blk);
  if (rc) return rc;
  char* p = static_cast<char*>(blk);
  auto take = [&](size_t b) { void* r = p; p += (b + 255) & ~size_t(255); return r; };
  GcvReq g{};
  g.op = op;
  g.level = level;
  g.prec = op->precision;
  g.b = b;
  g.w = sub->d_kind == 1 ? sub->w : nullptr;
  g.c1 = sub->c;
  g.c2 = nullptr;
  g.bh = static_cast<double*>(take(n * 8));
  g.e = static_cast<double*>(take(n * 8));
  g.tmp = static_cast<double*>(take(n * 8));
  g.in = static_cast<double*>(take(n * 8));
  g.scal = static_cast<double*>(take(NSCAL * 8));
  g.part = static_cast<double*>(take(part_doubles(m) * 8));
  g.bh_valid = false;
  g.grid = grid;
  g.mode = mode;
  rc = hip_check(ctx, hipMemsetAsync(g.scal, 0, NSCAL * 8, ctx->stream), "clear");
  std::vector<GcvReq> v{g};
  if (!rc) rc = gcv_run(ctx, v);
  double out[2] = {0, 0};
  if (!rc)
    rc = hip_check(ctx, hipMemcpyAsync(out, g.scal + S_GAMMA, sizeof(double), hipMemcpyDeviceToHost,
                                       ctx->stream), "read gamma");
  if (!rc)
    rc = hip_check(ctx, hipMemcpyAsync(out + 1, g.scal + S_G_FBEST, sizeof(double),
                                       hipMemcpyDeviceToHost, ctx->stream), "read gcv");
  if (!rc) rc = hip_check(ctx, hipStreamSynchronize(ctx->stream), "sync");
  else (void)hipStreamSynchronize(ctx->stream);  // queued work may still read blk
  dfree(ctx, blk);
  if (rc) return rc;
  *gamma_out = out[0];
  if (gcv_out) *gcv_out = out[1];
  return DBL_OK;
}

size_t dbl_request_bytes(const dbl_request* req) {
  if (!req) return 0;
  dbl_ctx tmp;
  tmp.device = -1;
  if (check_request(&tmp, *req)) return 0;
  return slot_bytes(*req);
}

int dbl_deblur(dbl_ctx* ctx, const void* b, const double* psf, int ph, int pw, int m, int solver,
               int wavelet, int levels, int transfer, const dbl_opts* opts, void* x,
               dbl_report* rep) {
  if (!ctx) return DBL_EINVAL;
  dbl_request r;
  std::memset(&r, 0, sizeof(r));
  r.b = b;
  r.x = x;
  r.psf = psf;
  r.ph = ph;
  r.pw = pw;
  r.m = m;
  r.solver = solver;
  r.wavelet = wavelet;
  r.levels = levels;
  r.transfer = transfer;
  if (opts) r.opts = *opts; else dbl_opts_default(&r.opts);
  return dbl_deblur_batch(ctx, 1, &r, rep);
}

int dbl_deblur_batch(dbl_ctx* ctx, int count, const dbl_request* reqs, dbl_report* reps) {
  if (!ctx) return DBL_EINVAL;
  if (count < 0 || (count > 0 && !reqs)) return set_err(ctx, DBL_EINVAL, "bad request list");
  if (count > 60000) return set_err(ctx, DBL_EINVAL, "too many requests");
  for (int i = 0; i < count; ++i) {
    int rc = check_request(ctx, reqs[i]);
    if (rc) return rc;
  }
  if (count == 0) return DBL_OK;
  if (ctx->device < 0) return set_err(ctx, DBL_EDEVICE, "context has no device");
  (void)hipSetDevice(ctx->device);
  if (int rc0 = stage_checkpoint(ctx)) return rc0;
  std::vector<Slot> slots(count);
  std::vector<Slot*> ptrs;
  int rc = DBL_OK;
  for (int i = 0; i < count && !rc; ++i) {
    rc = slot_init(ctx, reqs[i], &slots[i]);
    ptrs.push_back(&slots[i]);
  }
  if (!rc) rc = hip_check(ctx, hipEventRecord(ctx->ev0, ctx->stream), "event");
  while (!rc) {
    bool all = true;
    for (Slot* s : ptrs) all = all && s->done;
    if (all) break;
    rc = engine_step(ctx, ptrs);
  }
  if (!rc) rc = hip_check(ctx, hipEventRecord(ctx->ev1, ctx->stream), "event");
  if (!rc) rc = hip_check(ctx, hipStreamSynchronize(ctx->stream), "sync");
  float ms = 0.f;
  if (!rc) (void)hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1);
  for (int i = 0; i < count; ++i) {
    if (!rc && reps) {
      rc = slot_report(ctx, &slots[i], &reps[i]);
      reps[i].seconds = ms * 1e-3;
      bool bad = false;
      // iterations a tolerance skipped are NaN by design; only run ones count
      for (int l = 0; l < slots[i].levels; ++l)
        for (int k = 0; k < reps[i].iters[l]; ++k)
          if (!std::isfinite(reps[i].objective[l][k])) bad = true;
      if (bad) reps[i].status = DBL_ENUMERIC;
    }
  }
  (void)hipStreamSynchronize(ctx->stream);
  for (auto& s : slots) slot_free(ctx, &s);
  return rc;
}

}  // extern "C"
