// Autotuner for the CGLS phase launches of separable operators.
//
// Four compiled variants compute every phase launch with the same sums in
// the same order: the generic tile kernels (k_cgls_p1/p2) and the 32 x 32
// wavefront-layout kernels (k_cgls_p1_sep/p2_sep), each with the unbounded
// and the register-bounded ("wide") occupancy.  Which is fastest depends on
// the grid size, the radius bucket and how many tiles a launch holds, so the
// tuner times all four on synthetic jobs over a grid of those keys (HIP
// events on the library stream), keeps the fastest per key, and writes the
// table to a JSON cache that later contexts load instead of measuring.  A
// phase launch then takes the entry nearest to its own key.  Since every
// variant produces the same bits, tuning changes speed only, never results.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/deblur.h"
#include "launch.h"
#include "runtime.h"

using namespace dbl;

namespace {

int ilog2(long long v) {
  int l = 0;
  while (v > 1) {
    v >>= 1;
    ++l;
  }
  return l;
}

std::string device_name(int device) {
  hipDeviceProp_t p;
  if (hipGetDeviceProperties(&p, device) != hipSuccess) return "unknown";
  return std::string(p.gcnArchName) + " cu" + std::to_string(p.multiProcessorCount);
}

// Radius of a Gaussian kernel that falls in radius bucket rb.
int radius_for_bucket(int rb) { return rb == 8 ? 7 : rb; }

std::vector<double> gaussian(int r) {
  const double sig = std::max(0.5, r / 3.0);
  const int e = 2 * r + 1;
  std::vector<double> p((size_t)e * e);
  double s = 0.0;
  for (int j = 0; j < e; ++j)
    for (int i = 0; i < e; ++i) {
      const double v = std::exp(-((i - r) * (i - r) + (j - r) * (j - r)) / (2.0 * sig * sig));
      p[(size_t)j * e + i] = v;
      s += v;
    }
  for (double& v : p) v /= s;
  return p;
}

// Launch one phase with the variant applied.
hipError_t launch_variant(int phase, const LaunchArgs& base, int prec, int rb, int variant) {
  LaunchArgs la = base;
  la.tile32 = base.tile32 && variant >= 2;
  la.wide = variant & 1;
  return phase == 1 ? launch_cgls_p1(la, prec, 1, rb, rb) : launch_cgls_p2(la, prec, 1, rb, rb);
}

// Time every variant of both phases for `count` jobs on an m x m grid with
// the separable operator `op` (level 0, radius bucket rb); append entries.
int measure_key(dbl_ctx* ctx, const dbl_op* op, int prec, int rb, int m, int count,
                std::vector<TuneEntry>& out) {
  const size_t esz = prec == DBL_F64 ? 8 : 4, ssz = prec == DBL_BF16 ? 2 : esz;
  const size_t n = (size_t)m * m, nl = 2 * (size_t)m * (m - 1);
  auto al = [](size_t b) { return (b + 255) & ~size_t(255); };
  const size_t per = 6 * al(n * ssz) + 3 * al(nl * ssz) + al(n * esz) + al(nl * esz) +
                     al(NSCAL * 8) + al(part_doubles(m) * 8);
  void* blk = nullptr;
  int rc = dmalloc(ctx, per * count, &blk);
  if (rc) return rc;
  if ((rc = hip_check(ctx, hipMemsetAsync(blk, 0, per * count, ctx->stream), "clear"))) {
    dfree(ctx, blk);
    return rc;
  }
  Launch L1, L2;
  for (int q = 0; q < count; ++q) {
    char* p = static_cast<char*>(blk) + per * q;
    auto take = [&](size_t b) { void* r = p; p += al(b); return r; };
    void* P0 = take(n * ssz);
    void* P1 = take(n * ssz);
    void* S = take(n * ssz);
    void* R10 = take(n * ssz);
    void* R11 = take(n * ssz);
    void* Q1 = take(n * ssz);
    void* R20 = take(nl * ssz);
    void* R21 = take(nl * ssz);
    void* Q2 = take(nl * ssz);
    void* X = take(n * esz);
    void* W = take(nl * esz);
    double* scal = static_cast<double*>(take(NSCAL * 8));
    double* part = static_cast<double*>(take(part_doubles(m) * 8));
    const PartLayout PL = part_layout(part, m);
    Job j;
    std::memset(&j, 0, sizeof(j));
    j.m = m;
    j.op = op->d_ops;
    j.scal = scal;
    j.part = part;
    j.v[V_X] = X;
    j.v[V_S] = S;
    j.v[V_Q1] = Q1;
    j.v[V_Q2] = Q2;
    j.v[V_W] = W;
    Job a = j;  // phase 1 of an iteration > 0
    a.v[V_PA] = P0;
    a.v[V_PB] = P1;
    a.pw = PL.q;
    a.pr[0] = PL.s[0];
    a.pr[1] = PL.s[1];
    L1.add(a, m, (int)esz);
    Job b = j;  // phase 2 of the same iteration
    b.v[V_PB] = P1;
    b.v[V_R1A] = R10;
    b.v[V_R1B] = R11;
    b.v[V_R2A] = R20;
    b.v[V_R2B] = R21;
    b.pr[0] = PL.q;
    b.pr[1] = PL.s[0];
    b.pw = PL.s[1];
    L2.add(b, m, (int)esz);
  }
  LaunchArgs la1, la2;
  if (!(rc = L1.upload(ctx, la1))) rc = L2.upload(ctx, la2);
  for (int phase = 1; phase <= 2 && !rc; ++phase) {
    const LaunchArgs& la = phase == 1 ? la1 : la2;
    TuneEntry e{phase, prec, rb, ilog2(m), ilog2(la.ntiles), 0, {0, 0, 0, 0}};
    const int nvar = la.tile32 ? 4 : 2;
    for (int v = 0; v < nvar && !rc; ++v) {
      constexpr int WARM = 2, REPS = 5;
      for (int k = 0; k < WARM && !rc; ++k)
        rc = hip_check(ctx, launch_variant(phase, la, prec, rb, v), "tune launch");
      if (rc) break;
      if ((rc = hip_check(ctx, hipEventRecord(ctx->ev0, ctx->stream), "event"))) break;
      for (int k = 0; k < REPS && !rc; ++k)
        rc = hip_check(ctx, launch_variant(phase, la, prec, rb, v), "tune launch");
      if (rc) break;
      if ((rc = hip_check(ctx, hipEventRecord(ctx->ev1, ctx->stream), "event"))) break;
      if ((rc = hip_check(ctx, hipEventSynchronize(ctx->ev1), "event sync"))) break;
      float ms = 0.f;
      if ((rc = hip_check(ctx, hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1), "event time"))) break;
      e.us[v] = 1000.0 * ms / REPS;
    }
    if (!rc) {
      for (int v = 1; v < nvar; ++v)
        if (e.us[v] < e.us[e.variant]) e.variant = v;
      out.push_back(e);
    }
  }
  const int rs = hip_check(ctx, hipStreamSynchronize(ctx->stream), "sync");
  dfree(ctx, blk);
  return rc ? rc : rs;
}

int write_cache(const char* path, const std::string& dev, int prec,
                const std::vector<TuneEntry>& es) {
  FILE* f = std::fopen(path, "w");
  if (!f) return DBL_EINVAL;
  std::fprintf(f, "{\"device\": \"%s\", \"precision\": %d, \"variants\": [\"generic\", "
                  "\"generic wide\", \"tile32\", \"tile32 wide\"],\n \"entries\": [\n",
               dev.c_str(), prec);
  for (size_t k = 0; k < es.size(); ++k) {
    const TuneEntry& e = es[k];
    std::fprintf(f, "  {\"phase\": %d, \"rb\": %d, \"m\": %d, \"tiles\": %d, \"variant\": %d, "
                    "\"us\": [%.3f, %.3f, %.3f, %.3f]}%s\n",
                 e.phase, e.rb, 1 << e.mlog, 1 << e.tlog, e.variant, e.us[0], e.us[1], e.us[2],
                 e.us[3], k + 1 < es.size() ? "," : "");
  }
  std::fprintf(f, " ]}\n");
  return std::fclose(f) == 0 ? DBL_OK : DBL_EINVAL;
}

// Integer field `key` of the JSON object text [b, e); false when absent.
bool field(const char* b, const char* e, const char* key, long long* v) {
  const std::string pat = std::string("\"") + key + "\"";
  const char* p = std::search(b, e, pat.begin(), pat.end());
  if (p == e) return false;
  p += pat.size();
  while (p < e && (*p == ' ' || *p == ':')) ++p;
  if (p == e) return false;
  char* end = nullptr;
  *v = std::strtoll(p, &end, 10);
  return end != p && end <= e;
}

// Entries of a cache written by write_cache for this device and precision.
int read_cache(const char* path, const std::string& dev, int prec, std::vector<TuneEntry>& es) {
  FILE* f = std::fopen(path, "r");
  if (!f) return DBL_EINVAL;
  std::string s;
  char buf[4096];
  size_t k;
  while ((k = std::fread(buf, 1, sizeof(buf), f)) > 0) s.append(buf, k);
  std::fclose(f);
  const std::string devkey = "\"device\": \"" + dev + "\"";
  if (s.find(devkey) == std::string::npos) return DBL_EINVAL;  // another device
  long long pv = -1;
  if (!field(s.data(), s.data() + s.size(), "precision", &pv) || pv != prec) return DBL_EINVAL;
  const size_t at = s.find("\"entries\"");
  if (at == std::string::npos) return DBL_EINVAL;
  size_t pos = at;
  std::vector<TuneEntry> got;
  while ((pos = s.find('{', pos)) != std::string::npos) {
    const size_t end = s.find('}', pos);
    if (end == std::string::npos) return DBL_EINVAL;
    const char* b = s.data() + pos;
    const char* e = s.data() + end;
    long long ph, rb, m, t, v;
    if (!field(b, e, "phase", &ph) || !field(b, e, "rb", &rb) || !field(b, e, "m", &m) ||
        !field(b, e, "tiles", &t) || !field(b, e, "variant", &v))
      return DBL_EINVAL;
    if ((ph != 1 && ph != 2) || v < 0 || v > 3 || m < 1 || t < 1) return DBL_EINVAL;
    got.push_back(TuneEntry{(int)ph, prec, (int)rb, ilog2(m), ilog2(t), (int)v, {0, 0, 0, 0}});
    pos = end + 1;
  }
  if (got.empty()) return DBL_EINVAL;
  es = got;
  return DBL_OK;
}

}  // namespace

void dbl::tune_cgls_launch(const dbl_ctx* ctx, int phase, int prec, int sep, int rb,
                           LaunchArgs& la) {
  if (!sep || ctx->tune.empty()) return;
  const int ml = ilog2(la.m_max), tl = ilog2(la.ntiles);
  const TuneEntry* best = nullptr;
  int bd = 1 << 30;
  for (const TuneEntry& e : ctx->tune) {
    if (e.phase != phase || e.prec != prec || e.rb != rb) continue;
    const int d = 4 * std::abs(e.mlog - ml) + std::abs(e.tlog - tl);
    if (d < bd) {
      bd = d;
      best = &e;
    }
  }
  if (!best) return;
  la.tile32 = la.tile32 && best->variant >= 2;
  la.wide = best->variant & 1;
}

extern "C" int dbl_autotune(dbl_ctx* ctx, int precision, const char* cache_path, int flags,
                            int* n_entries) {
  if (!ctx) return DBL_EINVAL;
  if (precision < DBL_F32 || precision > DBL_BF16)
    return set_err(ctx, DBL_EINVAL, "precision must be DBL_F32, DBL_F64 or DBL_BF16");
  if (flags & ~(DBL_TUNE_REMEASURE | DBL_TUNE_QUICK))
    return set_err(ctx, DBL_EINVAL, "unknown autotune flags");
  if (ctx->device < 0) return set_err(ctx, DBL_EDEVICE, "context has no device");
  (void)hipSetDevice(ctx->device);
  const std::string dev = device_name(ctx->device);
  std::vector<TuneEntry> es;
  auto install = [&]() {
    ctx->tune.erase(std::remove_if(ctx->tune.begin(), ctx->tune.end(),
                                   [&](const TuneEntry& e) { return e.prec == precision; }),
                    ctx->tune.end());
    ctx->tune.insert(ctx->tune.end(), es.begin(), es.end());
    if (n_entries) *n_entries = (int)es.size();
    return DBL_OK;
  };
  if (cache_path && !(flags & DBL_TUNE_REMEASURE) &&
      read_cache(cache_path, dev, precision, es) == DBL_OK)
    return install();
  if (int rc0 = stage_checkpoint(ctx)) return rc0;
  const bool quick = flags & DBL_TUNE_QUICK;
  const std::vector<int> rbs = quick ? std::vector<int>{4, 8} : std::vector<int>{2, 4, 8, 12, 16};
  const std::vector<int> ms = quick ? std::vector<int>{64, 256}
                                    : std::vector<int>{32, 64, 128, 256, 512, 1024};
  const std::vector<int> counts = quick ? std::vector<int>{1, 16} : std::vector<int>{1, 4, 16, 64};
  const long long max_px = 1ll << 22;  // pixels per measured launch
  es.clear();
  for (int rb : rbs) {
    const int r = radius_for_bucket(rb);
    const std::vector<double> psf = gaussian(r);
    for (int m : ms) {
      if (m < 2 * r + 2) continue;
      dbl_op* op = nullptr;
      int rc = dbl_op_create(ctx, psf.data(), 2 * r + 1, 2 * r + 1, m, 1, DBL_HAAR, precision, &op);
      if (rc) return rc;
      if (!op->host.levels[0].sep || op->host.levels[0].rb != rb) {
        dbl_op_destroy(op);
        continue;
      }
      for (int c : counts) {
        if ((long long)c * m * m > max_px) continue;
        if ((rc = measure_key(ctx, op, precision, rb, m, c, es))) {
          dbl_op_destroy(op);
          return rc;
        }
      }
      dbl_op_destroy(op);
    }
  }
  if (cache_path && write_cache(cache_path, dev, precision, es) != DBL_OK)
    return set_err(ctx, DBL_EINVAL, "cannot write the autotune cache file");
  return install();
}

extern "C" int dbl_tune_choice(const dbl_ctx* ctx, int phase, int precision, int rb, int m,
                               int ntiles, int* variant) {
  if (!ctx || !variant || (phase != 1 && phase != 2) || m < 1 || ntiles < 1) return DBL_EINVAL;
  LaunchArgs la{};
  la.m_max = m;
  la.ntiles = ntiles;
  la.tile32 = ctx->tile32 && m >= 32;
  la.wide = -1;
  tune_cgls_launch(ctx, phase, precision, 1, rb, la);
  const bool wide = la.wide >= 0 ? la.wide != 0 : ntiles > cgls_wide_tiles();
  *variant = (la.tile32 ? 2 : 0) + (wide ? 1 : 0);
  return DBL_OK;
}
