// Runtime: device memory, job staging, operator upload and the V-cycle
// engine (Alg. 4 with the outer solvers of Algs. 1-3).
#include "runtime.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <stdexcept>
#include <tuple>

namespace dbl {

int set_err(dbl_ctx* ctx, int code, const std::string& msg) {
  if (ctx) ctx->err = msg;
  return code;
}

int hip_check(dbl_ctx* ctx, hipError_t e, const char* what) {
  if (e == hipSuccess) return DBL_OK;
  return set_err(ctx, DBL_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

int dmalloc(dbl_ctx* ctx, size_t bytes, void** p) {
  *p = nullptr;
  if (bytes == 0) bytes = 256;
  if (ctx->budget && ctx->used + bytes > ctx->budget && ctx->pool_bytes) pool_trim(ctx, 0);
  if (ctx->budget && ctx->used + bytes > ctx->budget)
    return set_err(ctx, DBL_ENOMEM, "device workspace budget exceeded");
  hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) {
    *p = nullptr;
    (void)hipGetLastError();
    return set_err(ctx, DBL_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
  }
  ctx->allocs[*p] = bytes;
  ctx->used += bytes;
  return DBL_OK;
}

void dfree(dbl_ctx* ctx, void* p) {
  if (!p) return;
  auto it = ctx->allocs.find(p);
  if (it != ctx->allocs.end()) {
    ctx->used -= it->second;
    ctx->allocs.erase(it);
  }
  (void)hipFree(p);
}

int pool_get(dbl_ctx* ctx, size_t bytes, void** p) {
  auto it = ctx->pool.find(bytes);
  if (it != ctx->pool.end()) {
    *p = it->second;
    ctx->pool.erase(it);
    ctx->pool_bytes -= bytes;
    return DBL_OK;
  }
  return dmalloc(ctx, bytes, p);
}

void pool_put(dbl_ctx* ctx, void* p, size_t bytes) {
  if (!p) return;
  ctx->pool.insert({bytes, p});
  ctx->pool_bytes += bytes;
  const size_t kKeep = size_t(8) << 30;
  if (ctx->pool_bytes > kKeep) pool_trim(ctx, kKeep / 2);
}

void pool_trim(dbl_ctx* ctx, size_t keep_bytes) {
  if (ctx->pool_bytes <= keep_bytes) return;
  (void)hipStreamSynchronize(ctx->stream);
  for (auto it = ctx->pool.begin(); it != ctx->pool.end() && ctx->pool_bytes > keep_bytes;) {
    ctx->pool_bytes -= it->first;
    dfree(ctx, it->second);
    it = ctx->pool.erase(it);
  }
}

// Copy `bytes` to the device through the staging buffer; the copy is queued
// on the context stream.  Staged data stays valid until the next checkpoint:
// when the buffer is full a larger one replaces it and the old one is only
// released at a checkpoint, after a stream synchronisation, so arrays staged
// for launches that have not been issued yet are never overwritten.
int stage(dbl_ctx* ctx, const void* src, size_t bytes, void** dptr) {
  const size_t need = (bytes + 255) & ~size_t(255);
  if (ctx->stage_off + need > ctx->stage_cap) {
    if (ctx->h_stage) ctx->retired.push_back({ctx->h_stage, ctx->d_stage});
    ctx->h_stage = nullptr;
    ctx->d_stage = nullptr;
    const size_t cap = std::max<size_t>(std::max(need, 2 * ctx->stage_cap), size_t(4) << 20);
    ctx->stage_cap = 0;
    ctx->stage_off = 0;
    int rc = hip_check(ctx, hipHostMalloc((void**)&ctx->h_stage, cap, hipHostMallocDefault),
                       "hipHostMalloc");
    if (rc) return rc;
    rc = dmalloc(ctx, cap, (void**)&ctx->d_stage);
    if (rc) {
      (void)hipHostFree(ctx->h_stage);
      ctx->h_stage = nullptr;
      return rc;
    }
    ctx->stage_cap = cap;
  }
  std::memcpy(ctx->h_stage + ctx->stage_off, src, bytes);
  int rc = hip_check(ctx,
                     hipMemcpyAsync(ctx->d_stage + ctx->stage_off, ctx->h_stage + ctx->stage_off,
                                    bytes, hipMemcpyHostToDevice, ctx->stream),
                     "stage copy");
  if (rc) return rc;
  *dptr = ctx->d_stage + ctx->stage_off;
  ctx->stage_off += need;
  return DBL_OK;
}

// Called only where no staged array is waiting for its launch: when the
// buffer is more than half used (or old buffers are retired), wait for the
// stream, free retired buffers and restart at offset 0.
int stage_checkpoint(dbl_ctx* ctx) {
  if (ctx->retired.empty() && ctx->stage_off <= ctx->stage_cap / 2) return DBL_OK;
  int rc = hip_check(ctx, hipStreamSynchronize(ctx->stream), "stage checkpoint");
  if (rc) return rc;
  for (auto& b : ctx->retired) {
    (void)hipHostFree(b.first);
    dfree(ctx, b.second);
  }
  ctx->retired.clear();
  ctx->stage_off = 0;
  return DBL_OK;
}

// ------------------------------------------------------------ profiling ----

hipEvent_t prof_event(dbl_ctx* ctx) {
  if (ctx->prof_pool.empty()) {
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
  }
  hipEvent_t e = ctx->prof_pool.back();
  ctx->prof_pool.pop_back();
  return e;
}

int prof_id(dbl_ctx* ctx, const char* name) {
  for (size_t i = 0; i < ctx->prof_names.size(); ++i)
    if (ctx->prof_names[i] == name) return (int)i;
  ctx->prof_names.push_back(name);
  ctx->prof_launches.push_back(0);
  ctx->prof_ms.push_back(0.0);
  ctx->prof_bytes.push_back(0.0);
  return (int)ctx->prof_names.size() - 1;
}

int prof_collect(dbl_ctx* ctx) {
  if (ctx->prof_pending.empty()) return DBL_OK;
  int rc = hip_check(ctx, hipStreamSynchronize(ctx->stream), "profile sync");
  if (rc) return rc;
  for (auto& p : ctx->prof_pending) {
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, p.a, p.b);
    ctx->prof_launches[p.id] += 1;
    ctx->prof_ms[p.id] += ms;
    ctx->prof_bytes[p.id] += p.bytes;
    ctx->prof_pool.push_back(p.a);
    ctx->prof_pool.push_back(p.b);
  }
  ctx->prof_pending.clear();
  return DBL_OK;
}

double job_bytes(const char* k, const Job& j, int prec) {
  const double n = (double)j.m * j.m, nl = 2.0 * j.m * (j.m - 1);
  const bool irls = j.flags & F_IRLS;
  const double e = prec == DBL_F64 ? 8.0 : 4.0;                            // x, b, w, c
  const double v = prec == DBL_F64 ? 8.0 : (prec == DBL_BF16 ? 2.0 : 4.0);  // CGLS state
  const double wb = irls ? nl * e : 0.0;
  const std::string s(k);
  // each operand read or written once.  The CGLS phases count the fused
  // minimum of an iteration (q = A^ p is not an operand: a fully fused
  // iteration recomputes it), so the bytes these kernels move beyond it (the
  // q1, q2 round trip and re-read halos) show up against this figure in the
  // memory counters, not in it.
  if (s == "cgls_p1") return 3 * n * v + wb;                          // s, p in; p out
  if (s == "cgls_p2") return (4 * n + 2 * nl) * v + 2 * n * e + wb;   // p in; x, r1, r2 in+out; s out
  if (s == "cgls_init" || s == "lsqr_init") return (2 * n + nl) * v + (2 * n + nl) * e;
  if (s == "lsqr_a") return (5 * n + 2 * nl) * v + 2 * n * e + wb;  // v,u,w in; u,w out; x
  if (s == "lsqr_b") return (3 * n + nl) * v + wb;                  // u, v in; v out
  if (s == "lsqr_fin") return n * v + 2 * n * e;                    // w in; x in and out
  if (s == "cgls_small")  // b, c, w in, x out; then the tiled phases' figure per iteration
    return (2 * n + 2 * nl) * e + j.i0 * ((7 * n + 2 * nl) * v + 2 * n * e + 2 * wb);
  double el = 0.0;  // elements of x, b, w, c moved
  if (s == "apply_A") el = 2 * n;
  else if (s == "apply_L" || s == "apply_LT") el = n + nl;
  else if (s == "restrict" || s == "prolong" || s == "dwt_fwd" || s == "dwt_inv")
    el = 1.25 * n;  // m x m <-> (m/2)^2 (m = fine)
  else if (s == "dtransfer") el = 1.25 * nl;  // coarse n_L in, fine n_L out
  else if (s == "dwt_fwd4" || s == "dwt_inv4") el = 2 * n;
  else if (s == "stats") el = 3 * n;
  else if (s == "aux") el = n + 2 * nl;
  return el * e;
}

// Tiles per axis of a launch over an m x m grid.  Image, gradient and GCV
// kernels use tile_edge(m) tiles (esz 4 or 8); esz 0 selects the 64 x 64
// output tiles of the FP64 GEMM.
int tiles_per_axis(int grid_m, int esz) {
  const int ts = esz == 0 ? 64 : tile_edge(grid_m);
  return grid_m < ts ? 1 : grid_m / ts;
}

size_t part_doubles(int m) {
  const size_t t4 = (size_t)tiles_per_axis(m, 4), t8 = (size_t)tiles_per_axis(m, 8);
  return 9 * t8 * t8 + (6 + 2 * DBL_GCV_GRID_MAX + 2) * t4 * t4 + 64;
}

PartLayout part_layout(double* base, int m) {
  const size_t t4 = (size_t)tiles_per_axis(m, 4), t8 = (size_t)tiles_per_axis(m, 8);
  const size_t nt = t8 * t8, ng = t4 * t4;  // nt bounds the tile count of either precision
  PartLayout L;
  double* p = base;
  L.q = p; p += nt;
  L.s[0] = p; p += 2 * nt;
  L.s[1] = p; p += 2 * nt;
  L.st = p; p += 4 * nt;
  L.gw = p; p += 2 * ng;
  L.gmm = p; p += 2 * ng;
  L.ggrid = p; p += 2 * DBL_GCV_GRID_MAX * ng;
  L.gb[0] = p; p += 2 * ng;
  L.gb[1] = p; p += 2 * ng;
  return L;
}

void Launch::add(const Job& j0, int grid_m, int esz, int group) {
  const int t = tiles_per_axis(grid_m, esz);
  add_grid(j0, t, t, group);
}

void Launch::add_grid(const Job& j0, int nti, int ntj, int group) {
  Job j = j0;
  j.nti = nti;
  j.ntj = ntj;
  const uint32_t idx = (uint32_t)jobs.size();
  if (jobs.empty() || group != last_group) seg_start.push_back((int)tiles.size());
  last_group = group;
  jobs.push_back(j);
  for (int t = 0; t < j.nti * j.ntj; ++t) tiles.push_back((idx << 16) | (uint32_t)t);
  tiles_upto.push_back((int)tiles.size());
  m_max = std::max(m_max, j.m);
  m_min = std::min(m_min, j.m);
}

void add_prolong(Launch& L, const Job& j, int esz) {
  if (j.m >= 64)
    L.add_grid(j, j.m / 32, j.m / 64);
  else
    L.add(j, j.m, esz);
}

void xcd_order(std::vector<uint32_t>& tiles, size_t s0, size_t s1, int nxcd) {
  const size_t n = s1 - s0;
  if (n < 2 || nxcd < 2) return;
  std::vector<uint32_t> run(tiles.begin() + s0, tiles.begin() + s1);
  // chunk start of each XCD: positions p in [s0, s1) with p % nxcd == x
  std::vector<size_t> cnt(nxcd, 0), next(nxcd, 0);
  for (size_t p = s0; p < s1; ++p) ++cnt[p % nxcd];
  size_t acc = 0;
  for (int x = 0; x < nxcd; ++x) {
    next[x] = acc;
    acc += cnt[x];
  }
  for (size_t p = s0; p < s1; ++p) tiles[p] = run[next[p % nxcd]++];
}

size_t Launch::pack(std::vector<char>& buf) const {
  std::vector<uint32_t> order = tiles;
  for (size_t q = 0; q < seg_start.size(); ++q) {
    const size_t s1 = q + 1 < seg_start.size() ? (size_t)seg_start[q + 1] : order.size();
    xcd_order(order, (size_t)seg_start[q], s1, XCDS);
  }
  const size_t oj = (buf.size() + 255) & ~size_t(255);
  const size_t nj = jobs.size() * sizeof(Job);
  const size_t ot = (oj + nj + 255) & ~size_t(255);
  buf.resize(ot + order.size() * sizeof(uint32_t), 0);
  std::memcpy(buf.data() + oj, jobs.data(), nj);
  std::memcpy(buf.data() + ot, order.data(), order.size() * sizeof(uint32_t));
  return oj;
}

void Launch::bind(const dbl_ctx* ctx, char* d, size_t off, LaunchArgs& la) const {
  const size_t ot = (off + jobs.size() * sizeof(Job) + 255) & ~size_t(255);
  la.jobs = reinterpret_cast<const Job*>(d + off);
  la.tiles = reinterpret_cast<const uint32_t*>(d + ot);
  la.ntiles = (int)tiles.size();
  la.m_max = m_max;
  la.stream = ctx->stream;
  la.tile32 = ctx->tile32 && m_min >= 32;
}

int Launch::upload(dbl_ctx* ctx, LaunchArgs& la) {
  std::vector<char> buf;
  const size_t off = pack(buf);
  void* d = nullptr;
  int rc = stage(ctx, buf.data(), buf.size(), &d);
  if (rc) return rc;
  bind(ctx, static_cast<char*>(d), off, la);
  return DBL_OK;
}

int upload_all(dbl_ctx* ctx, const std::vector<std::pair<const Launch*, LaunchArgs*>>& ls) {
  std::vector<char> buf;
  std::vector<size_t> offs;
  for (auto& l : ls) offs.push_back(l.first->pack(buf));
  if (buf.empty()) return DBL_OK;
  void* d = nullptr;
  int rc = stage(ctx, buf.data(), buf.size(), &d);
  if (rc) return rc;
  for (size_t q = 0; q < ls.size(); ++q)
    ls[q].first->bind(ctx, static_cast<char*>(d), offs[q], *ls[q].second);
  return DBL_OK;
}

// ----------------------------------------------------------- operators ----

namespace {

// Host image of an operator's device allocation.  Arrays are appended at
// 256-byte offsets; pointer fields of the level structures hold offset + 1
// (0 = no array) until the allocation exists, then fix() turns them into
// device addresses.
struct Blob {
  std::vector<char> bytes;
  size_t put(const void* src, size_t n) {
    const size_t off = (bytes.size() + 255) & ~size_t(255);
    bytes.resize(off + std::max<size_t>(n, 1), 0);
    if (src && n) std::memcpy(bytes.data() + off, src, n);
    return off;
  }
  template <typename T> T* ref(const std::vector<T>& v) {
    return reinterpret_cast<T*>(put(v.data(), v.size() * sizeof(T)) + 1);
  }
};

template <typename T> void fix(T*& p, char* base) {
  if (p) p = reinterpret_cast<T*>(base + (reinterpret_cast<uintptr_t>(p) - 1));
}

void put_t1(Blob& B, const Table1DHost& h, Table1D& d) {
  d.R = h.R;
  d.St = h.St;
  d.Sb = h.Sb;
  d.rows = h.rows;
  const std::vector<float> f(h.taps.begin(), h.taps.end());
  d.tf = B.ref(f);
  d.td = B.ref(h.taps);
}

void put_t2(Blob& B, const Table2DHost& h, Table2D& d) {
  d.R0 = h.R0;
  d.R1 = h.R1;
  d.St0 = h.St0;
  d.Sb0 = h.Sb0;
  d.St1 = h.St1;
  d.Sb1 = h.Sb1;
  d.rows0 = h.rows0;
  d.rows1 = h.rows1;
  std::vector<short2> e(h.val.size());
  for (size_t k = 0; k < e.size(); ++k) e[k] = make_short2(h.e0[k], h.e1[k]);
  const std::vector<float> f(h.val.begin(), h.val.end());
  d.off = B.ref(h.off);
  d.e = B.ref(e);
  d.vf = B.ref(f);
  d.vd = B.ref(h.val);
}

void fix_level(LevelOp& d, char* base) {
  Table1D* t1[4] = {&d.f0, &d.f1, &d.a0, &d.a1};
  for (Table1D* t : t1) {
    fix(t->tf, base);
    fix(t->td, base);
  }
  Table2D* t2[2] = {&d.f2, &d.a2};
  for (Table2D* t : t2) {
    fix(t->off, base);
    fix(t->e, base);
    fix(t->vf, base);
    fix(t->vd, base);
  }
}

}  // namespace

void op_free(dbl_op* op) {
  if (!op) return;
  if (op->blob) dfree(op->ctx, op->blob);
  if (op->sym_blk) dfree(op->ctx, op->sym_blk);
  delete op;
}

int op_build(dbl_ctx* ctx, const double* psf, int ph, int pw, int m, int levels, int wavelet,
             int precision, dbl_op** out) {
  *out = nullptr;
  dbl_op* op = new dbl_op();
  op->ctx = ctx;
  op->m = m;
  op->levels = levels;
  op->wavelet = wavelet;
  op->precision = precision;
  try {
    build_hierarchy(psf, ph, pw, m, levels, wavelet, op->host);
  } catch (const std::exception& ex) {
    delete op;
    return set_err(ctx, DBL_ENOTSUP, std::string("hierarchy: ") + ex.what());
  }
  op->sep = op->host.sep;
  Blob B;
  std::vector<LevelOp> lv(levels);
  for (int i = 0; i < levels; ++i) {
    const LevelHost& L = op->host.levels[i];
    LevelOp& d = lv[i];
    std::memset(&d, 0, sizeof(d));
    d.m = L.m;
    d.sep = L.sep ? 1 : 0;
    d.rb = L.rb;
    d.R = L.sep ? L.rb : L.R;
    if (L.sep) {
      put_t1(B, L.f0, d.f0);
      put_t1(B, L.f1, d.f1);
      put_t1(B, L.a0, d.a0);
      put_t1(B, L.a1, d.a1);
    } else {
      put_t2(B, L.f2, d.f2);
      put_t2(B, L.a2, d.a2);
    }
  }
  // padded variants for the larger radius buckets of separable levels
  std::vector<LevelOp> pad((size_t)levels * NBUCKETS);
  std::memset(pad.data(), 0, pad.size() * sizeof(LevelOp));
  for (int i = 0; i < levels; ++i) {
    const LevelHost& L = op->host.levels[i];
    if (!L.sep) continue;
    for (int k = 0; k < NBUCKETS; ++k) {
      const int b = RB_BUCKETS[k];
      if (b < L.rb) continue;
      LevelOp& d = pad[(size_t)i * NBUCKETS + k];
      d = lv[i];
      if (b == L.rb) continue;
      d.rb = b;
      d.R = b;
      Table1DHost t[4] = {L.f0, L.f1, L.a0, L.a1};
      Table1D* dt[4] = {&d.f0, &d.f1, &d.a0, &d.a1};
      for (int q = 0; q < 4; ++q) {
        pad_table(t[q], b);
        put_t1(B, t[q], *dt[q]);
      }
    }
  }
  // GCV symbol inputs per level: l(k) = 4 sin^2(pi k / 2m), then the
  // interior kernel
  std::vector<size_t> lam_off(levels);
  for (int i = 0; i < levels; ++i) {
    const LevelHost& L = op->host.levels[i];
    std::vector<double> h(L.m + L.kint.size());
    for (int k = 0; k < L.m; ++k) {
      const double s = std::sin(M_PI * k / (2.0 * L.m));
      h[k] = 4.0 * s * s;
    }
    std::memcpy(h.data() + L.m, L.kint.data(), L.kint.size() * 8);
    lam_off[i] = B.put(h.data(), h.size() * 8);
  }
  const size_t ops_off = B.put(nullptr, sizeof(LevelOp) * lv.size());
  const size_t pad_off = B.put(nullptr, sizeof(LevelOp) * pad.size());
  int rc = dmalloc(ctx, B.bytes.size(), &op->blob);
  if (rc) {
    delete op;
    return rc;
  }
  char* base = static_cast<char*>(op->blob);
  for (LevelOp& d : lv) fix_level(d, base);
  for (LevelOp& d : pad) fix_level(d, base);
  std::memcpy(B.bytes.data() + ops_off, lv.data(), sizeof(LevelOp) * lv.size());
  std::memcpy(B.bytes.data() + pad_off, pad.data(), sizeof(LevelOp) * pad.size());
  op->d_ops = reinterpret_cast<LevelOp*>(base + ops_off);
  op->d_pad = reinterpret_cast<LevelOp*>(base + pad_off);
  op->lam.resize(levels);
  for (int i = 0; i < levels; ++i) op->lam[i] = reinterpret_cast<double*>(base + lam_off[i]);
  op->sym.assign(levels, nullptr);
  op->sym_ready.assign(levels, 0);
  // one asynchronous copy through the staging ring
  void* staged = nullptr;
  rc = stage(ctx, B.bytes.data(), B.bytes.size(), &staged);
  if (!rc)
    rc = hip_check(ctx, hipMemcpyAsync(op->blob, staged, B.bytes.size(), hipMemcpyDeviceToDevice,
                                       ctx->stream),
                   "upload operator");
  if (rc) {
    op_free(op);
    return rc;
  }
  *out = op;
  return DBL_OK;
}

static std::string op_key(const double* psf, int ph, int pw, int m, int levels, int wavelet,
                          int precision) {
  std::string k;
  const int hdr[6] = {ph, pw, m, levels, wavelet, precision};
  k.append(reinterpret_cast<const char*>(hdr), sizeof(hdr));
  k.append(reinterpret_cast<const char*>(psf), sizeof(double) * (size_t)ph * pw);
  return k;
}

int op_acquire(dbl_ctx* ctx, const double* psf, int ph, int pw, int m, int levels, int wavelet,
               int precision, dbl_op** out) {
  const std::string key = op_key(psf, ph, pw, m, levels, wavelet, precision);
  auto it = ctx->op_cache.find(key);
  if (it != ctx->op_cache.end()) {
    it->second.refs += 1;
    it->second.last = ++ctx->op_clock;
    *out = it->second.op;
    return DBL_OK;
  }
  const size_t kMaxIdle = 64;
  if (ctx->op_cache.size() >= kMaxIdle) {
    // evict idle entries, oldest first, down to half the bound
    std::vector<std::pair<unsigned long long, std::string>> idle;
    for (auto& kv : ctx->op_cache)
      if (kv.second.refs == 0) idle.push_back({kv.second.last, kv.first});
    std::sort(idle.begin(), idle.end());
    for (size_t q = 0; q < idle.size() && ctx->op_cache.size() >= kMaxIdle / 2; ++q) {
      (void)hipStreamSynchronize(ctx->stream);
      op_free(ctx->op_cache[idle[q].second].op);
      ctx->op_cache.erase(idle[q].second);
    }
  }
  dbl_op* op = nullptr;
  int rc = op_build(ctx, psf, ph, pw, m, levels, wavelet, precision, &op);
  if (rc) return rc;
  ctx->op_cache[key] = {op, 1, ++ctx->op_clock};
  *out = op;
  return DBL_OK;
}

void op_release(dbl_ctx* ctx, dbl_op* op) {
  for (auto& kv : ctx->op_cache)
    if (kv.second.op == op) {
      kv.second.refs -= 1;
      return;
    }
}

void op_cache_clear(dbl_ctx* ctx) {
  for (auto& kv : ctx->op_cache) op_free(kv.second.op);
  ctx->op_cache.clear();
}

// --------------------------------------------------------------- slots ----

static size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

static bool wants_gcv(const dbl_opts& o) { return !o.mu_schedule && !(o.mu_fixed > 0.0); }

size_t slot_bytes(const dbl_request& req) {
  const size_t esz = req.opts.precision == DBL_F64 ? 8 : 4;
  const size_t ssz = req.opts.precision == DBL_BF16 ? 2 : esz;  // CGLS state vectors
  const size_t n = (size_t)req.m * req.m, nl = 2 * (size_t)req.m * (req.m - 1);
  size_t b = 0;
  b += 2 * align256(n * esz) + 6 * align256(n * ssz);   // x x2; p x2, s, r1 x2, q1
  // w, c1, c2 and r2 x2 (full width: Approach D transfers w / c into r2's
  // buffers and swaps them with the originals); q2
  b += 5 * align256(nl * esz) + align256(nl * ssz);
  for (int i = 1; i < req.levels; ++i) b += align256(((size_t)req.m >> i) * (req.m >> i) * esz);
  b += align256(NSCAL * 8) + align256(part_doubles(req.m) * 8);
  b += align256((size_t)req.levels * DBL_MAX_KOUT * 3 * 8);
  if (wants_gcv(req.opts)) b += 4 * align256(n * 8);
  return b;
}

int slot_init(dbl_ctx* ctx, const dbl_request& req, Slot* s) {
  s->req = req;
  s->opts = req.opts;
  s->prec = req.opts.precision;
  s->esz = s->prec == DBL_F64 ? 8 : 4;
  s->m = req.m;
  s->levels = req.levels;
  s->solver = req.solver;
  s->wavelet = req.wavelet;
  s->transfer = req.transfer;
  s->n0 = req.m * req.m;
  s->nl0 = 2 * req.m * (req.m - 1);
  s->gcv = wants_gcv(req.opts);
  const int K = req.opts.k_out;
  if (!s->gcv) {
    s->mu.assign((size_t)req.levels * K, req.opts.mu_fixed);
    if (req.opts.mu_schedule)
      for (size_t i = 0; i < s->mu.size(); ++i) s->mu[i] = req.opts.mu_schedule[i];
  }
  int rc = op_acquire(ctx, req.psf, req.ph, req.pw, req.m, req.levels, req.wavelet, s->prec,
                      &s->op);
  if (rc) return rc;
  const size_t bytes = slot_bytes(req);
  rc = pool_get(ctx, bytes, &s->block);
  if (rc) {
    op_release(ctx, s->op);
    s->op = nullptr;
    return rc;
  }
  char* p = static_cast<char*>(s->block);
  auto take = [&](size_t b) {
    void* r = p;
    p += align256(b);
    return r;
  };
  const size_t n = s->n0, nl = s->nl0, e = s->esz;
  const size_t v = s->prec == DBL_BF16 ? 2 : e;  // CGLS state vectors
  s->X[0] = take(n * e);
  s->X[1] = take(n * e);
  s->P[0] = take(n * v);
  s->P[1] = take(n * v);
  s->S = take(n * v);
  s->R1[0] = take(n * v);
  s->R1[1] = take(n * v);
  s->Q1 = take(n * v);
  s->R2[0] = take(nl * e);  // full width: Approach D swaps these with W / C1 / C2
  s->R2[1] = take(nl * e);
  s->Q2 = take(nl * v);
  s->W = take(nl * e);
  s->C1 = take(nl * e);
  s->C2 = take(nl * e);
  s->B.assign(req.levels, nullptr);
  s->B[0] = req.b;
  for (int i = 1; i < req.levels; ++i) s->B[i] = take(((size_t)req.m >> i) * (req.m >> i) * e);
  s->scal = static_cast<double*>(take(NSCAL * 8));
  s->part = static_cast<double*>(take(part_doubles(req.m) * 8));
  s->hist = static_cast<double*>(take((size_t)req.levels * DBL_MAX_KOUT * 3 * 8));
  if (s->gcv) {
    s->g_bh = static_cast<double*>(take(n * 8));
    s->g_e = static_cast<double*>(take(n * 8));
    s->g_tmp = static_cast<double*>(take(n * 8));
    s->g_in = static_cast<double*>(take(n * 8));
  }
  rc = hip_check(ctx, hipMemsetAsync(s->scal, 0, NSCAL * 8, ctx->stream), "clear scalars");
  if (!rc)
    rc = hip_check(ctx, hipMemsetAsync(s->hist, 0xff, (size_t)req.levels * DBL_MAX_KOUT * 3 * 8,
                                       ctx->stream),
                   "clear history");
  s->level = req.levels - 1;
  s->k = 0;
  s->cur = 0;
  for (int& it : s->iters) it = 0;
  s->rc_idx = -1;
  s->started = false;
  s->done = false;
  return rc;
}

void slot_free(dbl_ctx* ctx, Slot* s) {
  if (s->block) pool_put(ctx, s->block, slot_bytes(s->req));
  s->block = nullptr;
  if (s->op) op_release(ctx, s->op);
  s->op = nullptr;
}

int slot_report(dbl_ctx* ctx, Slot* s, dbl_report* rep) {
  if (!rep) return DBL_OK;
  std::vector<double> h((size_t)s->levels * DBL_MAX_KOUT * 3);
  int rc = hip_check(ctx, hipMemcpyAsync(h.data(), s->hist, h.size() * 8, hipMemcpyDeviceToHost,
                                         ctx->stream),
                     "read history");
  if (!rc) rc = hip_check(ctx, hipStreamSynchronize(ctx->stream), "sync");
  if (rc) return rc;
  rep->levels = s->levels;
  rep->k_out = s->opts.k_out;
  for (int i = 0; i < DBL_MAX_LEVELS; ++i) rep->sizes[i] = i < s->levels ? (s->m >> i) : 0;
  for (int i = 0; i < s->levels; ++i)
    for (int k = 0; k < s->opts.k_out; ++k) {
      const double* e = &h[((size_t)i * DBL_MAX_KOUT + k) * 3];
      rep->gamma[i][k] = e[0];
      rep->rc[i][k] = e[1];
      rep->objective[i][k] = e[2];
    }
  rep->status = s->status;
  for (int i = 0; i < DBL_MAX_LEVELS; ++i) rep->iters[i] = i < s->levels ? s->iters[i] : 0;
  return DBL_OK;
}

const LevelOp* op_dev(const dbl_op* op, int level, int rb) {
  const LevelHost& L = op->host.levels[level];
  if (!L.sep || rb == L.rb) return op->d_ops + level;
  return op->d_pad + (size_t)level * NBUCKETS + bucket_index(rb);
}

size_t small_lds_bytes(const dbl_ctx* ctx, const dbl_op* op, int level, bool irls, int* wlds) {
  *wlds = 0;
  if (!ctx->small_cgls) return 0;
  const LevelHost& L = op->host.levels[level];
  if (!L.sep) return small_cgls_lds(L.m, op->precision, small_halo(L), 0, irls, ctx->lds_limit,
                                    wlds, true);
  const int rows = L.f0.rows + L.f1.rows + L.a0.rows + L.a1.rows;
  return small_cgls_lds(L.m, op->precision, L.rb, rows, irls, ctx->lds_limit, wlds);
}

int small_halo(const LevelHost& L) { return L.sep ? L.rb : bucket_above(L.R); }

// -------------------------------------------------------------- engine ----

namespace {

struct GroupKey {
  int prec, sep, rb, H;
  // CGLS phases: jobs on grids of at least 32 (the 32 x 32 tile kernels)
  // launch apart from smaller ones, so a job's kernel depends on its own
  // grid alone, never on which jobs share its launch
  int t32 = 0;
  // CGLS phases: jobs of several radius buckets, each with tables padded to
  // its own bucket, share the launch; rb is the largest of them
  int multi = 0;
  bool operator<(const GroupKey& o) const {
    if (prec != o.prec) return prec < o.prec;
    if (sep != o.sep) return sep < o.sep;
    if (rb != o.rb) return rb < o.rb;
    if (H != o.H) return H < o.H;
    if (t32 != o.t32) return t32 < o.t32;
    return multi < o.multi;
  }
};

Job base_job(const Slot* s, int level) {
  Job j;
  std::memset(&j, 0, sizeof(j));
  j.m = s->m >> level;
  j.op = s->op->d_ops + level;
  j.scal = s->scal;
  j.part = s->part;
  j.hist = s->hist;
  return j;
}

// A general operator's group is keyed by the radius bucket above its radius:
// its tile kernels take that bucket as their halo, and the generic kernels
// lay each job out by the job's own radius (the launch's H only sizes the
// LDS), so operators of different radii in one bucket share launches and
// every job computes what it computes alone.
GroupKey key_of(const Slot* s, int level) {
  const LevelHost& L = s->op->host.levels[level];
  const int hb = bucket_above(L.R);
  return GroupKey{s->prec, L.sep ? 1 : 0, L.sep ? L.rb : 0, L.sep ? L.rb : (hb > 0 ? hb : L.R)};
}

// RC tolerance of the slot's current level (0: fixed outer count).
double level_tol(const Slot* s) {
  return s->level == 0 ? s->opts.tol_fine : s->opts.tol_coarse;
}

int solver_flags(const Slot* s) {
  if (s->solver == DBL_IRLS) return F_IRLS;
  if (s->solver == DBL_MM) return F_SHIFT | F_MM;
  return F_SHIFT | F_SB;
}

// Launch groups of the CGLS stage.  Jobs share a launch when they have the
// same precision and kind of operator and their tables are padded to the
// same radius bucket.  A group that cannot fill the chip on its own (fewer
// than MERGE_TILES tiles, or one-block jobs of one level size) is latency
// bound, so it joins the next larger bucket: its jobs run with their tables
// zero-padded to that bucket (the same operator, a few more multiply-adds).
// With `multi`, separable levels on the 32 x 32 tile kernels instead share
// mixed launches (kernels_cgls_multi.hip) in which every job keeps its own
// bucket: buckets up to 8 always (their kernels run at one occupancy), and
// bucket 12 too when it has fewer than ctx->multi_tiles tiles, too few to
// keep the chip busy in a launch of its own.  General levels on the tile
// kernels mix their buckets (the bucket above each operator's radius) by
// the same rule, in launches of their own.
struct GroupPlan {
  struct Entry {
    GroupKey key;       // the launch group (rb = the bucket the tables are padded to)
    size_t small_lds;   // > 0: one-block CGLS with this much LDS
    int wlds;           // one-block CGLS stages the IRLS weights in LDS
    int tab_rb = 0;     // > 0: the bucket of the job's tables in a mixed launch
    int tables() const { return tab_rb ? tab_rb : key.rb; }
  };
  std::map<const Slot*, Entry> e;
  const Entry& at(const Slot* s) const { return e.at(s); }
};

constexpr int MERGE_TILES = 256;

// One CGLS phase launch of a group (general operators in mixed-bucket
// groups take their own kernels).
hipError_t cgls_phase(const LaunchArgs& la, int phase, const GroupKey& g) {
  if (g.multi && !g.sep) return launch_cgls_gen_multi(la, phase, g.prec, g.H);
  return phase == 1 ? launch_cgls_p1(la, g.prec, g.sep, g.rb, g.H)
                    : launch_cgls_p2(la, g.prec, g.sep, g.rb, g.H);
}

GroupPlan plan_groups(dbl_ctx* ctx, const std::vector<Slot*>& slots, bool allow_small = true,
                      bool multi = false) {
  GroupPlan P;
  // one-block candidates by (precision, m): one bucket for all when every
  // member still fits in LDS with it
  std::map<std::tuple<int, int, int>, std::vector<const Slot*>> small;  // (prec, m, sep)
  std::map<GroupKey, std::vector<const Slot*>> tiled;
  // mixed-launch candidates by (precision, separable)
  std::map<std::pair<int, int>, std::vector<const Slot*>> mixed;
  multi = multi && ctx->multi_tiles >= 0 && ctx->tile32;
  for (const Slot* s : slots) {
    const int lv = s->level;
    const LevelHost& L = s->op->host.levels[lv];
    GroupPlan::Entry en{key_of(s, lv), 0, 0};
    if (allow_small)
      en.small_lds = small_lds_bytes(ctx, s->op, lv, s->solver == DBL_IRLS, &en.wlds);
    P.e[s] = en;
    if (en.small_lds) small[{s->prec, L.m, L.sep ? 1 : 0}].push_back(s);
    else if (multi && L.sep && L.m >= 32 && L.rb <= 12) mixed[{s->prec, 1}].push_back(s);
    else if (multi && !L.sep && L.m >= 32 && bucket_above(L.R) > 0 && bucket_above(L.R) <= 12)
      mixed[{s->prec, 0}].push_back(s);
    else tiled[en.key].push_back(s);
  }
  for (auto& kv : mixed) {
    const bool sepg = kv.first.second != 0;
    auto bucket = [&](const Slot* s) {
      const LevelHost& L = s->op->host.levels[s->level];
      return sepg ? L.rb : bucket_above(L.R);
    };
    std::map<int, size_t> per;  // tiles by bucket
    for (const Slot* s : kv.second) {
      const int mi = s->m >> s->level, t = mi / 32;
      per[bucket(s)] += (size_t)t * t;
    }
    // the buckets that share the launch
    auto joins = [&](int rb) { return rb <= 8 || per[rb] < (size_t)ctx->multi_tiles; };
    int top = 0, nb = 0;
    for (auto& b : per)
      if (joins(b.first)) {
        top = std::max(top, b.first);
        ++nb;
      }
    for (const Slot* s : kv.second) {
      const int rb = bucket(s);
      GroupPlan::Entry& en = P.e[s];
      if (nb < 2 || !joins(rb) || !(sepg ? cgls_multi_bucket(top) : cgls_gen_multi_bucket(top))) {
        tiled[en.key].push_back(s);  // a launch of its own bucket
        continue;
      }
      en.key.t32 = 1;
      en.key.multi = 1;
      if (sepg) {
        en.key.rb = en.key.H = top;
        en.tab_rb = rb;
      } else {
        en.key.H = top;  // general tables are not padded: rb stays 0
      }
    }
  }
  for (auto& kv : small) {
    const bool gen = std::get<2>(kv.first) == 0;
    int rbt = 0;
    for (const Slot* s : kv.second) rbt = std::max(rbt, small_halo(s->op->host.levels[s->level]));
    std::vector<std::pair<size_t, int>> got;
    bool ok = true;
    for (const Slot* s : kv.second) {
      const LevelHost& L = s->op->host.levels[s->level];
      int wl = 0;
      const size_t b =
          small_cgls_lds(L.m, s->prec, rbt, L.f0.rows + L.f1.rows + L.a0.rows + L.a1.rows,
                         s->solver == DBL_IRLS, ctx->lds_limit, &wl, gen);
      if (!b) ok = false;
      got.push_back({b, wl});
    }
    if (!ok) continue;
    for (size_t q = 0; q < kv.second.size(); ++q) {
      GroupPlan::Entry& en = P.e[kv.second[q]];
      en.key.rb = en.key.H = rbt;
      en.small_lds = got[q].first;
      en.wlds = got[q].second;
    }
  }
  // tiled groups: separable groups below MERGE_TILES tiles join the next
  // larger bucket of the same precision (cascading upward)
  std::map<GroupKey, size_t> tiles;
  for (auto& kv : tiled)
    for (const Slot* s : kv.second) {
      const int t = tiles_per_axis(s->m >> s->level, (int)s->esz);
      tiles[kv.first] += (size_t)t * t;
    }
  std::vector<GroupKey> keys;
  for (auto& kv : tiles) keys.push_back(kv.first);  // ordered by (prec, sep, rb)
  std::map<GroupKey, GroupKey> target;
  for (size_t q = 0; q < keys.size(); ++q) target[keys[q]] = keys[q];
  for (size_t q = 0; q + 1 < keys.size(); ++q) {
    const GroupKey& a = keys[q];
    const GroupKey& b = keys[q + 1];
    if (!a.sep || a.prec != b.prec || a.sep != b.sep || tiles[a] >= (size_t)MERGE_TILES) continue;
    tiles[b] += tiles[a];
    for (auto& t : target)
      if (!(t.second < a) && !(a < t.second)) t.second = b;
  }
  for (auto& kv : tiled)
    for (const Slot* s : kv.second) P.e[s].key = target[kv.first];
  return P;
}

// Launch helpers: one launch per precision for simple kernels.
using SimpleFn = hipError_t (*)(const LaunchArgs&, int);

int run_simple(dbl_ctx* ctx, SimpleFn fn, std::map<int, Launch>& byprec, const char* what) {
  for (auto& kv : byprec) {
    if (kv.second.empty()) continue;
    LaunchArgs la;
    int rc = kv.second.upload(ctx, la);
    if (rc) return rc;
    double b = 0.0;
    for (const Job& jj : kv.second.jobs) b += job_bytes(what, jj, kv.first);
    rc = hip_check(ctx, timed(ctx, what, b, [&] { return fn(la, kv.first); }), what);
    if (rc) return rc;
  }
  return DBL_OK;
}

// LSQR on the subproblems of the slots in `lq` (Sec. 3): per slot, init,
// then B_i and A_i for i = 1..k_in and the finishing update, all tiled
// (kernels_lsqr.hip), batched across slots like the CGLS phases.  Slots are
// ordered by decreasing k_in so that each iteration launches a prefix.
int run_lsqr(dbl_ctx* ctx, std::vector<Slot*> lq) {
  if (lq.empty()) return DBL_OK;
  int rc = DBL_OK;
  std::stable_sort(lq.begin(), lq.end(),
                   [](const Slot* a, const Slot* b) { return a->opts.k_in > b->opts.k_in; });
  const GroupPlan plan = plan_groups(ctx, lq, false);
  std::map<int, Launch> initL;
  std::map<GroupKey, Launch> bF, aF, bP[2], aP[2];
  std::map<std::pair<GroupKey, int>, Launch> finL;  // by (group, k_in)
  std::map<GroupKey, std::vector<int>> kin;
  for (Slot* s : lq) {
    const int lv = s->level;
    const int mi = s->m >> lv;
    const PartLayout PL = part_layout(s->part, mi);
    const size_t nt = (size_t)tiles_per_axis(mi, (int)s->esz) * tiles_per_axis(mi, (int)s->esz);
    double* PA[2] = {PL.s[0], PL.s[0] + nt};  // |u|^2 partials by iteration parity
    double* PB[2] = {PL.s[1], PL.s[1] + nt};  // |v|^2 partials by iteration parity
    const GroupPlan::Entry& pe = plan.at(s);
    const GroupKey gk = pe.key;
    Job j = base_job(s, lv);
    j.op = op_dev(s->op, lv, gk.rb ? gk.rb : s->op->host.levels[lv].rb);
    j.flags = solver_flags(s);
    j.v[V_X] = s->X[1 - s->cur];
    j.v[V_PA] = s->P[0];   // w
    j.v[V_S] = s->S;       // v
    j.v[V_R1A] = s->R1[0];  // u (image part)
    j.v[V_R2A] = s->R2[0];  // u (gradient part)
    j.v[V_W] = s->W;
    j.v[V_B] = const_cast<void*>(s->B[lv]);
    j.v[V_C1] = s->C1;
    j.v[V_C2] = s->C2;
    Job ji = j;
    ji.pw = PA[0];
    initL[s->prec].add(ji, mi, (int)s->esz);
    for (int i = 1; i <= 3; ++i) {  // i = 1 (first), 2 and 3 (the two parities)
      Job jb = j;
      jb.i0 = i;
      if (i == 1) jb.flags |= F_FIRST;
      jb.pr[0] = PA[(i - 1) & 1];
      jb.pr[1] = PB[(i - 1) & 1];
      jb.pw = PB[i & 1];
      Job ja = j;
      ja.i0 = i;
      if (i == 1) ja.flags |= F_FIRST;
      ja.pr[0] = PB[i & 1];
      ja.pr[1] = PA[(i - 1) & 1];
      ja.pw = PA[i & 1];
      Launch& B = i == 1 ? bF[gk] : bP[i & 1][gk];
      Launch& A = i == 1 ? aF[gk] : aP[i & 1][gk];
      B.add(jb, mi, (int)s->esz, s->opts.k_in);
      A.add(ja, mi, (int)s->esz, s->opts.k_in);
    }
    Job jf = j;
    jf.i0 = s->opts.k_in;
    jf.pr[0] = PA[s->opts.k_in & 1];
    finL[{gk, s->opts.k_in}].add(jf, mi, (int)s->esz);
    kin[gk].push_back(s->opts.k_in);
  }
  if ((rc = run_simple(ctx, launch_lsqr_init, initL, "lsqr_init"))) return rc;
  std::map<GroupKey, LaunchArgs> lbF, laF, lbP[2], laP[2];
  for (auto& kv : kin) {
    const GroupKey& g = kv.first;
    if ((rc = bF[g].upload(ctx, lbF[g])) || (rc = aF[g].upload(ctx, laF[g]))) return rc;
    for (int par = 0; par < 2; ++par)
      if ((rc = bP[par][g].upload(ctx, lbP[par][g])) || (rc = aP[par][g].upload(ctx, laP[par][g])))
        return rc;
  }
  int kmax = 0;
  for (auto& kv : kin)
    for (int k : kv.second) kmax = std::max(kmax, k);
  for (int it = 1; it <= kmax; ++it) {
    const int par = it & 1;
    for (int phase = 0; phase < 2; ++phase) {  // B_it, then A_it
      for (auto& kv : kin) {
        const GroupKey& g = kv.first;
        const std::vector<int>& ks = kv.second;
        int q = 0;
        while (q < (int)ks.size() && ks[q] >= it) ++q;
        if (!q) continue;
        const Launch& src = phase == 0 ? (it == 1 ? bF[g] : bP[par][g])
                                       : (it == 1 ? aF[g] : aP[par][g]);
        LaunchArgs la = phase == 0 ? (it == 1 ? lbF[g] : lbP[par][g])
                                   : (it == 1 ? laF[g] : laP[par][g]);
        la.ntiles = src.tiles_upto[q - 1];
        const char* name = phase == 0 ? "lsqr_b" : "lsqr_a";
        double b = 0.0;
        for (int jq = 0; jq < q; ++jq) b += job_bytes(name, src.jobs[jq], g.prec);
        if ((rc = hip_check(ctx, timed(ctx, name, b, [&] {
                              return phase == 0 ? launch_lsqr_b(la, g.prec, g.sep, g.rb, g.H)
                                                : launch_lsqr_a(la, g.prec, g.sep, g.rb, g.H);
                            }),
                            name)))
          return rc;
      }
    }
    for (auto& kv : finL) {
      if (kv.first.second != it) continue;
      const GroupKey& g = kv.first.first;
      LaunchArgs la;
      if ((rc = kv.second.upload(ctx, la))) return rc;
      double b = 0.0;
      for (const Job& jj : kv.second.jobs) b += job_bytes("lsqr_fin", jj, g.prec);
      if ((rc = hip_check(ctx, timed(ctx, "lsqr_fin", b, [&] {
                            return launch_lsqr_fin(la, g.prec);
                          }),
                          "lsqr fin")))
        return rc;
    }
  }
  return DBL_OK;
}

void add_fill(std::map<int, Launch>& L, const Slot* s, int level, void* img, void* grad,
              double val) {
  Job j = base_job(s, level);
  j.v[0] = img;
  j.v[1] = grad;
  j.p0 = val;
  L[s->prec].add(j, j.m, (int)s->esz);
}

void add_aux(std::map<int, Launch>& L, const Slot* s, int level, int mode, const void* x,
             void* w, void* c1, void* c2) {
  Job j = base_job(s, level);
  j.i0 = mode;
  j.p0 = s->opts.eps;
  j.p1 = s->opts.tau;
  j.v[V_X] = const_cast<void*>(x);
  j.v[V_W] = w;
  j.v[V_C1] = c1;
  j.v[V_C2] = c2;
  L[s->prec].add(j, j.m, (int)s->esz);
}

}  // namespace

int engine_step(dbl_ctx* ctx, std::vector<Slot*>& slots) {
  int rc = stage_checkpoint(ctx);
  if (rc) return rc;
  std::vector<Slot*> act;
  for (Slot* s : slots)
    if (!s->done && !s->status) act.push_back(s);
  if (act.empty()) return DBL_OK;

  // ---- A. entering a level ------------------------------------------------
  {
    // restriction of b down the hierarchy (first step only), by depth
    int maxdepth = 0;
    for (Slot* s : act)
      if (!s->started) maxdepth = std::max(maxdepth, s->levels - 1);
    for (int d = 1; d <= maxdepth; ++d) {
      std::map<int, Launch> L;
      for (Slot* s : act) {
        if (s->started || d > s->levels - 1) continue;
        Job j = base_job(s, d - 1);
        j.m = s->m >> (d - 1);  // fine size
        j.flags = s->wavelet;
        j.v[0] = const_cast<void*>(s->B[d - 1]);
        j.v[1] = const_cast<void*>(s->B[d]);
        j.p0 = 0.0;
        L[s->prec].add(j, j.m >> 1, (int)s->esz);
      }
      if ((rc = run_simple(ctx, launch_dwt_fwd, L, "dwt_fwd"))) return rc;
    }
    std::map<int, Launch> fillL, prolL, auxL, finL, xferL;
    std::vector<Slot*> dslots;
    for (Slot* s : act) {
      if (s->k != 0) continue;
      const int lv = s->level;
      if (!s->started) {
        // Approach I start at the coarsest grid (Sec. 4.1)
        add_fill(fillL, s, lv, s->X[s->cur], nullptr, 0.0);
        if (s->solver == DBL_IRLS) add_fill(fillL, s, lv, nullptr, s->W, 1.0);
        if (s->solver == DBL_MM) add_fill(fillL, s, lv, nullptr, s->C1, 0.0);
        if (s->solver == DBL_SB) {
          add_fill(fillL, s, lv, nullptr, s->C1, 0.0);
          add_fill(fillL, s, lv, nullptr, s->C2, 0.0);
        }
      } else if (s->transfer == DBL_XFER_X) {
        // X^(i) = W1 X^(i+1) W1^T, then auxiliaries from it
        Job j = base_job(s, lv);
        j.flags = s->wavelet;
        j.v[0] = s->X[s->cur];
        j.v[1] = s->X[1 - s->cur];
        j.p0 = 0.0;
        add_prolong(prolL[s->prec], j, (int)s->esz);
      } else {
        // coarse auxiliary state from the completed coarse solve
        if (s->solver == DBL_IRLS)
          add_aux(finL, s, lv + 1, AUX_IRLS_W, s->X[s->cur], s->W, nullptr, nullptr);
        if (s->solver == DBL_MM)
          add_aux(finL, s, lv + 1, AUX_MM_W, s->X[s->cur], nullptr, s->C1, nullptr);
        dslots.push_back(s);
      }
    }
    if ((rc = run_simple(ctx, launch_fill, fillL, "fill"))) return rc;
    if ((rc = run_simple(ctx, launch_dwt_inv, prolL, "dwt_inv"))) return rc;
    if ((rc = run_simple(ctx, launch_aux, finL, "aux"))) return rc;
    for (Slot* s : act) {
      if (s->k != 0 || !s->started || s->transfer != DBL_XFER_X) continue;
      s->cur = 1 - s->cur;
      const int lv = s->level;
      if (s->solver == DBL_IRLS) add_aux(auxL, s, lv, AUX_IRLS_W, s->X[s->cur], s->W, nullptr, nullptr);
      if (s->solver == DBL_MM) add_aux(auxL, s, lv, AUX_MM_W, s->X[s->cur], nullptr, s->C1, nullptr);
      if (s->solver == DBL_SB) add_aux(auxL, s, lv, AUX_SB_INIT, s->X[s->cur], nullptr, s->C1, s->C2);
    }
    // Approach D: block transfer of the auxiliaries, then start from x = 0
    std::map<int, Launch> fillD;
    for (Slot* s : dslots) {
      const int lv = s->level;
      auto add_x = [&](void* src, void* dst) {
        Job j = base_job(s, lv);
        j.flags = s->wavelet;
        j.v[0] = src;
        j.v[1] = dst;
        xferL[s->prec].add(j, j.m, (int)s->esz);
      };
      if (s->solver == DBL_IRLS) add_x(s->W, s->R2[0]);
      if (s->solver == DBL_MM) add_x(s->C1, s->R2[0]);
      if (s->solver == DBL_SB) {
        add_x(s->C1, s->R2[0]);
        add_x(s->C2, s->R2[1]);
      }
      add_fill(fillD, s, lv, s->X[s->cur], nullptr, 0.0);
    }
    if ((rc = run_simple(ctx, launch_dtransfer, xferL, "dtransfer"))) return rc;
    for (Slot* s : dslots) {
      if (s->solver == DBL_IRLS) std::swap(s->W, s->R2[0]);
      if (s->solver == DBL_MM) std::swap(s->C1, s->R2[0]);
      if (s->solver == DBL_SB) {
        std::swap(s->C1, s->R2[0]);
        std::swap(s->C2, s->R2[1]);
      }
    }
    if ((rc = run_simple(ctx, launch_fill, fillD, "fill"))) return rc;
    if ((rc = run_simple(ctx, launch_aux, auxL, "aux"))) return rc;
    for (Slot* s : act) s->started = true;
  }

  // ---- B. auxiliaries from the current iterate (Algs. 1, 2) --------------
  {
    std::map<int, Launch> L;
    for (Slot* s : act) {
      if (s->k == 0) continue;
      if (s->solver == DBL_IRLS) add_aux(L, s, s->level, AUX_IRLS_W, s->X[s->cur], s->W, nullptr, nullptr);
      if (s->solver == DBL_MM) add_aux(L, s, s->level, AUX_MM_W, s->X[s->cur], nullptr, s->C1, nullptr);
    }
    if ((rc = run_simple(ctx, launch_aux, L, "aux"))) return rc;
  }

  // ---- C. the parameter gamma ----------------------------------------------
  {
    std::vector<GcvReq> greqs;
    Launch setg;  // fixed parameters: one launch writes gamma, sqrt(gamma) of every slot
    for (Slot* s : act) {
      if (!s->gcv) {
        const double g = s->mu[(size_t)s->level * s->opts.k_out + s->k];
        Job j = base_job(s, s->level);
        j.p0 = g;
        j.p1 = std::sqrt(g);
        setg.add(j, 1, 4);
        continue;
      }
      // GCV schedule (Sec. 3): MM / SB at k = 0, 1, 2; IRLS every k with at
      // most two grids, else two passes (unweighted at k = 0, weighted at k = 3).
      int which = 0;  // 0 none, 1 current pair, 2 unweighted pair
      if (s->solver != DBL_IRLS) which = s->k <= 2 ? 1 : 0;
      else if (s->levels <= 2) which = 1;
      else which = s->k == 0 ? 2 : (s->k == 3 ? 1 : 0);
      if (!which) continue;
      GcvReq g{};
      g.op = s->op;
      g.level = s->level;
      g.prec = s->prec;
      g.b = s->B[s->level];
      g.w = (s->solver == DBL_IRLS && which == 1) ? s->W : nullptr;
      g.c1 = s->solver != DBL_IRLS ? s->C1 : nullptr;
      g.c2 = s->solver == DBL_SB ? s->C2 : nullptr;
      g.scal = s->scal;
      g.part = s->part;
      g.bh = s->g_bh;
      g.e = s->g_e;
      g.tmp = s->g_tmp;
      g.in = s->g_in;
      g.bh_valid = s->bh_valid;
      g.grid = s->opts.gcv_grid;
      const int n = (s->m >> s->level) * (s->m >> s->level);
      g.mode = s->opts.gcv_mode != DBL_GCV_AUTO ? s->opts.gcv_mode
               : n <= DBL_GCV_AUTO_EXACT_N         ? DBL_GCV_EXACT
                                                   : DBL_GCV_SPECTRAL;
      greqs.push_back(g);
      s->bh_valid = g.mode == DBL_GCV_SPECTRAL;  // the exact tier reuses the DCT buffer
    }
    if (!setg.empty()) {
      LaunchArgs la;
      if ((rc = setg.upload(ctx, la))) return rc;
      if ((rc = hip_check(ctx, timed(ctx, "set_gamma", 0.0, [&] { return launch_set_gamma(la); }),
                          "set gamma")))
        return rc;
    }
    if (!greqs.empty() && (rc = gcv_run(ctx, greqs))) return rc;
  }

  // ---- D. CGLS (or LSQR) on the augmented system ---------------------------
  std::vector<Slot*> lq;
  for (Slot* s : act)
    if (s->opts.inner_solver == DBL_INNER_LSQR) lq.push_back(s);
  if ((rc = run_lsqr(ctx, lq))) return rc;
  {
    // order slots by decreasing k_in so every iteration launches a prefix
    std::vector<Slot*> ord;
    for (Slot* s : act)
      if (s->opts.inner_solver != DBL_INNER_LSQR) ord.push_back(s);
    std::stable_sort(ord.begin(), ord.end(),
                     [](const Slot* a, const Slot* b) { return a->opts.k_in > b->opts.k_in; });
    std::map<int, Launch> initL;
    std::map<GroupKey, Launch> first, p1f, p1[2], p2[2];
    std::map<GroupKey, std::vector<int>> kin;
    std::map<std::pair<GroupKey, int>, Launch> smallL;  // by (group, m)
    std::map<std::pair<GroupKey, int>, size_t> smallB;
    const GroupPlan plan = plan_groups(ctx, ord, true, true);
    for (Slot* s : ord) {
      const int lv = s->level;
      const int nw = 1 - s->cur;
      const PartLayout PL = part_layout(s->part, s->m >> lv);
      const GroupPlan::Entry& pe = plan.at(s);
      Job j = base_job(s, lv);
      j.op = op_dev(s->op, lv, pe.tables() ? pe.tables() : s->op->host.levels[lv].rb);
      j.flags = solver_flags(s);
      j.v[V_X] = s->X[nw];
      j.v[V_S] = s->S;
      j.v[V_Q1] = s->Q1;
      j.v[V_Q2] = s->Q2;
      j.v[V_W] = s->W;
      j.v[V_B] = const_cast<void*>(s->B[lv]);
      j.v[V_C1] = s->C1;
      j.v[V_C2] = s->C2;
      GroupKey gk = pe.key;
      gk.t32 = j.m >= 32;
      if (pe.small_lds) {
        Job js = j;
        js.i0 = s->opts.k_in;
        if (pe.wlds) js.flags |= F_WLDS;
        const auto sk = std::make_pair(gk, js.m);
        smallL[sk].add(js, 1, 4);
        smallB[sk] = std::max(smallB[sk], pe.small_lds);
        continue;
      }
      Job ji = j;
      ji.v[V_PA] = s->P[0];
      ji.v[V_R1A] = s->R1[0];
      ji.v[V_R2A] = s->R2[0];
      initL[s->prec].add(ji, ji.m, (int)s->esz);
      Job jf = j;
      jf.flags |= F_FIRST;
      jf.v[V_R1A] = s->R1[0];
      jf.v[V_R1B] = s->R1[1];
      jf.v[V_R2A] = s->R2[0];
      jf.v[V_R2B] = s->R2[1];
      jf.pw = PL.s[0];
      first[gk].add(jf, jf.m, (int)s->esz);
      for (int par = 0; par < 2; ++par) {
        Job a = j;
        a.v[V_PA] = s->P[par];
        a.v[V_PB] = s->P[1 - par];
        a.pw = PL.q;
        a.pr[0] = PL.s[par];
        a.pr[1] = PL.s[1 - par];
        p1[par][gk].add(a, a.m, (int)s->esz, s->opts.k_in);
        if (par == 0) {
          Job a0 = a;
          a0.flags |= F_FIRST;  // iteration 0: beta = 0
          p1f[gk].add(a0, a0.m, (int)s->esz, s->opts.k_in);
        }
        Job b = j;
        b.v[V_PB] = s->P[1 - par];
        b.v[V_R1A] = s->R1[1 - par];
        b.v[V_R1B] = s->R1[par];
        b.v[V_R2A] = s->R2[1 - par];
        b.v[V_R2B] = s->R2[par];
        b.pr[0] = PL.q;
        b.pr[1] = PL.s[par];
        b.pw = PL.s[1 - par];
        p2[par][gk].add(b, b.m, (int)s->esz, s->opts.k_in);
      }
      kin[gk].push_back(s->opts.k_in);
    }
    // every table of the stage staged with one copy
    std::map<std::pair<GroupKey, int>, LaunchArgs> laS;
    std::map<int, LaunchArgs> laI;
    std::map<GroupKey, LaunchArgs> aF, a1f, a1[2], a2[2];
    std::vector<std::pair<const Launch*, LaunchArgs*>> up;
    for (auto& kv : smallL) up.push_back({&kv.second, &laS[kv.first]});
    for (auto& kv : initL)
      if (!kv.second.empty()) up.push_back({&kv.second, &laI[kv.first]});
    for (auto& kv : first) {
      const GroupKey& g = kv.first;
      up.push_back({&kv.second, &aF[g]});
      up.push_back({&p1f[g], &a1f[g]});
      for (int par = 0; par < 2; ++par) {
        up.push_back({&p1[par][g], &a1[par][g]});
        up.push_back({&p2[par][g], &a2[par][g]});
      }
    }
    if ((rc = upload_all(ctx, up))) return rc;
    for (auto& kv : smallL) {
      const GroupKey& g = kv.first.first;
      const int mm = kv.first.second;
      const LaunchArgs& la = laS[kv.first];
      double b = 0.0;
      for (const Job& jj : kv.second.jobs) b += job_bytes("cgls_small", jj, g.prec);
      const size_t lds = smallB[kv.first];
      if ((rc = hip_check(ctx, timed(ctx, "cgls_small", b, [&] {
                            return launch_cgls_small(la, g.prec, g.rb, mm, lds, !g.sep);
                          }),
                          "cgls small")))
        return rc;
    }
    for (auto& kv : laI) {
      double b = 0.0;
      for (const Job& jj : initL[kv.first].jobs) b += job_bytes("cgls_init", jj, kv.first);
      if ((rc = hip_check(ctx, timed(ctx, "cgls_init", b, [&] {
                            return launch_cgls_init(kv.second, kv.first);
                          }),
                          "cgls_init")))
        return rc;
    }
    for (auto& kv : first) {
      const GroupKey& g = kv.first;
      if (g.multi) {
        aF[g].multi = a1f[g].multi = true;
        for (int par = 0; par < 2; ++par) a1[par][g].multi = a2[par][g].multi = true;
      }
    }
    for (auto& kv : aF) {
      const GroupKey& g = kv.first;
      double b = 0.0;
      for (const Job& jj : first[g].jobs) b += job_bytes("cgls_p2", jj, g.prec);
      LaunchArgs la = kv.second;
      if (!g.multi) tune_cgls_launch(ctx, 2, g.prec, g.sep, g.rb, la);
      if ((rc = hip_check(ctx, timed(ctx, "cgls_p2", b, [&] {
                            return cgls_phase(la, 2, g);
                          }),
                          "cgls p2")))
        return rc;
    }
    int kmax = 0;
    for (auto& kv : kin)
      for (int k : kv.second) kmax = std::max(kmax, k);
    for (int it = 0; it < kmax; ++it) {
      const int par = it & 1;
      for (auto& kv : kin) {
        const GroupKey& g = kv.first;
        const std::vector<int>& ks = kv.second;
        int q = 0;
        while (q < (int)ks.size() && ks[q] > it) ++q;
        if (!q) continue;
        LaunchArgs la = it == 0 ? a1f[g] : a1[par][g];
        la.ntiles = p1[par][g].tiles_upto[q - 1];
        if (!g.multi) tune_cgls_launch(ctx, 1, g.prec, g.sep, g.rb, la);
        double b = 0.0;
        for (int jq = 0; jq < q; ++jq)
          b += job_bytes("cgls_p1", p1[par][g].jobs[jq], g.prec);
        if ((rc = hip_check(ctx, timed(ctx, "cgls_p1", b, [&] {
                              return cgls_phase(la, 1, g);
                            }),
                            "cgls p1")))
          return rc;
      }
      for (auto& kv : kin) {
        const GroupKey& g = kv.first;
        const std::vector<int>& ks = kv.second;
        int q = 0;
        while (q < (int)ks.size() && ks[q] > it) ++q;
        if (!q) continue;
        LaunchArgs la = a2[par][g];
        la.ntiles = p2[par][g].tiles_upto[q - 1];
        if (!g.multi) tune_cgls_launch(ctx, 2, g.prec, g.sep, g.rb, la);
        double b = 0.0;
        for (int jq = 0; jq < q; ++jq)
          b += job_bytes("cgls_p2", p2[par][g].jobs[jq], g.prec);
        if ((rc = hip_check(ctx, timed(ctx, "cgls_p2", b, [&] {
                              return cgls_phase(la, 2, g);
                            }),
                            "cgls p2")))
          return rc;
      }
    }
  }

  // ---- E. Split Bregman update (Alg. 3) and statistics ----------------------
  // Solves that stop on a tolerance get an entry of ctx->d_rc, which the
  // statistics kernel fills with this step's RC for the host's test in F.
  int n_rc = 0;
  for (Slot* s : act) s->rc_idx = level_tol(s) > 0.0 ? n_rc++ : -1;
  if (n_rc > ctx->rc_cap) {
    const int cap = std::max(64, 2 * n_rc);
    if ((rc = hip_check(ctx, hipStreamSynchronize(ctx->stream), "sync"))) return rc;
    if (ctx->d_rc) dfree(ctx, ctx->d_rc);
    if (ctx->h_rc) (void)hipHostFree(ctx->h_rc);
    ctx->d_rc = ctx->h_rc = nullptr;
    ctx->rc_cap = 0;
    void* d = nullptr;
    if ((rc = dmalloc(ctx, (size_t)cap * 8, &d))) return rc;
    ctx->d_rc = static_cast<double*>(d);
    if ((rc = hip_check(ctx, hipHostMalloc((void**)&ctx->h_rc, (size_t)cap * 8,
                                           hipHostMallocDefault),
                        "hipHostMalloc")))
      return rc;
    ctx->rc_cap = cap;
  }
  {
    std::map<int, Launch> L;
    for (Slot* s : act)
      if (s->solver == DBL_SB)
        add_aux(L, s, s->level, AUX_SB_UPDATE, s->X[1 - s->cur], nullptr, s->C1, s->C2);
    std::map<GroupKey, Launch> S;
    Launch F;
    for (Slot* s : act) {
      const PartLayout PL = part_layout(s->part, s->m >> s->level);
      Job j = base_job(s, s->level);
      j.flags = solver_flags(s);
      j.v[V_X] = s->X[1 - s->cur];
      j.v[V_XOLD] = s->X[s->cur];
      j.v[V_B] = const_cast<void*>(s->B[s->level]);
      j.p0 = s->opts.eps;
      j.p1 = s->opts.tau;
      j.i0 = s->level * DBL_MAX_KOUT + s->k;
      j.pw = PL.st;
      S[key_of(s, s->level)].add(j, j.m, (int)s->esz);
      Job jf = j;
      jf.pr[0] = PL.st;
      const int t = tiles_per_axis(j.m, (int)s->esz);
      jf.i1 = t * t;
      if (s->rc_idx >= 0) jf.v[V_RCOUT] = ctx->d_rc + s->rc_idx;
      F.add(jf, 1, 4);
    }
    // every table of the stage staged with one copy
    std::map<int, LaunchArgs> laL;
    std::map<GroupKey, LaunchArgs> laS;
    LaunchArgs laF;
    std::vector<std::pair<const Launch*, LaunchArgs*>> up;
    for (auto& kv : L)
      if (!kv.second.empty()) up.push_back({&kv.second, &laL[kv.first]});
    for (auto& kv : S) up.push_back({&kv.second, &laS[kv.first]});
    up.push_back({&F, &laF});
    if ((rc = upload_all(ctx, up))) return rc;
    for (auto& kv : laL) {
      double b = 0.0;
      for (const Job& jj : L[kv.first].jobs) b += job_bytes("aux", jj, kv.first);
      if ((rc = hip_check(ctx, timed(ctx, "aux", b, [&] { return launch_aux(kv.second, kv.first); }),
                          "aux")))
        return rc;
    }
    for (auto& kv : S) {
      const LaunchArgs& la = laS[kv.first];
      const GroupKey& g = kv.first;
      double b = 0.0;
      for (const Job& jj : kv.second.jobs) b += job_bytes("stats", jj, g.prec);
      if ((rc = hip_check(ctx, timed(ctx, "stats", b, [&] {
                            return launch_stats(la, g.prec, g.sep, g.rb, g.H);
                          }),
                          "stats")))
        return rc;
    }
    if ((rc = hip_check(ctx, timed(ctx, "stats_fin", 0.0, [&] { return launch_stats_fin(laF); }),
                        "stats fin")))
      return rc;
    if (n_rc > 0) {
      rc = hip_check(ctx, hipMemcpyAsync(ctx->h_rc, ctx->d_rc, (size_t)n_rc * 8,
                                         hipMemcpyDeviceToHost, ctx->stream),
                     "read RC");
      if (!rc) rc = hip_check(ctx, hipStreamSynchronize(ctx->stream), "sync RC");
      if (rc) return rc;
    }
  }

  // ---- F. advance ------------------------------------------------------------
  for (Slot* s : act) {
    s->cur = 1 - s->cur;
    s->k += 1;
    s->iters[s->level] = s->k;
    // eq. (stop); a NaN RC (iteration from x = 0) never stops the level
    const bool converged = s->rc_idx >= 0 && ctx->h_rc[s->rc_idx] < level_tol(s);
    if (s->level == 0 && s->opts.x_hist) {
      char* dst = static_cast<char*>(s->opts.x_hist) + (size_t)(s->k - 1) * s->n0 * s->esz;
      rc = hip_check(ctx, hipMemcpyAsync(dst, s->X[s->cur], (size_t)s->n0 * s->esz,
                                         hipMemcpyDeviceToDevice, ctx->stream),
                     "copy iterate history");
      if (rc) return rc;
    }
    if (s->k == s->opts.k_out || converged) {
      s->k = 0;
      if (s->level == 0) {
        s->done = true;
        rc = hip_check(ctx, hipMemcpyAsync(s->req.x, s->X[s->cur], (size_t)s->n0 * s->esz,
                                           hipMemcpyDeviceToDevice, ctx->stream),
                       "copy result");
        if (rc) return rc;
      } else {
        s->level -= 1;
        s->bh_valid = false;
      }
    }
  }
  return DBL_OK;
}

}  // namespace dbl
