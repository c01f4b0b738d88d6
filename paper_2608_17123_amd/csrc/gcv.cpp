// GCV driver (Sec. 3): spectral (DCT surrogate) or exact (generalised
// eigendecomposition of the pencil, n <= 16384) data, grid search and Brent
// refinement for a batch of subproblems; writes gamma and sqrt(gamma) into
// each scalar block.
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <cmath>
#include <cstring>

#include "dense.h"
#include "runtime.h"

namespace dbl {

namespace {

enum : int { G_B = 0, G_W, G_C1, G_C2, G_IN, G_TMP, G_BH, G_E, G_SYM, G_LAM, G_KINT, G_DCT,
             G_DONE };

const int BRENT_MAXIT = 100;
const int BRENT_CHECK0 = 16;  // Brent launches before the host first reads the done flags
const int BRENT_CHECK = 8;    // launches between later reads
const double BRENT_XTOL = 1e-8;

int ensure_dct(dbl_ctx* ctx, int m, double** out) {
  auto it = ctx->dct.find(m);
  if (it != ctx->dct.end()) {
    *out = it->second;
    return DBL_OK;
  }
  // orthonormal DCT-II, column-major: C[k + i m] = c_k cos(pi k (2i + 1) / (2m))
  std::vector<double> C((size_t)m * m);
  for (int i = 0; i < m; ++i)
    for (int k = 0; k < m; ++k)
      C[k + (size_t)i * m] = (k == 0 ? std::sqrt(1.0 / m) : std::sqrt(2.0 / m)) *
                             std::cos(M_PI * k * (2.0 * i + 1.0) / (2.0 * m));
  double* d = nullptr;
  int rc = hip_check(ctx, hipMalloc((void**)&d, C.size() * 8), "hipMalloc dct");
  if (rc) return rc;
  rc = hip_check(ctx, hipMemcpy(d, C.data(), C.size() * 8, hipMemcpyHostToDevice), "upload dct");
  if (rc) return rc;
  ctx->dct[m] = d;
  *out = d;
  return DBL_OK;
}

// GCV symbols a_k of every (operator, level) among the spectral requests that
// does not have one yet: the operator's symbol block (every level) is
// allocated once, and all missing levels are computed in one launch from the
// inputs the operator's upload carries (l(k) and the interior kernel).
int ensure_symbols(dbl_ctx* ctx, const std::vector<GcvReq>& reqs) {
  Launch La;
  std::vector<std::pair<dbl_op*, int>> built;
  for (const GcvReq& r : reqs) {
    if (r.mode == DBL_GCV_EXACT) continue;
    dbl_op* op = const_cast<dbl_op*>(r.op);
    if (op->sym_ready[r.level]) continue;
    if (!op->sym_blk) {
      size_t tot = 0;
      for (int i = 0; i < op->levels; ++i) {
        const size_t mi = (size_t)op->host.levels[i].m;
        tot += mi * mi;
      }
      int rc = dmalloc(ctx, tot * 8, (void**)&op->sym_blk);
      if (rc) return rc;
      double* p = op->sym_blk;
      for (int i = 0; i < op->levels; ++i) {
        const size_t mi = (size_t)op->host.levels[i].m;
        op->sym[i] = p;
        p += mi * mi;
      }
    }
    const LevelHost& L = op->host.levels[r.level];
    Job j;
    std::memset(&j, 0, sizeof(j));
    j.m = L.m;
    j.i0 = L.kint_r0;
    j.i1 = L.kint_r1;
    j.v[G_KINT] = op->lam[r.level] + L.m;
    j.v[G_SYM] = op->sym[r.level];
    La.add(j, L.m, 4);
    op->sym_ready[r.level] = 1;  // several requests may share an (op, level)
    built.push_back({op, r.level});
  }
  if (La.empty()) return DBL_OK;
  LaunchArgs la;
  int rc = La.upload(ctx, la);
  if (!rc) rc = hip_check(ctx, timed(ctx, "gcv_symbol", 0.0, [&] { return launch_gcv_symbol(la); }),
                          "gcv symbol");
  if (rc)
    for (auto& b : built) b.first->sym_ready[b.second] = 0;
  return rc;
}

int blas_check(dbl_ctx* ctx, rocblas_status st, const char* what) {
  if (st == rocblas_status_success) return DBL_OK;
  return set_err(ctx, DBL_EDEVICE, std::string(what) + ": rocBLAS/rocSOLVER status " +
                                       std::to_string((int)st));
}

// EXACT tier data of one request (n = m^2 <= DBL_GCV_EXACT_MAX_N), in FP64 on the device:
//   Ad  = A^(level) applied to every unit vector (the library's own stencil
//         kernel, FP64 tables) -- the dense level operator;
//   K   = Ad^T Ad (lower triangle, the FP64 matrix-core Gram kernel),
//         M = K + D^T D (D = diag(w) L or L);
//   (nu, V) = generalised eigenpairs of K v = nu M v with V^T M V = I
//         (rocSOLVER sygvd, ascending nu);
//   f = V^T Ad^T b, g = V^T L^T c (0 without a shift), ||b||^2 (the
//         column-dot kernel, fixed summation order).
// Results: nu in r.in, f in r.bh, g in r.e, ||b||^2 in scal[S_G_BB].
int exact_data(dbl_ctx* ctx, const GcvReq& r, Job& base) {
  const LevelHost& L = r.op->host.levels[r.level];
  const int m = L.m, n = m * m;
  int rc = DBL_OK;
  const size_t nn = (size_t)n * n;
  const size_t need = 3 * nn * 8 + 2 * (size_t)n * 8 + 256;
  if (ctx->gx_bytes < need) {
    if ((rc = hip_check(ctx, hipStreamSynchronize(ctx->stream), "sync"))) return rc;
    dfree(ctx, ctx->gx);
    ctx->gx = nullptr;
    ctx->gx_bytes = 0;
    if ((rc = dmalloc(ctx, need, &ctx->gx))) return rc;
    ctx->gx_bytes = need;
  }
  if (!ctx->blas) {
    rocblas_handle h = nullptr;
    if ((rc = blas_check(ctx, rocblas_create_handle(&h), "rocblas_create_handle"))) return rc;
    ctx->blas = h;
  }
  rocblas_handle h = static_cast<rocblas_handle>(ctx->blas);
  if ((rc = blas_check(ctx, rocblas_set_stream(h, ctx->stream), "rocblas_set_stream"))) return rc;
  double* X1 = static_cast<double*>(ctx->gx);  // identity, then M
  double* Ad = X1 + nn;
  double* K = Ad + nn;                           // K, then V
  double* nu = K + nn;
  double* E = nu + n;
  rocblas_int* info = reinterpret_cast<rocblas_int*>(E + n);
  // b in FP64 (r.in), ||b||^2
  {
    Launch P;
    Job j = base;
    j.i0 = 0;
    P.add(j, m, 4);
    LaunchArgs la;
    if ((rc = P.upload(ctx, la))) return rc;
    if ((rc = hip_check(ctx, launch_gcv_prep(la, r.prec), "gcv prep"))) return rc;
  }
  if ((rc = hip_check(ctx, launch_gemv_t64(r.in, n, n, 1, r.in, r.scal + S_G_BB, ctx->stream),
                      "||b||^2")))
    return rc;
  // dense operator: Ad = A I, column by column in one launch (one job per column)
  if ((rc = hip_check(ctx, launch_gcv_eye(X1, n, ctx->stream), "gcv eye"))) return rc;
  {
    Launch La;
    for (int c = 0; c < n; ++c) {
      Job j;
      std::memset(&j, 0, sizeof(j));
      j.m = m;
      j.op = r.op->d_ops + r.level;
      j.v[0] = X1 + (size_t)c * n;
      j.v[1] = Ad + (size_t)c * n;
      La.add(j, m, 8);
    }
    LaunchArgs la;
    if ((rc = La.upload(ctx, la))) return rc;
    const int sep = L.sep ? 1 : 0, H = L.sep ? L.rb : L.R;
    if ((rc = hip_check(ctx, launch_apply_A(la, 1, sep, L.rb, H), "dense operator"))) return rc;
  }
  // A^T b into r.tmp; K = Ad^T Ad (lower triangle)
  if ((rc = hip_check(ctx, launch_gemv_t64(Ad, n, n, n, r.in, r.tmp, ctx->stream), "A^T b")))
    return rc;
  if ((rc = hip_check(ctx, timed(ctx, "gcv_gram", 1.5 * (double)nn * 8.0,
                                 [&] { return launch_gram64(Ad, K, n, ctx->stream); }),
                      "A^T A")))
    return rc;
  // L^T c into r.in (shift), M = K + D^T D
  if (r.c1) {
    Launch P;
    Job j = base;
    j.i0 = 1;
    j.v[G_W] = nullptr;  // no weight partials needed here
    P.add(j, m, 4);
    LaunchArgs la;
    if ((rc = P.upload(ctx, la))) return rc;
    if ((rc = hip_check(ctx, launch_gcv_prep(la, r.prec), "gcv prep"))) return rc;
  }
  if ((rc = hip_check(ctx, hipMemcpyAsync(X1, K, nn * 8, hipMemcpyDeviceToDevice, ctx->stream),
                      "copy K")))
    return rc;
  if ((rc = hip_check(ctx, launch_gcv_add_dtd(X1, r.w, r.prec, m, ctx->stream), "D^T D")))
    return rc;
  if ((rc = blas_check(ctx, rocsolver_dsygvd(h, rocblas_eform_ax, rocblas_evect_original,
                                             rocblas_fill_lower, n, K, n, X1, n, nu, E, info),
                       "dsygvd")))
    return rc;
  rocblas_int hinfo = 0;
  if ((rc = hip_check(ctx, hipMemcpyAsync(&hinfo, info, sizeof(hinfo), hipMemcpyDeviceToHost,
                                          ctx->stream), "read info")))
    return rc;
  if ((rc = hip_check(ctx, hipStreamSynchronize(ctx->stream), "sync"))) return rc;
  if (hinfo != 0)
    return set_err(ctx, DBL_ENUMERIC, "generalised eigensolver failed (info " +
                                          std::to_string(hinfo) + ")");
  // f = V^T (A^T b) into r.bh; g = V^T (L^T c) into r.e; nu into r.in
  if ((rc = hip_check(ctx, launch_gemv_t64(K, n, n, n, r.tmp, r.bh, ctx->stream), "f")))
    return rc;
  if (r.c1) {
    if ((rc = hip_check(ctx, launch_gemv_t64(K, n, n, n, r.in, r.e, ctx->stream), "g")))
      return rc;
  } else if ((rc = hip_check(ctx, hipMemsetAsync(r.e, 0, (size_t)n * 8, ctx->stream), "g = 0"))) {
    return rc;
  }
  return hip_check(ctx, hipMemcpyAsync(r.in, nu, (size_t)n * 8, hipMemcpyDeviceToDevice,
                                       ctx->stream), "copy nu");
}

}  // namespace

int gcv_run(dbl_ctx* ctx, std::vector<GcvReq>& reqs) {
  int rc = DBL_OK;
  for (auto& r : reqs) {
    const int m = r.op->host.levels[r.level].m;
    if (r.mode == DBL_GCV_EXACT && m * m > DBL_GCV_EXACT_MAX_N)
      return set_err(ctx, DBL_ENOTSUP, "EXACT GCV needs n <= 16384; use SPECTRAL");
  }
  if ((rc = ensure_symbols(ctx, reqs))) return rc;
  std::vector<Job> base(reqs.size());
  std::vector<PartLayout> PLs(reqs.size());
  for (size_t q = 0; q < reqs.size(); ++q) {
    GcvReq& r = reqs[q];
    const int m = r.op->host.levels[r.level].m;
    PLs[q] = part_layout(r.part, m);
    const bool exact = r.mode == DBL_GCV_EXACT;
    double *sym = nullptr, *dct = nullptr, *lam = nullptr;
    if (!exact) {
      sym = r.op->sym[r.level];
      lam = r.op->lam[r.level];
      if ((rc = ensure_dct(ctx, m, &dct))) return rc;
    }
    Job& j = base[q];
    std::memset(&j, 0, sizeof(j));
    j.m = m;
    j.scal = r.scal;
    j.part = r.part;
    j.v[G_B] = const_cast<void*>(r.b);
    j.v[G_W] = const_cast<void*>(r.w);
    j.v[G_C1] = const_cast<void*>(r.c1);
    j.v[G_C2] = const_cast<void*>(r.c2);
    j.v[G_IN] = r.in;
    j.v[G_TMP] = r.tmp;
    j.v[G_BH] = r.bh;
    j.v[G_E] = r.e;
    j.v[G_SYM] = exact ? r.in : sym;  // exact: nu (written by exact_data)
    j.v[G_LAM] = exact ? nullptr : lam;
    j.v[G_DCT] = dct;
    if (exact) j.flags |= F_EXACT;
  }
  // EXACT tier data, one request at a time (shared dense workspace)
  for (size_t q = 0; q < reqs.size(); ++q)
    if (reqs[q].mode == DBL_GCV_EXACT && (rc = exact_data(ctx, reqs[q], base[q]))) return rc;
  auto run = [&](hipError_t (*fn)(const LaunchArgs&), Launch& L, const char* what) -> int {
    if (L.empty()) return DBL_OK;
    LaunchArgs la;
    int r2 = L.upload(ctx, la);
    if (r2) return r2;
    return hip_check(ctx, timed(ctx, what, 0.0, [&] { return fn(la); }), what);
  };
  auto run_prec = [&](std::map<int, Launch>& M, const char* what) -> int {
    for (auto& kv : M) {
      if (kv.second.empty()) continue;
      LaunchArgs la;
      int r2 = kv.second.upload(ctx, la);
      if (r2) return r2;
      if ((r2 = hip_check(ctx, timed(ctx, what, 0.0, [&] { return launch_gcv_prep(la, kv.first); }),
                          what)))
        return r2;
    }
    return DBL_OK;
  };
  // DCT(X) = C X C^T as two GEMMs: tmp = C in, out = tmp C^T.  The grids of
  // at least 128 take the 128 x 128 tile kernel when their tiles fill the
  // chip at least once (256 blocks; the kernel runs two waves per SIMD), else
  // every grid the 64 x 64 one (both give the same result bit for bit).
  auto dct2 = [&](const std::vector<size_t>& sel, int out_slot) -> int {
    Launch g1, g2, h1, h2;
    size_t t128 = 0;
    for (size_t q : sel)
      if (base[q].m >= 128) t128 += (size_t)(base[q].m / 128) * (base[q].m / 128);
    const bool use128 = t128 >= 256;
    for (size_t q : sel) {
      Job a = base[q];
      a.v[0] = base[q].v[G_DCT];
      a.v[1] = base[q].v[G_IN];
      a.v[2] = base[q].v[G_TMP];
      a.i0 = 0;
      Job b = base[q];
      b.v[0] = base[q].v[G_TMP];
      b.v[1] = base[q].v[G_DCT];
      b.v[2] = base[q].v[out_slot];
      b.i0 = 1;
      if (use128 && a.m >= 128) {
        h1.add_grid(a, a.m / 128, a.m / 128);
        h2.add_grid(b, b.m / 128, b.m / 128);
      } else {
        g1.add(a, a.m, 0);
        g2.add(b, b.m, 0);
      }
    }
    auto big = [](int tb) {
      return tb ? +[](const LaunchArgs& la) { return launch_gemm128(la, 1); }
                : +[](const LaunchArgs& la) { return launch_gemm128(la, 0); };
    };
    int r2 = run(launch_gemm64, g1, "gcv_dct_gemm");
    if (!r2) r2 = run(big(0), h1, "gcv_dct_gemm");
    if (!r2) r2 = run(launch_gemm64, g2, "gcv_dct_gemm");
    if (!r2) r2 = run(big(1), h2, "gcv_dct_gemm");
    return r2;
  };
  // 1. DCT of the data b (once per level)
  {
    std::map<int, Launch> P;
    std::vector<size_t> sel;
    for (size_t q = 0; q < reqs.size(); ++q) {
      if (reqs[q].bh_valid || reqs[q].mode == DBL_GCV_EXACT) continue;
      Job j = base[q];
      j.i0 = 0;
      P[reqs[q].prec].add(j, j.m, 4);
      sel.push_back(q);
    }
    if ((rc = run_prec(P, "gcv_prep"))) return rc;
    // boundary completion of b under the surrogate's reflexive model, two
    // passes: tmp = b + E(b), then in = b + E(tmp) (b is held in `in`)
    Launch c1, c2;
    for (size_t q : sel) {
      const LevelHost& L = reqs[q].op->host.levels[reqs[q].level];
      if (L.kint_r0 > 16 || L.kint_r1 > 16)
        return set_err(ctx, DBL_ENOTSUP, "GCV boundary completion needs a kernel radius <= 16");
      Job a = base[q];
      a.i0 = L.kint_r0;
      a.i1 = L.kint_r1;
      a.v[G_KINT] = static_cast<double*>(base[q].v[G_LAM]) + a.m;
      Job b = a;
      a.v[0] = base[q].v[G_IN];
      a.v[1] = base[q].v[G_IN];
      a.v[2] = base[q].v[G_TMP];
      b.v[0] = base[q].v[G_IN];
      b.v[1] = base[q].v[G_TMP];
      b.v[2] = base[q].v[G_IN];
      c1.add(a, a.m, 4);
      c2.add(b, b.m, 4);
    }
    if ((rc = run(launch_gcv_complete, c1, "gcv_complete"))) return rc;
    if ((rc = run(launch_gcv_complete, c2, "gcv_complete"))) return rc;
    if (!sel.empty() && (rc = dct2(sel, G_BH))) return rc;
  }
  // 2. L^T c (shift) and the IRLS weight scale, then DCT(L^T c)
  {
    std::map<int, Launch> P;
    std::vector<size_t> sel;
    for (size_t q = 0; q < reqs.size(); ++q) {
      if (reqs[q].mode == DBL_GCV_EXACT) continue;
      Job j = base[q];
      j.i0 = 1;
      j.pw = PLs[q].gw;
      P[reqs[q].prec].add(j, j.m, 4);
      if (reqs[q].c1) sel.push_back(q);
    }
    if ((rc = run_prec(P, "gcv_prep"))) return rc;
    if (!sel.empty() && (rc = dct2(sel, G_E))) return rc;
  }
  // 3. per-frequency data and grid bounds; 4. grid; 5. Brent (levels of at
  //    most 64 x 64: 4 and 5 in one block per job)
  {
    // done flags of the multi-launch Brent jobs (one FP64 per job)
    int nb = 0;
    for (size_t q = 0; q < reqs.size(); ++q) nb += base[q].m > 64 ? 1 : 0;
    if (nb > ctx->gflag_cap) {
      if ((rc = hip_check(ctx, hipStreamSynchronize(ctx->stream), "sync"))) return rc;
      if (ctx->d_gflag) dfree(ctx, ctx->d_gflag);
      if (ctx->h_gflag) (void)hipHostFree(ctx->h_gflag);
      ctx->d_gflag = ctx->h_gflag = nullptr;
      ctx->gflag_cap = 0;
      const int cap = std::max(64, 2 * nb);
      void* d = nullptr;
      if ((rc = dmalloc(ctx, (size_t)cap * 8, &d))) return rc;
      ctx->d_gflag = static_cast<double*>(d);
      if ((rc = hip_check(ctx, hipHostMalloc((void**)&ctx->h_gflag, (size_t)cap * 8,
                                             hipHostMallocDefault),
                          "hipHostMalloc")))
        return rc;
      ctx->gflag_cap = cap;
    }
    int ib = 0;
    Launch Ld, Lg, Lf, Lb[2], Ls[2];
    for (size_t q = 0; q < reqs.size(); ++q) {
      const PartLayout& PL = PLs[q];
      const bool exact = reqs[q].mode == DBL_GCV_EXACT;
      Job j = base[q];
      j.i0 = reqs[q].c1 ? 1 : 0;
      j.pr[0] = (reqs[q].w && !exact) ? PL.gw : nullptr;
      j.pw = PL.gmm;
      Ld.add(j, j.m, 4);
      if (j.m <= 64) {
        Job o = base[q];
        o.i0 = reqs[q].grid;
        const int t = tiles_per_axis(o.m, 4);
        o.i1 = t * t;
        o.pr[0] = PL.gmm;
        o.p0 = BRENT_XTOL;
        o.p1 = BRENT_MAXIT;
        Ls[0].add(o, 1, 4);
        continue;
      }
      Job g = base[q];
      g.i1 = reqs[q].grid;
      g.pr[0] = PL.gmm;
      g.pw = PL.ggrid;
      Lg.add(g, g.m, 4);
      Job f = base[q];
      f.i0 = reqs[q].grid;
      const int t = tiles_per_axis(f.m, 4);
      f.i1 = t * t;
      f.pr[0] = PL.ggrid;
      Lf.add(f, 1, 4);
      for (int par = 0; par < 2; ++par) {
        Job b = base[q];
        b.i0 = par;
        b.i1 = BRENT_MAXIT;
        b.p0 = BRENT_XTOL;
        b.pr[0] = PL.gb[par];
        b.pw = PL.gb[1 - par];
        b.v[G_DONE] = ctx->d_gflag + ib;
        Lb[par].add(b, b.m, 4);
      }
      ++ib;
    }
    if ((rc = run(launch_gcv_data, Ld, "gcv_data"))) return rc;
    for (int c = 0; c < 2; ++c)
      if ((rc = run(launch_gcv_solo, Ls[c], "gcv_solo"))) return rc;
    if (Lg.empty()) return DBL_OK;
    LaunchArgs lg;
    if ((rc = Lg.upload(ctx, lg))) return rc;
    if ((rc = hip_check(ctx, timed(ctx, "gcv_grid", 0.0, [&] { return launch_gcv_grid(lg, 0); }),
                        "gcv grid")))
      return rc;
    if ((rc = run(launch_gcv_gridfin, Lf, "gcv_gridfin"))) return rc;
    LaunchArgs lb[2];
    for (int par = 0; par < 2; ++par)
      if ((rc = Lb[par].upload(ctx, lb[par]))) return rc;
    // one start evaluation, up to BRENT_MAXIT steps, one final reduction.
    // Every launch leaves each job's done flag; after BRENT_CHECK0 launches,
    // and every BRENT_CHECK after that, the host reads them and stops once
    // all are set (the launches left would only copy the final states).
    int it = 0;
    while (it < BRENT_MAXIT + 2) {
      const int upto = std::min(BRENT_MAXIT + 2, it == 0 ? BRENT_CHECK0 : it + BRENT_CHECK);
      for (; it < upto; ++it)
        if ((rc = hip_check(ctx, timed(ctx, "gcv_brent", 0.0,
                                       [&] { return launch_gcv_brent(lb[it & 1]); }),
                            "gcv brent")))
          return rc;
      if (it >= BRENT_MAXIT + 2) break;
      rc = hip_check(ctx, hipMemcpyAsync(ctx->h_gflag, ctx->d_gflag, (size_t)ib * 8,
                                         hipMemcpyDeviceToHost, ctx->stream),
                     "read Brent flags");
      if (!rc) rc = hip_check(ctx, hipStreamSynchronize(ctx->stream), "sync Brent flags");
      if (rc) return rc;
      bool all = true;
      for (int q = 0; q < ib; ++q) all = all && ctx->h_gflag[q] != 0.0;
      if (all) break;
    }
  }
  return DBL_OK;
}

}  // namespace dbl
