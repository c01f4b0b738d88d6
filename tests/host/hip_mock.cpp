// Host-only stand-in for the HIP runtime, for dry runs of the library's
// engine on a machine without a GPU (test infrastructure, never linked into
// the library).
//
// Device memory is host memory: hipMalloc returns zeroed host blocks and
// records them; copies and fills run at once with memcpy / memset.  Kernel
// launches run nothing: each one is audited instead.  For a launch of a
// kernel that takes (const Job* jobs, const uint32_t* tiles) -- every kernel
// of the library -- the audit reads the staged job and tile tables (they sit
// in the fake device memory) and checks
//   * every tile entry names a job of the launch and a tile below nti * ntj,
//     and the tile grid matches the kernel's geometry for the job's size;
//   * every pointer the kernel can dereference for that job -- vector slots,
//     partial sums, scalar block, history, operator tables -- lies inside one
//     live allocation with the extent the kernel reads or writes there.
//     Slots a kernel reads only under a condition are checked when the job
//     makes the condition true.
// Violations are collected and printed by dryrun_main.cpp.
#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <cxxabi.h>
#include <dlfcn.h>

#include <cstdio>
#include <cstdlib>
#include <algorithm>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "../../paper_2608_17123_amd/csrc/common.h"
#include "../../paper_2608_17123_amd/csrc/launch.h"

using dbl::Job;

namespace mock {

std::map<const char*, size_t> allocs;  // base -> bytes (std::less on pointers: ordered)
std::vector<std::string> violations;
std::map<std::string, long> launches;  // kernel family -> launch count
long checked_pointers = 0;
// copies queued since the last launch, and per kernel family the copies
// queued right before its launches (the table uploads each launch waits for)
long pending_copies = 0;
std::map<std::string, long> copies_before;

const char* owner(const void* p, size_t bytes) {
  const char* c = static_cast<const char*>(p);
  auto it = allocs.upper_bound(c);
  if (it == allocs.begin()) return nullptr;
  --it;
  if (c >= it->first && c + bytes <= it->first + it->second) return it->first;
  return nullptr;
}

void fail(const std::string& kernel, int job, const std::string& what) {
  if (violations.size() < 200)
    violations.push_back(kernel + " job " + std::to_string(job) + ": " + what);
}

void need(const std::string& k, int jb, const char* what, const void* p, size_t bytes) {
  ++checked_pointers;
  if (!p) {
    fail(k, jb, std::string(what) + " is NULL but is dereferenced");
    return;
  }
  if (!owner(p, bytes)) {
    char buf[160];
    std::snprintf(buf, sizeof buf, "%s = %p (+%zu bytes) is not inside a live allocation", what,
                  p, bytes);
    fail(k, jb, buf);
  }
}

std::map<const void*, std::string> registered;  // host stub -> device (mangled) name

std::string kernel_name(const void* f) {
  auto it = registered.find(f);
  if (it != registered.end()) {
    int st = 0;
    char* d = abi::__cxa_demangle(it->second.c_str(), nullptr, nullptr, &st);
    std::string s = (st == 0 && d) ? d : it->second;
    std::free(d);
    return s;
  }
  Dl_info info;
  if (!dladdr(f, &info) || !info.dli_sname) return "?";
  int st = 0;
  char* d = abi::__cxa_demangle(info.dli_sname, nullptr, nullptr, &st);
  std::string s = (st == 0 && d) ? d : info.dli_sname;
  std::free(d);
  return s;
}

// template arguments of a demangled kernel name, e.g. "dbl::k_cgls_p2<float, float, 8, true>"
std::vector<std::string> targs(const std::string& s) {
  std::vector<std::string> out;
  const size_t a = s.find('<'), b = s.rfind('>');
  if (a == std::string::npos || b == std::string::npos) return out;
  std::string cur;
  for (size_t i = a + 1; i < b; ++i) {
    if (s[i] == ',') {
      out.push_back(cur);
      cur.clear();
    } else if (s[i] != ' ') {
      cur += s[i];
    }
  }
  out.push_back(cur);
  return out;
}

size_t tsize(const std::string& t) {
  if (t == "double") return 8;
  if (t == "dbl::bf16s") return 2;
  return 4;
}

void check_table1(const std::string& k, int jb, const char* what, const dbl::Table1D& t,
                  bool dbl_taps) {
  if (t.rows <= 0) return;
  const size_t e = (size_t)t.rows * (2 * t.R + 1);
  need(k, jb, what, dbl_taps ? (const void*)t.td : (const void*)t.tf, e * (dbl_taps ? 8 : 4));
}

void check_op(const std::string& k, int jb, const Job& j, bool dbl_taps) {
  need(k, jb, "op", j.op, sizeof(dbl::LevelOp));
  if (!j.op || !owner(j.op, sizeof(dbl::LevelOp))) return;
  const dbl::LevelOp& op = *j.op;
  if (op.sep) {
    check_table1(k, jb, "op.f0", op.f0, dbl_taps);
    check_table1(k, jb, "op.f1", op.f1, dbl_taps);
    check_table1(k, jb, "op.a0", op.a0, dbl_taps);
    check_table1(k, jb, "op.a1", op.a1, dbl_taps);
  } else {
    const dbl::Table2D* ts[2] = {&op.f2, &op.a2};
    for (const dbl::Table2D* t : ts) {
      const size_t cls = (size_t)t->rows0 * t->rows1;
      need(k, jb, "op.off", t->off, (cls + 1) * 4);
    }
  }
}

int tile_edge_of(int m) { return dbl::tile_edge(m); }

// The 32 x 32 tile CGLS kernels: a grid of at least 32, a separable operator
// whose four tables are padded to the kernel's radius bucket rb (every tap
// row 2 rb + 1 long, the seam classes inside the rows), and the dynamic LDS
// the kernel lays out (haloed tile, pass-A result, tap rows, gradient part).
void check_sep32(const std::string& k, int jb, const Job& j, int rb, size_t esz, int phase,
                 size_t shmem) {
  if (j.m < 32) fail(k, jb, "32 x 32 tile kernel on a grid of " + std::to_string(j.m));
  if (!j.op || !owner(j.op, sizeof(dbl::LevelOp))) return;
  const dbl::LevelOp& op = *j.op;
  if (!op.sep) {
    fail(k, jb, "32 x 32 tile kernel on a non-separable operator");
    return;
  }
  const dbl::Table1D* ts[4] = {&op.f0, &op.f1, &op.a0, &op.a1};
  for (const dbl::Table1D* t : ts) {
    if (t->R != rb) fail(k, jb, "table radius " + std::to_string(t->R) + " != bucket " +
                                    std::to_string(rb));
    if (t->rows != t->St + 1 + t->Sb) fail(k, jb, "table rows != St + 1 + Sb");
    if (t->St + t->Sb > j.m) fail(k, jb, "seam rows exceed the grid");
  }
  const size_t e = (size_t)(32 + 2 * rb) * (32 + 2 * rb + 1) + (size_t)(32 + 2 * rb) * 33 +
                   2 * (2 * rb + 1) + (phase == 2 ? 32 * 32 : 0);
  if (shmem < e * esz)
    fail(k, jb, "dynamic LDS " + std::to_string(shmem) + " < " + std::to_string(e * esz));
}

// The 32 x 32 tile kernels for general operators: a grid of at least 32, a
// non-separable operator of radius <= the kernel's halo rb whose interior
// lists fit the staging area, and the dynamic LDS the kernel lays out
// (haloed tile, staged list, in phase 2 the gradient part).
void check_gen32(const std::string& k, int jb, const Job& j, int rb, size_t esz, int phase,
                 size_t shmem) {
  if (j.m < 32) fail(k, jb, "32 x 32 tile kernel on a grid of " + std::to_string(j.m));
  if (!j.op || !owner(j.op, sizeof(dbl::LevelOp))) return;
  const dbl::LevelOp& op = *j.op;
  if (op.sep) {
    fail(k, jb, "general-operator tile kernel on a separable level");
    return;
  }
  const size_t gt = (size_t)(2 * rb + 1) * (2 * rb + 1);
  const dbl::Table2D* ts[2] = {&op.f2, &op.a2};
  for (const dbl::Table2D* t : ts) {
    if (t->R0 > rb || t->R1 > rb) fail(k, jb, "table radius above the halo " + std::to_string(rb));
    const size_t ncls = (size_t)t->rows0 * t->rows1;
    if (!owner(t->off, (ncls + 1) * 4)) continue;
    const int cls = t->St0 + t->St1 * t->rows0;
    if ((size_t)(t->off[cls + 1] - t->off[cls]) > gt)
      fail(k, jb, "interior tap list longer than the staging area");
  }
  const size_t xs = (size_t)(32 + 2 * rb) * (32 + 2 * rb + 1), gti = (gt + 1) & ~size_t(1);
  const size_t e = esz * xs + 4 * gti + esz * gt + (phase == 2 ? esz * 32 * 32 : 0);
  if (shmem < e) fail(k, jb, "dynamic LDS " + std::to_string(shmem) + " < " + std::to_string(e));
}

// A general tile kernel of a launch that mixes buckets up to rbmax: the job
// runs the body of the bucket above its operator's radius, which must be at
// most rbmax, and is audited as a launch of that bucket (the launch's LDS,
// sized for rbmax, covers it).
void check_gmulti(const std::string& k, int jb, const Job& j, int rbmax, size_t esz, int phase,
                  size_t shmem) {
  if (!j.op || !owner(j.op, sizeof(dbl::LevelOp))) return;
  const int R = j.op->R, rb = R <= 2 ? 2 : R <= 4 ? 4 : R <= 8 ? 8 : R <= 12 ? 12 : 16;
  if (rb > rbmax) fail(k, jb, "job bucket " + std::to_string(rb) + " above the launch's " +
                                  std::to_string(rbmax));
  check_gen32(k, jb, j, rb, esz, phase, shmem);
}

// The one-block CGLS: a separable operator with tables padded to the kernel's
// halo RB, or (gen) a general operator of radius <= RB whose interior class
// lists fit the staging area; the dynamic LDS covers the kernel's layout.
void check_small(const std::string& k, int jb, const Job& j, int RB, size_t esz, bool gen,
                 size_t shmem) {
  if (!j.op || !owner(j.op, sizeof(dbl::LevelOp))) return;
  const dbl::LevelOp& op = *j.op;
  if (gen != !op.sep) {
    fail(k, jb, gen ? "general-operator kernel on a separable level"
                    : "separable kernel on a general level");
    return;
  }
  int tab_elems = 0;
  if (gen) {
    if (op.R > RB) fail(k, jb, "operator radius " + std::to_string(op.R) + " > halo " +
                                   std::to_string(RB));
    const dbl::Table2D* ts[2] = {&op.f2, &op.a2};
    for (const dbl::Table2D* t : ts) {
      if (t->R0 > RB || t->R1 > RB) fail(k, jb, "table radius above the halo");
      const size_t ncls = (size_t)t->rows0 * t->rows1;
      if (!owner(t->off, (ncls + 1) * 4)) continue;
      const int cls = t->St0 + t->St1 * t->rows0;
      if (t->off[cls + 1] - t->off[cls] > dbl::small_gen_taps(RB))
        fail(k, jb, "interior tap list longer than the staging area");
    }
  } else {
    const dbl::Table1D* ts[4] = {&op.f0, &op.f1, &op.a0, &op.a1};
    for (const dbl::Table1D* t : ts) {
      if (t->R != RB) fail(k, jb, "table radius " + std::to_string(t->R) + " != halo " +
                                      std::to_string(RB));
      tab_elems += t->rows * (2 * RB + 1);
    }
  }
  const bool wl = j.flags & dbl::F_WLDS;
  const size_t need_lds = dbl::small_lds(j.m, RB, (int)esz, wl, tab_elems, gen).total;
  if (shmem < need_lds)
    fail(k, jb, "dynamic LDS " + std::to_string(shmem) + " < " + std::to_string(need_lds));
}

// The mixed-bucket tile kernels: every job's tables are padded to a bucket
// of its own, one the kernel has a body for (2, 4, 8, 12 up to its RBMAX),
// and each job then meets the 32 x 32 tile kernel's conditions for that
// bucket; the launch's LDS is sized for RBMAX, which covers every body.
void check_multi(const std::string& k, int jb, const Job& j, int rbmax, size_t esz, int phase,
                 size_t shmem) {
  if (rbmax != 4 && rbmax != 8 && rbmax != 12) fail(k, jb, "mixed launch up to bucket " +
                                                            std::to_string(rbmax));
  if (!j.op || !owner(j.op, sizeof(dbl::LevelOp))) return;
  const int rb = j.op->rb;
  if ((rb != 2 && rb != 4 && rb != 8 && rb != 12) || rb > rbmax) {
    fail(k, jb, "job bucket " + std::to_string(rb) + " outside the launch's bodies (up to " +
                    std::to_string(rbmax) + ")");
    return;
  }
  check_sep32(k, jb, j, rb, esz, phase, shmem);
}

void audit(const void* func, dim3 grid, dim3 block, void** args, size_t shmem) {
  const std::string name = kernel_name(func);
  // family: the unqualified kernel name ("void dbl::k_cgls_p2<...>(...)" -> k_cgls_p2)
  std::string fam = name;
  if (fam.rfind("void ", 0) == 0) fam = fam.substr(5);
  if (fam.rfind("dbl::", 0) == 0) fam = fam.substr(5);
  fam = fam.substr(0, std::min(fam.find('<'), fam.find('(')));
  launches[fam] += 1;
  copies_before[fam] += pending_copies;
  pending_copies = 0;
  const Job* jobs = *static_cast<const Job* const*>(args[0]);
  const uint32_t* tiles = *static_cast<const uint32_t* const*>(args[1]);
  const size_t nt = grid.x;
  need(fam, -1, "tile table", tiles, nt * 4);
  if (!owner(tiles, nt * 4)) return;
  // jobs are staged right before their tile table
  const char* jb0 = reinterpret_cast<const char*>(jobs);
  const long njobs = (reinterpret_cast<const char*>(tiles) - jb0) / (long)sizeof(Job);
  if (njobs <= 0 || !owner(jobs, njobs * sizeof(Job))) {
    fail(fam, -1, "job table not inside a live allocation before the tile table");
    return;
  }
  const std::vector<std::string> ta = targs(name);
  std::vector<char> seen(njobs, 0);
  for (size_t b = 0; b < nt; ++b) {
    const uint32_t t = tiles[b];
    const long ji = t >> 16;
    const int tix = int(t & 0xffffu);
    if (ji >= njobs) {
      fail(fam, (int)ji, "tile entry names a job past the job table");
      continue;
    }
    const Job& j = jobs[ji];
    if (tix >= j.nti * j.ntj) fail(fam, (int)ji, "tile index " + std::to_string(tix) +
                                                  " >= nti*ntj " + std::to_string(j.nti * j.ntj));
    seen[ji] = 1;
  }
  for (long ji = 0; ji < njobs; ++ji) {
    if (!seen[ji]) continue;
    const Job& j = jobs[ji];
    const int jb = (int)ji;
    const size_t m = (size_t)j.m, n = m * m, nl = 2 * m * (m - 1);
    const int ntile = j.nti * j.ntj;
    // geometry of the tiled kernels: nti x nti tiles of tile_edge(grid) pixels
    auto grid_is = [&](size_t gm) {
      const int te = tile_edge_of((int)gm);
      if (j.nti != j.ntj || (size_t)j.nti * te != gm)
        fail(fam, jb, "tile grid " + std::to_string(j.nti) + "x" + std::to_string(j.ntj) +
                          " does not cover a " + std::to_string(gm) + " grid");
    };
    auto v = [&](int s) { return j.v[s]; };
    const bool irls = j.flags & dbl::F_IRLS, shift = j.flags & dbl::F_SHIFT,
               sb = j.flags & dbl::F_SB, first = j.flags & dbl::F_FIRST;
    if (fam == "k_cgls_init") {
      const size_t T = tsize(ta[0]), S = tsize(ta[1]);
      grid_is(m);
      need(fam, jb, "V_X", v(dbl::V_X), n * T);
      need(fam, jb, "V_PA", v(dbl::V_PA), n * S);
      need(fam, jb, "V_R1A", v(dbl::V_R1A), n * S);
      need(fam, jb, "V_R2A", v(dbl::V_R2A), nl * S);
      need(fam, jb, "V_B", v(dbl::V_B), n * T);
      need(fam, jb, "scal", j.scal, dbl::NSCAL * 8);
      if (shift) need(fam, jb, "V_C1", v(dbl::V_C1), nl * T);
      if (shift && sb) need(fam, jb, "V_C2", v(dbl::V_C2), nl * T);
      if (v(dbl::V_X0)) {
        need(fam, jb, "V_X0", v(dbl::V_X0), n * T);
        need(fam, jb, "V_XOLD", v(dbl::V_XOLD), n * T);
        if (irls) need(fam, jb, "V_W", v(dbl::V_W), nl * T);
      }
    } else if (fam == "k_cgls_p1" || fam == "k_cgls_p1_wide" || fam == "k_cgls_p1_sep" ||
               fam == "k_cgls_p1_multi" || fam == "k_cgls_p1_gen" || fam == "k_cgls_p1_gmulti") {
      const size_t T = tsize(ta[0]), S = tsize(ta[1]);
      grid_is(m);
      check_op(fam, jb, j, T == 8);
      if (fam == "k_cgls_p1_sep") check_sep32(fam, jb, j, std::atoi(ta[2].c_str()), T, 1, shmem);
      if (fam == "k_cgls_p1_multi") check_multi(fam, jb, j, std::atoi(ta[2].c_str()), T, 1, shmem);
      if (fam == "k_cgls_p1_gen") check_gen32(fam, jb, j, std::atoi(ta[2].c_str()), T, 1, shmem);
      if (fam == "k_cgls_p1_gmulti") check_gmulti(fam, jb, j, std::atoi(ta[2].c_str()), T, 1, shmem);
      need(fam, jb, "V_S", v(dbl::V_S), n * S);
      need(fam, jb, "V_PA", v(dbl::V_PA), n * S);
      need(fam, jb, "V_PB", v(dbl::V_PB), n * S);
      need(fam, jb, "V_Q1", v(dbl::V_Q1), n * S);
      need(fam, jb, "V_Q2", v(dbl::V_Q2), nl * S);
      need(fam, jb, "scal", j.scal, dbl::NSCAL * 8);
      need(fam, jb, "pw", j.pw, (size_t)ntile * 8);
      if (irls) need(fam, jb, "V_W", v(dbl::V_W), nl * T);
      if (!first) {
        need(fam, jb, "pr[0]", j.pr[0], (size_t)ntile * 2 * 8);
        need(fam, jb, "pr[1]", j.pr[1], (size_t)ntile * 2 * 8);
      }
    } else if (fam == "k_cgls_p2" || fam == "k_cgls_p2_wide" || fam == "k_cgls_p2_sep" ||
               fam == "k_cgls_p2_multi" || fam == "k_cgls_p2_gen" || fam == "k_cgls_p2_gmulti") {
      const size_t T = tsize(ta[0]), S = tsize(ta[1]);
      grid_is(m);
      check_op(fam, jb, j, T == 8);
      if (fam == "k_cgls_p2_sep") check_sep32(fam, jb, j, std::atoi(ta[2].c_str()), T, 2, shmem);
      if (fam == "k_cgls_p2_multi") check_multi(fam, jb, j, std::atoi(ta[2].c_str()), T, 2, shmem);
      if (fam == "k_cgls_p2_gen") check_gen32(fam, jb, j, std::atoi(ta[2].c_str()), T, 2, shmem);
      if (fam == "k_cgls_p2_gmulti") check_gmulti(fam, jb, j, std::atoi(ta[2].c_str()), T, 2, shmem);
      need(fam, jb, "V_R1A", v(dbl::V_R1A), n * S);
      need(fam, jb, "V_R1B", v(dbl::V_R1B), n * S);
      need(fam, jb, "V_R2A", v(dbl::V_R2A), nl * S);
      need(fam, jb, "V_R2B", v(dbl::V_R2B), nl * S);
      need(fam, jb, "V_S", v(dbl::V_S), n * S);
      need(fam, jb, "scal", j.scal, dbl::NSCAL * 8);
      need(fam, jb, "pw", j.pw, (size_t)ntile * 2 * 8);
      if (irls) need(fam, jb, "V_W", v(dbl::V_W), nl * T);
      if (!first) {
        need(fam, jb, "V_X", v(dbl::V_X), n * T);
        need(fam, jb, "V_PB", v(dbl::V_PB), n * S);
        need(fam, jb, "V_Q1", v(dbl::V_Q1), n * S);
        need(fam, jb, "V_Q2", v(dbl::V_Q2), nl * S);
        need(fam, jb, "pr[0]", j.pr[0], (size_t)ntile * 8);
        need(fam, jb, "pr[1]", j.pr[1], (size_t)ntile * 2 * 8);
      }
    } else if (fam == "k_cgls_small") {
      const size_t T = tsize(ta[0]);
      const int RB = std::atoi(ta[1].c_str()), M = std::atoi(ta[2].c_str());
      if ((int)m != M) fail(fam, jb, "job size differs from the kernel's M");
      check_op(fam, jb, j, T == 8);
      check_small(fam, jb, j, RB, T, ta.size() > 3 && ta[3] == "true", shmem);
      need(fam, jb, "V_X", v(dbl::V_X), n * T);
      need(fam, jb, "V_B", v(dbl::V_B), n * T);
      need(fam, jb, "scal", j.scal, dbl::NSCAL * 8);
      if (irls) need(fam, jb, "V_W", v(dbl::V_W), nl * T);
      if (shift) need(fam, jb, "V_C1", v(dbl::V_C1), nl * T);
      if (shift && sb) need(fam, jb, "V_C2", v(dbl::V_C2), nl * T);
    } else if (fam == "k_aux") {
      const size_t T = tsize(ta[0]);
      grid_is(m);
      need(fam, jb, "V_X", v(dbl::V_X), n * T);
      if (j.i0 == dbl::AUX_IRLS_W) need(fam, jb, "V_W", v(dbl::V_W), nl * T);
      if (j.i0 == dbl::AUX_MM_W) need(fam, jb, "V_C1", v(dbl::V_C1), nl * T);
      if (j.i0 == dbl::AUX_SB_INIT || j.i0 == dbl::AUX_SB_UPDATE) {
        need(fam, jb, "V_C1", v(dbl::V_C1), nl * T);
        need(fam, jb, "V_C2", v(dbl::V_C2), nl * T);
      }
    } else if (fam == "k_stats") {
      const size_t T = tsize(ta[0]);
      grid_is(m);
      check_op(fam, jb, j, true);
      need(fam, jb, "V_X", v(dbl::V_X), n * T);
      need(fam, jb, "V_XOLD", v(dbl::V_XOLD), n * T);
      need(fam, jb, "V_B", v(dbl::V_B), n * T);
      need(fam, jb, "pw", j.pw, (size_t)ntile * 4 * 8);
    } else if (fam == "k_stats_fin") {
      need(fam, jb, "pr[0]", j.pr[0], (size_t)j.i1 * 4 * 8);
      need(fam, jb, "scal", j.scal, dbl::NSCAL * 8);
      need(fam, jb, "hist", j.hist, (size_t)(3 * j.i0 + 3) * 8);
      if (v(dbl::V_RCOUT)) need(fam, jb, "V_RCOUT", v(dbl::V_RCOUT), 8);
    } else if (fam == "k_fill") {
      const size_t T = tsize(ta[0]);
      grid_is(m);
      if (v(0)) need(fam, jb, "v[0]", v(0), n * T);
      if (v(1)) need(fam, jb, "v[1]", v(1), nl * T);
    } else if (fam == "k_set_gamma") {
      need(fam, jb, "scal", j.scal, 2 * 8);
    } else if (fam == "k_dwt_fwd") {
      const size_t T = tsize(ta[0]);
      grid_is(m / 2);
      need(fam, jb, "v[0]", v(0), n * T);
      need(fam, jb, "v[1]", v(1), (j.p0 != 0.0 ? n : n / 4) * T);
    } else if (fam == "k_dwt_inv") {
      const size_t T = tsize(ta[0]);
      // low-pass prolongation onto m >= 64: 32 x 64 tiles (the kernel takes
      // the width m / ntj), else the square tiles
      if (j.p0 == 0.0 && m >= 64) {
        const size_t w = 64;
        if ((size_t)j.nti * 32 != m || (size_t)j.ntj * w != m)
          fail(fam, jb, "prolongation tile grid " + std::to_string(j.nti) + "x" +
                            std::to_string(j.ntj) + " is not 32 x " + std::to_string(w) +
                            " tiles of " + std::to_string(m));
      } else {
        grid_is(m);
      }
      need(fam, jb, "v[0]", v(0), (j.p0 != 0.0 ? n : n / 4) * T);
      need(fam, jb, "v[1]", v(1), n * T);
    } else if (fam == "k_dtransfer") {
      const size_t T = tsize(ta[0]), mc = m / 2;
      grid_is(m);
      need(fam, jb, "v[0]", v(0), 2 * mc * (mc - 1) * T);
      need(fam, jb, "v[1]", v(1), nl * T);
    } else if (fam == "k_apply_sep" || fam == "k_apply_gen") {
      const size_t T = tsize(ta[0]);
      grid_is(m);
      check_op(fam, jb, j, T == 8);
      need(fam, jb, "v[0]", v(0), n * T);
      need(fam, jb, "v[1]", v(1), n * T);
    } else if (fam == "k_apply_stream") {
      check_op(fam, jb, j, false);
      need(fam, jb, "v[0]", v(0), n * 4);
      need(fam, jb, "v[1]", v(1), n * 4);
    } else if (fam == "k_grad" || fam == "k_gradT") {
      const size_t T = tsize(ta[0]);
      grid_is(m);
      need(fam, jb, "v[0]", v(0), (fam == "k_grad" ? n : nl) * T);
      need(fam, jb, "v[1]", v(1), (fam == "k_grad" ? nl : n) * T);
    } else if (fam == "k_gemm128_mfma") {
      // the spectral tier's DCT products: one block per 128 x 128 tile of an
      // m x m FP64 product, m a multiple of 128; A, B and out whole
      if (m % 128 != 0 || (size_t)j.nti * 128 != m || (size_t)j.ntj * 128 != m)
        fail(fam, jb, "128 x 128 tile grid " + std::to_string(j.nti) + "x" +
                          std::to_string(j.ntj) + " does not cover a " + std::to_string(m) +
                          " grid");
      for (int s = 0; s < 3; ++s)
        need(fam, jb, ("v[" + std::to_string(s) + "]").c_str(), v(s), n * 8);
      if ((ta[0] == "true") != (j.i0 != 0)) fail(fam, jb, "kernel form differs from the job's");
    } else if (fam == "k_cgls_hist") {
      need(fam, jb, "pr[0]", j.pr[0], (size_t)j.i1 * 2 * 8);
      need(fam, jb, "scal", j.scal, dbl::NSCAL * 8);
    } else {
      // other kernels (GCV, LSQR): every non-null pointer must lie inside an
      // allocation (extent one element)
      for (int s = 0; s < 16; ++s)
        if (j.v[s]) need(fam, jb, ("v[" + std::to_string(s) + "]").c_str(), j.v[s], 1);
      if (j.scal) need(fam, jb, "scal", j.scal, 8);
      if (j.pw) need(fam, jb, "pw", j.pw, 8);
      for (int s = 0; s < 3; ++s)
        if (j.pr[s]) need(fam, jb, "pr", j.pr[s], 8);
    }
  }
  (void)block;
  (void)shmem;
}

}  // namespace mock

// ---------------------------------------------------------------- runtime --
extern "C" {

struct CallCfg {
  dim3 g, b;
  size_t shm;
  hipStream_t s;
};
static std::vector<CallCfg> g_cfg;

hipError_t __hipPushCallConfiguration(dim3 gridDim, dim3 blockDim, size_t sharedMem,
                                    hipStream_t stream) {
  g_cfg.push_back({gridDim, blockDim, sharedMem, stream});
  return hipSuccess;
}
hipError_t __hipPopCallConfiguration(dim3* gridDim, dim3* blockDim, size_t* sharedMem,
                                     hipStream_t* stream) {
  const CallCfg c = g_cfg.back();
  g_cfg.pop_back();
  *gridDim = c.g;
  *blockDim = c.b;
  *sharedMem = c.shm;
  *stream = c.s;
  return hipSuccess;
}
hipError_t hipLaunchKernel(const void* f, dim3 g, dim3 b, void** args, size_t shm,
                           hipStream_t) {
  mock::audit(f, g, b, args, shm);
  return hipSuccess;
}

// kernel registration of the library's code objects: only the names are kept
void** __hipRegisterFatBinary(const void*) {
  static void* handle = nullptr;
  return &handle;
}
void __hipRegisterFunction(void**, const void* hostFunction, char*, const char* deviceName,
                           unsigned int, uint3*, uint3*, dim3*, dim3*, int*) {
  mock::registered[hostFunction] = deviceName;
}
// device variables: a fake device block of the variable's size per symbol
static std::map<const void*, size_t> g_var_size;
static std::map<const void*, void*> g_var_block;
void __hipRegisterVar(void**, void* var, char*, char*, int, size_t size, int, int) {
  g_var_size[var] = size;
}
hipError_t hipMalloc(void** p, size_t bytes);
hipError_t hipGetSymbolAddress(void** dev, const void* symbol) {
  auto it = g_var_block.find(symbol);
  if (it == g_var_block.end()) {
    auto sz = g_var_size.find(symbol);
    if (sz == g_var_size.end()) return hipErrorInvalidSymbol;
    void* p = nullptr;
    if (hipMalloc(&p, sz->second) != hipSuccess) return hipErrorOutOfMemory;
    it = g_var_block.emplace(symbol, p).first;
  }
  *dev = it->second;
  return hipSuccess;
}
void __hipUnregisterFatBinary(void**) {}

hipError_t hipMalloc(void** p, size_t bytes) {
  const size_t al = (bytes + 255) & ~size_t(255);
  *p = std::aligned_alloc(256, al ? al : 256);
  if (!*p) return hipErrorOutOfMemory;
  std::memset(*p, 0, al ? al : 256);
  mock::allocs[static_cast<const char*>(*p)] = bytes;
  return hipSuccess;
}
hipError_t hipFree(void* p) {
  if (!p) return hipSuccess;
  mock::allocs.erase(static_cast<const char*>(p));
  std::free(p);
  return hipSuccess;
}
hipError_t hipHostMalloc(void** p, size_t bytes, unsigned int) { return hipMalloc(p, bytes); }
hipError_t hipHostFree(void* p) { return hipFree(p); }
// A copy or fill that starts inside a (fake) device allocation must stay
// inside it; pointers outside every allocation are host memory.
static bool range_ok(const char* what, const void* p, size_t n) {
  const char* c = static_cast<const char*>(p);
  auto it = mock::allocs.upper_bound(c);
  if (it == mock::allocs.begin()) return true;
  --it;
  if (c >= it->first + it->second) return true;  // not device memory
  if (c + n <= it->first + it->second) return true;
  mock::fail(what, -1, "range of " + std::to_string(n) + " bytes runs past its allocation");
  return false;
}
hipError_t hipMemcpy(void* d, const void* s, size_t n, hipMemcpyKind) {
  if (range_ok("copy destination", d, n) && range_ok("copy source", s, n)) std::memmove(d, s, n);
  return hipSuccess;
}
hipError_t hipMemcpyAsync(void* d, const void* s, size_t n, hipMemcpyKind, hipStream_t) {
  ++mock::pending_copies;
  if (range_ok("copy destination", d, n) && range_ok("copy source", s, n)) std::memmove(d, s, n);
  return hipSuccess;
}
hipError_t hipMemsetAsync(void* d, int v, size_t n, hipStream_t) {
  if (range_ok("fill", d, n)) std::memset(d, v, n);
  return hipSuccess;
}
hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
hipError_t hipSetDevice(int) { return hipSuccess; }
hipError_t hipGetDeviceCount(int* c) {
  *c = 1;
  return hipSuccess;
}
hipError_t hipDeviceGetAttribute(int* v, hipDeviceAttribute_t a, int) {
  // the MI355X's LDS per workgroup (160 KB) and compute units
  *v = a == hipDeviceAttributeMaxSharedMemoryPerBlock ? 163840 : 256;
  return hipSuccess;
}
hipError_t hipGetLastError(void) { return hipSuccess; }
const char* hipGetErrorString(hipError_t) { return "mock"; }
hipError_t hipEventCreate(hipEvent_t* e) {
  *e = reinterpret_cast<hipEvent_t>(new int(0));
  return hipSuccess;
}
hipError_t hipEventDestroy(hipEvent_t e) {
  delete reinterpret_cast<int*>(e);
  return hipSuccess;
}
hipError_t hipEventRecord(hipEvent_t, hipStream_t) { return hipSuccess; }
hipError_t hipEventElapsedTime(float* ms, hipEvent_t, hipEvent_t) {
  *ms = 0.f;
  return hipSuccess;
}
hipError_t hipFuncSetAttribute(const void*, hipFuncAttribute, int) { return hipSuccess; }
hipError_t hipEventSynchronize(hipEvent_t) { return hipSuccess; }
hipError_t hipGetDevicePropertiesR0600(hipDeviceProp_tR0600* p, int) {
  std::memset(p, 0, sizeof(*p));
  std::strcpy(p->gcnArchName, "host-mock");
  p->multiProcessorCount = 256;
  return hipSuccess;
}

// the EXACT GCV tier's library calls are not part of a dry run
rocblas_status rocblas_create_handle(rocblas_handle*) { return rocblas_status_not_implemented; }
rocblas_status rocblas_destroy_handle(rocblas_handle) { return rocblas_status_success; }
rocblas_status rocblas_set_stream(rocblas_handle, hipStream_t) { return rocblas_status_success; }
rocblas_status rocblas_set_pointer_mode(rocblas_handle, rocblas_pointer_mode) {
  return rocblas_status_success;
}
rocblas_status rocblas_dsyrk(rocblas_handle, rocblas_fill, rocblas_operation, rocblas_int,
                             rocblas_int, const double*, const double*, rocblas_int,
                             const double*, double*, rocblas_int) {
  return rocblas_status_not_implemented;
}
rocblas_status rocblas_dgemv(rocblas_handle, rocblas_operation, rocblas_int, rocblas_int,
                             const double*, const double*, rocblas_int, const double*,
                             rocblas_int, const double*, double*, rocblas_int) {
  return rocblas_status_not_implemented;
}
rocblas_status rocblas_ddot(rocblas_handle, rocblas_int, const double*, rocblas_int,
                            const double*, rocblas_int, double*) {
  return rocblas_status_not_implemented;
}
rocblas_status rocsolver_dsygvd(rocblas_handle, const rocblas_eform, const rocblas_evect,
                                const rocblas_fill, const rocblas_int, double*, const rocblas_int,
                                double*, const rocblas_int, double*, double*, rocblas_int*) {
  return rocblas_status_not_implemented;
}

}  // extern "C"
