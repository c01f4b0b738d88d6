// Host FP64 construction of the level operators A^(i+1) = W^T A^(i) W
// (Sec. 4, Alg. 4) as class tables (see common.h).
//
// A blur with kernel P is A = sum_{a,b} P[a,b] S_b (x) S_a, S_d the zero-
// boundary shift (S_d x)[i] = x[i - d].  Since W = W1 (x) W1, every level is
//   A^(i) = sum_{a,b} P[a,b] M_b^(i) (x) M_a^(i),  M_d^(i+1) = W1^T M_d^(i) W1.
// A separable kernel P = u v^T collapses this to A^(i) = C1^(i) (x) C0^(i)
// with C0^(0) = T(u), C1^(0) = T(v) (banded Toeplitz).
//
// Each 1-D matrix is kept as a class table: circular-offset taps for the top
// St rows, one interior row and the bottom Sb rows.  Because a coarse row
// only depends on its distance to the periodic seam, a level can be built
// from a dense copy of the previous level at a reduced size (at most MAT
// rows): the extracted table is then the table of the full-size matrix.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <stdexcept>
#include <vector>

#include "host.h"

namespace dbl {

static const int MAT = 256;

struct Dense {
  int m = 0;
  std::vector<double> a;  // row-major m x m
  double& at(int i, int l) { return a[(size_t)i * m + l]; }
  double at(int i, int l) const { return a[(size_t)i * m + l]; }
};

static std::vector<double> lowpass(int wavelet) {
  if (wavelet == 0) return {std::sqrt(0.5), std::sqrt(0.5)};
  const double s3 = std::sqrt(3.0), d = 4.0 * std::sqrt(2.0);
  return {(1 + s3) / d, (3 + s3) / d, (3 - s3) / d, (1 - s3) / d};
}

static inline int circ(int d, int m) {  // representative of d mod m in [-m/2, m/2)
  int r = ((d % m) + m) % m;
  return r >= m / 2 ? r - m : r;
}

Table1DHost table_with(const Dense& C, int R, int St, int Sb) {
  Table1DHost t;
  t.R = R;
  t.St = St;
  t.Sb = Sb;
  const int m = C.m, NT = 2 * R + 1;
  t.rows = St + 1 + Sb;
  t.taps.assign((size_t)t.rows * NT, 0.0);
  auto fill_row = [&](int cls, int i) {
    for (int l = 0; l < m; ++l) {
      const double v = C.at(i, l);
      if (v == 0.0) continue;
      const int d = circ(l - i, m);
      if (d < -R || d > R) throw std::runtime_error("class table radius too small");
      t.taps[(size_t)cls * NT + d + R] = v;
    }
  };
  for (int c = 0; c < St; ++c) fill_row(c, c);
  if (m > St + Sb) fill_row(St, St + (m - St - Sb) / 2);
  for (int c = 0; c < Sb; ++c) fill_row(St + 1 + c, m - Sb + c);
  return t;
}

// Radius and seam extents of a dense circulant-banded matrix.
static void table_params(const Dense& C, int& R, int& St, int& Sb) {
  const int m = C.m;
  double amax = 0.0;
  R = 0;
  for (int i = 0; i < m; ++i)
    for (int l = 0; l < m; ++l) {
      const double v = C.at(i, l);
      if (v != 0.0) {
        R = std::max(R, std::abs(circ(l - i, m)));
        amax = std::max(amax, std::fabs(v));
      }
    }
  const int NT = 2 * R + 1;
  auto row = [&](int i) {
    std::vector<double> r(NT, 0.0);
    for (int l = 0; l < m; ++l) {
      const double v = C.at(i, l);
      if (v != 0.0) r[circ(l - i, m) + R] = v;
    }
    return r;
  };
  const int mid = m / 2;
  const std::vector<double> ref = row(mid);
  const double tol = 1e-15 * (amax > 0 ? amax : 1.0);
  auto same = [&](int i) {
    const std::vector<double> r = row(i);
    for (int k = 0; k < NT; ++k)
      if (std::fabs(r[k] - ref[k]) > tol) return false;
    return true;
  };
  St = 0;
  for (int i = 0; i < mid; ++i)
    if (!same(i)) St = i + 1;
  Sb = 0;
  for (int i = mid + 1; i < m; ++i)
    if (!same(i)) Sb = std::max(Sb, m - i);
}

static Dense materialize(const Table1DHost& t, int m) {
  Dense C;
  C.m = m;
  C.a.assign((size_t)m * m, 0.0);
  const int NT = 2 * t.R + 1;
  for (int i = 0; i < m; ++i) {
    const int cls = class_of(i, m, t.St, t.Sb);
    for (int e = -t.R; e <= t.R; ++e) {
      const double v = t.taps[(size_t)cls * NT + e + t.R];
      if (v == 0.0) continue;
      const int l = ((i + e) % m + m) % m;
      C.at(i, l) += v;
    }
  }
  return C;
}

static Dense coarsen(const Dense& C, const std::vector<double>& h) {
  const int m = C.m, mc = m / 2, K = (int)h.size();
  Dense D;
  D.m = mc;
  D.a.assign((size_t)mc * mc, 0.0);
  for (int j = 0; j < mc; ++j)
    for (int l = 0; l < mc; ++l) {
      double s = 0.0;
      for (int a = 0; a < K; ++a)
        for (int b = 0; b < K; ++b) s += h[a] * h[b] * C.at((2 * j + a) % m, (2 * l + b) % m);
      D.at(j, l) = s;
    }
  return D;
}

static Dense transpose(const Dense& C) {
  Dense T;
  T.m = C.m;
  T.a.resize(C.a.size());
  for (int i = 0; i < C.m; ++i)
    for (int l = 0; l < C.m; ++l) T.at(l, i) = C.at(i, l);
  return T;
}

static Dense toeplitz_taps(const std::vector<double>& t, int m) {
  // T[i, l] = t[i - l], t indexed -r..r
  const int r = ((int)t.size() - 1) / 2;
  Dense C;
  C.m = m;
  C.a.assign((size_t)m * m, 0.0);
  for (int i = 0; i < m; ++i)
    for (int d = -r; d <= r; ++d) {
      const int l = i - d;
      if (l >= 0 && l < m) C.at(i, l) = t[d + r];
    }
  return C;
}

// Chain of 1-D matrices over the levels.  Returns, per level, (forward,
// adjoint) class tables; `fixed` optionally forces common parameters.
struct Chain {
  std::vector<Dense> dense;      // dense copy per level at reduced size
  std::vector<int> true_m;
};

static Chain build_chain(const Dense& fine_reduced, int m, int levels,
                         const std::vector<double>& h) {
  Chain c;
  c.dense.push_back(fine_reduced);
  c.true_m.push_back(m);
  for (int i = 1; i < levels; ++i) {
    const Dense& prev = c.dense.back();
    int R, St, Sb;
    table_params(prev, R, St, Sb);
    const Table1DHost t = table_with(prev, R, St, Sb);
    const int mi_prev = c.true_m.back();
    const int msz = std::min(mi_prev, MAT);
    c.dense.push_back(coarsen(materialize(t, msz), h));
    c.true_m.push_back(mi_prev / 2);
  }
  return c;
}

static bool separable(const double* P, int ph, int pw, std::vector<double>& u,
                      std::vector<double>& v) {
  // P column-major: P[a + b * ph]
  int a0 = 0, b0 = 0;
  double best = 0.0;
  for (int b = 0; b < pw; ++b)
    for (int a = 0; a < ph; ++a)
      if (std::fabs(P[a + b * ph]) > best) { best = std::fabs(P[a + b * ph]); a0 = a; b0 = b; }
  if (best == 0.0) return false;
  const double piv = P[a0 + b0 * ph];
  u.resize(ph);
  v.resize(pw);
  for (int a = 0; a < ph; ++a) u[a] = P[a + b0 * ph];
  for (int b = 0; b < pw; ++b) v[b] = P[a0 + b * ph] / piv;
  for (int b = 0; b < pw; ++b)
    for (int a = 0; a < ph; ++a)
      if (std::fabs(P[a + b * ph] - u[a] * v[b]) > 1e-13 * std::fabs(piv)) return false;
  return true;
}

void pad_table(Table1DHost& t, int R) {
  if (t.R == R) return;
  const int NT0 = 2 * t.R + 1, NT = 2 * R + 1;
  std::vector<double> nt((size_t)t.rows * NT, 0.0);
  for (int r = 0; r < t.rows; ++r)
    for (int e = -t.R; e <= t.R; ++e) nt[(size_t)r * NT + e + R] = t.taps[(size_t)r * NT0 + e + t.R];
  t.taps.swap(nt);
  t.R = R;
}

// Drop all-zero outer rings of the interior kernel (the class tables it is
// read from are padded to the radius bucket).  Zero taps add exactly nothing
// to the GCV symbol or to the boundary completion, so only their cost goes.
static void trim_kint(LevelHost& L) {
  const int R0 = L.kint_r0, R1 = L.kint_r1, N0 = 2 * R0 + 1;
  auto at = [&](int a, int b) { return L.kint[(a + R0) + (size_t)(b + R1) * N0]; };
  int r0 = R0, r1 = R1;
  auto row_zero = [&](int a) {
    for (int b = -r1; b <= r1; ++b)
      if (at(a, b) != 0.0) return false;
    return true;
  };
  while (r0 > 0 && row_zero(r0) && row_zero(-r0)) --r0;
  auto col_zero = [&](int b) {
    for (int a = -r0; a <= r0; ++a)
      if (at(a, b) != 0.0) return false;
    return true;
  };
  while (r1 > 0 && col_zero(r1) && col_zero(-r1)) --r1;
  if (r0 == R0 && r1 == R1) return;
  const int n0 = 2 * r0 + 1, n1 = 2 * r1 + 1;
  std::vector<double> k((size_t)n0 * n1);
  for (int b = -r1; b <= r1; ++b)
    for (int a = -r0; a <= r0; ++a) k[(a + r0) + (size_t)(b + r1) * n0] = at(a, b);
  L.kint.swap(k);
  L.kint_r0 = r0;
  L.kint_r1 = r1;
}

static int bucket(int R) {
  for (int b : {2, 4, 8, 12, 16})
    if (R <= b) return b;
  return -1;
}

void build_hierarchy(const double* P, int ph, int pw, int m, int levels, int wavelet,
                     HierHost& out) {
  const std::vector<double> h = lowpass(wavelet);
  out.levels.clear();
  out.levels.resize(levels);
  std::vector<double> u, v;
  const int rh = ph / 2, rw = pw / 2;
  const int m0 = std::min(m, MAT);
  out.sep = separable(P, ph, pw, u, v);
  if (out.sep) {
    // u is indexed a = -rh..rh (rows), v by b = -rw..rw (columns).
    Chain c0 = build_chain(toeplitz_taps(u, m0), m, levels, h);
    Chain c1 = build_chain(toeplitz_taps(v, m0), m, levels, h);
    for (int i = 0; i < levels; ++i) {
      LevelHost& L = out.levels[i];
      L.m = m >> i;
      L.sep = true;
      const Dense* D[4] = {&c0.dense[i], &c1.dense[i], nullptr, nullptr};
      Dense t0 = transpose(c0.dense[i]), t1 = transpose(c1.dense[i]);
      D[2] = &t0;
      D[3] = &t1;
      Table1DHost* tabs[4] = {&L.f0, &L.f1, &L.a0, &L.a1};
      int Rmax = 0;
      for (int k = 0; k < 4; ++k) {
        int R, St, Sb;
        table_params(*D[k], R, St, Sb);
        *tabs[k] = table_with(*D[k], R, St, Sb);
        Rmax = std::max(Rmax, R);
      }
      L.R = Rmax;
      L.rb = bucket(Rmax);
      if (L.rb < 0) throw std::runtime_error("coarse operator radius exceeds 16");
      for (int k = 0; k < 4; ++k) pad_table(*tabs[k], L.rb);
      // interior kernel (convolution orientation) for the GCV surrogate:
      // K[a, b] = C0[i, i - a] C1[j, j - b] at interior rows.
      L.kint_r0 = L.f0.R;
      L.kint_r1 = L.f1.R;
      const int n0 = 2 * L.kint_r0 + 1, n1 = 2 * L.kint_r1 + 1;
      L.kint.assign((size_t)n0 * n1, 0.0);
      for (int b = -L.kint_r1; b <= L.kint_r1; ++b)
        for (int a = -L.kint_r0; a <= L.kint_r0; ++a)
          L.kint[(a + L.kint_r0) + (size_t)(b + L.kint_r1) * n0] =
              L.f0.taps[(size_t)L.f0.St * n0 + (-a) + L.f0.R] *
              L.f1.taps[(size_t)L.f1.St * n1 + (-b) + L.f1.R];
      trim_kint(L);
    }
    return;
  }
  // General kernel: one chain per shift offset d in [-r, r].
  const int r = std::max(rh, rw);
  std::vector<Chain> chains;
  chains.reserve(2 * r + 1);
  for (int d = -r; d <= r; ++d) {
    std::vector<double> t(2 * r + 1, 0.0);
    t[d + r] = 1.0;  // S_d[i, l] = 1 when i - l = d
    chains.push_back(build_chain(toeplitz_taps(t, m0), m, levels, h));
  }
  for (int i = 0; i < levels; ++i) {
    LevelHost& L = out.levels[i];
    L.m = m >> i;
    L.sep = false;
    for (int adj = 0; adj < 2; ++adj) {
      // common class parameters over all offsets
      int R = 0, St = 0, Sb = 0;
      std::vector<Dense> Ds;
      Ds.reserve(2 * r + 1);
      for (int d = -r; d <= r; ++d) {
        Ds.push_back(adj ? transpose(chains[d + r].dense[i]) : chains[d + r].dense[i]);
        int R1, St1, Sb1;
        table_params(Ds.back(), R1, St1, Sb1);
        R = std::max(R, R1);
        St = std::max(St, St1);
        Sb = std::max(Sb, Sb1);
      }
      std::vector<Table1DHost> T;
      for (auto& D : Ds) T.push_back(table_with(D, R, St, Sb));
      Table2DHost& tb = adj ? L.a2 : L.f2;
      tb.R0 = tb.R1 = R;
      tb.St0 = tb.St1 = St;
      tb.Sb0 = tb.Sb1 = Sb;
      tb.rows0 = tb.rows1 = St + 1 + Sb;
      const int NT = 2 * R + 1;
      tb.off.assign(1, 0);
      tb.e0.clear();
      tb.e1.clear();
      tb.val.clear();
      std::vector<double> acc((size_t)NT * NT);
      for (int c1 = 0; c1 < tb.rows1; ++c1)
        for (int c0 = 0; c0 < tb.rows0; ++c0) {
          std::fill(acc.begin(), acc.end(), 0.0);
          for (int b = -rw; b <= rw; ++b)
            for (int a = -rh; a <= rh; ++a) {
              const double pv = P[(a + rh) + (size_t)(b + rw) * ph];
              if (pv == 0.0) continue;
              const Table1DHost& Ta = T[a + r];
              const Table1DHost& Tb = T[b + r];
              for (int e1 = 0; e1 < NT; ++e1) {
                const double tb1 = Tb.taps[(size_t)c1 * NT + e1];
                if (tb1 == 0.0) continue;
                for (int e0 = 0; e0 < NT; ++e0) {
                  const double ta0 = Ta.taps[(size_t)c0 * NT + e0];
                  if (ta0 != 0.0) acc[e0 + (size_t)e1 * NT] += pv * ta0 * tb1;
                }
              }
            }
          for (int e1 = 0; e1 < NT; ++e1)
            for (int e0 = 0; e0 < NT; ++e0) {
              const double val = acc[e0 + (size_t)e1 * NT];
              if (val == 0.0) continue;
              tb.e0.push_back((short)(e0 - R));
              tb.e1.push_back((short)(e1 - R));
              tb.val.push_back(val);
            }
          tb.off.push_back((int)tb.val.size());
        }
    }
    L.R = std::max(1, std::max(L.f2.R0, L.a2.R0));  // the gradient needs a halo of 1
    L.rb = 0;
    if (L.R > 16) throw std::runtime_error("coarse operator radius exceeds 16");
    // interior kernel for the GCV surrogate: K[a, b] = tap at offset (-a, -b)
    const Table2DHost& tb = L.f2;
    const int cls = tb.St0 + tb.St1 * tb.rows0;
    L.kint_r0 = L.kint_r1 = tb.R0;
    const int n0 = 2 * tb.R0 + 1;
    L.kint.assign((size_t)n0 * n0, 0.0);
    for (int k = tb.off[cls]; k < tb.off[cls + 1]; ++k)
      L.kint[(-tb.e0[k] + tb.R0) + (size_t)(-tb.e1[k] + tb.R0) * n0] = tb.val[k];
    trim_kint(L);
  }
}

}  // namespace dbl
