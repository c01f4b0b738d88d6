// Host test of the XCD tile ordering of the launch tables (runtime.cpp):
// the reorder of every run is a permutation of the run, and the blocks with
// ids equal mod nxcd take one contiguous chunk of the run, in order.
#include <cstdint>
#include <cstdio>
#include <random>
#include <vector>

namespace dbl {
void xcd_order(std::vector<uint32_t>& tiles, size_t s0, size_t s1, int nxcd);
}

int main() {
  std::mt19937 rng(7);
  int fails = 0;
  for (int trial = 0; trial < 2000; ++trial) {
    const size_t n = rng() % 300;
    const size_t s0 = n ? rng() % (n + 1) : 0;
    const size_t s1 = s0 + (n > s0 ? rng() % (n - s0 + 1) : 0);
    const int nxcd = 1 + (int)(rng() % 9);
    std::vector<uint32_t> t(n);
    for (size_t i = 0; i < n; ++i) t[i] = (uint32_t)(1000 + i);
    std::vector<uint32_t> o = t;
    dbl::xcd_order(o, s0, s1, nxcd);
    // outside the run: untouched
    for (size_t i = 0; i < n; ++i)
      if ((i < s0 || i >= s1) && o[i] != t[i]) ++fails;
    // inside: each residue class reads a contiguous increasing chunk, and the
    // chunks tile the run in residue order
    size_t next = s0;
    for (int x = 0; x < nxcd && s1 - s0 >= 2 && nxcd >= 2; ++x) {
      for (size_t p = s0; p < s1; ++p) {
        if ((int)(p % nxcd) != x) continue;
        if (o[p] != t[next]) ++fails;
        ++next;
      }
    }
    if (s1 - s0 >= 2 && nxcd >= 2 && next != s1) ++fails;
    if ((s1 - s0 < 2 || nxcd < 2) && o != t) ++fails;
  }
  std::printf("%s\n", fails ? "FAIL" : "OK");
  return fails ? 1 : 0;
}
