// Host-side structures of the deblurring library.
#pragma once
#include <hip/hip_runtime.h>

#include <map>
#include <string>
#include <vector>

#include "../../include/deblur.h"
#include "common.h"
#include "launch.h"

namespace dbl {

struct Table1DHost {
  int R = 0, St = 0, Sb = 0, rows = 1;
  std::vector<double> taps;  // rows * (2R+1)
};

// Zero-pad a 1-D class table to radius R >= t.R (2R + 1 taps per row).
void pad_table(Table1DHost& t, int R);

// Radius buckets of the separable kernels (tables padded to one of these).
constexpr int NBUCKETS = 5;
constexpr int RB_BUCKETS[NBUCKETS] = {2, 4, 8, 12, 16};
inline int bucket_index(int rb) {
  for (int k = 0; k < NBUCKETS; ++k)
    if (RB_BUCKETS[k] == rb) return k;
  return -1;
}
// The smallest bucket >= R (-1 above the largest).
inline int bucket_above(int R) {
  for (int k = 0; k < NBUCKETS; ++k)
    if (R <= RB_BUCKETS[k]) return RB_BUCKETS[k];
  return -1;
}

struct Table2DHost {
  int R0 = 0, R1 = 0, St0 = 0, Sb0 = 0, St1 = 0, Sb1 = 0, rows0 = 1, rows1 = 1;
  std::vector<int> off;
  std::vector<short> e0, e1;
  std::vector<double> val;
};

struct LevelHost {
  int m = 0;
  bool sep = true;
  int R = 0, rb = 0;
  Table1DHost f0, f1, a0, a1;
  Table2DHost f2, a2;
  int kint_r0 = 0, kint_r1 = 0;
  std::vector<double> kint;  // interior kernel, convolution orientation, column-major
};

struct HierHost {
  bool sep = true;
  std::vector<LevelHost> levels;
};

void build_hierarchy(const double* P, int ph, int pw, int m, int levels, int wavelet,
                     HierHost& out);

}  // namespace dbl
