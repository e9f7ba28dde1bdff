// Compile-time tables shared by the host planner and the device engines (no upload needed).
#pragma once
#include <stdint.h>

#include "gbs_internal.h"

namespace gbs {

// C(a, b) for 0 <= a, b <= kMaxK (zero for b > a).
struct BinomTable {
  uint64_t v[kMaxK + 1][kMaxK + 1];
};

constexpr BinomTable make_binom() {
  BinomTable t{};
  for (int a = 0; a <= kMaxK; ++a) {
    t.v[a][0] = 1;
    for (int b = 1; b <= kMaxK; ++b) t.v[a][b] = a == 0 ? 0 : t.v[a - 1][b - 1] + t.v[a - 1][b];
  }
  return t;
}

constexpr BinomTable kBinom = make_binom();

// 1/q, correctly rounded, for the coefficient recursion q c_q = sum_j (t_j / 2) c_{q-j}.
struct InvTable {
  double v[kMaxK + 1];
};

constexpr InvTable make_inv() {
  InvTable t{};
  for (int q = 1; q <= kMaxK; ++q) t.v[q] = 1.0 / (double)q;
  return t;
}

constexpr InvTable kInv = make_inv();

}  // namespace gbs
