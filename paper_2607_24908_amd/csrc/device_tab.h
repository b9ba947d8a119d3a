// Piecewise-linear propagator tables (tabulated-propagator variant and the
// momentum-dependent flow built on it).
#pragma once

#include <hip/hip_runtime.h>

#pragma clang fp contract(off)

namespace frg {
namespace dev {

// Interpolated propagator of one row at table coordinate t = s / h (t >= 0):
// nodes k and k + 1 with f = t - k, and the last node beyond t_last = n_s - 1
// (k_last = n_s - 2).
__device__ __forceinline__ double interp(const double *__restrict__ row, double t, double t_last,
                                         int k_last) {
  t = fmin(t, t_last);
  int k = (int)t;
  k = k < k_last ? k : k_last;
  const double f = t - (double)k;
  const double g0 = row[k], g1 = row[k + 1];
  return __builtin_fma(f, g1 - g0, g0);
}

}  // namespace dev
}  // namespace frg
