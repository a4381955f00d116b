// Cubic (4-point Lagrange) interpolation of the tabulated correlation function
// (paper App. B: tabulated, interpolated with cubics).  Node k holds the value at
// s = (k - 1) h; a query s in [k-1, k) h uses nodes k-1 .. k+2.
#pragma once
#include <hip/hip_runtime.h>
#include "kconst.h"

namespace flints {

// Returns false (and clamps) when s lies beyond the table.
__host__ __device__ inline bool table_lookup(const double *tab, int ntab, int nf, double inv_h,
                                             double s, double *f) {
  double x = s * inv_h + 1.0;
  int k = (int)x;
  double t = x - (double)k;
  bool inr = true;
  if (k > ntab - 3) { k = ntab - 3; t = 1.0; inr = false; }
  if (k < 1) { k = 1; t = 0.0; }
  const double tm1 = t - 1.0, tm2 = t - 2.0, tp1 = t + 1.0;
  const double sixth = kconst(1.0 / 6.0);
  const double w0 = -t * tm1 * tm2 * sixth;
  const double w1 = tp1 * tm1 * tm2 * 0.5;
  const double w2 = -tp1 * t * tm2 * 0.5;
  const double w3 = tp1 * t * tm1 * sixth;
  const double *p = tab + (k - 1) * nf;
  for (int q = 0; q < nf; ++q)
    f[q] = w0 * p[q] + w1 * p[nf + q] + w2 * p[2 * nf + q] + w3 * p[3 * nf + q];
  return inr;
}

}  // namespace flints
