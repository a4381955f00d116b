// Internal plan representation shared by the HIP translation units.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string>
#include "../../include/flints.h"

namespace flints {

enum Counter {
  CNT_BAD_INPUT = 0,
  CNT_NUGGET_ESC = 1,
  CNT_CLAMPED_VAR = 2,
  CNT_FP64_FALLBACK = 3,
  CNT_SEARCH_FAIL = 4,
  CNT_TABLE_RANGE = 5,
  CNT_N = 8
};

// Plain-old-data view of a plan, passed by value to kernels.
struct PlanDev {
  int64_t nside, npix;
  int32_t K, spin, mode, nug_policy, var_kind, precision;
  int32_t n;           // rows of the neighbour system: K (spin 0) or 2K (spin 2)
  int32_t ntab, nfun;  // table nodes per function, functions per node
  double h, inv_h;     // node spacing in s = sin(beta/2); node k sits at s = (k - 1) h
  double smax;         // largest s the table covers
  double sigma2;       // prior variance per output field
  double eps;          // nugget epsilon (2^-26)
  double r0, rcap;     // search radii (angles, rad)
  double pivot_ratio_min, refine_tol;
  const double *tab;   // [ntab][nfun], normalised correlation values
  unsigned long long *counters;  // [CNT_N]
};

struct Plan {
  PlanDev d;
  int device;
  int lmax;
  double table_err;
  double *d_tab = nullptr;
  unsigned long long *d_counters = nullptr;
};

// Error reporting helpers (thread-local message).
void set_error(const std::string &msg);

// Table construction (tables.hip).  Fills plan->d_tab, d.ntab, d.h, table_err.
int build_table(Plan *p, const double *w_plus, const double *w_minus, double tol);

// Kernel launchers (interp.hip).
int launch_interpolate(const Plan *p, const double *map, const double *theta, const double *phi,
                       int64_t n, double *out, double *var, hipStream_t s);
int launch_interpolate_tqu(const Plan *p0, const Plan *p2, const double *map0, const double *map2,
                           const double *theta, const double *phi, int64_t n, double *out0,
                           double *var0, double *out2, double *var2, hipStream_t s);
bool tqu_shareable(const Plan *p0, const Plan *p2, const double *var0, const double *var2);
int launch_stencil(const Plan *p, const double *theta, const double *phi, int64_t n,
                   int64_t *idx, hipStream_t s);
int launch_table_eval(const Plan *p, const double *s, int64_t n, double *out, hipStream_t st);

}  // namespace flints
