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
  // Stencil tied to the containing pixel (FLINTS_STENCIL_PIXEL): per ring its
  // first class and quadrant size (0: one class for the whole ring), per class
  // the stencil of its representative pixel as (ring << 16 | j) and the
  // Cholesky factor of S + n I (packed rows, 1 / L_ii on the diagonal).
  int32_t stencil_mode;
  int32_t lsz;         // doubles per class factor, n (n + 1) / 2
  int32_t map_f32;     // maps hold float32 values (read and widened to FP64)
  int32_t pad_;
  const int64_t *cls_base;   // [4 nside] (index by ring)
  const int32_t *cls_quad;   // [4 nside]
  const int32_t *cls_stn;    // [nclass][K]
  const double *cls_L;       // [nclass][lsz]
};

struct Plan {
  PlanDev d;
  int device;
  int lmax;
  double table_err;
  int64_t nclass = 0;          // pixel classes of the fixed-stencil tables
  int64_t class_nuggets = 0;   // classes whose factorisation needed -lambda_min + eps
  int64_t *d_cls_base = nullptr;
  int32_t *d_cls_quad = nullptr;
  int32_t *d_cls_stn = nullptr;
  double *d_cls_L = nullptr;
  double fp32_reject = -1.0;   // FP32 probe: fraction of systems rejected (-1: not probed)
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
int launch_interpolate_tqu_noalloc(const Plan *p0, const Plan *p2, const double *map0,
                                   const double *map2, const double *theta, const double *phi,
                                   int64_t n, double *out0, double *var0, double *out2, double *var2,
                                   hipStream_t s);
bool tqu_shareable(const Plan *p0, const Plan *p2, const double *var0, const double *var2);
int launch_stencil(const Plan *p, const double *theta, const double *phi, int64_t n,
                   int64_t *idx, hipStream_t s);
int launch_table_eval(const Plan *p, const double *s, int64_t n, double *out, hipStream_t st);
// Stream-ordered workspace pool of the current device (interp_tqu.hip);
// nullptr if pools are unsupported.
hipMemPool_t workspace_pool();
// Supersampling (supersample.hip): every pixel centre of a RING map of nside_out.
int launch_supersample(const Plan *p, const double *map, int64_t nside_out, double *out, double *var,
                       hipStream_t s);
int launch_pixel_centres(int64_t nside, double *theta, double *phi, hipStream_t s);
// Lensing pipeline (sht.hip): spin-s synthesis of a RING map from a_lm, and
// the displaced pixel centres for a deflection map.
int launch_synthesize(int64_t N, int lmax, int spin, const double *alm, const double *blm, double *map,
                      hipStream_t s);
int launch_lensed_directions(int64_t N, const double *defl, double *theta, double *phi, hipStream_t s);
// Fixed-stencil tables (fixed.hip): classes, representative stencils and
// factors; and the per-target and stencil launchers of that mode.
int build_fixed(Plan *p);
void free_fixed(Plan *p);
int launch_fixed(const Plan *p, const double *map, const double *theta, const double *phi, int64_t n,
                 double *out, double *var, hipStream_t s);
int launch_fixed_stencil(const Plan *p, const double *theta, const double *phi, int64_t n, int64_t *idx,
                         hipStream_t s);
// FP32_IR conditioning probe (interp.hip): fraction of fixed probe systems the
// FP32 path rejects, in [0, 1], or < 0 with the error set.
double fp32_probe(Plan *p);

}  // namespace flints
