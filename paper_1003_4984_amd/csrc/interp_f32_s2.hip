// FP32 + refinement main passes, spin 2, with their FP64 fix-up passes.
#include "interp_kernels.h"

namespace flints {

int launch_fp32_s2(const Plan *p, const double *map, const double *theta, const double *phi,
                   int64_t n, double *out, double *var, hipStream_t s) {
  return launch_spin<2, false, true>(p, map, theta, phi, n, out, var, s);
}

}  // namespace flints
