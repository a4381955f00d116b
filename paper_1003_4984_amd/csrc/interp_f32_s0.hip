// FP32 + refinement main passes, spin 0, with their FP64 fix-up passes.
#include "interp_kernels.h"

namespace flints {

int launch_fp32_s0(const Plan *p, const double *map, const double *theta, const double *phi,
                   int64_t n, double *out, double *var, hipStream_t s) {
  return launch_spin<0, false, true>(p, map, theta, phi, n, out, var, s);
}

}  // namespace flints
