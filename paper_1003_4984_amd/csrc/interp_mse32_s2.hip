// Register-row launchers of the MSE variance, FP32 + refinement, spin 2.
#include "interp_kernels.h"

namespace flints {

int launch_mse_fp32_s2(const Plan *p, const double *map, const double *theta, const double *phi,
                       int64_t n, double *out, double *var, hipStream_t s) {
  return launch_spin<2, true, true>(p, map, theta, phi, n, out, var, s);
}

}  // namespace flints
