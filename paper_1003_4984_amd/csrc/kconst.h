// FP64 constant materialised at its point of use on the device.
//
// The interpolation kernels run persistent loops with very large bodies; the
// compiler otherwise hoists every FP64 constant (polynomial coefficients,
// interpolation weights, pi) into a register that stays live for the whole
// kernel, which pushes the factorisation phase into scratch spills.  An empty
// volatile asm on a scalar register pair cannot be hoisted, so the constant is
// rebuilt with two scalar moves where it is needed.  Host code gets the value.
#pragma once
#include <hip/hip_runtime.h>

namespace flints {

__host__ __device__ __forceinline__ double kconst(double v) {
#if defined(__HIP_DEVICE_COMPILE__)
  __asm__ volatile("" : "+s"(v));
#endif
  return v;
}

}  // namespace flints
