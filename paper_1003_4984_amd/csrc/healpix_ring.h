// HEALPix RING geometry for device and host code (Gorski et al. 2005 layout):
// 4*nside-1 iso-latitude rings; polar-cap ring i (< nside) has 4i pixels at
// z = 1 - i^2/(3 nside^2), phi_j = (j + 1/2) pi/(2i); belt rings have 4 nside
// pixels at z = (4 nside - 2 i)/(3 nside), phi_j = (j + s/2) pi/(2 nside) with
// s = 1 when (i - nside) is even; the south cap mirrors the north one.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <math.h>
#include "kconst.h"

namespace flints {

struct Ring {
  double z;      // cos(theta)
  double s;      // sin(theta), computed without cancellation near the poles
  double phi0;   // phi of the first pixel
  double dphi;   // pixel spacing in phi
  int64_t first; // RING index of the first pixel
  int32_t n;     // pixels in the ring
};

// Ring i (1-based, 1 <= i <= 4N-1).
__host__ __device__ inline Ring ring_geom(int64_t N, int32_t i) {
  Ring r;
  const double TWO_PI = kconst(6.28318530717958647692);
  if (i < N) {
    double omz = (double)i * (double)i / (3.0 * (double)N * (double)N);
    r.z = 1.0 - omz;
    r.s = sqrt(omz * (2.0 - omz));
    r.n = 4 * i;
    r.dphi = TWO_PI / (double)r.n;
    r.phi0 = 0.5 * r.dphi;
    r.first = 2 * (int64_t)i * (int64_t)(i - 1);
  } else if (i <= 3 * N) {
    r.z = 2.0 * (double)(2 * N - i) / (3.0 * (double)N);
    r.s = sqrt((1.0 - r.z) * (1.0 + r.z));
    r.n = (int32_t)(4 * N);
    r.dphi = TWO_PI / (double)r.n;
    r.phi0 = (((i - N) & 1) == 0) ? 0.5 * r.dphi : 0.0;
    r.first = 2 * N * (N - 1) + 4 * N * (int64_t)(i - N);
  } else {
    int32_t k = (int32_t)(4 * N - i);
    double omz = (double)k * (double)k / (3.0 * (double)N * (double)N);
    r.z = -(1.0 - omz);
    r.s = sqrt(omz * (2.0 - omz));
    r.n = 4 * k;
    r.dphi = TWO_PI / (double)r.n;
    r.phi0 = 0.5 * r.dphi;
    r.first = 12 * N * N - 2 * (int64_t)k * (int64_t)(k + 1);
  }
  return r;
}

__host__ __device__ inline int64_t isqrt64(int64_t x) {
  int64_t v = (int64_t)sqrt((double)x);
  while (v * v > x) --v;
  while ((v + 1) * (v + 1) <= x) ++v;
  return v;
}

// 1-based ring of RING pixel p.
__host__ __device__ inline int32_t pix_ring(int64_t N, int64_t p) {
  const int64_t ncap = 2 * N * (N - 1);
  const int64_t npix = 12 * N * N;
  if (p < ncap) return (int32_t)((1 + isqrt64(1 + 2 * p)) >> 1);
  if (p < npix - ncap) return (int32_t)((p - ncap) / (4 * N) + N);
  int64_t q = npix - 1 - p;
  return (int32_t)(4 * N - ((1 + isqrt64(1 + 2 * q)) >> 1));
}

// Continuous ring coordinate of colatitude cosine z (ring i sits at i exactly).
__host__ __device__ inline double ring_coord(int64_t N, double z) {
  const double twothird = kconst(2.0 / 3.0);
  if (z >= twothird) return (double)N * sqrt(3.0 * (1.0 - z));
  if (z <= -twothird) return 4.0 * (double)N - (double)N * sqrt(3.0 * (1.0 + z));
  return (double)N * (2.0 - 1.5 * z);
}

}  // namespace flints
