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

// Ring i (1-based, 1 <= i <= 4N-1).  The three zones' formulas are evaluated
// on selected arguments without branches (lanes of one wave often hold rings of
// different zones), so each call takes one square root and the results equal
// the zone-by-zone evaluation bit for bit.
__host__ __device__ inline Ring ring_geom(int64_t N, int32_t i) {
  Ring r;
  const double TWO_PI = kconst(6.28318530717958647692);
  const bool north = i < N, south = i > 3 * N, cap = north || south;
  const int32_t k = south ? (int32_t)(4 * N - i) : i;              // caps: rings from the pole
  const double omz = (double)k * (double)k / (3.0 * (double)N * (double)N);   // caps: 1 - |z|
  const double zb = 2.0 * (double)(2 * N - i) / (3.0 * (double)N);           // belt
  r.z = north ? 1.0 - omz : (south ? -(1.0 - omz) : zb);
  r.s = sqrt(cap ? omz * (2.0 - omz) : (1.0 - zb) * (1.0 + zb));
  r.n = 4 * (cap ? k : (int32_t)N);
  r.dphi = TWO_PI / (double)r.n;
  r.phi0 = (cap || ((i - N) & 1) == 0) ? 0.5 * r.dphi : 0.0;
  r.first = north ? 2 * (int64_t)i * (int64_t)(i - 1)
                  : (south ? 12 * N * N - 2 * (int64_t)k * (int64_t)(k + 1)
                           : 2 * N * (N - 1) + 4 * N * (int64_t)(i - N));
  return r;
}

// floor(sqrt(x)) for 0 <= x < 2^53: the correctly rounded square root of x is at
// most one above it, so one correction each way is exact.
__host__ __device__ inline int64_t isqrt64(int64_t x) {
  int64_t v = (int64_t)sqrt((double)x);
  v -= (v * v > x);
  v += ((v + 1) * (v + 1) <= x);
  return v;
}

// 1-based ring of RING pixel p (caps from the pixel's distance to the nearer
// pole, the belt by a 32-bit division: p - ncap < 8 N^2 < 2^32), without branches.
__host__ __device__ inline int32_t pix_ring(int64_t N, int64_t p) {
  const int64_t ncap = 2 * N * (N - 1);
  const int64_t npix = 12 * N * N;
  const bool north = p < ncap, south = p >= npix - ncap;
  const int64_t q = south ? npix - 1 - p : p;
  const int32_t rc = (int32_t)((1 + isqrt64(1 + 2 * q)) >> 1);
  const uint32_t pb = north || south ? 0u : (uint32_t)(p - ncap);
  const int32_t rb = (int32_t)(pb / (uint32_t)(4 * N)) + (int32_t)N;
  return north ? rc : (south ? (int32_t)(4 * N) - rc : rb);
}

// Continuous ring coordinate of colatitude cosine z (ring i sits at i exactly).
__host__ __device__ inline double ring_coord(int64_t N, double z) {
  const double twothird = kconst(2.0 / 3.0);
  if (z >= twothird) return (double)N * sqrt(3.0 * (1.0 - z));
  if (z <= -twothird) return 4.0 * (double)N - (double)N * sqrt(3.0 * (1.0 + z));
  return (double)N * (2.0 - 1.5 * z);
}

}  // namespace flints
