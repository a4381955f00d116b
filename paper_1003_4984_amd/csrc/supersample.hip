// Supersampling (paper Sec. 2.6, Table 1): a RING map of the plan's N_side is
// interpolated at every pixel centre of a RING map of another resolution
// (N_side -> 2 N_side in the paper).  The target directions are the pixel
// centres of the output map, generated on the device in RING order into a
// workspace from the library's pool; the interpolation is flints_interpolate
// over them, so the output is a RING map (spin 2: the Q map, then the U map).
#include "plan.h"
#include "healpix_ring.h"
#include <algorithm>
#include <string>

namespace flints {

// Pixel centres of RING pixels [0, n) at resolution N: theta from the ring's
// (sin, cos) pair (accurate at the poles), phi = phi0 + j dphi.
__global__ void k_pixel_centres(int64_t N, int64_t n, double *__restrict__ theta, double *__restrict__ phi) {
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += (int64_t)gridDim.x * blockDim.x) {
    const Ring R = ring_geom(N, pix_ring(N, p));
    theta[p] = atan2(R.s, R.z);
    phi[p] = R.phi0 + (double)(p - R.first) * R.dphi;
  }
}

int launch_pixel_centres(int64_t nside, double *theta, double *phi, hipStream_t s) {
  const int64_t n = 12 * nside * nside;
  const int threads = 256;
  const int64_t blocks = std::min<int64_t>((n + threads - 1) / threads, 65536);
  hipLaunchKernelGGL(k_pixel_centres, dim3((unsigned)blocks), dim3(threads), 0, s, nside, n, theta, phi);
  const hipError_t le = hipGetLastError();
  if (le != hipSuccess) {
    set_error(std::string("pixel-centre kernel launch failed: ") + hipGetErrorString(le));
    return FLINTS_EDEVICE;
  }
  return FLINTS_OK;
}

int launch_supersample(const Plan *p, const double *map, int64_t nside_out, double *out, double *var,
                       hipStream_t s) {
  const int64_t n = 12 * nside_out * nside_out;
  double *dir = nullptr;
  const size_t bytes = (size_t)n * 2 * sizeof(double);
  hipMemPool_t pool = workspace_pool();
  const hipError_t e = pool ? hipMallocFromPoolAsync((void **)&dir, bytes, pool, s)
                            : hipMallocAsync((void **)&dir, bytes, s);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    set_error("workspace allocation for the output pixel centres failed");
    return FLINTS_ENOMEM;
  }
  int rc = launch_pixel_centres(nside_out, dir, dir + n, s);
  if (rc == FLINTS_OK) rc = launch_interpolate(p, map, dir, dir + n, n, out, var, s);
  (void)hipFreeAsync(dir, s);
  return rc;
}

}  // namespace flints
