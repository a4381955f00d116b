// Entry of the single-plan path (dispatch by spin, precision and variance
// kind) and the stencil-only kernel.
#include "interp_kernels.h"
#include <cmath>
#include <vector>

namespace flints {

// Stencil only (a2/a3): K nearest pixel indices per target.
__global__ __launch_bounds__(STENCIL_WPB * WAVE) void k_stencil(PlanDev P, const double *__restrict__ theta,
                                                 const double *__restrict__ phi, int64_t n,
                                                 int64_t *__restrict__ idx, Layout L) {
  extern __shared__ double lds_dyn[];
  char *lds = (char *)lds_dyn;
  const int wpb = blockDim.x / WAVE;
  const int wave = threadIdx.x / WAVE;
  const int lane = threadIdx.x % WAVE;
  char *wb = lds + wave * L.wave_bytes;
  double *cu = (double *)(wb + L.off_cu);
  int *ci = (int *)(wb + L.off_ci);
  RingSpan *rs = (RingSpan *)(wb + L.off_rings);
  int *sel = (int *)(wb + L.off_sel);
  const int K = P.K;
  for (int64_t pt = xcd_block() * wpb + wave; pt < n; pt += (int64_t)gridDim.x * wpb) {
    const double th = theta[pt], ph = phi[pt];
    const bool good = (th >= 0.0) && (th <= kconst(PI_D)) && isfinite(ph);
    bool found = false;
    if (good) found = knn_search(P, th, ph, lane, cu, ci, rs, sel);
    for (int k = lane; k < K; k += WAVE) idx[pt * K + k] = found ? (int64_t)sel[k] : -1;
    wave_lds_sync();
  }
}


// FP32_IR conditioning probe: the plan's FP32 main pass and fix-up pass over
// 512 directions of a Fibonacci lattice on the sphere (z_k = 1 - (2k+1)/512,
// phi_k = k times the golden angle), with no map (zero data: the acceptance
// tests of the FP32 path do not depend on the data).  Every rejected system is
// recomputed in FP64 by the fix-up pass and counted; the count over 512 is the
// rejection fraction.  The plan's counters are zero again afterwards.
double fp32_probe(Plan *p) {
  constexpr int NP = 512;
  std::vector<double> hth(NP), hph(NP);
  const double ga = PI_D * (3.0 - std::sqrt(5.0));
  for (int k = 0; k < NP; ++k) {
    const double z = 1.0 - (2.0 * k + 1.0) / NP;
    hth[k] = std::acos(z);
    hph[k] = std::fmod(k * ga, TWO_PI_D);
  }
  const size_t nf = p->d.spin == 0 ? 1 : 2;
  double *dth = nullptr, *dph = nullptr, *dout = nullptr;
  auto cleanup = [&] {
    if (dth) (void)hipFree(dth);
    if (dph) (void)hipFree(dph);
    if (dout) (void)hipFree(dout);
  };
  if (hipMalloc(&dth, NP * sizeof(double)) != hipSuccess || hipMalloc(&dph, NP * sizeof(double)) != hipSuccess ||
      hipMalloc(&dout, NP * nf * sizeof(double)) != hipSuccess) {
    cleanup();
    set_error("device allocation of the FP32 probe failed");
    return -1.0;
  }
  unsigned long long c[CNT_N];
  bool ok = hipMemcpy(dth, hth.data(), NP * sizeof(double), hipMemcpyHostToDevice) == hipSuccess &&
            hipMemcpy(dph, hph.data(), NP * sizeof(double), hipMemcpyHostToDevice) == hipSuccess &&
            hipMemset(p->d_counters, 0, sizeof(c)) == hipSuccess;
  if (ok) ok = launch_interpolate(p, nullptr, dth, dph, NP, dout, nullptr, nullptr) == FLINTS_OK;
  if (ok)
    ok = hipStreamSynchronize(nullptr) == hipSuccess &&
         hipMemcpy(c, p->d_counters, sizeof(c), hipMemcpyDeviceToHost) == hipSuccess &&
         hipMemset(p->d_counters, 0, sizeof(c)) == hipSuccess && hipDeviceSynchronize() == hipSuccess;
  cleanup();
  if (!ok) {
    set_error("the FP32 conditioning probe failed");
    return -1.0;
  }
  return (double)c[CNT_FP64_FALLBACK] / NP;
}

int launch_interpolate(const Plan *p, const double *map, const double *theta, const double *phi,
                       int64_t n, double *out, double *var, hipStream_t s) {
  if (n == 0) return FLINTS_OK;
  if (p->d.stencil_mode == FLINTS_STENCIL_PIXEL) return launch_fixed(p, map, theta, phi, n, out, var, s);
  const bool mse = (p->d.var_kind == FLINTS_VAR_MSE) && var != nullptr;
  const bool f32 = p->d.precision == FLINTS_FP32_IR;
  if (mse) {
    if (p->d.spin == 0)
      return f32 ? launch_mse_fp32_s0(p, map, theta, phi, n, out, var, s)
                 : launch_mse_fp64_s0(p, map, theta, phi, n, out, var, s);
    return f32 ? launch_mse_fp32_s2(p, map, theta, phi, n, out, var, s)
               : launch_mse_fp64_s2(p, map, theta, phi, n, out, var, s);
  }
  if (f32) return p->d.spin == 0 ? launch_fp32_s0(p, map, theta, phi, n, out, var, s)
                                 : launch_fp32_s2(p, map, theta, phi, n, out, var, s);
  return p->d.spin == 0 ? launch_fp64_s0(p, map, theta, phi, n, out, var, s)
                        : launch_fp64_s2(p, map, theta, phi, n, out, var, s);
}

int launch_stencil(const Plan *p, const double *theta, const double *phi, int64_t n, int64_t *idx,
                   hipStream_t s) {
  if (n == 0) return FLINTS_OK;
  if (p->d.stencil_mode == FLINTS_STENCIL_PIXEL) return launch_fixed_stencil(p, theta, phi, n, idx, s);
  const DevLimits lim = device_limits();
  Layout L = make_layout(0, 1, p->d.K, 1, 1, 1, 2);
  const int wpb = STENCIL_WPB;
  const int lds = wpb * L.wave_bytes;
  hipFuncSetAttribute((const void *)k_stencil, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
  int64_t blocks = std::min<int64_t>((n + wpb - 1) / wpb, (int64_t)lim.ncu * 8);
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_stencil, dim3((unsigned)blocks), dim3(wpb * WAVE), lds, s, p->d, theta,
                     phi, n, idx, L);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    set_error(std::string("stencil kernel launch failed: ") + hipGetErrorString(e));
    return FLINTS_EDEVICE;
  }
  return FLINTS_OK;
}

}  // namespace flints
