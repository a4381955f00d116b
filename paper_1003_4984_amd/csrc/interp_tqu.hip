// T + Q/U with one stencil search per target: the shared-stencil passes, the
// pooled stencil buffer and the static workspace of the no-allocation call.
#include "interp_kernels.h"

namespace flints {

// Targets per chunk of the shared-stencil T + Q/U path (a multiple of 4; the
// stencil buffer holds K ints per target of one chunk: 2 GiB at K = 32).
constexpr int64_t TQU_CHUNK = int64_t(1) << 24;

// Workspaces (stencil buffers of the T + Q/U path, target directions of the
// supersampling call) come from a memory pool per device that keeps what is
// freed (release threshold unlimited), so after the first call the
// stream-ordered allocation reuses the same memory instead of asking the driver
// again.  Returns nullptr if the device has no pool support (the default pool
// is then used).
hipMemPool_t workspace_pool() {
  static std::mutex mu;
  static std::map<int, hipMemPool_t> pools;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return nullptr;
  std::lock_guard<std::mutex> g(mu);
  auto it = pools.find(dev);
  if (it != pools.end()) return it->second;
  hipMemPoolProps props;
  std::memset(&props, 0, sizeof(props));
  props.allocType = hipMemAllocationTypePinned;
  props.location.type = hipMemLocationTypeDevice;
  props.location.id = dev;
  hipMemPool_t pool = nullptr;
  if (hipMemPoolCreate(&pool, &props) != hipSuccess) {
    (void)hipGetLastError();
    pool = nullptr;
  } else {
    uint64_t keep = UINT64_MAX;
    if (hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep) != hipSuccess)
      (void)hipGetLastError();
  }
  pools[dev] = pool;
  return pool;
}

// Workspace of flints_interpolate_tqu_noalloc: the stencil hand-over buffer in
// a static device array (every device the library runs on holds its own copy
// until the process ends).  Host code never uses the name `scratch` as an
// address: the device address comes from hipGetSymbolAddress, once per device.
constexpr size_t NOALLOC_SCRATCH_BYTES = size_t(64) << 20;
static __device__ __align__(256) int scratch[NOALLOC_SCRATCH_BYTES / sizeof(int)];

static int *scratch_address() {
  static std::mutex mu;
  static std::map<int, int *> addr;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) {
    set_error("no current HIP device");
    return nullptr;
  }
  std::lock_guard<std::mutex> g(mu);
  auto it = addr.find(dev);
  if (it != addr.end()) return it->second;
  void *ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr) {
    set_error(std::string("device address of the static workspace: ") + hipGetErrorString(e));
    return nullptr;
  }
  addr[dev] = (int *)ptr;
  return (int *)ptr;
}

// Shared-stencil T + Q/U: per chunk the spin-2 main pass (which writes the
// stencils) and then the spin-0 main pass (which reads them), each with the
// layout and block size of its single-plan path; then both fix-up passes.
// The stencil buffer is stream-ordered (allocated and freed on s); if it
// cannot be allocated, each plan runs its own searching pass.
template <int NT0, int NT2, int T2>
static int launch_tqu_t(const Plan *p0, const Plan *p2, const double *map0, const double *map2,
                        const double *theta, const double *phi, int64_t n, double *out0, double *var0,
                        double *out2, double *var2, hipStream_t s, int *ws, int64_t ws_targets) {
  constexpr int SCR = T2 ? (T2 - 1) * TILE_D + 16 : 0;
  constexpr int PPW2 = T2 ? 1 : 4;
  const DevLimits lim = device_limits();
  const int K = p0->d.K;
  Layout L2 = make_layout(p2->d.ntab, p2->d.nfun, K, p2->d.n, PPW2, 1, 3, SCR);
  // The tile pass reads the correlation table through the caches instead of
  // an LDS copy: the 64-row systems then fit eight waves per CU (20,480 B of
  // LDS each at K = 32) instead of seven.
  if (T2) L2.tab_bytes = 0;
  const Layout L0 = make_layout(p0->d.ntab, p0->d.nfun, K, p0->d.n, 4, 1, 2);
  auto k2 = [] {
    if constexpr (T2 != 0) return k_interp_tile_st<T2>;
    else return k_interp_rs_st<NT2>;
  }();
  auto k0 = k_interp_rs_ld<NT0>;
  int wpb2 = 0, occ2 = 0, wpb0 = 0, occ0 = 0;
  if (!pick_wpb(k2, L2, lim, wpb2, occ2) || !pick_wpb(k0, L0, lim, wpb0, occ0)) return FLINTS_ELIMIT;
  const int lds2 = L2.tab_bytes + wpb2 * L2.wave_bytes;
  const int lds0 = L0.tab_bytes + wpb0 * L0.wave_bytes;
  // ws (when given) holds ws_targets stencils, a multiple of 4; otherwise the
  // buffer is allocated on the stream from the library's pool
  const int64_t chunk = std::min<int64_t>(ws ? ws_targets : TQU_CHUNK, (n + 3) & ~int64_t(3));
  int *stn = ws;
  if (!ws) {
    const size_t bytes = (size_t)chunk * K * sizeof(int);
    hipMemPool_t pool = workspace_pool();
    const hipError_t e = pool ? hipMallocFromPoolAsync((void **)&stn, bytes, pool, s)
                              : hipMallocAsync((void **)&stn, bytes, s);
    if (e != hipSuccess) {
      (void)hipGetLastError();   // no buffer: one searching pass per plan instead
      const int rc = launch_interpolate(p0, map0, theta, phi, n, out0, var0, s);
      return rc != FLINTS_OK ? rc : launch_interpolate(p2, map2, theta, phi, n, out2, var2, s);
    }
  }
  hipFuncSetAttribute((const void *)k2, hipFuncAttributeMaxDynamicSharedMemorySize, lds2);
  hipFuncSetAttribute((const void *)k0, hipFuncAttributeMaxDynamicSharedMemorySize, lds0);
  for (int64_t s0 = 0; s0 < n; s0 += chunk) {
    const int64_t s1 = std::min(n, s0 + chunk);
    const int64_t g2 = (s1 - s0 + PPW2 - 1) / PPW2, g0 = (s1 - s0 + 3) / 4;
    const int64_t b2 = std::max<int64_t>(std::min<int64_t>((g2 + wpb2 - 1) / wpb2, (int64_t)lim.ncu * occ2), 1);
    const int64_t b0 = std::max<int64_t>(std::min<int64_t>((g0 + wpb0 - 1) / wpb0, (int64_t)lim.ncu * occ0), 1);
    hipLaunchKernelGGL(k2, dim3((unsigned)b2), dim3(wpb2 * WAVE), lds2, s, p2->d, map2, theta, phi, n,
                       out2, var2, L2, stn, s0, s1);
    hipLaunchKernelGGL(k0, dim3((unsigned)b0), dim3(wpb0 * WAVE), lds0, s, p0->d, map0, theta, phi, n,
                       out0, var0, L0, (const int *)stn, s0, s1);
  }
  if (!ws) (void)hipFreeAsync(stn, s);
  auto esc2 = [] {
    if constexpr (T2 != 0) return k_fixup<TileEngine<T2, 2>, 2>;
    else return k_fixup<RowGroupEngine<NT2, 2>, 2>;
  }();
  auto esc0 = k_fixup<RowGroupEngine<NT0, 0>, 0>;
  const int64_t nch = (n + WAVE - 1) / WAVE;
  const int64_t e2 = std::max<int64_t>(std::min<int64_t>((nch + wpb2 - 1) / wpb2, (int64_t)lim.ncu * 4), 1);
  const int64_t e0 = std::max<int64_t>(std::min<int64_t>((nch + wpb0 - 1) / wpb0, (int64_t)lim.ncu * 4), 1);
  hipFuncSetAttribute((const void *)esc2, hipFuncAttributeMaxDynamicSharedMemorySize, lds2);
  hipLaunchKernelGGL(esc2, dim3((unsigned)e2), dim3(wpb2 * WAVE), lds2, s, p2->d, map2, theta, phi, n,
                     out2, var2, L2);
  hipFuncSetAttribute((const void *)esc0, hipFuncAttributeMaxDynamicSharedMemorySize, lds0);
  hipLaunchKernelGGL(esc0, dim3((unsigned)e0), dim3(wpb0 * WAVE), lds0, s, p0->d, map0, theta, phi, n,
                     out0, var0, L0);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    set_error(std::string("T + Q/U interpolation launch failed: ") + hipGetErrorString(e));
    return FLINTS_EDEVICE;
  }
  return FLINTS_OK;
}

// True when the shared-stencil path applies: FP64 plans with paper variance (or no
// variance requested) and one stencil for both, i.e. equal N_side, K and search
// radii, with K <= 32.
bool tqu_shareable(const Plan *p0, const Plan *p2, const double *var0, const double *var2) {
  const PlanDev &a = p0->d, &b = p2->d;
  const bool mse0 = a.var_kind == FLINTS_VAR_MSE && var0 != nullptr;
  const bool mse2 = b.var_kind == FLINTS_VAR_MSE && var2 != nullptr;
  return a.stencil_mode == FLINTS_STENCIL_NEAREST && b.stencil_mode == FLINTS_STENCIL_NEAREST &&
         a.precision == FLINTS_FP64 && b.precision == FLINTS_FP64 && !mse0 && !mse2 &&
         a.nside == b.nside && a.K == b.K && a.K <= 32 && a.r0 == b.r0 && a.rcap == b.rcap;
}

static int tqu_dispatch(const Plan *p0, const Plan *p2, const double *map0, const double *map2,
                        const double *theta, const double *phi, int64_t n, double *out0, double *var0,
                        double *out2, double *var2, hipStream_t s, int *ws, int64_t ws_targets) {
  const int K = p0->d.K;
  if (K <= 8)
    return launch_tqu_t<1, 1, 0>(p0, p2, map0, map2, theta, phi, n, out0, var0, out2, var2, s, ws, ws_targets);
  if (K <= 16)
    return launch_tqu_t<1, 2, 0>(p0, p2, map0, map2, theta, phi, n, out0, var0, out2, var2, s, ws, ws_targets);
  if (K <= 24)
    return launch_tqu_t<2, 0, 3>(p0, p2, map0, map2, theta, phi, n, out0, var0, out2, var2, s, ws, ws_targets);
  return launch_tqu_t<2, 0, 4>(p0, p2, map0, map2, theta, phi, n, out0, var0, out2, var2, s, ws, ws_targets);
}

int launch_interpolate_tqu(const Plan *p0, const Plan *p2, const double *map0, const double *map2,
                           const double *theta, const double *phi, int64_t n, double *out0,
                           double *var0, double *out2, double *var2, hipStream_t s) {
  if (n == 0) return FLINTS_OK;
  if (!tqu_shareable(p0, p2, var0, var2)) {
    const int rc = launch_interpolate(p0, map0, theta, phi, n, out0, var0, s);
    if (rc != FLINTS_OK) return rc;
    return launch_interpolate(p2, map2, theta, phi, n, out2, var2, s);
  }
  return tqu_dispatch(p0, p2, map0, map2, theta, phi, n, out0, var0, out2, var2, s, nullptr, 0);
}

// The same call with the stencil buffer in the static workspace: targets run
// in chunks of what it holds (64 MiB / (4 K) stencils, at least 262,144
// targets for K <= 64), so nothing is allocated.
int launch_interpolate_tqu_noalloc(const Plan *p0, const Plan *p2, const double *map0,
                                   const double *map2, const double *theta, const double *phi,
                                   int64_t n, double *out0, double *var0, double *out2, double *var2,
                                   hipStream_t s) {
  if (n == 0) return FLINTS_OK;
  if (!tqu_shareable(p0, p2, var0, var2)) {
    const int rc = launch_interpolate(p0, map0, theta, phi, n, out0, var0, s);
    if (rc != FLINTS_OK) return rc;
    return launch_interpolate(p2, map2, theta, phi, n, out2, var2, s);
  }
  const int K = p0->d.K;
  const int64_t cap = (int64_t)(NOALLOC_SCRATCH_BYTES / (sizeof(int) * (size_t)K)) & ~int64_t(3);
  if (cap < 4) {
    set_error("K is too large for the static workspace of the no-allocation call");
    return FLINTS_ELIMIT;
  }
  int *ws = scratch_address();
  if (!ws) return FLINTS_EDEVICE;
  return tqu_dispatch(p0, p2, map0, map2, theta, phi, n, out0, var0, out2, var2, s, ws, cap);
}


}  // namespace flints
