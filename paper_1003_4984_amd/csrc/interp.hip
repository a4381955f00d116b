// FLINTS single-plan kernels and launchers for gfx950 (CDNA4): the row-group
// path (n <= 32), the tile path (32 < n <= 64), the register-row path (MSE
// variance and the FP32 + refinement main pass), their fix-up passes and the
// stencil kernel.  The device code they run lives in device.h.
#include "device.h"
#include <algorithm>
#include <cstring>
#include <mutex>
#include <map>
#include <tuple>
#include <utility>

namespace flints {

// Main pass over all targets (FP32 selects the FP32 + refinement phase B).
template <int NMAX, int G, int SPIN, bool MSE, bool FP32>
__global__ __launch_bounds__(MAX_WPB * WAVE) void k_interp64(PlanDev P, const double *__restrict__ map,
                                                  const double *__restrict__ theta,
                                                  const double *__restrict__ phi, int64_t n,
                                                  double *__restrict__ out,
                                                  double *__restrict__ var, Layout L) {
  constexpr int PPW = WAVE / G;
  constexpr int NR = (SPIN == 0) ? 2 : 3;
  extern __shared__ double lds_dyn[];
  char *lds = (char *)lds_dyn;
  const double *tab = load_table(lds, P);
  const int wpb = blockDim.x / WAVE;
  const int wave = threadIdx.x / WAVE;
  const int lane = threadIdx.x % WAVE;
  const WaveBufs B = wave_bufs(lds, L, wave);
  const int nrow = P.n;
  const int K = P.K;
  const int64_t ngroups = (n + PPW - 1) / PPW;
  const int grp = lane / G;
  const int row = lane % G;
  const double nug = (P.nug_policy == FLINTS_NUG_ALWAYS) ? P.eps : 0.0;

  for (int64_t g = xcd_block() * wpb + wave; g < ngroups; g += (int64_t)gridDim.x * wpb) {
    unsigned act_mask = 0;
#pragma unroll 1
    for (int q = 0; q < PPW; ++q) {
      const int64_t pt = g * PPW + q;
      if (pt >= n) break;
      if (phase_a_search(P, theta[pt], phi[pt], lane, B.cu, B.ci, B.rs, B.sel + q * K))
        act_mask |= 1u << q;
    }
#pragma unroll 1
    for (int q = 0; q < PPW; ++q) {
      if (!((act_mask >> q) & 1u)) continue;
      const int64_t pt = g * PPW + q;
      phase_a_build<SPIN, NR>(P, tab, map, theta[pt], phi[pt], lane, B.sel + q * K, B.nb,
                              B.mat + q * L.matsz, B.rhs + q * nrow * NR);
    }
    const bool gact = (act_mask >> grp) & 1u;
    const bool ract = gact && row < nrow;
    int rowv = row;
    __asm__ volatile("" : "+v"(rowv));   // keeps row-dependent LDS addresses out of LICM
    GroupOut o;
    bool ok;
    if (FP32)
      ok = fp32_phase_b<NMAX, G, SPIN, NR, MSE>(P, B.mat + grp * L.matsz, B.rhs + grp * nrow * NR,
                                               rowv, grp, ract, nrow, nug, o);
    else
      ok = fp64_phase_b<NMAX, G, SPIN, NR, MSE>(B.mat + grp * L.matsz, B.rhs + grp * nrow * NR,
                                               rowv, grp, ract, nrow, nug, o);
    if (row == 0) {
      const int64_t pt = g * PPW + grp;
      if (pt < n)
        store_point<SPIN>(P, pt, n, gact, ok, FP32 ? FAIL32_BITS : FAIL64_BITS, o, nug, MSE, out, var);
    }
  }
}

// Fix-up pass over tagged points, one at a time.  A point rejected by the FP32
// path is recomputed in FP64 (counted as an FP64 fallback); an FP64
// factorisation failure gets the nugget of paper Sec. 2.4, n = mu + eps with mu
// the smallest shift for which S + mu I factorises (bisection on [n0, rows + 1];
// the upper end is positive definite by Gershgorin since |S_ij| <= 1).
// Untagged chunks cost one coalesced read of `out` per 64 points.
template <int NMAX, int G, int SPIN, bool MSE>
__global__ __launch_bounds__(MAX_WPB * WAVE) void k_escalate(PlanDev P, const double *__restrict__ map,
                                                  const double *__restrict__ theta,
                                                  const double *__restrict__ phi, int64_t n,
                                                  double *__restrict__ out,
                                                  double *__restrict__ var, Layout L) {
  constexpr int NR = (SPIN == 0) ? 2 : 3;
  extern __shared__ double lds_dyn[];
  char *lds = (char *)lds_dyn;
  const double *tab = load_table(lds, P);
  const int wpb = blockDim.x / WAVE;
  const int wave = threadIdx.x / WAVE;
  const int lane = threadIdx.x % WAVE;
  const WaveBufs B = wave_bufs(lds, L, wave);
  const int nrow = P.n;
  const int grp = lane / G;
  const int row = lane % G;
  const double nug0 = (P.nug_policy == FLINTS_NUG_ALWAYS) ? P.eps : 0.0;
  const int64_t nchunks = (n + WAVE - 1) / WAVE;
  for (int64_t ch = xcd_block() * wpb + wave; ch < nchunks; ch += (int64_t)gridDim.x * wpb) {
    const int64_t p0 = ch * WAVE + lane;
    const unsigned long long bits =
        p0 < n ? (unsigned long long)__double_as_longlong(out[p0]) : 0ull;
    const bool t64 = bits == FAIL64_BITS, t32 = bits == FAIL32_BITS;
    unsigned long long mask = __ballot(t64 || t32);
    const unsigned long long m32 = __ballot(t32);
    while (mask) {
      const int bit = __ffsll((long long)mask) - 1;
      mask &= mask - 1ull;
      const bool from32 = (m32 >> bit) & 1ull;
      const int64_t pt = ch * WAVE + bit;
      const bool found = phase_a_search(P, theta[pt], phi[pt], lane, B.cu, B.ci, B.rs, B.sel);
      if (found)
        phase_a_build<SPIN, NR>(P, tab, map, theta[pt], phi[pt], lane, B.sel, B.nb, B.mat, B.rhs);
      const bool gact = found && grp == 0;
      const bool ract = gact && row < nrow;
      GroupOut o;
      double nug = nug0;
      bool ok = false;
      if (from32) {
        ok = __all(fp64_phase_b<NMAX, G, SPIN, NR, MSE>(B.mat, B.rhs, row, grp, ract, nrow, nug, o) || !gact);
        if (lane == 0) atomicAdd(P.counters + CNT_FP64_FALLBACK, 1ull);
      }
      if (!ok) {
        double lo = nug0, hi = (double)nrow + 1.0;
#pragma unroll 1
        for (int it = 0; it < 64; ++it) {
          const double mu = 0.5 * (lo + hi);
          double a[NMAX];
          double r[NR];
          double diag;
          load_rows<NMAX, NR>(B.mat, B.rhs, row, ract, nrow, a, r);
          const bool ok2 = __all(chol_rows<NMAX, G, NR>(a, r, row, grp, mu, diag) || !gact);
          if (ok2) hi = mu; else lo = mu;
        }
        nug = hi + P.eps;
#pragma unroll 1
        for (int it = 0; it < 8 && !ok; ++it) {
          ok = __all(fp64_phase_b<NMAX, G, SPIN, NR, MSE>(B.mat, B.rhs, row, grp, ract, nrow, nug, o) ||
                     !gact);
          if (!ok) nug *= 2.0;
        }
        if (lane == 0) atomicAdd(P.counters + CNT_NUGGET_ESC, 1ull);
      }
      if (lane == 0) store_point<SPIN>(P, pt, n, gact, ok, FAIL64_BITS, o, nug, MSE, out, var);
    }
  }
}

// Main pass for systems of n <= 32 rows: four points per wave, one per 16-lane
// row group.  Every point of the group is searched first; then each is
// assembled in the wave's single system buffer and loaded into the registers
// of its row group before the next point reuses the buffer, and phase B runs
// for all four at once.
template <int NT, int SPIN>
__global__ __launch_bounds__(MAX_WPB * WAVE) void k_interp_rs(PlanDev P, const double *__restrict__ map,
                                                   const double *__restrict__ theta,
                                                   const double *__restrict__ phi, int64_t n,
                                                   double *__restrict__ out,
                                                   double *__restrict__ var, Layout L) {
  extern __shared__ double lds_dyn[];
  char *lds = (char *)lds_dyn;
  const double *tab = load_table(lds, P);
  const int wpb = blockDim.x / WAVE;
  const int wave = threadIdx.x / WAVE;
  const int lane = threadIdx.x % WAVE;
  const WaveBufs B = wave_bufs(lds, L, wave);
  const int64_t ngroups = (n + 3) / 4;
  for (int64_t g = xcd_block() * wpb + wave; g < ngroups; g += (int64_t)gridDim.x * wpb)
    group_rs<NT, SPIN>(P, tab, map, theta, phi, n, out, var, B, g * 4, lane);
}

// Fix-up pass of the row-group and tile paths (same policy as k_escalate).
template <class Eng, int SPIN>
__global__ __launch_bounds__(MAX_WPB * WAVE) void k_fixup(PlanDev P, const double *__restrict__ map,
                                               const double *__restrict__ theta,
                                               const double *__restrict__ phi, int64_t n,
                                               double *__restrict__ out,
                                               double *__restrict__ var, Layout L) {
  extern __shared__ double lds_dyn[];
  char *lds = (char *)lds_dyn;
  const double *tab = load_table(lds, P);
  const int wpb = blockDim.x / WAVE;
  const int wave = threadIdx.x / WAVE;
  const int lane = threadIdx.x % WAVE;
  const WaveBufs B = wave_bufs(lds, L, wave);
  const int64_t nchunks = (n + WAVE - 1) / WAVE;
  for (int64_t ch = xcd_block() * wpb + wave; ch < nchunks; ch += (int64_t)gridDim.x * wpb)
    fixup_chunk<Eng, SPIN>(P, tab, map, theta, phi, n, out, var, B, ch * WAVE, lane);
}

// Main pass for 32 < n <= 16 T: one point per wave, blocked tile Cholesky.
template <int T, int SPIN>
__global__ __launch_bounds__(MAX_WPB * WAVE) void k_interp_tile(PlanDev P, const double *__restrict__ map,
                                                     const double *__restrict__ theta,
                                                     const double *__restrict__ phi, int64_t n,
                                                     double *__restrict__ out,
                                                     double *__restrict__ var, Layout L) {
  extern __shared__ double lds_dyn[];
  char *lds = (char *)lds_dyn;
  const double *tab = load_table(lds, P);
  const int wpb = blockDim.x / WAVE;
  const int wave = threadIdx.x / WAVE;
  const int lane = threadIdx.x % WAVE;
  const WaveBufs B = wave_bufs(lds, L, wave);
  for (int64_t pt = xcd_block() * wpb + wave; pt < n; pt += (int64_t)gridDim.x * wpb)
    point_tile<T, SPIN>(P, tab, map, theta, phi, n, out, var, B, pt, lane);
}

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

// ---------------------------------------------------------------- launchers
struct DevLimits {
  int ncu = 0;
  int lds_max = 0;
};

static DevLimits device_limits() {
  static std::mutex mu;
  static std::map<int, DevLimits> cache;
  int dev = 0;
  hipGetDevice(&dev);
  std::lock_guard<std::mutex> g(mu);
  auto it = cache.find(dev);
  if (it != cache.end()) return it->second;
  DevLimits d;
  hipDeviceGetAttribute(&d.ncu, hipDeviceAttributeMultiprocessorCount, dev);
  hipDeviceGetAttribute(&d.lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
  cache[dev] = d;
  return d;
}

// Launches the main pass and the fix-up pass over the same LDS layout.  Waves
// per block: the count that puts the most waves on a CU given the LDS (table
// shared per block) and the kernel's register use; cached per kernel and layout.
template <typename KM, typename KE>
static int launch_pair(KM kern, KE esc, const Plan *p, const Layout &L, int ppw, const double *map,
                       const double *theta, const double *phi, int64_t n, double *out, double *var,
                       hipStream_t s) {
  const DevLimits lim = device_limits();
  static std::mutex mu;
  static std::map<std::tuple<int, const void *, int, int>, std::pair<int, int>> cache;
  int wpb = 0, occ = 0;
  {
    std::lock_guard<std::mutex> g(mu);
    int dev = 0;
    hipGetDevice(&dev);
    const auto key = std::make_tuple(dev, (const void *)kern, L.tab_bytes, L.wave_bytes);
    auto it = cache.find(key);
    if (it != cache.end()) {
      wpb = it->second.first;
      occ = it->second.second;
    } else {
      int best_waves = 0;
      for (int w = 1; w <= MAX_WPB; ++w) {
        const int l = L.tab_bytes + w * L.wave_bytes;
        if (l > lim.lds_max) break;
        hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, l);
        int o = 0;
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&o, kern, w * WAVE, l);
        if (o * w >= best_waves) { best_waves = o * w; wpb = w; occ = o; }
      }
      cache[key] = std::make_pair(wpb, occ);
    }
  }
  if (wpb == 0) {
    set_error("plan needs more LDS than the device offers (reduce K or the table size)");
    return FLINTS_ELIMIT;
  }
  const int lds = L.tab_bytes + wpb * L.wave_bytes;
  hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
  if (occ < 1) occ = 1;
  const int64_t ngroups = (n + ppw - 1) / ppw;
  int64_t blocks = std::min<int64_t>((ngroups + wpb - 1) / wpb, (int64_t)lim.ncu * occ);
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(wpb * WAVE), lds, s, p->d, map, theta,
                     phi, n, out, var, L);
  hipFuncSetAttribute((const void *)esc, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
  const int64_t eblocks = std::min<int64_t>(((n + WAVE - 1) / WAVE + wpb - 1) / wpb, (int64_t)lim.ncu * 4);
  hipLaunchKernelGGL(esc, dim3((unsigned)std::max<int64_t>(eblocks, 1)), dim3(wpb * WAVE), lds, s, p->d,
                     map, theta, phi, n, out, var, L);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    set_error(std::string("interpolation kernel launch failed: ") + hipGetErrorString(e));
    return FLINTS_EDEVICE;
  }
  return FLINTS_OK;
}

// Register-row path (one row per lane, groups of G lanes).
template <int NMAX, int G, int SPIN, bool MSE, bool FP32>
static int launch_t(const Plan *p, const double *map, const double *theta, const double *phi,
                    int64_t n, double *out, double *var, hipStream_t s) {
  constexpr int PPW = WAVE / G;
  constexpr int NR = (SPIN == 0) ? 2 : 3;
  const Layout L = make_layout(p->d.ntab, p->d.nfun, p->d.K, p->d.n, PPW, PPW, NR);
  return launch_pair(k_interp64<NMAX, G, SPIN, MSE, FP32>, k_escalate<NMAX, G, SPIN, MSE>, p, L, PPW,
                     map, theta, phi, n, out, var, s);
}

// Row-group path for n <= 16 NT (FP64), and the FP32 main pass of the same
// sizes whose rejected points are recomputed by the row-group fix-up.
template <int NT, int SPIN, bool FP32>
static int launch_rs(const Plan *p, const double *map, const double *theta, const double *phi,
                     int64_t n, double *out, double *var, hipStream_t s) {
  constexpr int NR = (SPIN == 0) ? 2 : 3;
  if (FP32) {
    constexpr int G = 16 * NT, PPW = WAVE / G;
    const Layout L = make_layout(p->d.ntab, p->d.nfun, p->d.K, p->d.n, PPW, PPW, NR);
    return launch_pair(k_interp64<16 * NT, G, SPIN, false, true>, k_fixup<RowGroupEngine<NT, SPIN>, SPIN>,
                       p, L, PPW, map, theta, phi, n, out, var, s);
  }
  const Layout L = make_layout(p->d.ntab, p->d.nfun, p->d.K, p->d.n, 4, 1, NR);
  return launch_pair(k_interp_rs<NT, SPIN>, k_fixup<RowGroupEngine<NT, SPIN>, SPIN>, p, L, 4, map,
                     theta, phi, n, out, var, s);
}

// Tile path for 16 (T - 1) < n <= 16 T (FP64), and the FP32 main pass of the
// same sizes whose rejected points are recomputed by the tile fix-up.
template <int T, int SPIN, bool FP32>
static int launch_tile(const Plan *p, const double *map, const double *theta, const double *phi,
                       int64_t n, double *out, double *var, hipStream_t s) {
  constexpr int NR = (SPIN == 0) ? 2 : 3;
  constexpr int SCR = (T - 1) * TILE_D + 16;   // staged tiles and pivots overlay the packed system
  if (FP32) {
    constexpr int G = 64, PPW = 1;
    const Layout L = make_layout(p->d.ntab, p->d.nfun, p->d.K, p->d.n, PPW, PPW, NR, SCR);
    return launch_pair(k_interp64<16 * T, G, SPIN, false, true>, k_fixup<TileEngine<T, SPIN>, SPIN>, p,
                       L, PPW, map, theta, phi, n, out, var, s);
  }
  const Layout L = make_layout(p->d.ntab, p->d.nfun, p->d.K, p->d.n, 1, 1, NR, SCR);
  return launch_pair(k_interp_tile<T, SPIN>, k_fixup<TileEngine<T, SPIN>, SPIN>, p, L, 1, map, theta,
                     phi, n, out, var, s);
}

template <int SPIN, bool MSE, bool FP32>
static int launch_spin(const Plan *p, const double *map, const double *theta, const double *phi,
                       int64_t n, double *out, double *var, hipStream_t s) {
  const int nrow = p->d.n;
  if (!MSE && nrow <= 16) return launch_rs<1, SPIN, FP32>(p, map, theta, phi, n, out, var, s);
  if (!MSE && nrow <= 32) return launch_rs<2, SPIN, FP32>(p, map, theta, phi, n, out, var, s);
  if (!MSE && nrow <= 48) return launch_tile<3, SPIN, FP32>(p, map, theta, phi, n, out, var, s);
  if (!MSE) return launch_tile<4, SPIN, FP32>(p, map, theta, phi, n, out, var, s);
  if (nrow <= 16) return launch_t<16, 16, SPIN, MSE, FP32>(p, map, theta, phi, n, out, var, s);
  if (nrow <= 32) return launch_t<32, 32, SPIN, MSE, FP32>(p, map, theta, phi, n, out, var, s);
  if (nrow <= 48) return launch_t<48, 64, SPIN, MSE, FP32>(p, map, theta, phi, n, out, var, s);
  return launch_t<64, 64, SPIN, MSE, FP32>(p, map, theta, phi, n, out, var, s);
}

template <int SPIN>
static int launch_prec(const Plan *p, const double *map, const double *theta, const double *phi,
                       int64_t n, double *out, double *var, hipStream_t s) {
  const bool mse = (p->d.var_kind == FLINTS_VAR_MSE) && var != nullptr;
  const bool f32 = p->d.precision == FLINTS_FP32_IR;
  if (f32)
    return mse ? launch_spin<SPIN, true, true>(p, map, theta, phi, n, out, var, s)
               : launch_spin<SPIN, false, true>(p, map, theta, phi, n, out, var, s);
  return mse ? launch_spin<SPIN, true, false>(p, map, theta, phi, n, out, var, s)
             : launch_spin<SPIN, false, false>(p, map, theta, phi, n, out, var, s);
}

int launch_interpolate(const Plan *p, const double *map, const double *theta, const double *phi,
                       int64_t n, double *out, double *var, hipStream_t s) {
  if (n == 0) return FLINTS_OK;
  if (p->d.spin == 0) return launch_prec<0>(p, map, theta, phi, n, out, var, s);
  return launch_prec<2>(p, map, theta, phi, n, out, var, s);
}

int launch_stencil(const Plan *p, const double *theta, const double *phi, int64_t n, int64_t *idx,
                   hipStream_t s) {
  if (n == 0) return FLINTS_OK;
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
