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

// Main passes of T + Q/U over targets [s0, s1) with shared stencils: the
// spin-2 pass (tiles, or row groups for 2K <= 32 rows) writes each target's
// stencil to stn, the spin-0 pass (row groups) reads it.  s0 is a multiple of
// 4 and s1 is a multiple of 4 or n, so no group of four crosses a chunk.
template <int T>
__global__ __launch_bounds__(MAX_WPB * WAVE) void k_interp_tile_st(
    PlanDev P, const double *__restrict__ map, const double *__restrict__ theta,
    const double *__restrict__ phi, int64_t n, double *__restrict__ out, double *__restrict__ var,
    Layout L, int *__restrict__ stn, int64_t s0, int64_t s1) {
  extern __shared__ double lds_dyn[];
  char *lds = (char *)lds_dyn;
  const double *tab = load_table(lds, P);
  const int wpb = blockDim.x / WAVE;
  const int wave = threadIdx.x / WAVE;
  const int lane = threadIdx.x % WAVE;
  const WaveBufs B = wave_bufs(lds, L, wave);
  for (int64_t pt = s0 + xcd_block() * wpb + wave; pt < s1; pt += (int64_t)gridDim.x * wpb)
    point_tile_st<T, 2>(P, tab, map, theta, phi, n, out, var, B, pt, lane, stn, s0);
}

template <int NT>
__global__ __launch_bounds__(MAX_WPB * WAVE) void k_interp_rs_st(
    PlanDev P, const double *__restrict__ map, const double *__restrict__ theta,
    const double *__restrict__ phi, int64_t n, double *__restrict__ out, double *__restrict__ var,
    Layout L, int *__restrict__ stn, int64_t s0, int64_t s1) {
  extern __shared__ double lds_dyn[];
  char *lds = (char *)lds_dyn;
  const double *tab = load_table(lds, P);
  const int wpb = blockDim.x / WAVE;
  const int wave = threadIdx.x / WAVE;
  const int lane = threadIdx.x % WAVE;
  const WaveBufs B = wave_bufs(lds, L, wave);
  const int64_t ngroups = (s1 - s0 + 3) / 4;
  for (int64_t g = xcd_block() * wpb + wave; g < ngroups; g += (int64_t)gridDim.x * wpb)
    group_rs_st<NT, 2>(P, tab, map, theta, phi, n, out, var, B, s0 + g * 4, lane, stn, s0);
}

template <int NT>
__global__ __launch_bounds__(MAX_WPB * WAVE) void k_interp_rs_ld(
    PlanDev P, const double *__restrict__ map, const double *__restrict__ theta,
    const double *__restrict__ phi, int64_t n, double *__restrict__ out, double *__restrict__ var,
    Layout L, const int *__restrict__ stn, int64_t s0, int64_t s1) {
  extern __shared__ double lds_dyn[];
  char *lds = (char *)lds_dyn;
  const double *tab = load_table(lds, P);
  const int wpb = blockDim.x / WAVE;
  const int wave = threadIdx.x / WAVE;
  const int lane = threadIdx.x % WAVE;
  const WaveBufs B = wave_bufs(lds, L, wave);
  const int64_t ngroups = (s1 - s0 + 3) / 4;
  for (int64_t g = xcd_block() * wpb + wave; g < ngroups; g += (int64_t)gridDim.x * wpb)
    group_rs_ld<NT, 0>(P, tab, map, theta, phi, n, out, var, B, s0 + g * 4, lane, stn, s0);
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
// Waves per block for kernel kern over layout L: the count that puts the most
// waves on a CU given the LDS (tables shared per block) and the kernel's
// register use; cached per kernel and layout.  Returns false (error set) if
// not even one wave fits.
template <typename KM>
static bool pick_wpb(KM kern, const Layout &L, const DevLimits &lim, int &wpb, int &occ) {
  static std::mutex mu;
  static std::map<std::tuple<int, const void *, int, int>, std::pair<int, int>> cache;
  wpb = 0;
  occ = 0;
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
    return false;
  }
  if (occ < 1) occ = 1;
  return true;
}

// Launches the main pass and the fix-up pass over the same LDS layout.
template <typename KM, typename KE>
static int launch_pair(KM kern, KE esc, const Plan *p, const Layout &L, int ppw, const double *map,
                       const double *theta, const double *phi, int64_t n, double *out, double *var,
                       hipStream_t s) {
  const DevLimits lim = device_limits();
  int wpb = 0, occ = 0;
  if (!pick_wpb(kern, L, lim, wpb, occ)) return FLINTS_ELIMIT;
  const int lds = L.tab_bytes + wpb * L.wave_bytes;
  hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
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

// Targets per chunk of the shared-stencil T + Q/U path (a multiple of 4; the
// stencil buffer holds K ints per target of one chunk: 2 GiB at K = 32).
constexpr int64_t TQU_CHUNK = int64_t(1) << 24;

// Shared-stencil T + Q/U: per chunk the spin-2 main pass (which writes the
// stencils) and then the spin-0 main pass (which reads them), each with the
// layout and block size of its single-plan path; then both fix-up passes.
// The stencil buffer is stream-ordered (allocated and freed on s); if it
// cannot be allocated, each plan runs its own searching pass.
template <int NT0, int NT2, int T2>
static int launch_tqu_t(const Plan *p0, const Plan *p2, const double *map0, const double *map2,
                        const double *theta, const double *phi, int64_t n, double *out0, double *var0,
                        double *out2, double *var2, hipStream_t s) {
  constexpr int SCR = T2 ? (T2 - 1) * TILE_D + 16 : 0;
  constexpr int PPW2 = T2 ? 1 : 4;
  const DevLimits lim = device_limits();
  const int K = p0->d.K;
  const Layout L2 = make_layout(p2->d.ntab, p2->d.nfun, K, p2->d.n, PPW2, 1, 3, SCR);
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
  const int64_t chunk = std::min<int64_t>(TQU_CHUNK, (n + 3) & ~int64_t(3));
  int *stn = nullptr;
  if (hipMallocAsync((void **)&stn, (size_t)chunk * K * sizeof(int), s) != hipSuccess) {
    (void)hipGetLastError();   // no buffer: one searching pass per plan instead
    const int rc = launch_interpolate(p0, map0, theta, phi, n, out0, var0, s);
    return rc != FLINTS_OK ? rc : launch_interpolate(p2, map2, theta, phi, n, out2, var2, s);
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
  (void)hipFreeAsync(stn, s);
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
  return a.precision == FLINTS_FP64 && b.precision == FLINTS_FP64 && !mse0 && !mse2 &&
         a.nside == b.nside && a.K == b.K && a.K <= 32 && a.r0 == b.r0 && a.rcap == b.rcap;
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
  const int K = p0->d.K;
  if (K <= 8)
    return launch_tqu_t<1, 1, 0>(p0, p2, map0, map2, theta, phi, n, out0, var0, out2, var2, s);
  if (K <= 16)
    return launch_tqu_t<1, 2, 0>(p0, p2, map0, map2, theta, phi, n, out0, var0, out2, var2, s);
  if (K <= 24)
    return launch_tqu_t<2, 0, 3>(p0, p2, map0, map2, theta, phi, n, out0, var0, out2, var2, s);
  return launch_tqu_t<2, 0, 4>(p0, p2, map0, map2, theta, phi, n, out0, var0, out2, var2, s);
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
