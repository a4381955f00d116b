// Kernel templates and launch helpers of the single-plan and T + Q/U paths.
// The launchers are instantiated in separate translation units (one per spin
// and precision class, interp_*.hip) so that they compile in parallel; the
// device code they run lives in device.h.
#pragma once
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
  const double *tab = kernel_table(lds, P, L);
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
  const double *tab = kernel_table(lds, P, L);
  const int wpb = blockDim.x / WAVE;
  const int wave = threadIdx.x / WAVE;
  const int lane = threadIdx.x % WAVE;
  const WaveBufs B = wave_bufs(lds, L, wave);
  for (int64_t pt = xcd_block() * wpb + wave; pt < n; pt += (int64_t)gridDim.x * wpb)
    point_tile<T, SPIN>(P, tab, map, theta, phi, n, out, var, B, pt, lane);
}

// Main pass for 64 < n <= 128 (spin 2 with 32 < K <= 64) with the LDS
// elimination.  The packed systems (up to 66 KB) leave no room for an LDS copy
// of the table, which is read through the caches (layouts with no table bytes).
// NW waves per target (2 or 4): block b holds one system (the
// layout's first wave area) and two int flags after it.  Wave 0 searches and
// gathers the records; all waves assemble and eliminate (panel rows and tile
// groups dealt between them, block barriers per block of columns); wave 0 stores.
// Every barrier is reached by every wave: the loops' bounds are block-uniform.
template <int SPIN, int NW>
__global__ __launch_bounds__(NW * WAVE) void k_interp_lds2(PlanDev P, const double *__restrict__ map,
                                               const double *__restrict__ theta,
                                               const double *__restrict__ phi, int64_t n,
                                               double *__restrict__ out,
                                               double *__restrict__ var, Layout L) {
  constexpr int NR = (SPIN == 0) ? 2 : 3;
  extern __shared__ double lds_dyn[];
  char *lds = (char *)lds_dyn;
  const double *tab = kernel_table(lds, P, L);
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);   // wave-uniform
  const int lane = threadIdx.x % WAVE;
  const WaveBufs B = wave_bufs(lds, L, 0);
  int *flag = (int *)(lds + L.tab_bytes + L.wave_bytes);   // search result of wave 0
  const double nug = (P.nug_policy == FLINTS_NUG_ALWAYS) ? P.eps : 0.0;
  for (int64_t pt = xcd_block(); pt < n; pt += (int64_t)gridDim.x) {
    const double th = theta[pt], ph = phi[pt];
    if (w == 0) {
      const bool f = phase_a_search(P, th, ph, lane, B.cu, B.ci, B.rs, B.sel);
      // records without the data column: the right-hand sides overlay them
      if (f) neighbour_records<SPIN, NR, false>(P, th, ph, lane, B.sel, B.nb, B.rhs, map);
      if (lane == 0) flag[0] = f ? 1 : 0;
    }
    __syncthreads();
    const bool found = flag[0] != 0;
    GroupOut o;
    bool ok = true;
    if (found) {
      lds_assemble<SPIN, NR>(P, tab, map, B.sel, B.nb, lane, B.mat, B.rhs, w, NW);
      __syncthreads();
      ok = lds_phase_b<SPIN, NR>(B.mat, B.rhs, B.rbuf, lane, P.n, nug, o, w, NW);
    }
    if (w == 0 && lane == 0) store_point<SPIN>(P, pt, n, found, ok, FAIL64_BITS, o, nug, false, out, var);
    __syncthreads();   // the next target's search reuses the system's LDS
  }
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
  const double *tab = kernel_table(lds, P, L);
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

// ---------------------------------------------------------------- launchers
struct DevLimits {
  int ncu = 0;
  int lds_max = 0;
};

inline DevLimits device_limits() {
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
inline bool pick_wpb(KM kern, const Layout &L, const DevLimits &lim, int &wpb, int &occ) {
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
inline int launch_pair(KM kern, KE esc, const Plan *p, const Layout &L, int ppw, const double *map,
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
inline int launch_t(const Plan *p, const double *map, const double *theta, const double *phi,
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
inline int launch_rs(const Plan *p, const double *map, const double *theta, const double *phi,
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
inline int launch_tile(const Plan *p, const double *map, const double *theta, const double *phi,
                       int64_t n, double *out, double *var, hipStream_t s) {
  constexpr int NR = (SPIN == 0) ? 2 : 3;
  constexpr int SCR = (T - 1) * TILE_D + 16;   // staged tiles and pivots overlay the packed system
  if (FP32) {
    constexpr int G = 64, PPW = 1;
    const Layout L = make_layout(p->d.ntab, p->d.nfun, p->d.K, p->d.n, PPW, PPW, NR, SCR);
    return launch_pair(k_interp64<16 * T, G, SPIN, false, true>, k_fixup<TileEngine<T, SPIN>, SPIN>, p,
                       L, PPW, map, theta, phi, n, out, var, s);
  }
  Layout L = make_layout(p->d.ntab, p->d.nfun, p->d.K, p->d.n, 1, 1, NR, SCR);
  // the table is read through the caches when its LDS copy would cost waves
  const DevLimits lim = device_limits();
  if (lim.lds_max / L.wave_bytes > (lim.lds_max - L.tab_bytes) / L.wave_bytes &&
      (lim.lds_max - L.tab_bytes) / L.wave_bytes < MAX_WPB)
    L.tab_bytes = 0;
  return launch_pair(k_interp_tile<T, SPIN>, k_fixup<TileEngine<T, SPIN>, SPIN>, p, L, 1, map, theta,
                     phi, n, out, var, s);
}

// LDS elimination for 64 < n <= 128 (FP64, paper variance).
// Main pass with two or four waves per target (k_interp_lds2), fix-up with one
// wave per target (the LDS engine of k_fixup: the same elimination in 4-column
// blocks).
template <int SPIN>
inline int launch_lds(const Plan *p, const double *map, const double *theta, const double *phi,
                      int64_t n, double *out, double *var, hipStream_t s) {
  constexpr int NR = (SPIN == 0) ? 2 : 3;
  // right-hand sides and spare slots over the records, then the packed system;
  // the table is read through the caches
  const Layout L = make_layout_lds(p->d.K, p->d.n, NR);
  const DevLimits lim = device_limits();
  const int lds2 = L.wave_bytes + 16;
  if (lds2 > lim.lds_max) {
    set_error("plan needs more LDS than the device offers");
    return FLINTS_ELIMIT;
  }
  // Two waves per target, or four where a CU holds at most two systems, so
  // that every SIMD runs two waves.  Systems per CU: the occupancy API's count,
  // bounded by the LDS rounded up to 512-byte granules (at 112 rows, 54,576 B,
  // the API counts three two-wave blocks but the measured rate is that of two;
  // four waves run 25 % faster there, and 24 % slower at 104 rows, where three fit).
  constexpr int LDS_GRANULE = 512;
  const int fit = lim.lds_max / ((lds2 + LDS_GRANULE - 1) / LDS_GRANULE * LDS_GRANULE);
  auto kern = k_interp_lds2<SPIN, 2>;
  int nw = 2, occ = 0;
  hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, lds2);
  hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kern, nw * WAVE, lds2);
  occ = std::min(occ, fit);
  if (occ <= 2) {
    kern = k_interp_lds2<SPIN, 4>;
    nw = 4;
    hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, lds2);
    hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kern, nw * WAVE, lds2);
    occ = std::min(occ, fit);
  }
  if (occ < 1) occ = 1;
  const int64_t blocks = std::max<int64_t>(std::min<int64_t>(n, (int64_t)lim.ncu * occ), 1);
  hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(nw * WAVE), lds2, s, p->d, map, theta, phi, n, out,
                     var, L);
  auto esc = k_fixup<LdsEngine<SPIN>, SPIN>;
  int wpb = 0, eocc = 0;
  if (!pick_wpb(esc, L, lim, wpb, eocc)) return FLINTS_ELIMIT;
  const int lds = L.tab_bytes + wpb * L.wave_bytes;
  hipFuncSetAttribute((const void *)esc, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
  const int64_t eblocks = std::min<int64_t>(((n + WAVE - 1) / WAVE + wpb - 1) / wpb, (int64_t)lim.ncu * 4);
  hipLaunchKernelGGL(esc, dim3((unsigned)std::max<int64_t>(eblocks, 1)), dim3(wpb * WAVE), lds, s, p->d, map,
                     theta, phi, n, out, var, L);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    set_error(std::string("interpolation kernel launch failed: ") + hipGetErrorString(e));
    return FLINTS_EDEVICE;
  }
  return FLINTS_OK;
}

template <int SPIN, bool MSE, bool FP32>
inline int launch_spin(const Plan *p, const double *map, const double *theta, const double *phi,
                       int64_t n, double *out, double *var, hipStream_t s) {
  const int nrow = p->d.n;
  if (nrow > 128) {
    set_error("systems of more than 128 rows are not supported");
    return FLINTS_ELIMIT;
  }
  if (nrow > 64) {
    // the LDS elimination (FP64, paper variance); plan creation refuses the MSE
    // variance above 64 rows and runs FP32 plans of this size in FP64
    if constexpr (MSE || FP32) {
      set_error("systems of more than 64 rows run in FP64 with the paper variance only");
      return FLINTS_ELIMIT;
    } else {
      return launch_lds<SPIN>(p, map, theta, phi, n, out, var, s);
    }
  }
  if (!MSE && nrow <= 16) return launch_rs<1, SPIN, FP32>(p, map, theta, phi, n, out, var, s);
  if (!MSE && nrow <= 32) return launch_rs<2, SPIN, FP32>(p, map, theta, phi, n, out, var, s);
  if (!MSE && nrow <= 48) return launch_tile<3, SPIN, FP32>(p, map, theta, phi, n, out, var, s);
  if (!MSE) return launch_tile<4, SPIN, FP32>(p, map, theta, phi, n, out, var, s);
  if (nrow <= 16) return launch_t<16, 16, SPIN, MSE, FP32>(p, map, theta, phi, n, out, var, s);
  if (nrow <= 32) return launch_t<32, 32, SPIN, MSE, FP32>(p, map, theta, phi, n, out, var, s);
  if (nrow <= 48) return launch_t<48, 64, SPIN, MSE, FP32>(p, map, theta, phi, n, out, var, s);
  return launch_t<64, 64, SPIN, MSE, FP32>(p, map, theta, phi, n, out, var, s);
}


// Instantiated launchers (one translation unit each).
int launch_fp64_s0(const Plan *p, const double *map, const double *theta, const double *phi,
                   int64_t n, double *out, double *var, hipStream_t s);
int launch_fp64_s2(const Plan *p, const double *map, const double *theta, const double *phi,
                   int64_t n, double *out, double *var, hipStream_t s);
int launch_fp32_s0(const Plan *p, const double *map, const double *theta, const double *phi,
                   int64_t n, double *out, double *var, hipStream_t s);
int launch_fp32_s2(const Plan *p, const double *map, const double *theta, const double *phi,
                   int64_t n, double *out, double *var, hipStream_t s);
int launch_mse_fp64_s0(const Plan *p, const double *map, const double *theta, const double *phi,
                       int64_t n, double *out, double *var, hipStream_t s);
int launch_mse_fp64_s2(const Plan *p, const double *map, const double *theta, const double *phi,
                       int64_t n, double *out, double *var, hipStream_t s);
int launch_mse_fp32_s0(const Plan *p, const double *map, const double *theta, const double *phi,
                       int64_t n, double *out, double *var, hipStream_t s);
int launch_mse_fp32_s2(const Plan *p, const double *map, const double *theta, const double *phi,
                       int64_t n, double *out, double *var, hipStream_t s);

}  // namespace flints
