// Device code shared by the FLINTS kernels for gfx950 (CDNA4): phase A (search,
// records, assembly), the phase-B engines and the per-point / per-group bodies
// that the single-plan kernels (interp.hip) and the batched persistent kernels
// (batch.hip) both run, so that a point gets the same arithmetic in either.
//
// A 64-lane wavefront owns a group of target points (four on the row-group
// path, one on the tile path, 64/G on the register-row path).  Phase A runs once
// per point of the group with the whole wave:
//   a2/a3  K-nearest search: rings crossing a disc of radius r around the target
//          are listed one per lane, their pixel windows are flattened across the
//          wave, every lane tests one candidate pixel (chord distance in FP64 from
//          a difference vector written in the target's rotated frame), survivors
//          are compacted into LDS, and each candidate's rank (distance, then pixel
//          index) is counted against all others; ranks < K form the stencil.
//   a4/a5  per-neighbour record: offset from the target, local e_theta / e_phi,
//          gathered map values (RING order, so neighbouring targets reuse lines).
//   a6     every pair (a, b) of {target, neighbours}: half chord s, correlation
//          from the LDS table (cubic), spin-2 parallel-transport phases from the
//          bearings, written as the packed lower triangle of S plus the
//          right-hand sides (target covariances and data) in LDS.
// Phase B factorises S + nI with the right-hand sides (target covariances and
// data) carried through the elimination, which gives y = L^-1 b and
// z = L^-1 data, so
//   value = y . z = b^T (S+nI)^-1 data   (paper Eq. best_temperature_field / major_eq)
//   var   = sigma^2 (1 - y . y)          (paper Eq. gaussvar / gaussvar_pol)
// without a backward solve.  Four engines:
//   row group (n <= 32)   one point per 16-lane row group, lower-triangular rows
//                          in registers, pivot values by DPP row broadcast;
//   tile (32 < n <= 64)   one point per wave, blocked on 16 x 16 tiles, panels
//                          eliminated by row groups, trailing update on FP64 MFMA;
//   LDS (64 < n <= 128)   blocked L D L^T of the packed system in LDS, two or
//                          four waves per point (one in the fix-up);
//   register row          one row per lane with readlane broadcasts (the MSE
//                          variance, which needs a backward solve, and the FP32 +
//                          refinement main pass).
// A failed factorisation (non-positive pivot) triggers the nugget escalation of
// paper Sec. 2.4: bisection for the smallest shift mu with S + mu I positive
// definite, then n = mu + eps.
#pragma once
#include "plan.h"
#include "healpix_ring.h"
#include "table_interp.h"
#include "kconst.h"
#include <algorithm>
#include <cstring>
#include <mutex>
#include <map>
#include <tuple>
#include <utility>

namespace flints {

constexpr int WAVE = 64;
constexpr int MAX_WPB = 8;      // waves per block of the interpolation kernels (launch bound 512)
constexpr int STENCIL_WPB = 4;  // waves per block of the stencil kernel (launch bound 256)
constexpr int CAND_CAP = 320;
constexpr int NBF = 8;   // doubles per neighbour record
constexpr double PI_D = 3.14159265358979323846;
constexpr double TWO_PI_D = 6.28318530717958647692;

__device__ inline void wave_lds_sync() { __asm__ volatile("s_waitcnt lgkmcnt(0)" ::: "memory"); }
__device__ inline void compiler_fence() { __asm__ volatile("" ::: "memory"); }
__host__ __device__ inline int tri(int r) { return r * (r + 1) / 2; }

// sin and cos of x for |x| <= 2 pi (colatitudes, disc radii and half
// longitude differences).  x is reduced by the nearest multiple k of pi/2 with
// pi/2 split into a double and its remainder (x - k*hi is exact for |k| <= 4),
// then sin and cos of |r| <= pi/4 come from their Taylor series (truncation
// < 1e-19).
__device__ inline void sincos_bounded(double x, double &s, double &c) {
  constexpr double PIO2_HI = 1.5707963267948966;      // pi/2 rounded to double
  constexpr double PIO2_LO = 6.123233995736766e-17;   // pi/2 - PIO2_HI
  constexpr double TWO_OVER_PI = 0.6366197723675814;
  // sin r = r - r^3 (1/3! - r^2/5! + ... + r^14/17!), coefficients 1/(2i+1)! with signs
  constexpr double SC[8] = {-1.0 / 355687428096000.0, 1.0 / 1307674368000.0, -1.0 / 6227020800.0,
                            1.0 / 39916800.0, -1.0 / 362880.0, 1.0 / 5040.0, -1.0 / 120.0, 1.0 / 6.0};
  // cos r = 1 + r^2 (-1/2! + r^2/4! - ... + r^14/16!)
  constexpr double CC[8] = {1.0 / 20922789888000.0, -1.0 / 87178291200.0, 1.0 / 479001600.0,
                            -1.0 / 3628800.0, 1.0 / 40320.0, -1.0 / 720.0, 1.0 / 24.0, -0.5};
  const double k = rint(x * kconst(TWO_OVER_PI));
  const double r = fma(-k, kconst(PIO2_LO), fma(-k, kconst(PIO2_HI), x));
  const double r2 = r * r;
  double ps = kconst(SC[0]);
#pragma unroll
  for (int i = 1; i < 8; ++i) ps = fma(ps, r2, kconst(SC[i]));
  const double sr = fma(-r * r2, ps, r);
  double pc = kconst(CC[0]);
#pragma unroll
  for (int i = 1; i < 8; ++i) pc = fma(pc, r2, kconst(CC[i]));
  const double cr = fma(r2, pc, 1.0);
  const int q = ((int)k) & 3;
  s = (q == 0) ? sr : (q == 1) ? cr : (q == 2) ? -sr : -cr;
  c = (q == 0) ? cr : (q == 1) ? -sr : (q == 2) ? -cr : sr;
}

// Broadcast a double held by lane `src` (wave-uniform index) to all lanes.
__device__ inline double readlane_d(double v, int src) {
  const unsigned long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(unsigned)(b & 0xffffffffull), src);
  const int hi = __builtin_amdgcn_readlane((int)(unsigned)(b >> 32), src);
  return __longlong_as_double(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}

__device__ inline float readlane_d(float v, int src) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), src));
}

// Value of `v` in row k of this lane's group (groups of G lanes).
template <int G, typename T>
__device__ inline T group_bcast(T v, int k, int grp) {
  T r = readlane_d(v, k);
#pragma unroll
  for (int g = 1; g < WAVE / G; ++g) {
    const T t = readlane_d(v, g * G + k);
    r = (grp == g) ? t : r;
  }
  return r;
}


struct RingSpan {
  double z, s, phi0, dphi;
  double sdiff;   // s_ring - s_target, formed without cancellation
  long long first;
  int n, j0, off, pad;
};

struct Layout {
  int tab_bytes, wave_bytes;
  int off_cu, off_ci, off_rings, off_sel, off_nb, off_mat, off_rhs, off_col, off_rbuf;
  int matsz;
};

// Words between fields of the neighbour records (field-major, K + 1 records).
__host__ __device__ inline int nb_stride(int K) { return (K + 2) & ~1; }

inline int al16(int x) { return (x + 15) & ~15; }

// Per-wave LDS: the stencils of the wave's points, then a region used first by
// the K-nearest search (candidates, ring spans) and afterwards by the assembly
// (one neighbour-record slot, the packed systems and right-hand sides of all
// PPW points).  The search of every point of the group runs before any
// assembly, so the two uses never overlap.
inline Layout make_layout(int ntab, int nf, int K, int n, int ppw, int nsys, int NR, int min_mat = 0) {
  Layout L;
  L.tab_bytes = al16(ntab * nf * 8);
  int o = 0;
  L.off_sel = o;   o = al16(o + ppw * K * 4);
  const int u0 = o;
  // search view
  int s = u0;
  L.off_cu = s;    s = al16(s + (CAND_CAP + 4) * 8);
  L.off_ci = s;    s = al16(s + (CAND_CAP + 4) * 4);
  L.off_rings = s; s = al16(s + WAVE * (int)sizeof(RingSpan));
  // assembly view
  int a = u0;
  L.off_nb = a;    a = al16(a + nb_stride(K) * NBF * 8);
  L.matsz = std::max(n * (n + 1) / 2, min_mat);
  L.off_mat = a;   a = al16(a + nsys * L.matsz * 8);
  L.off_rhs = a;   a = al16(a + nsys * n * NR * 8);
  L.off_col = a;
  L.off_rbuf = a;
  L.wave_bytes = s > a ? s : a;
  return L;
}

// Layout of the LDS elimination: the right-hand sides and WAVE spare doubles
// (the stores of masked-off lanes) overlay the neighbour records, which are dead
// once the pairs and target covariances are formed (the build writes the
// right-hand sides last); the packed system follows.  No table copy.
inline Layout make_layout_lds(int K, int n, int NR) {
  Layout L = make_layout(0, 1, K, n, 1, 1, NR);
  L.tab_bytes = 0;
  const int u0 = L.off_nb;
  L.off_rhs = u0;
  L.off_rbuf = al16(u0 + n * NR * 8);
  const int rec_end = al16(u0 + nb_stride(K) * NBF * 8), spare_end = al16(L.off_rbuf + WAVE * 8);
  const int region = rec_end > spare_end ? rec_end : spare_end;
  L.matsz = n * (n + 1) / 2;
  L.off_mat = region;
  L.off_col = al16(L.off_mat + L.matsz * 8);
  const int s = al16(L.off_rings + WAVE * (int)sizeof(RingSpan));   // end of the search view
  L.wave_bytes = s > L.off_col ? s : L.off_col;
  return L;
}

// Block index with the grid regrouped by XCD.  The dispatcher hands blocks to
// the 8 XCDs of an MI355X round robin (block b runs on XCD b mod 8), and each
// XCD has its own L2; numbering the blocks of one XCD consecutively makes the
// targets it works on at any moment one contiguous RING range, so the map lines
// their stencils share are fetched into one L2 instead of eight.
constexpr int NXCD = 8;
__device__ inline int64_t xcd_block() {
  const int nb = gridDim.x, b = blockIdx.x;
  if (nb % NXCD) return b;
  return (int64_t)(b % NXCD) * (nb / NXCD) + b / NXCD;
}

__device__ inline void count_event(unsigned long long *ctr, bool cond, int lane) {
  unsigned long long m = __ballot(cond);
  if (m && lane == 0) atomicAdd(ctr, (unsigned long long)__popcll(m));
}

// ---------------------------------------------------------------- a2/a3 search
// Candidates within angle r of the target, compacted into (cu, ci).  Returns the
// number found (entries beyond CAND_CAP are counted but not stored).
__device__ int enumerate_disc(const PlanDev &P, double th, double zt, double st, double phr,
                              double r, int lane, double *cu, int *ci, RingSpan *rs) {
  const int64_t N = P.nside;
  double sr, chr;
  sincos_bounded(0.5 * r, sr, chr);
  const double ur = 2.0 * sr * sr;  // 1 - cos r
  const double cr = 1.0 - 2.0 * sr * sr;
  const double pi = kconst(PI_D);
  const bool pn = (th - r) <= 0.0, ps = (th + r) >= pi;
  double s1, c1, s2, c2;
  sincos_bounded(th - r, s1, c1);
  sincos_bounded(th + r, s2, c2);
  const double zhi = pn ? 1.0 : c1;
  const double zlo = ps ? -1.0 : c2;
  int i0 = (int)floor(ring_coord(N, zhi)) - 1;
  if (i0 < 1) i0 = 1;
  int i1 = (int)ceil(ring_coord(N, zlo)) + 1;
  if (i1 > (int)(4 * N - 1)) i1 = (int)(4 * N - 1);
  int count = 0;
  for (int ib = i0; ib <= i1; ib += WAVE) {
    const int i = ib + lane;
    int m = 0, j0 = 0;
    if (i <= i1) {
      const Ring R = ring_geom(N, i);
      m = R.n;
      if (!(pn || ps)) {
        const double c = (cr - zt * R.z) / (st * R.s);
        if (c > 1.0 + 1e-6) {
          m = 0;
        } else if (c > -1.0) {
          const double half = acos(fmin(c, 1.0)) + R.dphi;
          if (half < pi) {
            const double inv = (double)R.n * kconst(0.5 / PI_D);
            const int jlo = (int)floor((phr - half - R.phi0) * inv);
            const int jhi = (int)ceil((phr + half - R.phi0) * inv);
            const int span = jhi - jlo + 1;
            if (span < R.n) {
              j0 = jlo;
              m = span;
            }
          }
        }
      }
      RingSpan S;
      S.z = R.z; S.s = R.s; S.phi0 = R.phi0; S.dphi = R.dphi;
      S.sdiff = (zt - R.z) * (zt + R.z) / (R.s + st);
      S.first = R.first; S.n = R.n;
      int jm = j0 % R.n;
      if (jm < 0) jm += R.n;
      S.j0 = jm;
      S.off = 0;
      S.pad = 0;
      rs[lane] = S;
    }
    int incl = m;
#pragma unroll
    for (int d = 1; d < WAVE; d <<= 1) {
      const int v = __shfl_up(incl, d);
      if (lane >= d) incl += v;
    }
    const int total = __shfl(incl, WAVE - 1);
    const int nrg = min(WAVE, i1 - ib + 1);
    if (i <= i1) rs[lane].off = incl - m;
    for (int c0 = 0; c0 < total; c0 += WAVE) {
      const int c = c0 + lane;
      bool keep = false;
      double u = 0.0;
      int pix = 0;
      if (c < total) {
        int lo = 0, hi = nrg - 1;
        while (lo < hi) {
          const int mid = (lo + hi + 1) >> 1;
          if (rs[mid].off <= c) lo = mid; else hi = mid - 1;
        }
        const RingSpan S = rs[lo];
        int j = S.j0 + (c - S.off);
        if (j >= S.n) j -= S.n;
        const double dphi = S.phi0 + (double)j * S.dphi - phr;
        double sh, ch;
        sincos_bounded(0.5 * dphi, sh, ch);
        const double dx = S.sdiff - 2.0 * S.s * sh * sh;
        const double dy = 2.0 * S.s * sh * ch;
        const double dz = S.z - zt;
        u = 0.5 * (dx * dx + dy * dy + dz * dz);
        keep = (u <= ur);
        pix = (int)(S.first + j);
      }
      const unsigned long long mk = __ballot(keep);
      const int pos = count + __popcll(mk & ((1ull << lane) - 1ull));
      if (keep && pos < CAND_CAP) {
        cu[pos] = u;
        ci[pos] = pix;
      }
      count += __popcll(mk);
    }
  }
  return count;
}

// K nearest pixels of (th, ph), ascending (distance, index), into sel[0..K).
__device__ bool knn_search(const PlanDev &P, double th, double ph, int lane, double *cu, int *ci,
                           RingSpan *rs, int *sel) {
  double zt, st;
  sincos_bounded(th, st, zt);
  const double twopi = kconst(TWO_PI_D);
  const double phr = ph - twopi * floor(ph / twopi);
  const int K = P.K;
  double r = P.r0, rlo = 0.0, rhi = 0.0;
  int count = 0;
  bool ok = false;
  for (int att = 0; att < 24; ++att) {
    count = enumerate_disc(P, th, zt, st, phr, r, lane, cu, ci, rs);
    if (count >= K && count <= CAND_CAP) { ok = true; break; }
    if (count < K) {
      if (r >= P.rcap) break;
      rlo = r;
      r = (rhi > 0.0) ? 0.5 * (r + rhi) : fmin(1.5 * r, P.rcap);
    } else {
      rhi = r;
      r = 0.5 * (rlo + r);
    }
  }
  if (!ok) return false;
  // pad to a multiple of 4 with keys that rank after every real candidate
  const int cpad = (count + 3) & ~3;
  if (lane < cpad - count) {
    cu[count + lane] = __builtin_inf();
    ci[count + lane] = 0x7fffffff;
  }
  for (int c = lane; c < count; c += WAVE) {
    const double uc = cu[c];
    const int ic = ci[c];
    int rank = 0;
    for (int c2 = 0; c2 < cpad; c2 += 4) {
      const double2 ua = *(const double2 *)(cu + c2);
      const double2 ub = *(const double2 *)(cu + c2 + 2);
      const int4 iv = *(const int4 *)(ci + c2);
      rank += (ua.x < uc) || (ua.x == uc && iv.x < ic);
      rank += (ua.y < uc) || (ua.y == uc && iv.y < ic);
      rank += (ub.x < uc) || (ub.x == uc && iv.z < ic);
      rank += (ub.y < uc) || (ub.y == uc && iv.w < ic);
    }
    if (rank < K) sel[rank] = ic;
  }
  return true;
}

// ---------------------------------------------------------------- a4/a5 records
// Neighbour records, field-major (record a's field f at nb[f * nbs + a], nbs =
// nb_stride(K)) so that lanes reading the records of consecutive neighbours
// read consecutive words.  Record 0 is the target.  Fields: chord offset from
// the target in the target's (e_theta, e_phi, z) frame (0-2), the point's own
// e_theta (3-5) and e_phi (6-7) in that frame.  The gathered map values go
// straight to the data column of the right-hand sides (column NR - 1 of the
// neighbour's rows).

// Map value i (float32 maps are widened exactly); zero without a map.
__device__ __forceinline__ double map_value(const PlanDev &P, const double *__restrict__ map, int64_t i) {
  if (!map) return 0.0;
  return P.map_f32 ? (double)((const float *)map)[i] : map[i];
}

// DATA false: the data column of the right-hand sides is not written (the LDS
// elimination, whose right-hand sides overlay the records, writes it later).
template <int SPIN, int NR, bool DATA = true>
__device__ void neighbour_records(const PlanDev &P, double th, double ph, int lane, const int *sel,
                                  double *nb, double *rhs, const double *__restrict__ map) {
  double zt, st;
  sincos_bounded(th, st, zt);
  const double twopi = kconst(TWO_PI_D);
  const double phr = ph - twopi * floor(ph / twopi);
  const int K = P.K;
  const int ns = nb_stride(K);
  for (int a = lane; a <= K; a += WAVE) {
    double f[NBF];
    if (a == 0) {
      f[0] = 0.0; f[1] = 0.0; f[2] = 0.0;
      f[3] = zt;  f[4] = 0.0; f[5] = -st;
      f[6] = 0.0; f[7] = 1.0;
    } else {
      const int64_t p = sel[a - 1];
      const Ring R = ring_geom(P.nside, pix_ring(P.nside, p));
      const double dphi = R.phi0 + (double)(p - R.first) * R.dphi - phr;
      double sh, ch;
      sincos_bounded(0.5 * dphi, sh, ch);
      const double sd = 2.0 * sh * ch, cd = 1.0 - 2.0 * sh * sh;
      const double sdiff = (zt - R.z) * (zt + R.z) / (R.s + st);
      f[0] = sdiff - 2.0 * R.s * sh * sh;
      f[1] = R.s * sd;
      f[2] = R.z - zt;
      f[3] = R.z * cd; f[4] = R.z * sd; f[5] = -R.s;
      f[6] = -sd;      f[7] = cd;
      // data column of the neighbour's rows (no map: the conditioning probe)
      if constexpr (DATA) {
        if (SPIN == 0) {
          rhs[(a - 1) * NR + NR - 1] = map_value(P, map, p);
        } else {
          rhs[2 * (a - 1) * NR + NR - 1] = map_value(P, map, p);
          rhs[(2 * (a - 1) + 1) * NR + NR - 1] = map_value(P, map, P.npix + p);
        }
      }
    }
#pragma unroll
    for (int i = 0; i < NBF; ++i) nb[i * ns + a] = f[i];
  }
}

// ---------------------------------------------------------------- a6 assembly
// 1 / d to full precision: the hardware estimate refined by two Newton steps.
__device__ __forceinline__ double recip(double d) {
  double r = __builtin_amdgcn_rcp(d);
  r = fma(r, fma(-d, r, 1.0), r);
  r = fma(r, fma(-d, r, 1.0), r);
  return r;
}

// Covariance entries of the pair (a, b) from their records.  Spin 0: c[0] =
// zeta(beta_ab) / zeta(0).  Spin 2: the 2 x 2 block Cov(Q_a, Q_b), Cov(Q_a, U_b),
// Cov(U_a, Q_b), Cov(U_a, U_b) from <P_a P_b*> = xi+ e^{2i(psi_ab - psi_ba)} and
// <P_a P_b> = xi- e^{2i(psi_ab + psi_ba)}, the bearings psi taken from the chord
// projected on each point's (e_theta, e_phi).  Returns false if the distance is
// beyond the table.
// sqrt(x) for x >= 0 by the reciprocal-square-root estimate and the same
// Goldschmidt refinement steps as the correctly rounded routine, without its
// rescaling of arguments below 2^-767 (squared chords between pixel centres and
// targets are far above that); sqrt(0) = 0.
__device__ __forceinline__ double sqrt_nonneg(double x) {
  const double r = __builtin_amdgcn_rsq(x);
  double g = x * r, h = 0.5 * r;
  const double e = fma(-h, g, 0.5);
  g = fma(g, e, g);
  h = fma(h, e, h);
  double d = fma(-g, g, x);
  g = fma(d, h, g);
  d = fma(-g, g, x);
  g = fma(d, h, g);
  return x > 0.0 ? g : 0.0;
}

template <int SPIN>
__device__ __forceinline__ bool pair_cov(const PlanDev &P, const double *tab, const double *nb, int ns,
                                         int a, int b, bool paper, double (&c)[4]) {
  const double dx = nb[a] - nb[b], dy = nb[ns + a] - nb[ns + b], dz = nb[2 * ns + a] - nb[2 * ns + b];
  const double s = 0.5 * sqrt_nonneg(dx * dx + dy * dy + dz * dz);
  if (SPIN == 0) {
    double f;
    const bool in = table_lookup(tab, P.ntab, 1, P.inv_h, s, &f);
    c[0] = f;
    return in;
  }
  double f[2];
  const bool in = table_lookup(tab, P.ntab, 2, P.inv_h, s, f);
  const double xa = dx * nb[3 * ns + a] + dy * nb[4 * ns + a] + dz * nb[5 * ns + a];
  const double ya = dx * nb[6 * ns + a] + dy * nb[7 * ns + a];
  const double xb = dx * nb[3 * ns + b] + dy * nb[4 * ns + b] + dz * nb[5 * ns + b];
  const double yb = dx * nb[6 * ns + b] + dy * nb[7 * ns + b];
  const double na = xa * xa + ya * ya, nbn = xb * xb + yb * yb;
  // the projections vanish together only for coincident points (beta = 0),
  // where the bearings are undefined and both phases are taken as 1
  const double prod = na * nbn;
  const bool sep = prod > 0.0;
  const double inv = recip(sep ? prod : 1.0);
  const double ia = nbn * inv, ib = na * inv;
  const double ca = sep ? (xa * xa - ya * ya) * ia : 1.0, sa = sep ? 2.0 * xa * ya * ia : 0.0;
  const double cb = sep ? (xb * xb - yb * yb) * ib : 1.0, sb = sep ? 2.0 * xb * yb * ib : 0.0;
  const double gr = f[0] * (ca * cb + sa * sb), gi = f[0] * (sa * cb - ca * sb);
  const double pr = paper ? 0.0 : f[1] * (ca * cb - sa * sb);
  const double pim = paper ? 0.0 : f[1] * (sa * cb + ca * sb);
  c[0] = gr + pr;   // QQ
  c[1] = pim - gi;  // QU
  c[2] = pim + gi;  // UQ
  c[3] = gr - pr;   // UU
  return in;
}

// The off-diagonal pairs (a, b), 1 <= b < a <= K, of the packed system: pair
// q = (a - 1)(a - 2) / 2 + (b - 1) on lane q mod (nw WAVE) of wave w.  Returns
// true if a pair distance lay beyond the table.
template <int SPIN>
__device__ __forceinline__ bool assemble_pairs(const PlanDev &P, const double *tab, const double *nb, int ns,
                                               int lane, double *mat, bool paper, int w, int nw) {
  bool range_bad = false;
  // (a, b) comes from q in closed form, so the loop has a fixed trip count
  const int npairs = P.K * (P.K - 1) / 2;
#pragma unroll 1
  for (int q = lane + w * WAVE; q < npairs; q += nw * WAVE) {
    // m = a - 1 from the hardware square root (within an ulp), then made exact
    const unsigned uq = (unsigned)q;
    unsigned m = (unsigned)(0.5f * (1.0f + __builtin_amdgcn_sqrtf(1.0f + 8.0f * (float)q)));
    m -= (m * (m - 1u) / 2u > uq);
    m += ((m + 1u) * m / 2u <= uq);
    const int a = (int)m + 1, b = (int)(uq - m * (m - 1u) / 2u) + 1;
    double c[4];
    range_bad |= !pair_cov<SPIN>(P, tab, nb, ns, a, b, paper, c);
    if (SPIN == 0) {
      mat[tri(a - 1) + (b - 1)] = c[0];
    } else {
      const int ra = 2 * (a - 1), rb = 2 * (b - 1);
      mat[tri(ra) + rb] = c[0];
      mat[tri(ra) + rb + 1] = c[1];
      mat[tri(ra + 1) + rb] = c[2];
      mat[tri(ra + 1) + rb + 1] = c[3];
    }
  }
  return range_bad;
}

// Packed lower triangle of S (row-major, unit diagonal before the nugget) and
// the right-hand sides [b | data] (spin 0) or [b_Q | b_U | data] (spin 2) in
// LDS.  First pass: one neighbour per lane, its target covariances, data and
// diagonal; second pass: the off-diagonal pairs (a, b), 1 <= b < a <= K, with no
// per-pair branches.
// w, nw: this wave's share when nw waves assemble one system together (the
// loops stride over nw * WAVE lanes); one wave by default.
template <int SPIN, int NR>
__device__ void assemble(const PlanDev &P, const double *tab, const double *nb, int lane,
                         double *mat, double *rhs, int w = 0, int nw = 1) {
  const int K = P.K;
  const int ns = nb_stride(K);
  const bool paper = (P.mode == FLINTS_S2_PAPER);
  bool range_bad = false;
  for (int a = 1 + lane + w * WAVE; a <= K; a += nw * WAVE) {
    double c[4];
    range_bad |= !pair_cov<SPIN>(P, tab, nb, ns, a, 0, paper, c);
    if (SPIN == 0) {
      const int ra = a - 1;
      mat[tri(ra) + ra] = 1.0;
      rhs[ra * NR + 0] = c[0];
    } else {
      const int ra = 2 * (a - 1);
      mat[tri(ra) + ra] = 1.0;
      mat[tri(ra + 1) + ra] = 0.0;
      mat[tri(ra + 1) + ra + 1] = 1.0;
      rhs[ra * NR + 0] = c[0];          // Cov(Q_a, Q_0)
      rhs[ra * NR + 1] = c[1];          // Cov(Q_a, U_0)
      rhs[(ra + 1) * NR + 0] = c[2];    // Cov(U_a, Q_0)
      rhs[(ra + 1) * NR + 1] = c[3];    // Cov(U_a, U_0)
    }
  }
  range_bad |= assemble_pairs<SPIN>(P, tab, nb, ns, lane, mat, paper, w, nw);
  count_event(P.counters + CNT_TABLE_RANGE, range_bad, lane);
}

// Assembly for the LDS elimination, whose right-hand sides overlay the
// neighbour records: the pairs are written and the target covariances of
// neighbour a = 1 + lane + w WAVE (K <= 64: at most one per lane) computed into
// registers while the records are read; after a barrier (nw waves) or a fence
// (one wave) the right-hand sides are written, the data column read from the
// map again.  The records must be complete (and visible) on entry.
template <int SPIN, int NR>
__device__ void lds_assemble(const PlanDev &P, const double *tab, const double *__restrict__ map,
                             const int *sel, const double *nb, int lane, double *mat, double *rhs, int w,
                             int nw) {
  const int K = P.K;
  const int ns = nb_stride(K);
  const bool paper = (P.mode == FLINTS_S2_PAPER);
  bool range_bad = false;
  const int a = 1 + lane + w * WAVE;
  const bool has = a <= K;
  double c[4] = {0.0, 0.0, 0.0, 0.0};
  if (has) {
    range_bad |= !pair_cov<SPIN>(P, tab, nb, ns, a, 0, paper, c);
    if (SPIN == 0) {
      mat[tri(a - 1) + a - 1] = 1.0;
    } else {
      const int ra = 2 * (a - 1);
      mat[tri(ra) + ra] = 1.0;
      mat[tri(ra + 1) + ra] = 0.0;
      mat[tri(ra + 1) + ra + 1] = 1.0;
    }
  }
  range_bad |= assemble_pairs<SPIN>(P, tab, nb, ns, lane, mat, paper, w, nw);
  count_event(P.counters + CNT_TABLE_RANGE, range_bad, lane);
  if (nw > 1) __syncthreads(); else compiler_fence();   // the records are no longer read
  if (has) {
    const int64_t p = sel[a - 1];
    if (SPIN == 0) {
      rhs[(a - 1) * NR + 0] = c[0];
      rhs[(a - 1) * NR + NR - 1] = map_value(P, map, p);
    } else {
      const int ra = 2 * (a - 1);
      rhs[ra * NR + 0] = c[0];
      rhs[ra * NR + 1] = c[1];
      rhs[(ra + 1) * NR + 0] = c[2];
      rhs[(ra + 1) * NR + 1] = c[3];
      rhs[ra * NR + NR - 1] = map_value(P, map, p);
      rhs[(ra + 1) * NR + NR - 1] = map_value(P, map, P.npix + p);
    }
  }
}

// ---------------------------------------------------------------- phase B
// Full symmetric row `row` of the group's system into registers (the upper part
// is read from the mirrored packed entry); rows past n and rows of inactive
// groups become identity rows with zero right-hand sides, which leave the
// factorisation of the real rows untouched.
template <int NMAX, int NR>
__device__ inline void load_rows(const double *mat, const double *rhs, int row, bool act, int nrow,
                                 double (&a)[NMAX], double (&r)[NR]) {
#pragma unroll
  for (int j = 0; j < NMAX; ++j) {
    const int idx = (j <= row) ? tri(row) + j : tri(j) + row;
    // columns past n stay exactly zero in real rows (padding must not see garbage)
    a[j] = act ? ((j < nrow) ? mat[idx] : 0.0) : (j == row ? 1.0 : 0.0);
  }
#pragma unroll
  for (int q = 0; q < NR; ++q) r[q] = act ? rhs[row * NR + q] : 0.0;
}

__device__ inline double rsqrt_t(double x) { return rsqrt(x); }
__device__ inline float rsqrt_t(float x) { return rsqrtf(x); }

// Right-looking Cholesky of the group's rows (all NMAX steps) with the
// right-hand sides carried along.  Every active lane updates its whole row, so
// the trailing matrix stays symmetric and the column needed at step k equals row
// k, held by one lane: pivot, column and the pivot row's right-hand sides are
// broadcast with readlane (no LDS traffic).  Rows that have already pivoted do
// not update, so at the end lane i holds row i of L (columns < i), L_ii, and in
// its upper half A^(i)_ij = L_ji L_ii (column i of L, scaled): both triangular
// solves are then register-local (see back_solve).  Steps are generated by
// template recursion so every register index is a compile-time constant.
template <typename T, int NMAX, int G, int NR, int K>
__device__ __forceinline__ void chol_step(T (&a)[NMAX], T (&r)[NR], int row, int grp, T nug,
                                          bool &ok, T &mydiag) {
  const T d = group_bcast<G>(a[K], K, grp) + nug;
  ok = ok && (d > T(0));
  const T rs = rsqrt_t(d);
  const T c = (row > K) ? a[K] * rs * rs : T(0);
  // broadcasts issued four at a time, so the VALU write of each SGPR pair is
  // separated from its first read by independent work (no hazard stalls)
  constexpr int CH = 4;
#pragma unroll
  for (int j0 = K + 1; j0 < NMAX; j0 += CH) {
    T s[CH];
#pragma unroll
    for (int u = 0; u < CH; ++u)
      if (j0 + u < NMAX) s[u] = group_bcast<G>(a[j0 + u], K, grp);
#pragma unroll
    for (int u = 0; u < CH; ++u)
      if (j0 + u < NMAX) a[j0 + u] = fma(-c, s[u], a[j0 + u]);
  }
#pragma unroll
  for (int q = 0; q < NR; ++q) r[q] = fma(-c, group_bcast<G>(r[q], K, grp), r[q]);
  const T piv = d * rs;
  if (row == K) mydiag = piv;
  a[K] = (row == K) ? piv : ((row > K) ? a[K] * rs : a[K]);
  if constexpr (K + 1 < NMAX) chol_step<T, NMAX, G, NR, K + 1>(a, r, row, grp, nug, ok, mydiag);
}

template <int NMAX, int G, int NR, typename T>
__device__ __forceinline__ bool chol_rows(T (&a)[NMAX], T (&r)[NR], int row, int grp, T nug,
                                          T &mydiag) {
  bool ok = true;
  mydiag = T(1);
  chol_step<T, NMAX, G, NR, 0>(a, r, row, grp, nug, ok, mydiag);
  return ok;
}

// Backward substitution L^T w = y after chol_rows: lane i accumulates
// sum_{k>i} A^(i)_ik w_k = L_ii sum_{k>i} L_ki w_k from its own upper half as the
// w_k (k descending) are broadcast, then w_i = (y_i - acc_i / L_ii) / L_ii.
template <typename T, int NMAX, int G, int NW, int K>
__device__ __forceinline__ void back_step(const T (&a)[NMAX], const T (&y)[NW], T inv, int row,
                                          int grp, T (&acc)[NW], T (&w)[NW]) {
#pragma unroll
  for (int q = 0; q < NW; ++q) {
    const T t = (y[q] - acc[q] * inv) * inv;
    const T wk = group_bcast<G>(t, K, grp);
    if (row == K) w[q] = wk;
    acc[q] = (row < K) ? fma(a[K], wk, acc[q]) : acc[q];
  }
  if constexpr (K > 0) back_step<T, NMAX, G, NW, K - 1>(a, y, inv, row, grp, acc, w);
}

template <int NMAX, int G, int NW, typename T>
__device__ __forceinline__ void back_solve(const T (&a)[NMAX], const T (&y)[NW], T diag, int row,
                                           int grp, T (&w)[NW]) {
  T acc[NW], inv = T(1) / diag;
#pragma unroll
  for (int q = 0; q < NW; ++q) { acc[q] = T(0); w[q] = T(0); }
  back_step<T, NMAX, G, NW, NMAX - 1>(a, y, inv, row, grp, acc, w);
}

// Forward substitution L t = v with L in the lanes' lower halves (row i holds
// L_ij, j < i), pivots broadcast in increasing order.
template <typename T, int NMAX, int G, int NW, int K>
__device__ __forceinline__ void fwd_step(const T (&a)[NMAX], T (&v)[NW], T inv, int row, int grp,
                                         T (&t)[NW]) {
#pragma unroll
  for (int q = 0; q < NW; ++q) {
    const T tk = group_bcast<G>(v[q] * inv, K, grp);
    if (row == K) t[q] = tk;
    v[q] = (row > K) ? fma(-a[K], tk, v[q]) : v[q];
  }
  if constexpr (K + 1 < NMAX) fwd_step<T, NMAX, G, NW, K + 1>(a, v, inv, row, grp, t);
}

template <int NMAX, int G, int NW, typename T>
__device__ __forceinline__ void fwd_solve(const T (&a)[NMAX], T (&v)[NW], T diag, int row,
                                          int grp, T (&t)[NW]) {
  const T inv = T(1) / diag;
#pragma unroll
  for (int q = 0; q < NW; ++q) t[q] = T(0);
  fwd_step<T, NMAX, G, NW, 0>(a, v, inv, row, grp, t);
}

template <int G>
__device__ inline double group_sum(double v) {
#pragma unroll
  for (int o = G / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, G);
  return v;
}

// ---------------------------------------------------------------- kernel
// Output values that tag a point for the fix-up pass (quiet NaNs with private
// payloads): FP64 factorisation failed (nugget escalation needed), or the FP32
// factorisation / refinement was rejected (recompute in FP64).
constexpr unsigned long long FAIL64_BITS = 0x7ff80000000f1a7ull;
constexpr unsigned long long FAIL32_BITS = 0x7ff80000000f132ull;

// Phase A, first half, for one point with the whole wave: validity and the
// K-nearest search.  Returns false if the point is invalid or its stencil was
// not found.
__device__ inline bool phase_a_search(const PlanDev &P, double th, double ph, int lane, double *cu,
                                      int *ci, RingSpan *rs, int *sel) {
  const bool good = (th >= 0.0) && (th <= kconst(PI_D)) && isfinite(ph);
  if (!good) {
    if (lane == 0) atomicAdd(P.counters + CNT_BAD_INPUT, 1ull);
    return false;
  }
  if (!knn_search(P, th, ph, lane, cu, ci, rs, sel)) {
    if (lane == 0) atomicAdd(P.counters + CNT_SEARCH_FAIL, 1ull);
    return false;
  }
  return true;
}

// Phase A, second half: neighbour records and the covariance assembly.
template <int SPIN, int NR>
__device__ inline void phase_a_build(const PlanDev &P, const double *tab,
                                     const double *__restrict__ map, double th, double ph, int lane,
                                     const int *sel, double *nb, double *mat, double *rhs) {
  neighbour_records<SPIN, NR>(P, th, ph, lane, sel, nb, rhs, map);
  assemble<SPIN, NR>(P, tab, nb, lane, mat, rhs);
}

struct WaveBufs {
  double *cu; int *ci; RingSpan *rs; int *sel; double *nb; double *mat; double *rhs; double *rbuf;
};

__device__ inline WaveBufs wave_bufs(char *lds, const Layout &L, int wave) {
  char *wb = lds + L.tab_bytes + wave * L.wave_bytes;
  WaveBufs B;
  B.cu = (double *)(wb + L.off_cu);
  B.ci = (int *)(wb + L.off_ci);
  B.rs = (RingSpan *)(wb + L.off_rings);
  B.sel = (int *)(wb + L.off_sel);
  B.nb = (double *)(wb + L.off_nb);
  B.mat = (double *)(wb + L.off_mat);
  B.rhs = (double *)(wb + L.off_rhs);
  B.rbuf = (double *)(wb + L.off_rbuf);
  return B;
}

__device__ inline const double *load_table(char *lds, const PlanDev &P) {
  const int ntabd = P.ntab * P.nfun;
  for (int i = threadIdx.x; i < ntabd; i += blockDim.x) ((double *)lds)[i] = P.tab[i];
  __syncthreads();
  return (const double *)lds;
}

// The correlation table a kernel reads: its LDS copy, or (layouts with no table
// bytes) the plan's table in device memory, read through the caches.
__device__ inline const double *kernel_table(char *lds, const PlanDev &P, const Layout &L) {
  return L.tab_bytes ? load_table(lds, P) : P.tab;
}

template <int G>
__device__ inline double group_min(double v) {
#pragma unroll
  for (int o = G / 2; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, G));
  return v;
}
template <int G>
__device__ inline double group_max(double v) {
#pragma unroll
  for (int o = G / 2; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, G));
  return v;
}

// Per-group results handed to store_point.
struct GroupOut {
  double v0, v1, qd0, qd1, w0, w1;
};

// ---------------------------------------------------------------- phase B, n <= 32
// One system per 16-lane row of the wave (four points per wave).  Lane x of a
// row group holds the lower-triangular rows x + 16 t (t < NT) of its point, row
// x + 16 t in a[t][0 .. 16 t + 15] with the column as register index, plus the
// right-hand sides of those rows.  The right-looking elimination needs, at step
// k, the pivot a_kk and column k (a_jk of every row j > k): both sit in one lane
// of the same 16-lane row, so each value reaches the whole row group through a
// DPP row broadcast (one VALU move per value, no scalar registers).  The pivot
// row is never scaled: row i is updated with c_i = a_ik / a_kk times the raw
// a_jk, and the right-hand sides likewise, so after the last step r_i = L_ii y_i.

// Value of v held by lane K of this lane's 16-lane row.
template <int K>
__device__ __forceinline__ double rbcast(double v) {
  return __builtin_amdgcn_mov_dpp(v, 0x150 + K, 0xf, 0xf, false);  // row_newbcast:K
}

// Compile-time loop: f(integral_constant<int, i>) for i in [B, E).
template <int B, int E, typename F>
__device__ __forceinline__ void cfor(F &&f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    cfor<B + 1, E>(f);
  }
}

// Column updates of one elimination step as v_fmac_f64 with a row_newbcast DPP
// source: the broadcast value feeds the multiply directly, so no separate move
// is issued.  For each column j: p_j += ncp * d_j(lane k), then d_j += ncd *
// d_j(lane k) (lane k's d_j is the pivot row's entry; ncd = 0 on lane k, so the
// source is unchanged).  Every block starts with s_nop 1, the two wait states a
// DPP read needs after a VALU write of its source; inside a block no DPP source
// is written before it is read.
#define FLINTS_FMAC_DPP(dst, src, c) "v_fmac_f64_dpp " dst ", " src ", " c " row_newbcast:%[k] row_mask:0xf bank_mask:0xf\n\t"

template <int K>
__device__ __forceinline__ void dpp_pd1(double &p0, double &d0, double ncp, double ncd) {
  __asm__ volatile("s_nop 1\n\t" FLINTS_FMAC_DPP("%[p0]", "%[d0]", "%[cp]") FLINTS_FMAC_DPP("%[d0]", "%[d0]", "%[cd]")
                   : [p0] "+v"(p0), [d0] "+v"(d0) : [cp] "v"(ncp), [cd] "v"(ncd), [k] "i"(K));
}
template <int K>
__device__ __forceinline__ void dpp_pd4(double &p0, double &d0, double &p1, double &d1, double &p2, double &d2,
                                        double &p3, double &d3, double ncp, double ncd) {
  __asm__ volatile("s_nop 1\n\t"
                   FLINTS_FMAC_DPP("%[p0]", "%[d0]", "%[cp]") FLINTS_FMAC_DPP("%[d0]", "%[d0]", "%[cd]")
                   FLINTS_FMAC_DPP("%[p1]", "%[d1]", "%[cp]") FLINTS_FMAC_DPP("%[d1]", "%[d1]", "%[cd]")
                   FLINTS_FMAC_DPP("%[p2]", "%[d2]", "%[cp]") FLINTS_FMAC_DPP("%[d2]", "%[d2]", "%[cd]")
                   FLINTS_FMAC_DPP("%[p3]", "%[d3]", "%[cp]") FLINTS_FMAC_DPP("%[d3]", "%[d3]", "%[cd]")
                   : [p0] "+v"(p0), [d0] "+v"(d0), [p1] "+v"(p1), [d1] "+v"(d1), [p2] "+v"(p2), [d2] "+v"(d2),
                     [p3] "+v"(p3), [d3] "+v"(d3)
                   : [cp] "v"(ncp), [cd] "v"(ncd), [k] "i"(K));
}
template <int K>
__device__ __forceinline__ void dpp_d1(double &d0, double ncd) {
  __asm__ volatile("s_nop 1\n\t" FLINTS_FMAC_DPP("%[d0]", "%[d0]", "%[cd]")
                   : [d0] "+v"(d0) : [cd] "v"(ncd), [k] "i"(K));
}
template <int K>
__device__ __forceinline__ void dpp_d4(double &d0, double &d1, double &d2, double &d3, double ncd) {
  __asm__ volatile("s_nop 1\n\t" FLINTS_FMAC_DPP("%[d0]", "%[d0]", "%[cd]") FLINTS_FMAC_DPP("%[d1]", "%[d1]", "%[cd]")
                   FLINTS_FMAC_DPP("%[d2]", "%[d2]", "%[cd]") FLINTS_FMAC_DPP("%[d3]", "%[d3]", "%[cd]")
                   : [d0] "+v"(d0), [d1] "+v"(d1), [d2] "+v"(d2), [d3] "+v"(d3) : [cd] "v"(ncd), [k] "i"(K));
}
// Pivot of step K + 1 from lane K + 1, read after the wait states its DPP source
// needs (it was just updated by the first column block).
template <int K>
__device__ __forceinline__ double dpp_pivot(double &dsrc) {
  double r;
  __asm__ volatile("s_nop 1\n\tv_mov_b64_dpp %[r], %[s] row_newbcast:%[k] row_mask:0xf bank_mask:0xf"
                   : [r] "=&v"(r) : [s] "v"(dsrc), [k] "i"(K));
  return r;
}
// dst_t += c_t * src(lane L) for one or two destinations sharing the source.
template <int L>
__device__ __forceinline__ void dpp_fma1(double &d0, double src, double c0) {
  __asm__ volatile("s_nop 1\n\t" FLINTS_FMAC_DPP("%[d0]", "%[s]", "%[c0]")
                   : [d0] "+v"(d0) : [s] "v"(src), [c0] "v"(c0), [k] "i"(L));
}
template <int L>
__device__ __forceinline__ void dpp_fma2(double &d0, double &d1, double src, double c0, double c1) {
  __asm__ volatile("s_nop 1\n\t" FLINTS_FMAC_DPP("%[d0]", "%[s]", "%[c0]") FLINTS_FMAC_DPP("%[d1]", "%[s]", "%[c1]")
                   : [d0] "+v"(d0), [d1] "+v"(d1) : [s] "v"(src), [c0] "v"(c0), [c1] "v"(c1), [k] "i"(L));
}
#undef FLINTS_FMAC_DPP

// Columns J0 .. 15 of step K, in blocks of four.
template <int K, int J0, bool PANEL>
__device__ __forceinline__ void dpp_columns(double (&d)[16], double (&p)[16], double ncp, double ncd) {
  if constexpr (J0 + 4 <= 16) {
    if constexpr (PANEL)
      dpp_pd4<K>(p[J0], d[J0], p[J0 + 1], d[J0 + 1], p[J0 + 2], d[J0 + 2], p[J0 + 3], d[J0 + 3], ncp, ncd);
    else
      dpp_d4<K>(d[J0], d[J0 + 1], d[J0 + 2], d[J0 + 3], ncd);
    dpp_columns<K, J0 + 4, PANEL>(d, p, ncp, ncd);
  } else if constexpr (J0 < 16) {
    if constexpr (PANEL) dpp_pd1<K>(p[J0], d[J0], ncp, ncd);
    else dpp_d1<K>(d[J0], ncd);
    dpp_columns<K, J0 + 1, PANEL>(d, p, ncp, ncd);
  }
}

template <int NT, int NR>
struct RowSys {
  double a[NT][16 * NT];   // a[t][j] used for j < 16 (t + 1)
  double r[NT][NR];
};

// Identity rows with zero right-hand sides (inactive points and padding rows
// factorise trivially and leave the real rows untouched).
template <int NT, int NR>
__device__ __forceinline__ void rowsys_identity(RowSys<NT, NR> &S, int x) {
#pragma unroll
  for (int t = 0; t < NT; ++t) {
#pragma unroll
    for (int j = 0; j < 16 * (t + 1); ++j) S.a[t][j] = (j == x + 16 * t) ? 1.0 : 0.0;
#pragma unroll
    for (int q = 0; q < NR; ++q) S.r[t][q] = 0.0;
  }
}

// Rows x + 16 t of the packed system (lower triangle, row-major) into registers,
// with the nugget added on the diagonal.  Entries right of the diagonal are zero.
template <int NT, int NR>
__device__ __forceinline__ void rowsys_load(RowSys<NT, NR> &S, const double *mat, const double *rhs,
                                            int x_in, int nrow, double nug) {
  int x = x_in;
  __asm__ volatile("" : "+v"(x));   // row-dependent LDS addresses stay out of LICM
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int i = x + 16 * t;
    const bool real = i < nrow;
    const int ic = real ? i : 0;
#pragma unroll
    for (int j = 0; j < 16 * (t + 1); ++j) {
      const double v = mat[tri(ic) + (j < ic ? j : ic)];
      S.a[t][j] = real ? (j < i ? v : (j == i ? v + nug : 0.0)) : (j == i ? 1.0 : 0.0);
    }
#pragma unroll
    for (int q = 0; q < NR; ++q) S.r[t][q] = real ? rhs[ic * NR + q] : 0.0;
  }
}

// Step K of the row-group elimination.  d = a_KK and inv = 1 / d arrive from
// step K - 1, which computes them as soon as column K + 1 is final so that the
// reciprocal overlaps the rest of that step's updates.  dg keeps the pivot of
// each of the lane's rows: r_i^2 / d_i = y_i^2 needs no square root.
// Four consecutive columns L0 .. L0 + 3 (one 16-lane block) of a row-group
// step: dst_t[i] += c_t * src(lane L0 + i), one or two row arrays.
template <int L0>
__device__ __forceinline__ void dpp_cols4x1(double &a0, double &a1, double &a2, double &a3, double src, double c0) {
  __asm__ volatile("s_nop 1\n\t"
                   "v_fmac_f64_dpp %[a0], %[s], %[c0] row_newbcast:%[l0] row_mask:0xf bank_mask:0xf\n\t"
                   "v_fmac_f64_dpp %[a1], %[s], %[c0] row_newbcast:%[l1] row_mask:0xf bank_mask:0xf\n\t"
                   "v_fmac_f64_dpp %[a2], %[s], %[c0] row_newbcast:%[l2] row_mask:0xf bank_mask:0xf\n\t"
                   "v_fmac_f64_dpp %[a3], %[s], %[c0] row_newbcast:%[l3] row_mask:0xf bank_mask:0xf"
                   : [a0] "+v"(a0), [a1] "+v"(a1), [a2] "+v"(a2), [a3] "+v"(a3)
                   : [s] "v"(src), [c0] "v"(c0), [l0] "i"(L0), [l1] "i"(L0 + 1), [l2] "i"(L0 + 2), [l3] "i"(L0 + 3));
}
template <int L0>
__device__ __forceinline__ void dpp_cols4x2(double &a0, double &a1, double &a2, double &a3, double &b0, double &b1,
                                            double &b2, double &b3, double src, double c0, double c1) {
  __asm__ volatile("s_nop 1\n\t"
                   "v_fmac_f64_dpp %[a0], %[s], %[c0] row_newbcast:%[l0] row_mask:0xf bank_mask:0xf\n\t"
                   "v_fmac_f64_dpp %[b0], %[s], %[c1] row_newbcast:%[l0] row_mask:0xf bank_mask:0xf\n\t"
                   "v_fmac_f64_dpp %[a1], %[s], %[c0] row_newbcast:%[l1] row_mask:0xf bank_mask:0xf\n\t"
                   "v_fmac_f64_dpp %[b1], %[s], %[c1] row_newbcast:%[l1] row_mask:0xf bank_mask:0xf\n\t"
                   "v_fmac_f64_dpp %[a2], %[s], %[c0] row_newbcast:%[l2] row_mask:0xf bank_mask:0xf\n\t"
                   "v_fmac_f64_dpp %[b2], %[s], %[c1] row_newbcast:%[l2] row_mask:0xf bank_mask:0xf\n\t"
                   "v_fmac_f64_dpp %[a3], %[s], %[c0] row_newbcast:%[l3] row_mask:0xf bank_mask:0xf\n\t"
                   "v_fmac_f64_dpp %[b3], %[s], %[c1] row_newbcast:%[l3] row_mask:0xf bank_mask:0xf"
                   : [a0] "+v"(a0), [a1] "+v"(a1), [a2] "+v"(a2), [a3] "+v"(a3), [b0] "+v"(b0), [b1] "+v"(b1),
                     [b2] "+v"(b2), [b3] "+v"(b3)
                   : [s] "v"(src), [c0] "v"(c0), [c1] "v"(c1), [l0] "i"(L0), [l1] "i"(L0 + 1), [l2] "i"(L0 + 2),
                     [l3] "i"(L0 + 3));
}

// Columns J0 .. N - 1 of row-group step K (after column K + 1, which carries the
// next pivot): blocks of four within a 16-column block, else one at a time.
template <int NT, int NR, int K, int J0>
__device__ __forceinline__ void rowsys_columns(RowSys<NT, NR> &S, const double (&nc)[NT]) {
  constexpr int N = 16 * NT, TK = K / 16;
  if constexpr (J0 < N) {
    constexpr int T0 = (J0 / 16 > TK ? J0 / 16 : TK);
    if constexpr (J0 % 16 <= 12 && J0 + 4 <= N && (J0 + 3) / 16 == J0 / 16) {
      if constexpr (T0 + 1 < NT)
        dpp_cols4x2<J0 % 16>(S.a[T0][J0], S.a[T0][J0 + 1], S.a[T0][J0 + 2], S.a[T0][J0 + 3], S.a[T0 + 1][J0],
                             S.a[T0 + 1][J0 + 1], S.a[T0 + 1][J0 + 2], S.a[T0 + 1][J0 + 3], S.a[J0 / 16][K],
                             nc[T0], nc[T0 + 1]);
      else
        dpp_cols4x1<J0 % 16>(S.a[T0][J0], S.a[T0][J0 + 1], S.a[T0][J0 + 2], S.a[T0][J0 + 3], S.a[J0 / 16][K],
                             nc[T0]);
      rowsys_columns<NT, NR, K, J0 + 4>(S, nc);
    } else {
      if constexpr (T0 + 1 < NT) dpp_fma2<J0 % 16>(S.a[T0][J0], S.a[T0 + 1][J0], S.a[J0 / 16][K], nc[T0], nc[T0 + 1]);
      else dpp_fma1<J0 % 16>(S.a[T0][J0], S.a[J0 / 16][K], nc[T0]);
      rowsys_columns<NT, NR, K, J0 + 1>(S, nc);
    }
  }
}

template <int NT, int NR, int K>
__device__ __forceinline__ void rowsys_step(RowSys<NT, NR> &S, double (&dg)[NT], int x, bool &ok,
                                            double d, double inv) {
  constexpr int TK = K / 16, XK = K % 16, N = 16 * NT;
  ok = ok && (d > 0.0);
  double c[NT];
#pragma unroll
  for (int t = TK; t < NT; ++t) c[t] = (x + 16 * t > K) ? S.a[t][K] * inv : 0.0;
  double dn = 1.0, invn = 1.0;
  double nc[NT];
#pragma unroll
  for (int t = TK; t < NT; ++t) nc[t] = -c[t];
  // column j takes a_ij -= c_i a_jK for the lane's rows i = x + 16 t >= j; the
  // source a_jK is lane j % 16's register a[j / 16][K], fed to the FMAs by DPP
  static_assert(NT <= 2, "row-group engine holds at most two row arrays");
  if constexpr (K + 1 < N) {
    constexpr int j = K + 1, T0 = (j / 16 > TK ? j / 16 : TK);
    if constexpr (T0 + 1 < NT) dpp_fma2<j % 16>(S.a[T0][j], S.a[T0 + 1][j], S.a[j / 16][K], nc[T0], nc[T0 + 1]);
    else dpp_fma1<j % 16>(S.a[T0][j], S.a[j / 16][K], nc[T0]);
    dn = dpp_pivot<j % 16>(S.a[j / 16][j]);   // next pivot, final after this update
    invn = recip(dn);
    rowsys_columns<NT, NR, K, K + 2>(S, nc);
  }
  // right-hand sides: the source r[TK][q] of lane XK is also a destination, so
  // the other array is updated first (no DPP read after a write of its source;
  // lane XK's own r[TK][q] is unchanged since its coefficient is zero)
#pragma unroll
  for (int q = 0; q < NR; ++q) {
    if constexpr (TK + 1 < NT) dpp_fma2<XK>(S.r[TK + 1][q], S.r[TK][q], S.r[TK][q], nc[TK + 1], nc[TK]);
    else dpp_fma1<XK>(S.r[TK][q], S.r[TK][q], nc[TK]);
  }
  dg[TK] = (x == XK) ? d : dg[TK];
  if constexpr (K + 1 < N) rowsys_step<NT, NR, K + 1>(S, dg, x, ok, dn, invn);
}

// Factorise, then value = y . z and quad = y . y per point as in fp64_phase_b
// (y_i = r_i / L_ii, so y_i y'_i = r_i r'_i / d_i).  Results are valid in every
// lane of the row group; ok is uniform in the group.
template <int NT, int SPIN, int NR>
__device__ inline bool rowsys_phase_b(RowSys<NT, NR> &S, int x, int nrow, GroupOut &o) {
  double dg[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) dg[t] = 1.0;
  bool ok = true;
  const double d0 = rbcast<0>(S.a[0][0]);
  rowsys_step<NT, NR, 0>(S, dg, x, ok, d0, recip(d0));
  double v0 = 0.0, v1 = 0.0, q0 = 0.0, q1 = 0.0;
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const double inv = (x + 16 * t < nrow) ? recip(dg[t]) : 0.0;
    const double r0 = S.r[t][0], r1 = S.r[t][1];
    if (SPIN == 0) {
      v0 = fma(r0 * r1, inv, v0);
      q0 = fma(r0 * r0, inv, q0);
    } else {
      const double r2 = S.r[t][NR - 1];
      v0 = fma(r0 * r2, inv, v0);
      v1 = fma(r1 * r2, inv, v1);
      q0 = fma(r0 * r0, inv, q0);
      q1 = fma(r1 * r1, inv, q1);
    }
  }
  o.v0 = group_sum<16>(v0);
  o.qd0 = group_sum<16>(q0);
  o.v1 = o.qd1 = o.w0 = o.w1 = 0.0;
  if (SPIN != 0) {
    o.v1 = group_sum<16>(v1);
    o.qd1 = group_sum<16>(q1);
  }
  return ok;
}

// ---------------------------------------------------------------- phase B, 32 < n <= 64
// Blocked right-looking Cholesky of one system per wave on 16 x 16 tiles.  For
// block column J the wave's four 16-lane row groups each take one block row
// J + rho (rho = 0 .. 3): every group holds a replica of the diagonal tile (row x
// of it in lane x) and its own panel tile, and eliminates the 16 columns with
// DPP row broadcasts as in the row-group path, which factors the diagonal tile
// and solves the panel L_rJ = A_rJ L_JJ^-T at once.  The trailing tiles then
// take A_rs -= L_rJ L_sJ^T on the FP64 matrix cores (v_mfma_f64_16x16x4f64),
// with the panels staged through LDS into the MFMA operand layout.  Trailing
// tiles live in registers in the MFMA accumulator layout: lane l, element v
// holds tile entry (4 v + l / 16, l % 16).  The right-hand sides ride along in
// the elimination and return to LDS between block columns.

typedef double dbl4 __attribute__((ext_vector_type(4)));

constexpr int TSTR = 18;             // row stride (doubles) of a staged 16 x 16 tile
constexpr int TILE_D = 16 * TSTR;    // doubles per staged tile

template <int T>
struct TileSys {
  dbl4 c[T][T];   // c[r][s], 1 <= s <= r < T
};

// S + nI entry (i, j) of the packed system, identity beyond n.
__device__ __forceinline__ double packed_entry(const double *mat, int i, int j, int nrow, double nug) {
  const bool real = (i < nrow) && (j < nrow);
  const int hi = i > j ? i : j, lo = i > j ? j : i;
  const double v = mat[real ? tri(hi) + lo : 0];
  return real ? (i == j ? v + nug : v) : (i == j ? 1.0 : 0.0);
}

template <int T>
__device__ __forceinline__ void tiles_load(TileSys<T> &S, const double *mat, int l, int nrow, double nug) {
#pragma unroll
  for (int r = 1; r < T; ++r)
#pragma unroll
    for (int s = 1; s <= r; ++s)
#pragma unroll
      for (int v = 0; v < 4; ++v)
        S.c[r][s][v] = packed_entry(mat, 16 * r + 4 * v + (l >> 4), 16 * s + (l & 15), nrow, nug);
}

struct TileAcc {
  double v0, v1, q0, q1;
};

template <int T, int SPIN, int NR, int J>
__device__ __forceinline__ void tile_step(TileSys<T> &S, double *scr, double *rhs, const double *mat,
                                          int l, int nrow, double nug, TileAcc &acc, bool &ok) {
  const int rho = l >> 4, x = l & 15;
  const int rp = J + rho;                       // block row of this row group
  const bool prow = (rho > 0) && (rp < T);      // group carries a panel tile
  double d[16], p[16], dr[NR], pr[NR];
  if constexpr (J == 0) {
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      d[j] = packed_entry(mat, x, j, nrow, nug);
      p[j] = prow ? packed_entry(mat, 16 * rp + x, j, nrow, nug) : 0.0;
    }
  } else {
#pragma unroll
    for (int r = J; r < T; ++r)
#pragma unroll
      for (int v = 0; v < 4; ++v) scr[(r - J) * TILE_D + (4 * v + rho) * TSTR + x] = S.c[r][J][v];
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      d[j] = scr[x * TSTR + j];
      p[j] = prow ? scr[rho * TILE_D + x * TSTR + j] : 0.0;
    }
  }
  const int ir = 16 * J + x, ip = 16 * rp + x;
#pragma unroll
  for (int q = 0; q < NR; ++q) {
    dr[q] = (ir < nrow) ? rhs[ir * NR + q] : 0.0;
    pr[q] = (prow && ip < nrow) ? rhs[ip * NR + q] : 0.0;
  }
  double *piv = scr + (T - 1) * TILE_D;   // pivots a_kk of this block column
  double pv = rbcast<0>(d[0]);
  double iv = recip(pv);
  cfor<0, 16>([&](auto kc) {
    constexpr int k = decltype(kc)::value;
    ok = ok && (pv > 0.0);
    piv[k] = pv;                   // same value from every lane
    const double cd = (x > k) ? d[k] * iv : 0.0;
    const double cp = p[k] * iv;
    double pn = 1.0, ivn = 1.0;
    if constexpr (k + 1 < 16) {
      // column k + 1 first: it holds the next pivot, whose reciprocal then
      // overlaps the remaining columns
      if constexpr (J + 1 < T) dpp_pd1<k>(p[k + 1], d[k + 1], -cp, -cd);
      else dpp_d1<k>(d[k + 1], -cd);
      pn = dpp_pivot<k + 1>(d[k + 1]);
      ivn = recip(pn);
      dpp_columns<k, k + 2, (J + 1 < T)>(d, p, -cp, -cd);
    }
#pragma unroll
    for (int q = 0; q < NR; ++q) {
      if constexpr (J + 1 < T) dpp_pd1<k>(pr[q], dr[q], -cp, -cd);
      else dpp_d1<k>(dr[q], -cd);
    }
    p[k] = cp;                     // the panel keeps c_ik = a_ik / a_kk
    pv = pn;
    iv = ivn;
  });
  if constexpr (J + 1 < T) {
    // the panel is consumed only under `prow`; pin it here so its elimination is
    // not sunk into that branch (which would keep every broadcast value live)
#pragma unroll
    for (int j = 0; j < 16; ++j) __asm__ volatile("" ::"v"(p[j]));
#pragma unroll
    for (int q = 0; q < NR; ++q) __asm__ volatile("" ::"v"(pr[q]));
  }
  // rows of block J are final: y_i = r_i / L_ii (counted once, by row group 0)
  if (rho == 0 && ir < nrow) {
    const double inv = recip(piv[x]);   // y_i y'_i = r_i r'_i / d_i
    const double r0 = dr[0], r1 = dr[1];
    if (SPIN == 0) {
      acc.v0 = fma(r0 * r1, inv, acc.v0);
      acc.q0 = fma(r0 * r0, inv, acc.q0);
    } else {
      const double r2 = dr[NR - 1];
      acc.v0 = fma(r0 * r2, inv, acc.v0);
      acc.v1 = fma(r1 * r2, inv, acc.v1);
      acc.q0 = fma(r0 * r0, inv, acc.q0);
      acc.q1 = fma(r1 * r1, inv, acc.q1);
    }
  }
  if constexpr (J + 1 < T) {
    if (prow && ip < nrow) {
#pragma unroll
      for (int q = 0; q < NR; ++q) rhs[ip * NR + q] = pr[q];
    }
    // panels C_rJ (c_ik = a_ik / a_kk, r > J) to LDS, then into the MFMA operand
    // layout: fr[r][m] at lane l = C_rJ(l % 16, 4 m + l / 16).  The trailing
    // update L_rJ L_sJ^T = sum_k c_ik a_jk takes a_jk = c_jk a_kk as the B operand,
    // so no square root is needed anywhere in the block column.
    if (prow) {
#pragma unroll
      for (int j = 0; j < 16; ++j) scr[(rho - 1) * TILE_D + x * TSTR + j] = p[j];
    }
    double fr[T][4], dk[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) dk[m] = piv[4 * m + rho];
#pragma unroll
    for (int r = J + 1; r < T; ++r)
#pragma unroll
      for (int m = 0; m < 4; ++m) fr[r][m] = scr[(r - J - 1) * TILE_D + x * TSTR + 4 * m + rho];
#pragma unroll
    for (int r = J + 1; r < T; ++r)
#pragma unroll
      for (int s = J + 1; s <= r; ++s)
#pragma unroll
        for (int m = 0; m < 4; ++m)
          S.c[r][s] = __builtin_amdgcn_mfma_f64_16x16x4f64(-fr[r][m], fr[s][m] * dk[m], S.c[r][s], 0, 0, 0);
    tile_step<T, SPIN, NR, J + 1>(S, scr, rhs, mat, l, nrow, nug, acc, ok);
  }
}

// Factorise the wave's system (packed in mat, right-hand sides in rhs) and
// return value / quad sums as fp64_phase_b does.  scr may overlay mat (mat is
// read in full before the first staged tile is written); rhs is overwritten.
template <int T, int SPIN, int NR>
__device__ inline bool tile_phase_b(const double *mat, double *rhs, double *scr, int lane_in, int nrow,
                                    double nug, GroupOut &o) {
  int l = lane_in;
  __asm__ volatile("" : "+v"(l));   // lane-dependent LDS addresses stay out of LICM
  TileSys<T> S;
  tiles_load<T>(S, mat, l, nrow, nug);
  TileAcc acc{0.0, 0.0, 0.0, 0.0};
  bool ok = true;
  tile_step<T, SPIN, NR, 0>(S, scr, rhs, mat, l, nrow, nug, acc, ok);
  o.v0 = group_sum<WAVE>(acc.v0);
  o.qd0 = group_sum<WAVE>(acc.q0);
  o.v1 = o.qd1 = o.w0 = o.w1 = 0.0;
  if (SPIN != 0) {
    o.v1 = group_sum<WAVE>(acc.v1);
    o.qd1 = group_sum<WAVE>(acc.q1);
  }
  return ok;
}


// FP64 phase B: factorise S + nI with the right-hand sides carried, then
// value = y.z and quad = y.y per point (y = L^-1 b, z = L^-1 data); with MSE
// also |w|^2 for w = L^-T y (register-local backward solve).
template <int NMAX, int G, int SPIN, int NR, bool MSE>
__device__ inline bool fp64_phase_b(const double *mat, const double *rhs, int row, int grp,
                                    bool ract, int nrow, double nug, GroupOut &o) {
  constexpr int NW = (SPIN == 0) ? 1 : 2;
  double a[NMAX];
  double r[NR];
  load_rows<NMAX, NR>(mat, rhs, row, ract, nrow, a, r);
  double diag;
  const bool ok = chol_rows<NMAX, G, NR>(a, r, row, grp, nug, diag);
  const double inv = 1.0 / diag;
  const double y0 = ract ? r[0] * inv : 0.0;
  const double y1 = ract ? r[1] * inv : 0.0;
  const double y2 = (ract && NR > 2) ? r[NR - 1] * inv : 0.0;
  o.v1 = o.qd1 = o.w0 = o.w1 = 0.0;
  if (SPIN == 0) {
    o.v0 = group_sum<G>(y0 * y1);
    o.qd0 = group_sum<G>(y0 * y0);
  } else {
    o.v0 = group_sum<G>(y0 * y2);
    o.v1 = group_sum<G>(y1 * y2);
    o.qd0 = group_sum<G>(y0 * y0);
    o.qd1 = group_sum<G>(y1 * y1);
  }
  if (MSE) {
    double yy[NW], w[NW];
    yy[0] = y0;
    if (NW > 1) yy[NW - 1] = y1;
    back_solve<NMAX, G, NW>(a, yy, diag, row, grp, w);
    o.w0 = group_sum<G>(ract ? w[0] * w[0] : 0.0);
    if (NW > 1) o.w1 = group_sum<G>(ract ? w[NW - 1] * w[NW - 1] : 0.0);
  }
  return ok;
}

// FP64 residual res = b - (S + nI) w for the NW right-hand sides, S read from the
// packed system in LDS and w_j broadcast from row j.
template <int NMAX, int G, int NW, int NR>
__device__ inline void residual64(const double *mat, const double *rhs, int row_in, bool ract, int nrow,
                                  double nug, const double (&w)[NW], int grp, double (&res)[NW]) {
  int row = row_in;
  __asm__ volatile("" : "+v"(row));   // recompute the row addresses here instead of keeping them live
#pragma unroll
  for (int q = 0; q < NW; ++q) res[q] = ract ? rhs[row * NR + q] - nug * w[q] : 0.0;
#pragma unroll
  for (int j = 0; j < NMAX; ++j) {
    const int idx = (j <= row) ? tri(row) + j : tri(j) + row;
    const double sij = (ract && j < nrow) ? mat[idx] : 0.0;
#pragma unroll
    for (int q = 0; q < NW; ++q) res[q] = fma(-sij, group_bcast<G>(w[q], j, grp), res[q]);
    if ((j & 7) == 7) __builtin_amdgcn_sched_barrier(0);   // bound the loads in flight
  }
}

// FP32 + refinement phase B: covariance entries stay FP64 in LDS;
// S + nI is rounded to FP32 and factorised, w = (S + nI)^-1 b is solved in FP32,
// one refinement step uses the FP64 residual and an FP32 correction solve, and
// value / variance use FP64 accumulation with the final FP64 residual r:
// var = sigma^2 (1 - b.w - w.r) (stationary in w).  The point is rejected (and
// recomputed in FP64) if the FP32 factorisation fails, if min L_kk / max L_kk is
// below the pivot-ratio threshold, or if |dw| > refine_tol |w|.
template <int NMAX, int G, int SPIN, int NR, bool MSE>
__device__ inline bool fp32_phase_b(const PlanDev &P, const double *mat, const double *rhs, int row_in,
                                    int grp, bool ract, int nrow, double nug, GroupOut &o) {
  constexpr int NW = (SPIN == 0) ? 1 : 2;
  int row = row_in;
  __asm__ volatile("" : "+v"(row));
  float a[NMAX];
  float rb[NW];
#pragma unroll
  for (int j = 0; j < NMAX; ++j) {
    const int idx = (j <= row) ? tri(row) + j : tri(j) + row;
    a[j] = ract ? ((j < nrow) ? (float)mat[idx] : 0.0f) : (j == row ? 1.0f : 0.0f);
  }
#pragma unroll
  for (int q = 0; q < NW; ++q) rb[q] = ract ? (float)rhs[row * NR + q] : 0.0f;
  float diag;
  bool ok = chol_rows<NMAX, G, NW>(a, rb, row, grp, (float)nug, diag);
  const double dmin = group_min<G>(ract ? (double)diag : 1e300);
  const double dmax = group_max<G>(ract ? (double)diag : 0.0);
  ok = ok && (dmin >= P.pivot_ratio_min * dmax);
  float y[NW], w32[NW];
#pragma unroll
  for (int q = 0; q < NW; ++q) y[q] = rb[q] / diag;
  back_solve<NMAX, G, NW>(a, y, diag, row, grp, w32);
  double w[NW], res[NW];
#pragma unroll
  for (int q = 0; q < NW; ++q) w[q] = ract ? (double)w32[q] : 0.0;
  residual64<NMAX, G, NW, NR>(mat, rhs, row, ract, nrow, nug, w, grp, res);
  float rv[NW], t[NW], dw[NW];
#pragma unroll
  for (int q = 0; q < NW; ++q) rv[q] = (float)res[q];
  fwd_solve<NMAX, G, NW>(a, rv, diag, row, grp, t);
  back_solve<NMAX, G, NW>(a, t, diag, row, grp, dw);
  double dn = 0.0, wn = 0.0;
#pragma unroll
  for (int q = 0; q < NW; ++q) {
    w[q] = ract ? w[q] + (double)dw[q] : 0.0;
    dn += ract ? (double)dw[q] * (double)dw[q] : 0.0;
    wn += w[q] * w[q];
  }
  dn = group_sum<G>(dn);
  wn = group_sum<G>(wn);
  ok = ok && (dn <= P.refine_tol * P.refine_tol * wn) && isfinite(dn);
  residual64<NMAX, G, NW, NR>(mat, rhs, row, ract, nrow, nug, w, grp, res);
  const double d = ract ? rhs[row * NR + NR - 1] : 0.0;
  o.v1 = o.qd1 = o.w0 = o.w1 = 0.0;
  const double b0 = ract ? rhs[row * NR + 0] : 0.0;
  o.v0 = group_sum<G>(w[0] * d);
  o.qd0 = group_sum<G>(w[0] * (b0 + res[0]));
  if (MSE) o.w0 = group_sum<G>(w[0] * w[0]);
  if (NW > 1) {
    const double b1 = ract ? rhs[row * NR + 1] : 0.0;
    o.v1 = group_sum<G>(w[NW - 1] * d);
    o.qd1 = group_sum<G>(w[NW - 1] * (b1 + res[NW - 1]));
    if (MSE) o.w1 = group_sum<G>(w[NW - 1] * w[NW - 1]);
  }
  return ok;
}

// Writes the outputs of point pt (called by lane row == 0 of its group).
// `tag` marks a rejected point for the fix-up pass.
template <int SPIN>
__device__ inline void store_point(const PlanDev &P, int64_t pt, int64_t n, bool gact, bool ok,
                                   unsigned long long tag, const GroupOut &o, double nug, bool mse,
                                   double *out, double *var) {
  const double nan = __builtin_nan("");
  const double s2 = P.sigma2;
  const bool good = gact && ok;
  const double bad = (gact && !ok) ? __longlong_as_double((long long)tag) : nan;
  if (SPIN == 0) {
    double vv = s2 * (1.0 - o.qd0);
    if (mse) vv -= s2 * nug * o.w0;
    if (good && vv < 0.0) { atomicAdd(P.counters + CNT_CLAMPED_VAR, 1ull); vv = 0.0; }
    out[pt] = good ? o.v0 : bad;
    if (var) var[pt] = good ? vv : nan;
  } else {
    double vq = s2 * (1.0 - o.qd0), vu = s2 * (1.0 - o.qd1);
    if (mse) { vq -= s2 * nug * o.w0; vu -= s2 * nug * o.w1; }
    if (good && (vq < 0.0 || vu < 0.0)) {
      atomicAdd(P.counters + CNT_CLAMPED_VAR, 1ull);
      vq = fmax(vq, 0.0);
      vu = fmax(vu, 0.0);
    }
    out[pt] = good ? o.v0 : bad;
    out[n + pt] = good ? o.v1 : bad;
    if (var) {
      var[pt] = good ? vq : nan;
      var[n + pt] = good ? vu : nan;
    }
  }
}

// ---------------------------------------------------------------- phase B, 64 < n <= 128
// Systems above 64 rows (spin 2 with 32 < K <= 64): S + nI = L D L^T (unit lower
// L, D the pivots) by blocked right-looking elimination of the wave's packed
// system in LDS, LDS_BS columns per block:
//   (1) every lane factors the block's pivot rows (LDS_BS x LDS_BS) with their
//       right-hand sides in registers, accumulating value and quad over the
//       final r_c r'_c / d_c (z = L^-1 b, b^T (S + nI)^-1 b = sum z_c^2 / d_c);
//   (2) the panel rows i below the block (one lane each) take the block's
//       updates in registers, are stored back, and update their right-hand
//       sides, r_i -= sum_c a_ic r_c / d_c;
//   (3) the trailing triangle takes the rank-LDS_BS update
//       a_ij -= sum_c a_ic a_jc / d_c (i >= j past the block) in 16 x 16 tiles,
//       a 2 x 2 block of entries per lane (tile rows tr, tr + 8 and columns tc,
//       tc + 8): a lane reads its multipliers a_jc / d_c once per column tile
//       and the loads of two row tiles are issued before their stores.
// A block has LDS_BS serial pivots but one pass over the trailing triangle.
// Every lane ends with the same sums.  Stores of masked-off lanes go to the
// lane's spare slot dum[lane] (WAVE doubles outside the system), so the stores
// need no branch.
// With nw > 1 waves of one block on the system (w = this wave), the panel rows
// and the tile groups are dealt round robin and block barriers separate the
// phases; every wave must call it, the assembled system visible to all of
// them.  Returns false if a pivot is not positive.
// LDS_BS is 8: against 4 it takes 8 to 12 % off at 72 to 96 rows (fewer blocks;
// the extra registers do not lower the occupancy, which LDS bounds).
constexpr int LDS_TB = 2;   // row tiles whose loads are issued together

template <int SPIN, int NR, int LDS_BS = 8>
__device__ inline bool lds_phase_b(double *mat, double *rhs, double *dum, int lane, int nrow, double nug,
                                   GroupOut &o, int w = 0, int nw = 1) {
  bool ok = true;
  double v0 = 0.0, v1 = 0.0, q0 = 0.0, q1 = 0.0;
  double *const spare = dum + lane;
  const int tr = lane >> 3, tc = lane & 7;   // tile rows tr, tr + 8; columns tc, tc + 8
#pragma unroll 1
  for (int K0 = 0; K0 < nrow; K0 += LDS_BS) {
    compiler_fence();   // block K0 reads what the previous block wrote from other lanes
    const int nb = min(LDS_BS, nrow - K0);   // columns of this block (the last may be short)
    // (1) pivot block and its right-hand sides (identity past the system)
    double Pm[LDS_BS][LDS_BS], Rb[LDS_BS][NR], idv[LDS_BS];
#pragma unroll
    for (int r = 0; r < LDS_BS; ++r) {
#pragma unroll
      for (int c = 0; c <= r; ++c)
        Pm[r][c] = (r < nb) ? mat[tri(K0 + r) + K0 + c] : (c == r ? 1.0 : 0.0);
#pragma unroll
      for (int q = 0; q < NR; ++q) Rb[r][q] = (r < nb) ? rhs[(K0 + r) * NR + q] : 0.0;
    }
#pragma unroll
    for (int c = 0; c < LDS_BS; ++c) {
      const bool live = c < nb;
      const double dc = Pm[c][c] + (live ? nug : 0.0);
      ok = ok && (!live || dc > 0.0);
      idv[c] = recip(dc);
      if (live) {
        if (SPIN == 0) {
          v0 = fma(Rb[c][0] * Rb[c][1], idv[c], v0);
          q0 = fma(Rb[c][0] * Rb[c][0], idv[c], q0);
        } else {
          v0 = fma(Rb[c][0] * Rb[c][NR - 1], idv[c], v0);
          v1 = fma(Rb[c][1] * Rb[c][NR - 1], idv[c], v1);
          q0 = fma(Rb[c][0] * Rb[c][0], idv[c], q0);
          q1 = fma(Rb[c][1] * Rb[c][1], idv[c], q1);
        }
      }
#pragma unroll
      for (int r = c + 1; r < LDS_BS; ++r) {
        const double f = Pm[r][c] * idv[c];
#pragma unroll
        for (int c2 = c + 1; c2 <= r; ++c2) Pm[r][c2] = fma(-f, Pm[c2][c], Pm[r][c2]);
#pragma unroll
        for (int q = 0; q < NR; ++q) Rb[r][q] = fma(-f, Rb[c][q], Rb[r][q]);
      }
    }
    const int m0 = K0 + LDS_BS;   // first row and column past the block
    if (m0 >= nrow) break;        // block-uniform: the last block has no panel
    // (2) panel rows i >= m0: the block's columns of row i, then its right-hand sides
#pragma unroll 1
    for (int i = m0 + lane + w * WAVE; i < nrow; i += nw * WAVE) {
      const int ti = tri(i) + K0;
      double x[LDS_BS];
#pragma unroll
      for (int c = 0; c < LDS_BS; ++c) x[c] = mat[ti + c];
#pragma unroll
      for (int c = 0; c < LDS_BS; ++c) {
        const double g = x[c] * idv[c];
#pragma unroll
        for (int c2 = c + 1; c2 < LDS_BS; ++c2) x[c2] = fma(-g, Pm[c2][c], x[c2]);
      }
#pragma unroll
      for (int c = 0; c < LDS_BS; ++c) mat[ti + c] = x[c];
#pragma unroll
      for (int q = 0; q < NR; ++q) {
        double acc = rhs[i * NR + q];
#pragma unroll
        for (int c = 0; c < LDS_BS; ++c) acc = fma(-x[c] * idv[c], Rb[c][q], acc);
        rhs[i * NR + q] = acc;
      }
    }
    if (nw > 1) __syncthreads(); else compiler_fence();   // the panel is visible to every wave
    // (3) trailing triangle (rows and columns >= m0).  Loads of clamped indices
    // stay inside the system: tri(i) + j < tri(n) for i, j < n.
    const int nt = (nrow - m0 + 15) >> 4;
    const int tlast = tri(nrow - 1);
    int item = 0;   // tile groups, dealt round robin over the waves
#pragma unroll 1
    for (int J = 0; J < nt; ++J) {
      int jmin[2];        // entry (i, j) is stored iff jmin <= i < nrow (nrow: column past the system)
      double *pj[2];      // column j (clamped into the system) of row 0: entry (i, j) at pj + tri(i)
      double fj[2][LDS_BS];
#pragma unroll
      for (int cc = 0; cc < 2; ++cc) {
        const int j = m0 + 16 * J + tc + 8 * cc;
        const int jc = j < nrow ? j : nrow - 1;
        jmin[cc] = j < nrow ? j : nrow;
        pj[cc] = mat + jc;
        const int tj = tri(jc) + K0;
#pragma unroll
        for (int c = 0; c < LDS_BS; ++c) fj[cc][c] = mat[tj + c] * idv[c];
      }
#pragma unroll 1
      for (int I0 = J; I0 < nt; I0 += LDS_TB) {
        if ((item++) % nw != w) continue;
        const int ib = m0 + 16 * I0 + tr;
        const int tb = tri(ib);
        double x[LDS_TB][2][2];
        double *pst[LDS_TB][2][2];   // where each entry is stored (its slot or the spare)
#pragma unroll
        for (int u = 0; u < LDS_TB; ++u)
#pragma unroll
          for (int rr = 0; rr < 2; ++rr) {
            const int d = 16 * u + 8 * rr;
            const int i = ib + d;
            const bool iv = i < nrow;
            const int ti = iv ? tb + d * ib + d * (d + 1) / 2 : tlast;
            double a[LDS_BS];
#pragma unroll
            for (int c = 0; c < LDS_BS; ++c) a[c] = mat[ti + K0 + c];
#pragma unroll
            for (int cc = 0; cc < 2; ++cc) {
              double *const pe = pj[cc] + ti;
              double v = *pe;
#pragma unroll
              for (int c = 0; c < LDS_BS; ++c) v = fma(-a[c], fj[cc][c], v);
              x[u][rr][cc] = v;
              pst[u][rr][cc] = (iv && jmin[cc] <= i) ? pe : spare;
            }
          }
        compiler_fence();
#pragma unroll
        for (int u = 0; u < LDS_TB; ++u)
#pragma unroll
          for (int rr = 0; rr < 2; ++rr)
#pragma unroll
            for (int cc = 0; cc < 2; ++cc) *pst[u][rr][cc] = x[u][rr][cc];
      }
    }
    if (nw > 1) __syncthreads();   // block K0 complete in every wave before the next reads it
  }
  compiler_fence();
  o.v0 = v0;
  o.v1 = v1;
  o.qd0 = q0;
  o.qd1 = q1;
  o.w0 = o.w1 = 0.0;
  return ok;
}

// Phase-B engines of the fix-up pass: solve the tagged point (searched and
// assembled into the wave's first system buffer) with nugget nug, using
// exactly the arithmetic of the matching main pass.  `first` is false when an
// earlier attempt may have overwritten the assembled system.
template <int NT, int SPIN>
struct RowGroupEngine {
  static constexpr int NR = (SPIN == 0) ? 2 : 3;
  __device__ static void build(const PlanDev &P, const double *tab, const double *map, double th, double ph,
                               int lane, const WaveBufs &B) {
    phase_a_build<SPIN, NR>(P, tab, map, th, ph, lane, B.sel, B.nb, B.mat, B.rhs);
  }
  __device__ static bool solve(const PlanDev &P, const double *, const double *, double, double, int lane,
                               const WaveBufs &B, bool found, bool, double nug, GroupOut &o) {
    RowSys<NT, NR> S;
    rowsys_identity(S, lane & 15);
    if (found && (lane >> 4) == 0) rowsys_load(S, B.mat, B.rhs, lane & 15, P.n, nug);
    return __all(rowsys_phase_b<NT, SPIN, NR>(S, lane & 15, P.n, o));
  }
};

template <int T, int SPIN>
struct TileEngine {
  static constexpr int NR = (SPIN == 0) ? 2 : 3;
  __device__ static void build(const PlanDev &P, const double *tab, const double *map, double th, double ph,
                               int lane, const WaveBufs &B) {
    phase_a_build<SPIN, NR>(P, tab, map, th, ph, lane, B.sel, B.nb, B.mat, B.rhs);
  }
  __device__ static bool solve(const PlanDev &P, const double *tab, const double *map, double th,
                               double ph, int lane, const WaveBufs &B, bool found, bool first,
                               double nug, GroupOut &o) {
    if (!found) return true;
    if (!first) phase_a_build<SPIN, NR>(P, tab, map, th, ph, lane, B.sel, B.nb, B.mat, B.rhs);
    return __all(tile_phase_b<T, SPIN, NR>(B.mat, B.rhs, B.mat, lane, P.n, nug, o));
  }
};

// The LDS engine is the exception: its one-wave fix-up eliminates in 4-column
// blocks (8 would spill there), so its sums are grouped differently from the
// main pass's 8-column blocks and agree with them to rounding, not bit for bit.
template <int SPIN>
struct LdsEngine {
  static constexpr int NR = (SPIN == 0) ? 2 : 3;
  // records without the data column, then the assembly that writes the
  // right-hand sides (which overlay the records) last
  __device__ static void build(const PlanDev &P, const double *tab, const double *map, double th, double ph,
                               int lane, const WaveBufs &B) {
    neighbour_records<SPIN, NR, false>(P, th, ph, lane, B.sel, B.nb, B.rhs, map);
    compiler_fence();
    lds_assemble<SPIN, NR>(P, tab, map, B.sel, B.nb, lane, B.mat, B.rhs, 0, 1);
  }
  __device__ static bool solve(const PlanDev &P, const double *tab, const double *map, double th,
                               double ph, int lane, const WaveBufs &B, bool found, bool first,
                               double nug, GroupOut &o) {
    if (!found) return true;
    if (!first) build(P, tab, map, th, ph, lane, B);
    return lds_phase_b<SPIN, NR, 4>(B.mat, B.rhs, B.rbuf, lane, P.n, nug, o);
  }
};


// ---------------------------------------------------------------- shared bodies
// Phase A (assembly) and phase B of the four points starting at p0 on the
// wave's row groups, their stencils already in sel[q K] (bit q of act_mask set
// where the search succeeded): each is assembled in the wave's single system
// buffer and loaded into its row group before the next point reuses the buffer,
// then phase B runs for all four at once.
template <int NT, int SPIN>
__device__ inline void group_rs_solve(const PlanDev &P, const double *tab, const double *__restrict__ map,
                                      const double *__restrict__ theta, const double *__restrict__ phi,
                                      int64_t n, double *__restrict__ out, double *__restrict__ var,
                                      const WaveBufs &B, const int *sel, int64_t p0, int lane,
                                      unsigned act_mask) {
  constexpr int PPW = 4;
  constexpr int NR = (SPIN == 0) ? 2 : 3;
  const int grp = lane >> 4;
  const int x = lane & 15;
  const int nrow = P.n, K = P.K;
  const double nug = (P.nug_policy == FLINTS_NUG_ALWAYS) ? P.eps : 0.0;
  RowSys<NT, NR> S;
  rowsys_identity(S, x);
#pragma unroll 1
  for (int q = 0; q < PPW; ++q) {
    if (!((act_mask >> q) & 1u)) continue;
    const int64_t pt = p0 + q;
    phase_a_build<SPIN, NR>(P, tab, map, theta[pt], phi[pt], lane, sel + q * K, B.nb, B.mat, B.rhs);
    if (grp == q) rowsys_load(S, B.mat, B.rhs, x, nrow, nug);
  }
  GroupOut o;
  const bool ok = rowsys_phase_b<NT, SPIN, NR>(S, x, nrow, o);
  if (x == 0) {
    const int64_t pt = p0 + grp;
    if (pt < n)
      store_point<SPIN>(P, pt, n, (act_mask >> grp) & 1u, ok, FAIL64_BITS, o, nug, false, out, var);
  }
}

// Four points (first at p0) on the wave's row groups: search all, then
// assemble and solve them together.
template <int NT, int SPIN>
__device__ inline void group_rs(const PlanDev &P, const double *tab, const double *__restrict__ map,
                                const double *__restrict__ theta, const double *__restrict__ phi,
                                int64_t n, double *__restrict__ out, double *__restrict__ var,
                                const WaveBufs &B, int64_t p0, int lane) {
  constexpr int PPW = 4;
  const int K = P.K;
  unsigned act_mask = 0;
#pragma unroll 1
  for (int q = 0; q < PPW; ++q) {
    const int64_t pt = p0 + q;
    if (pt >= n) break;
    if (phase_a_search(P, theta[pt], phi[pt], lane, B.cu, B.ci, B.rs, B.sel + q * K))
      act_mask |= 1u << q;
  }
  group_rs_solve<NT, SPIN>(P, tab, map, theta, phi, n, out, var, B, B.sel, p0, lane, act_mask);
}

// Assembly, blocked tile Cholesky and output of one point on the whole wave,
// its stencil already in sel (found is false if the search failed).
template <int T, int SPIN>
__device__ inline void tile_solve(const PlanDev &P, const double *tab, const double *__restrict__ map,
                                  double th, double ph, int64_t n, double *__restrict__ out,
                                  double *__restrict__ var, const WaveBufs &B, const int *sel,
                                  int64_t pt, bool found, int lane) {
  constexpr int NR = (SPIN == 0) ? 2 : 3;
  const double nug = (P.nug_policy == FLINTS_NUG_ALWAYS) ? P.eps : 0.0;
  GroupOut o;
  bool ok = true;
  if (found) {
    phase_a_build<SPIN, NR>(P, tab, map, th, ph, lane, sel, B.nb, B.mat, B.rhs);
    ok = tile_phase_b<T, SPIN, NR>(B.mat, B.rhs, B.mat, lane, P.n, nug, o);
  }
  if (lane == 0) store_point<SPIN>(P, pt, n, found, ok, FAIL64_BITS, o, nug, false, out, var);
}

// One point on the whole wave with the blocked tile Cholesky.
template <int T, int SPIN>
__device__ inline void point_tile(const PlanDev &P, const double *tab, const double *__restrict__ map,
                                  const double *__restrict__ theta, const double *__restrict__ phi,
                                  int64_t n, double *__restrict__ out, double *__restrict__ var,
                                  const WaveBufs &B, int64_t pt, int lane) {
  const double th = theta[pt], ph = phi[pt];
  const bool found = phase_a_search(P, th, ph, lane, B.cu, B.ci, B.rs, B.sel);
  tile_solve<T, SPIN>(P, tab, map, th, ph, n, out, var, B, B.sel, pt, found, lane);
}

// ---------------------------------------------------------------- shared stencils (T + Q/U)
// The K-nearest stencil of a target depends only on the target, N_side and K
// (paper Sec. 2.5 picks the neighbours before any covariance is formed).  For
// temperature and polarisation at the same targets, the spin-2 pass writes each
// target's stencil to device memory and the spin-0 pass reads it instead of
// searching again.  stn holds K pixel indices per target of the chunk that
// starts at target s0; all K entries are -1 where the search failed or the
// target is invalid.
__device__ inline void store_stencil(int *__restrict__ stn, int64_t i, int K, const int *sel, bool found,
                                     int lane) {
  for (int k = lane; k < K; k += WAVE) stn[i * K + k] = found ? sel[k] : -1;
}

// point_tile that also writes the stencil.
template <int T, int SPIN>
__device__ inline void point_tile_st(const PlanDev &P, const double *tab, const double *__restrict__ map,
                                     const double *__restrict__ theta, const double *__restrict__ phi,
                                     int64_t n, double *__restrict__ out, double *__restrict__ var,
                                     const WaveBufs &B, int64_t pt, int lane, int *__restrict__ stn,
                                     int64_t s0) {
  const double th = theta[pt], ph = phi[pt];
  const bool found = phase_a_search(P, th, ph, lane, B.cu, B.ci, B.rs, B.sel);
  store_stencil(stn, pt - s0, P.K, B.sel, found, lane);
  tile_solve<T, SPIN>(P, tab, map, th, ph, n, out, var, B, B.sel, pt, found, lane);
}

// group_rs that also writes the stencils.
template <int NT, int SPIN>
__device__ inline void group_rs_st(const PlanDev &P, const double *tab, const double *__restrict__ map,
                                   const double *__restrict__ theta, const double *__restrict__ phi,
                                   int64_t n, double *__restrict__ out, double *__restrict__ var,
                                   const WaveBufs &B, int64_t p0, int lane, int *__restrict__ stn,
                                   int64_t s0) {
  constexpr int PPW = 4;
  const int K = P.K;
  unsigned act_mask = 0;
#pragma unroll 1
  for (int q = 0; q < PPW; ++q) {
    const int64_t pt = p0 + q;
    if (pt >= n) break;
    const bool found = phase_a_search(P, theta[pt], phi[pt], lane, B.cu, B.ci, B.rs, B.sel + q * K);
    store_stencil(stn, pt - s0, K, B.sel + q * K, found, lane);
    if (found) act_mask |= 1u << q;
  }
  group_rs_solve<NT, SPIN>(P, tab, map, theta, phi, n, out, var, B, B.sel, p0, lane, act_mask);
}

// group_rs with the stencils read from stn instead of searched.  Validity is
// checked and counted as in the search, so the plan's counters are those of a
// searching pass.
template <int NT, int SPIN>
__device__ inline void group_rs_ld(const PlanDev &P, const double *tab, const double *__restrict__ map,
                                   const double *__restrict__ theta, const double *__restrict__ phi,
                                   int64_t n, double *__restrict__ out, double *__restrict__ var,
                                   const WaveBufs &B, int64_t p0, int lane, const int *__restrict__ stn,
                                   int64_t s0) {
  constexpr int PPW = 4;
  const int K = P.K;
  // the group's directions and stencils, each read in one round trip: the
  // stencils of p0 .. p0 + 3 are contiguous (no group of four crosses a chunk)
  const int64_t pend = min(n, p0 + PPW);
  const int64_t pl = p0 + (lane & (PPW - 1));
  const bool lv = lane < PPW && pl < pend;
  const double thl = lv ? theta[pl] : 0.0, phl = lv ? phi[pl] : 0.0;
  const int nst = (int)(pend - p0) * K;
  const int *src = stn + (p0 - s0) * K;
  for (int e = lane; e < nst; e += WAVE) B.sel[e] = src[e];
  unsigned act_mask = 0;
#pragma unroll 1
  for (int q = 0; q < PPW; ++q) {
    const int64_t pt = p0 + q;
    if (pt >= n) break;
    const double th = readlane_d(thl, q), ph = readlane_d(phl, q);
    const bool good = (th >= 0.0) && (th <= kconst(PI_D)) && isfinite(ph);
    if (!good) {
      if (lane == 0) atomicAdd(P.counters + CNT_BAD_INPUT, 1ull);
      continue;
    }
    if (B.sel[q * K] < 0) {
      if (lane == 0) atomicAdd(P.counters + CNT_SEARCH_FAIL, 1ull);
      continue;
    }
    act_mask |= 1u << q;
  }
  group_rs_solve<NT, SPIN>(P, tab, map, theta, phi, n, out, var, B, B.sel, p0, lane, act_mask);
}

// Fix-up of the 64 outputs starting at p0 (row-group and tile paths): each
// tagged point is searched and assembled again and solved by the engine; an
// FP32-rejected point is recomputed with the FP64 engine, an FP64 factorisation
// failure gets the nugget of paper Sec. 2.4, n = mu + eps with mu the smallest
// shift for which S + mu I factorises (bisection on [n0, rows + 1]; the upper
// end is positive definite by Gershgorin since |S_ij| <= 1).
template <class Eng, int SPIN>
__device__ inline void fixup_chunk(const PlanDev &P, const double *tab, const double *__restrict__ map,
                                   const double *__restrict__ theta, const double *__restrict__ phi,
                                   int64_t n, double *__restrict__ out, double *__restrict__ var,
                                   const WaveBufs &B, int64_t p0, int lane) {
  constexpr int NR = (SPIN == 0) ? 2 : 3;
  const int nrow = P.n;
  const double nug0 = (P.nug_policy == FLINTS_NUG_ALWAYS) ? P.eps : 0.0;
  const int64_t pl = p0 + lane;
  const unsigned long long bits = pl < n ? (unsigned long long)__double_as_longlong(out[pl]) : 0ull;
  const bool t64 = bits == FAIL64_BITS, t32 = bits == FAIL32_BITS;
  unsigned long long mask = __ballot(t64 || t32);
  const unsigned long long m32 = __ballot(t32);
  while (mask) {
    const int bit = __ffsll((long long)mask) - 1;
    mask &= mask - 1ull;
    const bool from32 = (m32 >> bit) & 1ull;
    const int64_t pt = p0 + bit;
    const double th = theta[pt], ph = phi[pt];
    const bool found = phase_a_search(P, th, ph, lane, B.cu, B.ci, B.rs, B.sel);
    if (found) Eng::build(P, tab, map, th, ph, lane, B);
    GroupOut o;
    double nug = nug0;
    bool ok = false, first = true;
    if (from32) {
      ok = Eng::solve(P, tab, map, th, ph, lane, B, found, first, nug, o);
      first = false;
      if (lane == 0) atomicAdd(P.counters + CNT_FP64_FALLBACK, 1ull);
    }
    if (!ok) {
      double lo = nug0, hi = (double)nrow + 1.0;
#pragma unroll 1
      for (int it = 0; it < 64; ++it) {
        const double mu = 0.5 * (lo + hi);
        GroupOut tmp;
        const bool ok2 = Eng::solve(P, tab, map, th, ph, lane, B, found, first, mu, tmp);
        first = false;
        if (ok2) hi = mu; else lo = mu;
      }
      nug = hi + P.eps;
#pragma unroll 1
      for (int it = 0; it < 8 && !ok; ++it) {
        ok = Eng::solve(P, tab, map, th, ph, lane, B, found, false, nug, o);
        if (!ok) nug *= 2.0;
      }
      if (lane == 0) atomicAdd(P.counters + CNT_NUGGET_ESC, 1ull);
    }
    if (lane == 0) store_point<SPIN>(P, pt, n, found, ok, FAIL64_BITS, o, nug, false, out, var);
  }
}

}  // namespace flints
