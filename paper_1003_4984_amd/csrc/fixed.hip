// Stencil tied to the containing pixel, with tabulated factors (paper Sec. 2.3
// and Sec. 2.4: the neighbours of a direction are those of the pixel it falls
// in, so the neighbour covariance S depends only on that pixel, and S^-1 is
// computed once per pixel geometry, using the symmetries of the pixelisation
// to store one per ring position rather than one per pixel).
//
// Reading: the stencil of a pixel is the K pixel centres nearest to its centre
// (the paper takes the pixel and its neighbours, 9, or NESTED extensions of
// them, 36); the containing pixel is the RING pixel ang2pix returns.  The
// covariance of a stencil depends only on the relative geometry of its points,
// which a rotation about the polar axis preserves, and spin-2 bearings are
// measured against each point's own (e_theta, e_phi), which such a rotation
// also preserves.  Two rotations map the pixelisation onto itself:
//   * a quarter turn (every ring has 4i or 4 N_side pixels);
//   * a turn by one belt pixel (2 pi / 4 N_side), for the belt rings.
// So a pixel class is (ring, position within a quarter), and in belt rings
// whose stencils cannot reach a polar-cap ring the whole ring is one class.
// Each class stores its representative's stencil (pixels as ring and index)
// and the Cholesky factor of its S + n I; a target's stencil is the
// representative's rotated onto the target's pixel, and the per-target work is
// the K covariances to the target, the gathered values and two triangular
// solves with the stored factor: O(K^2) instead of O(K^3).
//
// Plan time: one wave per class (search as in the K-nearest path around the
// representative's centre, covariance assembly, register-row Cholesky with
// the nugget of Sec. 2.4).  Per target: one lane per target.
#include "device.h"
#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

namespace flints {

// ------------------------------------------------------------------ geometry
// RING pixel containing the direction (z = cos theta, st = sin theta, phr in
// [0, 2 pi)), with its ring (1-based) and index in the ring.  The HEALPix
// construction (Gorski et al. 2005): with t = 2 phi / pi in [0, 4), the pixel
// boundaries of the equatorial zone (|z| <= 2/3) are the lines
// N (1/2 + t) -/+ (3/4) N z = integer, and those of a polar cap the lines
// t' r = integer and (1 - t') r = integer with t' = frac(t) and
// r = N sqrt(3 (1 - |z|)) (1 - |z| formed as st^2 / (1 + |z|), exact near the
// poles).
__device__ inline int64_t ang2pix_ring(int64_t N, double z, double st, double phr, int &ring, int &j) {
  const double tt = phr * kconst(2.0 / PI_D);
  const double za = fabs(z);
  if (za <= kconst(2.0 / 3.0)) {
    const double t1 = (double)N * (0.5 + tt), t2 = (double)N * z * 0.75;
    const int64_t jp = (int64_t)(t1 - t2), jm = (int64_t)(t1 + t2);
    int64_t ir = N + 1 + jp - jm;                 // 1 .. 2N + 1, counted from z = 2/3
    ir = ir < 1 ? 1 : (ir > 2 * N + 1 ? 2 * N + 1 : ir);
    const int64_t kshift = 1 - (ir & 1);
    int64_t ip = (jp + jm - N + kshift + 1) / 2;
    ip %= 4 * N;
    if (ip < 0) ip += 4 * N;
    ring = (int)(N - 1 + ir);
    j = (int)ip;
    return 2 * N * (N - 1) + (ir - 1) * 4 * N + ip;
  }
  const double tp = tt - floor(tt);
  const double omz = st * st / (1.0 + za);
  const double tmp = (double)N * sqrt(3.0 * omz);
  const int64_t jp = (int64_t)(tp * tmp), jm = (int64_t)((1.0 - tp) * tmp);
  int64_t ir = jp + jm + 1;                       // ring counted from the nearer pole
  ir = ir < 1 ? 1 : (ir > N ? N : ir);
  int64_t ip = (int64_t)(tt * (double)ir);
  ip %= 4 * ir;
  if (ip < 0) ip += 4 * ir;
  j = (int)ip;
  if (z > 0.0) {
    ring = (int)ir;
    return 2 * ir * (ir - 1) + ip;
  }
  ring = (int)(4 * N - ir);
  return 12 * N * N - 2 * ir * (ir + 1) + ip;
}

// Class of the pixel (ring, j) and the rotation that carries the class's
// representative onto it: quarter turns q (quadrant classes), or j belt-pixel
// steps (whole-ring classes).
struct ClassRef {
  int64_t c;
  int32_t quad;   // 0: whole-ring class, rotate by `steps` belt pixels
  int32_t steps;  // quadrant classes: quarter turns
};

__device__ inline ClassRef pixel_class(const PlanDev &P, int ring, int j) {
  ClassRef r;
  const int32_t qs = P.cls_quad[ring];
  r.quad = qs;
  if (qs == 0) {
    r.c = P.cls_base[ring];
    r.steps = j;
  } else {
    r.c = P.cls_base[ring] + j % qs;
    r.steps = j / qs;
  }
  return r;
}

// Stencil entry k of a class (ring << 16 | j of the representative's
// neighbour) rotated onto the target's pixel: ring and pixel index.
__device__ inline int64_t rotated_pixel(int64_t N, int32_t v, const ClassRef &cr, int &ring) {
  ring = v >> 16;
  const int jr = v & 0xffff;
  const Ring R = ring_geom(N, ring);
  int64_t jj;
  if (cr.quad == 0) jj = ((int64_t)jr + cr.steps) % R.n;
  else jj = ((int64_t)jr + (int64_t)cr.steps * (R.n / 4)) % R.n;
  return R.first + jj;
}

// ------------------------------------------------------------------ plan time
// One wave per class: the representative's centre, its K nearest pixels, the
// covariance S (as assembled for any target), S + n I = L L^T by register rows
// (lane i holds row i), escalating the nugget by bisection when the
// factorisation fails (paper Sec. 2.4, as in the fix-up passes), and the
// packed rows of L with 1 / L_ii on the diagonal.
template <int NMAX, int SPIN>
__global__ __launch_bounds__(MAX_WPB * WAVE) void k_fixed_build(PlanDev P, int64_t nclass,
                                                     int32_t *__restrict__ stn_out,
                                                     double *__restrict__ L_out,
                                                     unsigned long long *__restrict__ esc, Layout Lay) {
  constexpr int NR = (SPIN == 0) ? 2 : 3;
  extern __shared__ double lds_dyn[];
  char *lds = (char *)lds_dyn;
  const double *tab = load_table(lds, P);
  const int wpb = blockDim.x / WAVE;
  const int wave = threadIdx.x / WAVE;
  const int lane = threadIdx.x % WAVE;
  const WaveBufs B = wave_bufs(lds, Lay, wave);
  const int64_t N = P.nside;
  const int K = P.K, nrow = P.n;
  const int nring = (int)(4 * N - 1);
  const double nug0 = (P.nug_policy == FLINTS_NUG_ALWAYS) ? P.eps : 0.0;
  for (int64_t c = xcd_block() * wpb + wave; c < nclass; c += (int64_t)gridDim.x * wpb) {
    // ring of the class: the last ring whose first class is <= c
    int lo = 1, hi = nring;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (P.cls_base[mid] <= c) lo = mid; else hi = mid - 1;
    }
    const Ring R = ring_geom(N, lo);
    const int jrep = (int)(c - P.cls_base[lo]);
    const double th = atan2(R.s, R.z);
    const double ph = R.phi0 + (double)jrep * R.dphi;
    const bool found = knn_search(P, th, ph, lane, B.cu, B.ci, B.rs, B.sel);
    if (!found) {
      // no stencil within the search cap: a tagged class (the interpolation
      // reports its targets as search failures)
      for (int k = lane; k < K; k += WAVE) stn_out[c * K + k] = -1;
      wave_lds_sync();
      continue;
    }
    for (int k = lane; k < K; k += WAVE) {
      const int64_t p = B.sel[k];
      const int rg = pix_ring(N, p);
      stn_out[c * K + k] = (rg << 16) | (int)(p - ring_geom(N, rg).first);
    }
    phase_a_build<SPIN, NR>(P, tab, nullptr, th, ph, lane, B.sel, B.nb, B.mat, B.rhs);
    const bool ract = lane < nrow;
    double a[NMAX], r[NR], diag;
    double nug = nug0;
    load_rows<NMAX, NR>(B.mat, B.rhs, lane, ract, nrow, a, r);
    bool ok = __all(chol_rows<NMAX, WAVE, NR>(a, r, lane, 0, nug, diag));
    if (!ok) {
      double blo = nug0, bhi = (double)nrow + 1.0;
#pragma unroll 1
      for (int it = 0; it < 64; ++it) {
        const double mu = 0.5 * (blo + bhi);
        load_rows<NMAX, NR>(B.mat, B.rhs, lane, ract, nrow, a, r);
        if (__all(chol_rows<NMAX, WAVE, NR>(a, r, lane, 0, mu, diag))) bhi = mu; else blo = mu;
      }
      nug = bhi + P.eps;
#pragma unroll 1
      for (int it = 0; it < 8 && !ok; ++it) {
        load_rows<NMAX, NR>(B.mat, B.rhs, lane, ract, nrow, a, r);
        ok = __all(chol_rows<NMAX, WAVE, NR>(a, r, lane, 0, nug, diag));
        if (!ok) nug *= 2.0;
      }
      if (lane == 0) atomicAdd(esc, 1ull);
    }
    if (ract) {
      double *Lr = L_out + c * (int64_t)P.lsz + tri(lane);
#pragma unroll
      for (int jc = 0; jc < NMAX; ++jc)
        if (jc < lane) Lr[jc] = a[jc];
      Lr[lane] = 1.0 / a[lane];
    }
    wave_lds_sync();
  }
}

struct RingTables {
  std::vector<int64_t> base;  // [4N]
  std::vector<int32_t> quad;  // [4N]
  int64_t nclass = 0;
};

// Classes per ring: polar-cap rings (4i pixels) and belt rings whose stencils
// may reach a cap ring take one class per position within a quarter; other
// belt rings are one class.  A belt ring's stencils lie within the search cap
// rcap of its pixels, so it is one class when every cap ring is farther than
// rcap in colatitude.
static RingTables ring_tables(const PlanDev &d) {
  const int64_t N = d.nside;
  RingTables t;
  t.base.assign(4 * N, 0);
  t.quad.assign(4 * N, 0);
  const double th_ncap = N > 1 ? std::atan2(ring_geom(N, (int)N - 1).s, ring_geom(N, (int)N - 1).z) : -1e300;
  const double th_scap = N > 1 ? std::atan2(ring_geom(N, (int)(3 * N + 1)).s, ring_geom(N, (int)(3 * N + 1)).z)
                               : 1e300;
  int64_t next = 0;
  for (int r = 1; r <= (int)(4 * N - 1); ++r) {
    const Ring R = ring_geom(N, r);
    int32_t q;
    if (r < N || r > 3 * N) {
      q = R.n / 4;
    } else {
      const double th = std::atan2(R.s, R.z);
      const double gap = std::min(th - th_ncap, th_scap - th);
      q = gap > d.rcap * 1.000001 ? 0 : (int32_t)N;
    }
    t.base[r] = next;
    t.quad[r] = q;
    next += q == 0 ? 1 : q;
  }
  t.nclass = next;
  return t;
}

template <int NMAX, int SPIN>
static int run_build(Plan *p, int64_t nclass, unsigned long long *d_esc) {
  constexpr int NR = (SPIN == 0) ? 2 : 3;
  const Layout L = make_layout(p->d.ntab, p->d.nfun, p->d.K, p->d.n, 1, 1, NR);
  int dev = 0, ncu = 0, lds_max = 0;
  hipGetDevice(&dev);
  hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
  auto kern = k_fixed_build<NMAX, SPIN>;
  int wpb = 0, occ = 0, best = 0;
  for (int w = 1; w <= MAX_WPB; ++w) {
    const int l = L.tab_bytes + w * L.wave_bytes;
    if (l > lds_max) break;
    hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, l);
    int o = 0;
    hipOccupancyMaxActiveBlocksPerMultiprocessor(&o, kern, w * WAVE, l);
    if (o * w >= best) { best = o * w; wpb = w; occ = o; }
  }
  if (wpb == 0) {
    set_error("the fixed-stencil build needs more LDS than the device offers");
    return FLINTS_ELIMIT;
  }
  const int lds = L.tab_bytes + wpb * L.wave_bytes;
  hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
  const int64_t blocks = std::max<int64_t>(1, std::min<int64_t>((nclass + wpb - 1) / wpb,
                                                                 (int64_t)ncu * std::max(occ, 1)));
  hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(wpb * WAVE), lds, nullptr, p->d, nclass,
                     p->d_cls_stn, p->d_cls_L, d_esc, L);
  return hipGetLastError() == hipSuccess ? FLINTS_OK : FLINTS_EDEVICE;
}

void free_fixed(Plan *p) {
  if (p->d_cls_base) (void)hipFree(p->d_cls_base);
  if (p->d_cls_quad) (void)hipFree(p->d_cls_quad);
  if (p->d_cls_stn) (void)hipFree(p->d_cls_stn);
  if (p->d_cls_L) (void)hipFree(p->d_cls_L);
  p->d_cls_base = nullptr;
  p->d_cls_quad = nullptr;
  p->d_cls_stn = nullptr;
  p->d_cls_L = nullptr;
}

int build_fixed(Plan *p) {
  PlanDev &d = p->d;
  const RingTables t = ring_tables(d);
  p->nclass = t.nclass;
  d.lsz = d.n * (d.n + 1) / 2;
  const size_t stn_bytes = (size_t)t.nclass * d.K * sizeof(int32_t);
  const size_t L_bytes = (size_t)t.nclass * d.lsz * sizeof(double);
  unsigned long long *d_esc = nullptr;
  if (hipMalloc(&p->d_cls_base, t.base.size() * sizeof(int64_t)) != hipSuccess ||
      hipMalloc(&p->d_cls_quad, t.quad.size() * sizeof(int32_t)) != hipSuccess ||
      hipMalloc(&p->d_cls_stn, stn_bytes) != hipSuccess || hipMalloc(&p->d_cls_L, L_bytes) != hipSuccess ||
      hipMalloc(&d_esc, sizeof(unsigned long long)) != hipSuccess) {
    (void)hipGetLastError();
    if (d_esc) (void)hipFree(d_esc);
    free_fixed(p);
    set_error("device allocation of the fixed-stencil tables failed (" +
              std::to_string((stn_bytes + L_bytes) >> 20) + " MiB for " + std::to_string(t.nclass) +
              " pixel classes)");
    return FLINTS_ENOMEM;
  }
  unsigned long long esc = 0;
  bool ok = hipMemcpy(p->d_cls_base, t.base.data(), t.base.size() * sizeof(int64_t), hipMemcpyHostToDevice) ==
                hipSuccess &&
            hipMemcpy(p->d_cls_quad, t.quad.data(), t.quad.size() * sizeof(int32_t), hipMemcpyHostToDevice) ==
                hipSuccess &&
            hipMemset(d_esc, 0, sizeof(esc)) == hipSuccess;
  d.cls_base = p->d_cls_base;
  d.cls_quad = p->d_cls_quad;
  d.cls_stn = p->d_cls_stn;
  d.cls_L = p->d_cls_L;
  int rc = ok ? FLINTS_OK : FLINTS_EDEVICE;
  if (rc == FLINTS_OK) {
    if (d.spin == 0) {
      rc = d.n <= 16 ? run_build<16, 0>(p, t.nclass, d_esc)
           : d.n <= 32 ? run_build<32, 0>(p, t.nclass, d_esc)
                       : run_build<48, 0>(p, t.nclass, d_esc);
    } else {
      rc = d.n <= 16 ? run_build<16, 2>(p, t.nclass, d_esc) : run_build<32, 2>(p, t.nclass, d_esc);
    }
  }
  if (rc == FLINTS_OK &&
      (hipDeviceSynchronize() != hipSuccess ||
       hipMemcpy(&esc, d_esc, sizeof(esc), hipMemcpyDeviceToHost) != hipSuccess))
    rc = FLINTS_EDEVICE;
  (void)hipFree(d_esc);
  if (rc != FLINTS_OK) {
    if (rc == FLINTS_EDEVICE) set_error("building the fixed-stencil tables failed on the device");
    free_fixed(p);
    return rc;
  }
  p->class_nuggets = (int64_t)esc;
  return FLINTS_OK;
}

// ------------------------------------------------------------------ per target
// Covariance between neighbour k (chord offset x, y, z from the target in the
// target's frame, its own e_theta (a3, a4, a5) and e_phi (a6, a7) in that frame)
// and the target (e_theta = (zt, 0, -st), e_phi = (0, 1, 0)): spin 0 the
// normalised correlation, spin 2 the 2 x 2 block Cov((Q_k, U_k), (Q_0, U_0))
// from <P P*> = xi+ e^{2i(psi_k0 - psi_0k)} and <P P> = xi- e^{2i(psi_k0 + psi_0k)}
// with the bearings taken from the chord projected on each point's frame.
template <int SPIN>
__device__ __forceinline__ bool cov_to_target(const double *tab, int ntab, double inv_h, bool paper, double x,
                                              double y, double z, double a3, double a4, double a5, double a6,
                                              double a7, double zt, double st, double (&c)[4]) {
  const double s = 0.5 * sqrt(x * x + y * y + z * z);
  if (SPIN == 0) {
    double f;
    const bool in = table_lookup(tab, ntab, 1, inv_h, s, &f);
    c[0] = f;
    return in;
  }
  double f[2];
  const bool in = table_lookup(tab, ntab, 2, inv_h, s, f);
  const double xa = x * a3 + y * a4 + z * a5, ya = x * a6 + y * a7;
  const double xb = x * zt - z * st, yb = y;
  const double na = xa * xa + ya * ya, nb = xb * xb + yb * yb;
  const double prod = na * nb;
  const bool sep = prod > 0.0;
  const double inv = recip(sep ? prod : 1.0);
  const double ia = nb * inv, ib = na * inv;
  const double ca = sep ? (xa * xa - ya * ya) * ia : 1.0, sa = sep ? 2.0 * xa * ya * ia : 0.0;
  const double cb = sep ? (xb * xb - yb * yb) * ib : 1.0, sb = sep ? 2.0 * xb * yb * ib : 0.0;
  const double gr = f[0] * (ca * cb + sa * sb), gi = f[0] * (sa * cb - ca * sb);
  const double pr = paper ? 0.0 : f[1] * (ca * cb - sa * sb);
  const double pim = paper ? 0.0 : f[1] * (sa * cb + ca * sb);
  c[0] = gr + pr;   // Cov(Q_k, Q_0)
  c[1] = pim - gi;  // Cov(Q_k, U_0)
  c[2] = pim + gi;  // Cov(U_k, Q_0)
  c[3] = gr - pr;   // Cov(U_k, U_0)
  return in;
}

// One lane per target: pixel, class, rotated stencil, the target covariances
// b and data d in registers (rows up to NM, interleaved Q / U for spin 2),
// forward substitution y = L^-1 b, z = L^-1 d with the class's factor, then
// value = y . z and var = sigma^2 (1 - y . y) (Eq. best_temperature_field /
// gaussvar; Eq. major_eq / gaussvar_pol).
constexpr int FIXED_TPB = 256;

template <int NM, int SPIN>
__global__ __launch_bounds__(FIXED_TPB) void k_fixed(PlanDev P, const double *__restrict__ map,
                                                     const double *__restrict__ theta,
                                                     const double *__restrict__ phi, int64_t n,
                                                     double *__restrict__ out, double *__restrict__ var) {
  constexpr int NB = (SPIN == 0) ? 1 : 2;   // right-hand sides of covariances
  extern __shared__ double lds_dyn[];
  const double *tab = load_table((char *)lds_dyn, P);
  const int64_t N = P.nside;
  const int K = P.K, nrow = P.n;
  const bool paper = (P.mode == FLINTS_S2_PAPER);
  const double s2 = P.sigma2;
  const double nan = __builtin_nan("");
  const int lane = threadIdx.x % WAVE;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t start = xcd_block() * blockDim.x + threadIdx.x;
  const int64_t nround = (n + stride - 1) / stride;    // every lane runs the same trip count
  for (int64_t it = 0; it < nround; ++it) {
    const int64_t pt = start + it * stride;
    const bool live = pt < n;
    const double th = live ? theta[pt] : 0.0, ph = live ? phi[pt] : 0.0;
    const bool good = live && (th >= 0.0) && (th <= kconst(PI_D)) && isfinite(ph);
    count_event(P.counters + CNT_BAD_INPUT, live && !good, lane);
    double zt, st;
    sincos_bounded(good ? th : 0.5, st, zt);
    const double twopi = kconst(TWO_PI_D);
    const double phr = good ? ph - twopi * floor(ph / twopi) : 0.0;
    int ring = 1, jr = 0;
    ang2pix_ring(N, zt, st, phr, ring, jr);
    const ClassRef cr = pixel_class(P, ring, jr);
    const int32_t *cs = P.cls_stn + cr.c * K;
    const bool stn_ok = good && cs[0] >= 0;
    count_event(P.counters + CNT_SEARCH_FAIL, good && !stn_ok, lane);
    double b[NB][NM], dv[NM];
    bool range_bad = false;
#pragma unroll
    for (int i = 0; i < NM; ++i) {
      dv[i] = 0.0;
#pragma unroll
      for (int q = 0; q < NB; ++q) b[q][i] = 0.0;
    }
#pragma unroll
    for (int k = 0; k < NM / (SPIN == 0 ? 1 : 2); ++k) {
      if (k < K && stn_ok) {
        int rg = 0;
        const int64_t p = rotated_pixel(N, cs[k], cr, rg);
        const Ring R = ring_geom(N, rg);
        const double dphi = R.phi0 + (double)(p - R.first) * R.dphi - phr;
        double sh, ch;
        sincos_bounded(0.5 * dphi, sh, ch);
        const double sd = 2.0 * sh * ch, cd = 1.0 - 2.0 * sh * sh;
        const double sdiff = (zt - R.z) * (zt + R.z) / (R.s + st);
        const double x = sdiff - 2.0 * R.s * sh * sh, y = R.s * sd, z = R.z - zt;
        double c[4];
        range_bad |= !cov_to_target<SPIN>(tab, P.ntab, P.inv_h, paper, x, y, z, R.z * cd, R.z * sd, -R.s, -sd,
                                          cd, zt, st, c);
        if (SPIN == 0) {
          b[0][k] = c[0];
          dv[k] = map_value(P, map, p);
        } else {
          b[0][2 * k] = c[0];
          b[0][2 * k + 1] = c[2];
          b[NB - 1][2 * k] = c[1];
          b[NB - 1][2 * k + 1] = c[3];
          dv[2 * k] = map_value(P, map, p);
          dv[2 * k + 1] = map_value(P, map, P.npix + p);
        }
      }
    }
    count_event(P.counters + CNT_TABLE_RANGE, range_bad, lane);
    // forward substitution with the packed rows of L (1 / L_ii on the diagonal)
    const double *Lc = P.cls_L + (stn_ok ? cr.c : 0) * (int64_t)P.lsz;
    double vq[NB], qq[NB];
#pragma unroll
    for (int q = 0; q < NB; ++q) vq[q] = qq[q] = 0.0;
#pragma unroll
    for (int i = 0; i < NM; ++i) {
      if (i < nrow) {
        const double *Li = Lc + tri(i);
#pragma unroll
        for (int jc = 0; jc < i; ++jc) {
          const double l = Li[jc];
          dv[i] = fma(-l, dv[jc], dv[i]);
#pragma unroll
          for (int q = 0; q < NB; ++q) b[q][i] = fma(-l, b[q][jc], b[q][i]);
        }
        const double inv = Li[i];
        dv[i] *= inv;
#pragma unroll
        for (int q = 0; q < NB; ++q) {
          b[q][i] *= inv;
          vq[q] = fma(b[q][i], dv[i], vq[q]);
          qq[q] = fma(b[q][i], b[q][i], qq[q]);
        }
      }
    }
    if (live) {
      const bool ok = stn_ok;
      bool clamp = false;
#pragma unroll
      for (int q = 0; q < NB; ++q) {
        double vv = s2 * (1.0 - qq[q]);
        clamp |= ok && vv < 0.0;
        vv = fmax(vv, 0.0);
        out[q * n + pt] = ok ? vq[q] : nan;
        if (var) var[q * n + pt] = ok ? vv : nan;
      }
      count_event(P.counters + CNT_CLAMPED_VAR, clamp, lane);
    } else {
      count_event(P.counters + CNT_CLAMPED_VAR, false, lane);
    }
  }
}

// Stencil of each target: the class stencil rotated onto its pixel.
__global__ __launch_bounds__(FIXED_TPB) void k_fixed_stencil(PlanDev P, const double *__restrict__ theta,
                                                             const double *__restrict__ phi, int64_t n,
                                                             int64_t *__restrict__ idx) {
  const int64_t N = P.nside;
  const int K = P.K;
  for (int64_t pt = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; pt < n; pt += (int64_t)gridDim.x * blockDim.x) {
    const double th = theta[pt], ph = phi[pt];
    const bool good = (th >= 0.0) && (th <= kconst(PI_D)) && isfinite(ph);
    double zt, st;
    sincos_bounded(good ? th : 0.5, st, zt);
    const double twopi = kconst(TWO_PI_D);
    const double phr = good ? ph - twopi * floor(ph / twopi) : 0.0;
    int ring = 1, jr = 0;
    ang2pix_ring(N, zt, st, phr, ring, jr);
    const ClassRef cr = pixel_class(P, ring, jr);
    const int32_t *cs = P.cls_stn + cr.c * K;
    const bool ok = good && cs[0] >= 0;
    for (int k = 0; k < K; ++k) {
      int rg = 0;
      idx[pt * K + k] = ok ? rotated_pixel(N, cs[k], cr, rg) : -1;
    }
  }
}

template <int NM, int SPIN>
static int launch_fixed_t(const Plan *p, const double *map, const double *theta, const double *phi, int64_t n,
                          double *out, double *var, hipStream_t s) {
  int dev = 0, ncu = 0;
  hipGetDevice(&dev);
  hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  auto kern = k_fixed<NM, SPIN>;
  const int lds = ((p->d.ntab * p->d.nfun * 8) + 15) & ~15;
  hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
  int occ = 0;
  hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kern, FIXED_TPB, lds);
  const int64_t blocks = std::max<int64_t>(1, std::min<int64_t>((n + FIXED_TPB - 1) / FIXED_TPB,
                                                                 (int64_t)ncu * std::max(occ, 1)));
  hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(FIXED_TPB), lds, s, p->d, map, theta, phi, n, out, var);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    set_error(std::string("fixed-stencil kernel launch failed: ") + hipGetErrorString(e));
    return FLINTS_EDEVICE;
  }
  return FLINTS_OK;
}

int launch_fixed(const Plan *p, const double *map, const double *theta, const double *phi, int64_t n,
                 double *out, double *var, hipStream_t s) {
  if (n == 0) return FLINTS_OK;
  const int nr = p->d.n;
  if (p->d.spin == 0) {
    if (nr <= 16) return launch_fixed_t<16, 0>(p, map, theta, phi, n, out, var, s);
    if (nr <= 32) return launch_fixed_t<32, 0>(p, map, theta, phi, n, out, var, s);
    return launch_fixed_t<48, 0>(p, map, theta, phi, n, out, var, s);
  }
  if (nr <= 16) return launch_fixed_t<16, 2>(p, map, theta, phi, n, out, var, s);
  return launch_fixed_t<32, 2>(p, map, theta, phi, n, out, var, s);
}

int launch_fixed_stencil(const Plan *p, const double *theta, const double *phi, int64_t n, int64_t *idx,
                         hipStream_t s) {
  if (n == 0) return FLINTS_OK;
  const int64_t blocks = std::min<int64_t>((n + FIXED_TPB - 1) / FIXED_TPB, 65536);
  hipLaunchKernelGGL(k_fixed_stencil, dim3((unsigned)blocks), dim3(FIXED_TPB), 0, s, p->d, theta, phi, n, idx);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    set_error(std::string("fixed-stencil kernel launch failed: ") + hipGetErrorString(e));
    return FLINTS_EDEVICE;
  }
  return FLINTS_OK;
}

}  // namespace flints
