// Correlation-function tables (plan time, FP64, on the device).
//
// The paper tabulates the correlation function in beta and interpolates it with
// cubics (App. B).  Here the table variable is s = sin(beta/2) = |n_a - n_b| / 2,
// the half chord, which the interpolation kernel gets from a difference vector
// with one square root and no inverse trigonometry.  Each node is the exact
// band-limited sum evaluated by an l-recurrence written for the deficits
// 1 - P_l and 1 - d^l_{22} in u = 1 - cos(beta) = 2 s^2 (full relative precision
// near beta = 0):
//   spin 0  f(s)  = zeta(beta) / zeta(0),  zeta = sum_{l>=1} (2l+1)/(4pi) C_l P_l
//   spin 2  f+(s) = xi_+(beta) / xi_+(0),  xi_+ = sum (2l+1)/(4pi) (EE+BB) d^l_{22}
//           f-(s) = xi_-(beta) / xi_+(0),  xi_- = sum (2l+1)/(4pi) (EE-BB) d^l_{2,-2}
// Node k sits at s = (k - 1) h (node 0 at s = -h; the functions are even in s).
// The node count is refined until the cubic interpolant matches the exact sum at
// every interval midpoint within the requested tolerance, or stops improving
// (the FP64 recurrence itself carries ~1e-13..1e-12 relative rounding at l ~ 4096).
#include "plan.h"
#include "table_interp.h"
#include <vector>
#include <cmath>
#include <algorithm>

namespace flints {

// Exact normalised correlation value(s) at half chord s.
__device__ inline void exact_corr(const double *__restrict__ wp, const double *__restrict__ wm,
                                  int lmax, int spin, double inv_norm, double s, double *f) {
  const double u = 2.0 * s * s;
  if (spin == 0) {
    // (l+1) q_{l+1} = (2l+1)(u + (1-u) q_l) - l q_{l-1},  q_l = 1 - P_l(1 - u)
    double qm = 0.0, q = u, g = wp[1] * u;
    for (int l = 1; l < lmax; ++l) {
      double qn = ((2.0 * l + 1.0) * (u + (1.0 - u) * q) - (double)l * qm) / (double)(l + 1);
      qm = q;
      q = qn;
      g += wp[l + 1] * q;
    }
    f[0] = 1.0 - g * inv_norm;
    return;
  }
  // e_l = 1 - d^l_{22}:  l(l-1)(l+3) e_{l+1} = (2l+1)[(l(l+1)(1-u) - 4) e_l + l(l+1) u]
  //                                            - (l+1)(l-2)(l+2) e_{l-1}
  // g_l = d^l_{2,-2}:    l(l-1)(l+3) g_{l+1} = (2l+1)(l(l+1)(1-u) + 4) g_l - (l+1)(l-2)(l+2) g_{l-1}
  double em = 1.0, e = u - 0.25 * u * u;
  double gm = 0.0, gg = 0.25 * u * u;
  double gp = wp[2] * e, xm = wm[2] * gg;
  for (int l = 2; l < lmax; ++l) {
    const double A = (double)l * (double)(l - 1) * (double)(l + 3);
    const double B = 2.0 * l + 1.0;
    const double L2 = (double)l * (double)(l + 1);
    const double C = (double)(l + 1) * (double)(l - 2) * (double)(l + 2);
    double en = (B * ((L2 * (1.0 - u) - 4.0) * e + L2 * u) - C * em) / A;
    double gn = (B * (L2 * (1.0 - u) + 4.0) * gg - C * gm) / A;
    em = e; e = en;
    gm = gg; gg = gn;
    gp += wp[l + 1] * e;
    xm += wm[l + 1] * gg;
  }
  f[0] = 1.0 - gp * inv_norm;
  f[1] = xm * inv_norm;
}

__global__ void k_table_nodes(const double *wp, const double *wm, int lmax, int spin,
                              double inv_norm, double h, double offset, int count, double *out) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= count) return;
  const int nf = spin == 0 ? 1 : 2;
  double f[2];
  exact_corr(wp, wm, lmax, spin, inv_norm, ((double)k + offset) * h, f);
  for (int q = 0; q < nf; ++q) out[(size_t)k * nf + q] = f[q];
}

__global__ void k_table_eval(const double *tab, int ntab, int nf, double inv_h, const double *s,
                             int64_t n, double *out, unsigned long long *range_cnt) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double f[2];
  bool inr = table_lookup(tab, ntab, nf, inv_h, s[i], f);
  if (!inr && range_cnt) atomicAdd(range_cnt, 1ull);
  for (int q = 0; q < nf; ++q) out[i * nf + q] = f[q];
}

int launch_table_eval(const Plan *p, const double *s, int64_t n, double *out, hipStream_t st) {
  if (n == 0) return FLINTS_OK;
  int threads = 256;
  int64_t blocks = (n + threads - 1) / threads;
  hipLaunchKernelGGL(k_table_eval, dim3((unsigned)blocks), dim3(threads), 0, st, p->d.tab,
                     p->d.ntab, p->d.nfun, p->d.inv_h, s, n, out,
                     p->d.counters + CNT_TABLE_RANGE);
  if (hipGetLastError() != hipSuccess) {
    set_error("table_eval kernel launch failed");
    return FLINTS_EDEVICE;
  }
  return FLINTS_OK;
}

// Device buffer owned for the duration of the table build; freed on every
// return path unless released to the plan.
struct DevBuf {
  double *p = nullptr;
  DevBuf() = default;
  DevBuf(const DevBuf &) = delete;
  DevBuf &operator=(const DevBuf &) = delete;
  ~DevBuf() { reset(); }
  void reset(double *q = nullptr) {
    if (p) (void)hipFree(p);
    p = q;
  }
  double *release() {
    double *q = p;
    p = nullptr;
    return q;
  }
};

#define HIPCHK(x)                                                   \
  do {                                                              \
    hipError_t e_ = (x);                                            \
    if (e_ != hipSuccess) {                                         \
      set_error(std::string("HIP error in table build: ") +         \
                hipGetErrorString(e_));                             \
      return FLINTS_EDEVICE;                                        \
    }                                                               \
  } while (0)

int build_table(Plan *p, const double *w_plus, const double *w_minus, double tol) {
  const int lmax = p->lmax;
  const int spin = p->d.spin;
  const int nf = spin == 0 ? 1 : 2;
  const int NTAB_MAX = 8192;
  double norm = 0.0;
  for (int l = 0; l <= lmax; ++l) norm += w_plus[l];
  const double inv_norm = 1.0 / norm;

  DevBuf d_wp, d_wm, best_tab;
  HIPCHK(hipMalloc(&d_wp.p, sizeof(double) * (lmax + 1)));
  HIPCHK(hipMalloc(&d_wm.p, sizeof(double) * (lmax + 1)));
  HIPCHK(hipMemcpy(d_wp.p, w_plus, sizeof(double) * (lmax + 1), hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(d_wm.p, w_minus ? w_minus : w_plus, sizeof(double) * (lmax + 1),
                   hipMemcpyHostToDevice));

  int nint = 128;                 // intervals over [0, smax]
  double best_err = 1e300;
  int best_ntab = 0;
  double best_h = 0.0;
  for (int iter = 0; iter < 12; ++iter) {
    const int ntab = nint + 4;
    const double h = p->d.smax / (double)nint;
    DevBuf d_tab, d_tmp, d_s, d_int;
    HIPCHK(hipMalloc(&d_tab.p, sizeof(double) * ntab * nf));
    int th = 128;
    hipLaunchKernelGGL(k_table_nodes, dim3((ntab + th - 1) / th), dim3(th), 0, 0, d_wp.p, d_wm.p,
                       lmax, spin, inv_norm, h, -1.0, ntab, d_tab.p);
    // exact values at interval midpoints s = (m + 1/2) h, m = 0 .. nint-1
    HIPCHK(hipMalloc(&d_tmp.p, sizeof(double) * nint * nf));
    hipLaunchKernelGGL(k_table_nodes, dim3((nint + th - 1) / th), dim3(th), 0, 0, d_wp.p, d_wm.p,
                       lmax, spin, inv_norm, h, 0.5, nint, d_tmp.p);
    std::vector<double> hs(nint);
    for (int m = 0; m < nint; ++m) hs[m] = (m + 0.5) * h;
    HIPCHK(hipMalloc(&d_s.p, sizeof(double) * nint));
    HIPCHK(hipMalloc(&d_int.p, sizeof(double) * nint * nf));
    HIPCHK(hipMemcpy(d_s.p, hs.data(), sizeof(double) * nint, hipMemcpyHostToDevice));
    hipLaunchKernelGGL(k_table_eval, dim3((nint + th - 1) / th), dim3(th), 0, 0, d_tab.p, ntab,
                       nf, 1.0 / h, d_s.p, (int64_t)nint, d_int.p, (unsigned long long *)nullptr);
    HIPCHK(hipGetLastError());
    std::vector<double> ex(nint * nf), ip(nint * nf);
    HIPCHK(hipMemcpy(ex.data(), d_tmp.p, sizeof(double) * nint * nf, hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(ip.data(), d_int.p, sizeof(double) * nint * nf, hipMemcpyDeviceToHost));
    double err = 0.0;
    bool finite = true;
    for (int i = 0; i < nint * nf; ++i) {
      double e = std::fabs(ex[i] - ip[i]);
      if (!std::isfinite(e)) finite = false;
      err = std::max(err, e);
    }
    if (!finite) {
      set_error("correlation table is not finite (check the spectrum)");
      return FLINTS_EINVAL;
    }
    const bool improved = err < 0.5 * best_err;
    if (err < best_err) {
      best_tab.reset(d_tab.release());
      best_err = err; best_ntab = ntab; best_h = h;
    }
    if (best_err <= tol || !improved || ntab >= NTAB_MAX) break;
    double grow = std::pow(best_err / tol, 0.25) * 1.15;
    grow = std::min(std::max(grow, 1.25), 8.0);
    nint = std::min(NTAB_MAX - 4, (int)std::ceil(nint * grow));
  }
  p->d_tab = best_tab.release();
  p->d.tab = p->d_tab;
  p->d.ntab = best_ntab;
  p->d.nfun = nf;
  p->d.h = best_h;
  p->d.inv_h = 1.0 / best_h;
  p->table_err = best_err;
  return FLINTS_OK;
}

}  // namespace flints
