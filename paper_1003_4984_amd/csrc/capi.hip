// C ABI of libflints: validation, plan lifecycle, statistics and error text.
// Every entry point catches its own failures and reports them through a return
// code plus a thread-local message; nothing throws across the boundary.
#include "plan.h"
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

namespace flints {

static thread_local std::string g_last_error;

void set_error(const std::string &msg) { g_last_error = msg; }
// Start of an entry point: clears this thread's message and any HIP error left
// by earlier calls of the caller, so that launch checks see only this call's.
static void begin_call() {
  g_last_error.clear();
  (void)hipGetLastError();
}

static bool finite_nonneg(const double *v, int n) {
  for (int i = 0; i < n; ++i)
    if (!std::isfinite(v[i]) || v[i] < 0.0) return false;
  return true;
}

}  // namespace flints

using namespace flints;

extern "C" {

void flints_default_opts(flints_opts *o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->precision = FLINTS_FP64;
  o->spin2_mode = FLINTS_S2_FULL;
  o->nugget = FLINTS_NUG_ALWAYS;
  o->var_kind = FLINTS_VAR_PAPER;
  o->table_tol = 1e-12;
  o->pivot_ratio_min = 0.0;
  o->refine_tol = 0.0;
  o->fp32_max_reject = 0.0;
  o->stencil = FLINTS_STENCIL_NEAREST;
  o->map_type = FLINTS_MAP_F64;
}

const char *flints_last_error(void) { return g_last_error.c_str(); }

flints_plan_t flints_plan(int64_t nside, int lmax, const double *cl, int K, int spin) {
  return flints_plan_ex(nside, lmax, cl, K, spin, nullptr);
}

flints_plan_t flints_plan_ex(int64_t nside, int lmax, const double *cl, int K, int spin,
                             const flints_opts *opts) {
  begin_call();
  flints_opts o;
  flints_default_opts(&o);
  if (opts) o = *opts;
  if (o.table_tol <= 0.0) o.table_tol = 1e-12;
  if (nside < 1 || nside > 8192) { set_error("nside must be in [1, 8192]"); return nullptr; }
  if (spin != 0 && spin != 2) { set_error("spin must be 0 or 2"); return nullptr; }
  if (lmax < (spin == 0 ? 1 : 2) || lmax > 16384) {
    set_error("lmax must be in [1, 16384] (spin 2: >= 2)");
    return nullptr;
  }
  if (!cl) { set_error("cl is NULL"); return nullptr; }
  const int64_t npix = 12 * nside * nside;
  if (K < 1 || K > 64 || K > npix) {
    set_error("K must be in [1, min(64, npix)]");
    return nullptr;
  }
  if (o.precision != FLINTS_FP64 && o.precision != FLINTS_FP32_IR) { set_error("bad precision"); return nullptr; }
  if (o.spin2_mode != FLINTS_S2_FULL && o.spin2_mode != FLINTS_S2_PAPER) { set_error("bad spin2_mode"); return nullptr; }
  if (o.nugget != FLINTS_NUG_ALWAYS && o.nugget != FLINTS_NUG_ON_FAILURE) { set_error("bad nugget policy"); return nullptr; }
  if (o.var_kind != FLINTS_VAR_PAPER && o.var_kind != FLINTS_VAR_MSE) { set_error("bad var_kind"); return nullptr; }
  if (o.stencil != FLINTS_STENCIL_NEAREST && o.stencil != FLINTS_STENCIL_PIXEL) { set_error("bad stencil"); return nullptr; }
  if (o.map_type != FLINTS_MAP_F64 && o.map_type != FLINTS_MAP_F32) { set_error("bad map_type"); return nullptr; }
  if (spin == 2 && K > 32 && o.stencil == FLINTS_STENCIL_NEAREST && o.var_kind == FLINTS_VAR_MSE) {
    // systems above 64 rows run the LDS elimination, which forms the paper variance only
    set_error("FLINTS_VAR_MSE supports systems of at most 64 rows (spin 2: K <= 32)");
    return nullptr;
  }
  if (o.stencil == FLINTS_STENCIL_PIXEL) {
    if ((spin == 0 && K > 48) || (spin == 2 && K > 16)) {
      set_error("FLINTS_STENCIL_PIXEL supports at most 48 rows (spin 0: K <= 48, spin 2: K <= 16)");
      return nullptr;
    }
    if (o.var_kind != FLINTS_VAR_PAPER) {
      set_error("FLINTS_STENCIL_PIXEL supports FLINTS_VAR_PAPER only");
      return nullptr;
    }
    if (nside > 8191) {
      set_error("FLINTS_STENCIL_PIXEL supports nside <= 8191");
      return nullptr;
    }
  }
  const int ncl = (spin == 0 ? 1 : 2) * (lmax + 1);
  if (!finite_nonneg(cl, ncl)) { set_error("cl must be finite and non-negative"); return nullptr; }

  // weights (2l+1)/(4 pi) C_l; spin 0 sums from l = 1, spin 2 from l = 2
  std::vector<double> wp(lmax + 1, 0.0), wm(lmax + 1, 0.0);
  const double inv4pi = 1.0 / (4.0 * 3.14159265358979323846);
  for (int l = 0; l <= lmax; ++l) {
    const double f = (2.0 * l + 1.0) * inv4pi;
    if (spin == 0) {
      if (l >= 1) wp[l] = f * cl[l];
    } else if (l >= 2) {
      const double ee = cl[l], bb = cl[lmax + 1 + l];
      wp[l] = f * (ee + bb);
      wm[l] = f * (ee - bb);
    }
  }
  double s0 = 0.0;
  for (int l = 0; l <= lmax; ++l) s0 += wp[l];
  if (!(s0 > 0.0)) { set_error("the spectrum has no power in the summed range"); return nullptr; }

  Plan *p = new (std::nothrow) Plan();
  if (!p) { set_error("host allocation failed"); return nullptr; }
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) {
    delete p;
    set_error("no HIP device available");
    return nullptr;
  }
  p->device = dev;
  p->lmax = lmax;
  PlanDev &d = p->d;
  d.nside = nside;
  d.npix = npix;
  d.K = K;
  d.spin = spin;
  d.mode = o.spin2_mode;
  d.nug_policy = o.nugget;
  d.var_kind = o.var_kind;
  d.precision = o.precision;
  d.n = spin == 0 ? K : 2 * K;
  if (d.n > 64) d.precision = FLINTS_FP64;   // the elimination above 64 rows is FP64 only
  d.eps = 1.4901161193847656e-08;  // 2^-26 = sqrt(double epsilon), paper Sec. 2.4
  d.sigma2 = spin == 0 ? s0 : 0.5 * s0;
  d.pivot_ratio_min = o.pivot_ratio_min > 0.0 ? o.pivot_ratio_min : 1e-3;
  d.refine_tol = o.refine_tol > 0.0 ? o.refine_tol : 1e-3;
  // Search radii from the expected pixel count in a cap: N(r) = 6 nside^2 (1 - cos r).
  // r0 holds max(1.3K, K + 8) pixel centres on average (pixel counts in a disc
  // vary little on the HEALPix lattice, so the first disc nearly always holds K
  // and its candidates fit one pass of a wavefront); rcap ~5K; the table covers
  // pair separations up to 2 rcap, i.e. s = sin(beta/2) <= sin(rcap).
  const double n2 = (double)nside * (double)nside;
  auto cap_radius = [&](double count) {
    double c = 1.0 - count / (6.0 * n2);
    if (c <= -1.0) return 3.14159265358979323846;
    return std::acos(c);
  };
  d.r0 = cap_radius(std::max(1.3 * K, K + 8.0));
  d.rcap = std::max(d.r0, cap_radius(5.0 * K + 8.0));
  d.smax = d.rcap >= 0.5 * 3.14159265358979323846 ? 1.0 : std::min(1.0, std::sin(d.rcap) * 1.0001);

  int rc = build_table(p, wp.data(), spin == 2 ? wm.data() : nullptr, o.table_tol);
  if (rc != FLINTS_OK) {
    delete p;
    return nullptr;
  }
  if (hipMalloc(&p->d_counters, sizeof(unsigned long long) * CNT_N) != hipSuccess ||
      hipMemset(p->d_counters, 0, sizeof(unsigned long long) * CNT_N) != hipSuccess) {
    hipFree(p->d_tab);
    delete p;
    set_error("device allocation of plan counters failed");
    return nullptr;
  }
  d.counters = p->d_counters;
  d.stencil_mode = o.stencil;
  d.map_f32 = o.map_type == FLINTS_MAP_F32 ? 1 : 0;
  if (o.stencil == FLINTS_STENCIL_PIXEL) {
    d.precision = FLINTS_FP64;           // the tabulated factors are FP64
    if (build_fixed(p) != FLINTS_OK) {
      flints_plan_destroy(reinterpret_cast<flints_plan_t>(p));
      return nullptr;
    }
  }
  if (d.precision == FLINTS_FP32_IR) {
    const double maxrej = o.fp32_max_reject > 0.0 ? o.fp32_max_reject : 0.5;
    const double rej = fp32_probe(p);
    if (rej < 0.0) {
      flints_plan_destroy(reinterpret_cast<flints_plan_t>(p));
      return nullptr;
    }
    p->fp32_reject = rej;
    if (rej > maxrej) d.precision = FLINTS_FP64;   // FP32 would only add work here
  }
  return reinterpret_cast<flints_plan_t>(p);
}

static Plan *as_plan(flints_plan_t h) { return reinterpret_cast<Plan *>(h); }

int flints_interpolate(flints_plan_t plan, const void *map, const double *theta, const double *phi,
                       int64_t n, void *out, void *var, void *stream) {
  begin_call();
  if (!plan) { set_error("plan is NULL"); return FLINTS_EINVAL; }
  if (n < 0) { set_error("n must be >= 0"); return FLINTS_EINVAL; }
  if (n == 0) return FLINTS_OK;
  if (!map || !theta || !phi || !out) { set_error("map, theta, phi and out must be non-NULL"); return FLINTS_EINVAL; }
  Plan *p = as_plan(plan);
  return launch_interpolate(p, (const double *)map, theta, phi, n, (double *)out, (double *)var,
                            (hipStream_t)stream);
}

static int check_tqu(flints_plan_t plan_t, flints_plan_t plan_qu, const void *map_t, const void *map_qu,
                     const double *theta, const double *phi, int64_t n, const void *out_t,
                     const void *out_qu) {
  if (!plan_t || !plan_qu) { set_error("plans must be non-NULL"); return FLINTS_EINVAL; }
  const Plan *p0 = as_plan(plan_t), *p2 = as_plan(plan_qu);
  if (p0->d.spin != 0 || p2->d.spin != 2) {
    set_error("plan_t must be a spin-0 plan and plan_qu a spin-2 plan");
    return FLINTS_EINVAL;
  }
  if (p0->d.nside != p2->d.nside || p0->d.K != p2->d.K) {
    set_error("plan_t and plan_qu must have the same nside and K");
    return FLINTS_EINVAL;
  }
  if (n < 0) { set_error("n must be >= 0"); return FLINTS_EINVAL; }
  if (n > 0 && (!map_t || !map_qu || !theta || !phi || !out_t || !out_qu)) {
    set_error("maps, theta, phi and outputs must be non-NULL");
    return FLINTS_EINVAL;
  }
  return FLINTS_OK;
}

int flints_interpolate_tqu(flints_plan_t plan_t, flints_plan_t plan_qu, const void *map_t,
                           const void *map_qu, const double *theta, const double *phi, int64_t n,
                           void *out_t, void *var_t, void *out_qu, void *var_qu, void *stream) {
  begin_call();
  const int rc = check_tqu(plan_t, plan_qu, map_t, map_qu, theta, phi, n, out_t, out_qu);
  if (rc != FLINTS_OK || n == 0) return rc;
  return launch_interpolate_tqu(as_plan(plan_t), as_plan(plan_qu), (const double *)map_t,
                                (const double *)map_qu, theta, phi, n, (double *)out_t, (double *)var_t,
                                (double *)out_qu, (double *)var_qu, (hipStream_t)stream);
}

int flints_interpolate_tqu_noalloc(flints_plan_t plan_t, flints_plan_t plan_qu, const void *map_t,
                                   const void *map_qu, const double *theta, const double *phi,
                                   int64_t n, void *out_t, void *var_t, void *out_qu, void *var_qu,
                                   void *stream) {
  begin_call();
  const int rc = check_tqu(plan_t, plan_qu, map_t, map_qu, theta, phi, n, out_t, out_qu);
  if (rc != FLINTS_OK || n == 0) return rc;
  return launch_interpolate_tqu_noalloc(as_plan(plan_t), as_plan(plan_qu), (const double *)map_t,
                                        (const double *)map_qu, theta, phi, n, (double *)out_t,
                                        (double *)var_t, (double *)out_qu, (double *)var_qu,
                                        (hipStream_t)stream);
}

int flints_pixel_centres(int64_t nside, double *theta, double *phi, void *stream) {
  begin_call();
  if (nside < 1 || nside > 16384) { set_error("nside must be in [1, 16384]"); return FLINTS_EINVAL; }
  if (!theta || !phi) { set_error("theta and phi must be non-NULL"); return FLINTS_EINVAL; }
  return launch_pixel_centres(nside, theta, phi, (hipStream_t)stream);
}

int flints_synthesize(int64_t nside, int lmax, int spin, const void *alm, const void *blm, void *map,
                      void *stream) {
  begin_call();
  if (nside < 1 || nside > 8192) { set_error("nside must be in [1, 8192]"); return FLINTS_EINVAL; }
  if (lmax < 0 || lmax > 16384) { set_error("lmax must be in [0, 16384]"); return FLINTS_EINVAL; }
  if (spin < 0 || spin > 2) { set_error("spin must be 0, 1 or 2"); return FLINTS_EINVAL; }
  if (!alm || !map) { set_error("alm and map must be non-NULL"); return FLINTS_EINVAL; }
  if (spin != 2 && blm) { set_error("blm is taken by spin-2 synthesis only (pass NULL)"); return FLINTS_EINVAL; }
  return launch_synthesize(nside, lmax, spin, (const double *)alm, (const double *)blm, (double *)map,
                           (hipStream_t)stream);
}

int flints_lensed_directions(int64_t nside, const void *defl, void *theta, void *phi, void *stream) {
  begin_call();
  if (nside < 1 || nside > 16384) { set_error("nside must be in [1, 16384]"); return FLINTS_EINVAL; }
  if (!defl || !theta || !phi) { set_error("defl, theta and phi must be non-NULL"); return FLINTS_EINVAL; }
  return launch_lensed_directions(nside, (const double *)defl, (double *)theta, (double *)phi,
                                  (hipStream_t)stream);
}

int flints_supersample(flints_plan_t plan, const void *map, int64_t nside_out, void *out, void *var,
                       void *stream) {
  begin_call();
  if (!plan) { set_error("plan is NULL"); return FLINTS_EINVAL; }
  if (nside_out < 1 || nside_out > 16384) { set_error("nside_out must be in [1, 16384]"); return FLINTS_EINVAL; }
  if (!map || !out) { set_error("map and out must be non-NULL"); return FLINTS_EINVAL; }
  return launch_supersample(as_plan(plan), (const double *)map, nside_out, (double *)out, (double *)var,
                            (hipStream_t)stream);
}

int flints_tqu_shared(flints_plan_t plan_t, flints_plan_t plan_qu, int with_var_t, int with_var_qu) {
  begin_call();
  if (!plan_t || !plan_qu) { set_error("plans must be non-NULL"); return FLINTS_EINVAL; }
  const double some = 0.0;   // stands for a variance array; only its presence matters
  return tqu_shareable(as_plan(plan_t), as_plan(plan_qu), with_var_t ? &some : nullptr,
                     with_var_qu ? &some : nullptr) ? 1 : 0;
}

int flints_stencil(flints_plan_t plan, const double *theta, const double *phi, int64_t n,
                   int64_t *idx, void *stream) {
  begin_call();
  if (!plan) { set_error("plan is NULL"); return FLINTS_EINVAL; }
  if (n < 0) { set_error("n must be >= 0"); return FLINTS_EINVAL; }
  if (n == 0) return FLINTS_OK;
  if (!theta || !phi || !idx) { set_error("theta, phi and idx must be non-NULL"); return FLINTS_EINVAL; }
  return launch_stencil(as_plan(plan), theta, phi, n, idx, (hipStream_t)stream);
}

int flints_table_eval(flints_plan_t plan, const double *s, int64_t n, double *out, void *stream) {
  begin_call();
  if (!plan) { set_error("plan is NULL"); return FLINTS_EINVAL; }
  if (n < 0) { set_error("n must be >= 0"); return FLINTS_EINVAL; }
  if (n == 0) return FLINTS_OK;
  if (!s || !out) { set_error("s and out must be non-NULL"); return FLINTS_EINVAL; }
  return launch_table_eval(as_plan(plan), s, n, out, (hipStream_t)stream);
}

int flints_plan_info(flints_plan_t plan, flints_plan_info_t *info) {
  begin_call();
  if (!plan || !info) { set_error("plan and info must be non-NULL"); return FLINTS_EINVAL; }
  const Plan *p = as_plan(plan);
  info->nside = p->d.nside;
  info->lmax = p->lmax;
  info->K = p->d.K;
  info->spin = p->d.spin;
  info->ntab = p->d.ntab;
  info->table_step = p->d.h;
  info->table_smax = p->d.smax;
  info->table_err = p->table_err;
  info->sigma2 = p->d.sigma2;
  info->search_r0 = p->d.r0;
  info->search_rcap = p->d.rcap;
  info->nugget_eps = p->d.eps;
  info->precision = p->d.precision;
  info->fp32_probe_reject = p->fp32_reject;
  info->stencil = p->d.stencil_mode;
  info->map_type = p->d.map_f32 ? FLINTS_MAP_F32 : FLINTS_MAP_F64;
  info->pixel_classes = p->nclass;
  info->class_nuggets = p->class_nuggets;
  info->table_bytes = (int64_t)p->d.ntab * p->d.nfun * 8 +
                      (p->nclass ? p->nclass * ((int64_t)p->d.K * 4 + (int64_t)p->d.lsz * 8) +
                                       (int64_t)(4 * p->d.nside) * 12
                                 : 0);
  return FLINTS_OK;
}

int flints_plan_stats(flints_plan_t plan, flints_stats *st, void *stream) {
  begin_call();
  if (!plan || !st) { set_error("plan and stats must be non-NULL"); return FLINTS_EINVAL; }
  unsigned long long c[CNT_N];
  hipStream_t s = (hipStream_t)stream;
  if (hipMemcpyAsync(c, as_plan(plan)->d_counters, sizeof(c), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess) {
    set_error("reading plan counters failed");
    return FLINTS_EDEVICE;
  }
  st->bad_inputs = (int64_t)c[CNT_BAD_INPUT];
  st->nugget_escalations = (int64_t)c[CNT_NUGGET_ESC];
  st->clamped_vars = (int64_t)c[CNT_CLAMPED_VAR];
  st->fp64_fallbacks = (int64_t)c[CNT_FP64_FALLBACK];
  st->search_failures = (int64_t)c[CNT_SEARCH_FAIL];
  st->table_range = (int64_t)c[CNT_TABLE_RANGE];
  return FLINTS_OK;
}

int flints_plan_reset_stats(flints_plan_t plan, void *stream) {
  begin_call();
  if (!plan) { set_error("plan is NULL"); return FLINTS_EINVAL; }
  if (hipMemsetAsync(as_plan(plan)->d_counters, 0, sizeof(unsigned long long) * CNT_N,
                     (hipStream_t)stream) != hipSuccess) {
    set_error("resetting plan counters failed");
    return FLINTS_EDEVICE;
  }
  return FLINTS_OK;
}

void flints_plan_destroy(flints_plan_t plan) {
  if (!plan) return;
  Plan *p = as_plan(plan);
  if (p->d_tab) hipFree(p->d_tab);
  if (p->d_counters) hipFree(p->d_counters);
  free_fixed(p);
  delete p;
}

}  // extern "C"
