/*
 * flints.h -- C ABI of the MI355X FLINTS interpolation library (libflints.so).
 *
 * FLINTS (Lavaux & Wandelt, "Fast and optimal CMB lensing using statistical
 * interpolation on the sphere") predicts the value of an isotropic Gaussian
 * random field at an arbitrary direction from the values sampled on a stencil
 * of HEALPix pixels, using the field's angular power spectrum: the Gaussian
 * conditional mean (kriging), together with its error variance.
 *
 * For every target direction the library
 *   1. finds the K nearest RING pixel centres (chord distance, ties to the
 *      smaller pixel index) -- the stencil of paper Sec. 2.3, read as "K nearest";
 *   2. gathers their values from a RING-ordered map;
 *   3. assembles the K x K neighbour covariance S and the target-neighbour vector
 *      b from the correlation function tabulated at plan time -- spin 0:
 *      Sec. 2.1, Eq. correlation_func / fundamental_variance; spin 2: Sec. 2.2,
 *      Eq. spins_correl / v_spins, with parallel-transport phases;
 *   4. factorises S + n I (Cholesky, nugget n of Sec. 2.4) and solves;
 *   5. returns the weighted value (Eq. best_temperature_field, Eq. major_eq)
 *      and, if asked, the kriging variance (Eq. gaussvar, Eq. gaussvar_pol).
 *
 * Conventions
 *   - All device arrays are plain device pointers (hipMalloc'ed or equivalent);
 *     the caller owns every array passed in.  A plan owns its device tables.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).  All
 *     device work of a call is enqueued on that stream; calls return once the
 *     work is enqueued, without synchronising.
 *   - Return codes: FLINTS_OK (0) or a negative FLINTS_E* code; the message of
 *     the last failure on the calling thread is available from
 *     flints_last_error().  Nothing throws across this ABI.
 *   - Per-point problems never abort a launch: a target with theta outside
 *     [0, pi] or a non-finite angle yields NaN outputs and is counted in the
 *     plan's statistics.
 */
#ifndef FLINTS_H
#define FLINTS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct flints_plan_s *flints_plan_t;   /* opaque, immutable after creation */

enum {
  FLINTS_OK = 0,
  FLINTS_EINVAL = -1,    /* invalid argument (message says which) */
  FLINTS_ENOMEM = -2,    /* device or host allocation failed */
  FLINTS_EDEVICE = -3,   /* a HIP runtime call failed */
  FLINTS_ELIMIT = -4     /* request exceeds a documented size limit */
};

enum { FLINTS_FP64 = 0, FLINTS_FP32_IR = 1 };
enum { FLINTS_S2_FULL = 0, FLINTS_S2_PAPER = 1 };
enum { FLINTS_NUG_ALWAYS = 0, FLINTS_NUG_ON_FAILURE = 1 };
enum { FLINTS_VAR_PAPER = 0, FLINTS_VAR_MSE = 1 };
enum { FLINTS_STENCIL_NEAREST = 0, FLINTS_STENCIL_PIXEL = 1 };
enum { FLINTS_MAP_F64 = 0, FLINTS_MAP_F32 = 1 };

typedef struct {
  /* FLINTS_FP64: every step in double precision.
   * FLINTS_FP32_IR: covariance entries and residuals in FP64, factorisation and
   *   solves in FP32 with one step of iterative refinement; neighbourhoods whose
   *   FP32 factorisation fails the pivot-ratio or refinement-convergence test are
   *   recomputed in FP64 (counted in flints_stats.fp64_fallbacks). */
  int precision;
  /* Spin 2 only.  FLINTS_S2_FULL (default): exact Gaussian conditional mean of
   * (Q, U) from both <P P*> (xi_+) and <P P> (xi_-), a real 2K x 2K system.
   * FLINTS_S2_PAPER: the Hermitian complex K x K estimator of Sec. 2.2 (xi_- = 0). */
  int spin2_mode;
  /* FLINTS_NUG_ALWAYS (default): S + eps I with eps = 2^-26 (= 1.49e-8, the value
   * Sec. 2.4 gives for double precision); if that factorisation still fails the
   * nugget becomes -lambda_min(S) + eps.  FLINTS_NUG_ON_FAILURE: the paper's
   * literal rule, no nugget unless the factorisation of S fails. */
  int nugget;
  /* FLINTS_VAR_PAPER (default): sigma^2 (1 - b^T w), Eq. gaussvar with S + n I.
   * FLINTS_VAR_MSE: additionally subtracts sigma^2 n |w|^2, the exact mean
   * squared error of the regularised weights. */
  int var_kind;
  /* Maximum absolute error of the tabulated, cubic-interpolated correlation
   * function relative to its zero-lag value (0 = default 1e-12). */
  double table_tol;
  /* FP32_IR thresholds (0 = defaults): minimum ratio min_k L_kk / max_k L_kk of
   * the FP32 factor, and maximum |dw| / |w| of the refinement step. */
  double pivot_ratio_min;
  double refine_tol;
  /* FP32_IR plans probe their neighbour systems when created: the FP32
   * factorisation and refinement run (with zero data) on 512 fixed directions
   * spread over the sphere, and if more than this fraction of them is rejected
   * the plan computes in FP64 from the start, since an FP32 attempt that is
   * recomputed in FP64 only adds work (0 = default 0.5; >= 1 never skips).
   * The fraction found is reported by flints_plan_info. */
  double fp32_max_reject;
  /* FLINTS_STENCIL_NEAREST (default): the K pixel centres nearest to each
   *   target, and a factorisation per target (O(K^3) per target).
   * FLINTS_STENCIL_PIXEL: the paper's stencil tied to the pixel containing the
   *   target (Sec. 2.3), read as the K pixel centres nearest to that pixel's
   *   centre, with the Cholesky factor of every pixel class tabulated at plan
   *   time (Sec. 2.4, one factor per ring position using the quarter-turn and
   *   belt rotations of the pixelisation), so a target costs two triangular
   *   solves (O(K^2)).  Needs at most 48 rows (spin 0: K <= 48; spin 2:
   *   K <= 16), FLINTS_VAR_PAPER, and computes in FP64; the tables take
   *   about N_side^2 classes x (4 K + 4 n (n + 1)) bytes (n = K or 2K) of
   *   device memory, reported by flints_plan_info. */
  int stencil;
  /* FLINTS_MAP_F64 (default): maps hold doubles.  FLINTS_MAP_F32: maps hold
   * floats (half the gather bytes); each value is widened to double exactly
   * and everything else is unchanged, so the outputs equal those of an
   * FLINTS_MAP_F64 plan given the same values as doubles. */
  int map_type;
} flints_opts;

/* Fill *o with the defaults above. */
void flints_default_opts(flints_opts *o);

/*
 * Create a plan (paper Sec. 2.5, preparation steps 1-2: resolution, band limit
 * and the tabulated correlation function).
 *   nside  HEALPix resolution, 1 <= nside <= 8192.
 *   lmax   band limit, 1 <= lmax <= 16384 (spin 2: >= 2).
 *   cl     host array.  spin 0: C^TT_l for l = 0..lmax (l = 0 ignored, Eq.
 *          correlation_func sums from l = 1).  spin 2: C^EE_l for l = 0..lmax
 *          followed by C^BB_l for l = 0..lmax (l < 2 ignored).  Must be finite
 *          and non-negative; read during the call only.
 *   K      stencil size, 1 <= K <= min(64, 12 nside^2) (spin 2: a real 2K x 2K
 *          system).  Spin-2 plans with K > 32 (64 < 2K <= 128 rows) run an
 *          FP64 elimination in LDS: FLINTS_FP32_IR runs them in FP64, and
 *          FLINTS_VAR_MSE is refused for them (NULL).
 *   spin   0 (temperature) or 2 (Q, U polarisation).
 * The correlation function is built on the current HIP device in FP64 and kept
 * in device memory.  Returns NULL on error (see flints_last_error()).
 */
flints_plan_t flints_plan(int64_t nside, int lmax, const double *cl, int K, int spin);
flints_plan_t flints_plan_ex(int64_t nside, int lmax, const double *cl, int K, int spin,
                             const flints_opts *opts);

/*
 * Interpolate a RING map at n target directions (paper Sec. 2.5, steps 4-6).
 *   map    device, RING order.  spin 0: double[npix].  spin 2: double[2*npix],
 *          the Q plane followed by the U plane (float instead of double for
 *          plans made with FLINTS_MAP_F32).
 *   theta  device double[n], colatitude in [0, pi].
 *   phi    device double[n], longitude, any real (reduced modulo 2 pi).
 *   out    device.  spin 0: double[n].  spin 2: double[2*n] = (Q[n], U[n]).
 *   var    device, nullable (variance is then not written).  Same layout as out.
 * Q and U are Stokes parameters in the local (e_theta, e_phi) frame with
 * P = Q + iU = sum 2a_lm 2Y_lm, 2a_lm = -(E_lm + i B_lm), and
 * sY_lm = (-1)^s sqrt((2l+1)/4pi) e^{i m phi} d^l_{m,-s}(theta) (paper App. A).
 * n = 0 is a no-op.  Concurrent calls with one plan on different streams are
 * allowed.
 */
int flints_interpolate(flints_plan_t plan, const void *map, const double *theta,
                       const double *phi, int64_t n, void *out, void *var, void *stream);

/*
 * Temperature and polarisation at the same targets (T + Q + U) with one
 * stencil search per target.  The stencil of a target (its K nearest pixel
 * centres, paper Sec. 2.5, step 4) depends only on the target, N_side and K,
 * so for a spin-0 plan and a spin-2 plan of equal N_side and K the spin-2 pass
 * writes each target's stencil to device memory and the spin-0 pass reads it
 * instead of searching again.  Everything after the search is the per-plan
 * arithmetic of flints_interpolate, and the outputs equal
 * flints_interpolate(plan_t, map_t, ...) followed by
 * flints_interpolate(plan_qu, map_qu, ...) bit for bit.
 *   plan_t   spin-0 plan; plan_qu spin-2 plan with the same nside and K.
 *   map_t    device double[npix]; map_qu device double[2*npix] (Q then U).
 *   theta, phi  device double[n], shared by both fields.
 *   out_t    device double[n]; out_qu device double[2*n] = (Q[n], U[n]).
 *   var_t, var_qu  device, nullable, same layouts as the outputs.
 * The search is shared when both plans are FLINTS_FP64 with paper variance
 * (or their variance is not requested) and their search radii agree (see
 * flints_tqu_shared); other plan pairs, or a failed allocation of the stencil
 * buffer, run as the two separate calls on the same stream.  The buffer holds
 * K ints per target for chunks of up to 2^24 targets (2 GiB at K = 32) and is
 * allocated and freed on the stream from a memory pool of the library that
 * keeps freed memory (hipMallocFromPoolAsync / hipFreeAsync), so repeated
 * calls reuse it.  Invalid
 * targets and failed searches are counted in both plans.  Returns
 * FLINTS_EINVAL for NULL plans or pointers, spins other than (0, 2), or
 * differing nside or K; n = 0 is a no-op.
 */
int flints_interpolate_tqu(flints_plan_t plan_t, flints_plan_t plan_qu, const void *map_t,
                           const void *map_qu, const double *theta, const double *phi, int64_t n,
                           void *out_t, void *var_t, void *out_qu, void *var_qu, void *stream);

/*
 * flints_interpolate_tqu for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, hosts that forbid hipMalloc):
 * the same arguments, outputs and counters as flints_interpolate_tqu, but the
 * stencil hand-over buffer is a static 64 MiB device array of the library
 * instead of a stream-ordered allocation, and nothing is allocated or freed.
 * Targets run in chunks of what the array holds, 64 MiB / (4 K) stencils
 * (524,288 targets at K = 32), so n is not limited; a K whose stencil of four
 * targets would not fit returns FLINTS_ELIMIT (no plan has one).  Each device
 * holds its own array from the first call on it until the process ends; the
 * caller passes inputs and outputs as for flints_interpolate_tqu.  All calls
 * on one device share that array: calls that overlap on one device (other
 * streams, other host threads) race and must be serialised by the caller.
 * Plan pairs that flints_tqu_shared reports as not shared run as two
 * flints_interpolate calls, which use no workspace.
 */
int flints_interpolate_tqu_noalloc(flints_plan_t plan_t, flints_plan_t plan_qu, const void *map_t,
                                   const void *map_qu, const double *theta, const double *phi,
                                   int64_t n, void *out_t, void *var_t, void *out_qu, void *var_qu,
                                   void *stream);

/*
 * Centres of all RING pixels of resolution nside (the target directions of
 * flints_supersample, computed by the same kernel):
 *   theta, phi  device double[12 nside^2].  1 <= nside <= 16384.
 */
int flints_pixel_centres(int64_t nside, double *theta, double *phi, void *stream);

/*
 * Supersampling (paper Sec. 2.6, Table 1: a map of resolution N_side
 * interpolated onto the pixel centres of resolution 2 N_side): interpolate the
 * plan's RING map at every pixel centre of a RING map of resolution nside_out.
 * The target directions are generated on the device (RING order of nside_out,
 * pixel centres as in flints_plan's geometry), then the call is
 * flints_interpolate over them.
 *   map        as flints_interpolate (the plan's N_side).
 *   nside_out  1 <= nside_out <= 16384; npix_out = 12 nside_out^2 targets.
 *   out        device double[npix_out] (spin 2: [2][npix_out], the Q map then
 *              the U map), a RING map of nside_out.
 *   var        device, nullable, same layout.
 * A workspace of 16 B per output pixel (the directions) is taken from the
 * library's stream-ordered pool for the duration of the call.  Returns
 * FLINTS_ENOMEM if it cannot be allocated.
 */
int flints_supersample(flints_plan_t plan, const void *map, int64_t nside_out, void *out, void *var,
                       void *stream);

/*
 * Spin-s harmonic synthesis onto the RING pixel centres (the lensing pipeline
 * of paper Sec. 3.1 makes the unlensed T, Q, U maps and the deflection
 * d = grad(phi) this way; spin-weighted harmonics as in App. A,
 * sY_lm = (-1)^s sqrt((2l+1)/4pi) e^{i m phi} d^l_{m,-s}(theta), Condon-Shortley
 * phase, polarisation Q + iU = sum 2a_lm 2Y_lm with 2a_lm = -(E_lm + i B_lm)).
 *   nside  1 <= nside <= 8192.  lmax  0 <= lmax <= 16384 (any lmax; orders
 *          above the ring's Nyquist frequency alias as the sum itself does).
 *   spin   0: alm = T_lm, map = T                          (device double[npix])
 *          1: alm = phi_lm, map = (d_theta, d_phi) = grad phi (device double[2][npix])
 *          2: alm = E_lm, blm = B_lm (NULL: B = 0), map = (Q, U) (device double[2][npix])
 *   alm, blm  device, complex doubles interleaved (re, im), m >= 0 only, in
 *          m-major order: (l, m) at index m (2 lmax + 3 - m) / 2 + (l - m),
 *          (lmax+1)(lmax+2)/2 entries; the fields are real, so the m < 0
 *          coefficients are (-1)^m conj(a_lm) and the m = 0 imaginary parts
 *          are ignored.  blm must be NULL unless spin = 2.
 *   map    device, written in full (planes of npix = 12 nside^2 doubles).
 * Workspace from the library's stream-ordered pool: 16 B (spin 0) or 32 B
 * (spin 1, 2) per (ring, m) for the ring coefficients, then per group of rings
 * of equal transform length two complex buffers of that length per ring.
 * Returns FLINTS_ENOMEM if they cannot be allocated.  Stream-ordered.
 */
int flints_synthesize(int64_t nside, int lmax, int spin, const void *alm, const void *blm, void *map,
                      void *stream);

/*
 * Displaced pixel centres of the lensing remap (paper Sec. 3.1, vector form):
 * n' = cos|d| n + sin|d| (d_theta e_theta + d_phi e_phi) / |d| at every RING pixel
 * centre n of nside (n' = n where d = 0; no special case at the poles).
 *   defl   device double[2][npix]: d_theta then d_phi (radians), as
 *          flints_synthesize spin 1 writes it.
 *   theta, phi  device double[npix]: colatitude in [0, pi], longitude in [0, 2 pi).
 * Elementwise and stream-ordered; no workspace.
 */
int flints_lensed_directions(int64_t nside, const void *defl, void *theta, void *phi, void *stream);

/* 1 if flints_interpolate_tqu shares the stencil search between these plans
 * (with_var_*: whether variances will be requested), 0 if it runs two
 * separate calls, < 0 on error.  Host-only; launches nothing. */
int flints_tqu_shared(flints_plan_t plan_t, flints_plan_t plan_qu, int with_var_t, int with_var_qu);

/*
 * Stencil of each target: the K nearest RING pixels, ascending distance, ties to
 * the smaller index (paper Sec. 2.3 step, read as K nearest).
 *   idx    device int64[n*K], row-major; rows of invalid targets are -1.
 */
int flints_stencil(flints_plan_t plan, const double *theta, const double *phi, int64_t n,
                   int64_t *idx, void *stream);

/*
 * Evaluate the plan's tabulated correlation function (paper App. B: tabulated
 * and interpolated with cubics) at n chord half-lengths s = sin(beta/2).
 *   s      device double[n], 0 <= s <= plan's table range.
 *   out    device double[n*nf], nf = 1 (spin 0: zeta/zeta(0)) or 2 (spin 2:
 *          xi_+/xi_+(0), xi_-/xi_+(0)), row-major.
 */
int flints_table_eval(flints_plan_t plan, const double *s, int64_t n, double *out, void *stream);

typedef struct {
  int64_t nside;
  int lmax, K, spin;
  int ntab;              /* table nodes per function */
  double table_step;     /* node spacing in s = sin(beta/2) */
  double table_smax;     /* largest s covered */
  double table_err;      /* measured max interpolation error (relative) */
  double sigma2;         /* prior variance per output field */
  double search_r0, search_rcap;   /* stencil search radii (rad) */
  double nugget_eps;
  int precision;         /* arithmetic the plan runs: FLINTS_FP64, or FLINTS_FP32_IR if
                            the FP32 path was kept after the creation probe */
  double fp32_probe_reject;        /* FP32_IR plans: fraction of probe systems the
                                      FP32 path rejected (-1 for FP64 plans) */
  int stencil;                     /* FLINTS_STENCIL_NEAREST or FLINTS_STENCIL_PIXEL */
  int64_t pixel_classes;           /* FLINTS_STENCIL_PIXEL: tabulated classes */
  int64_t class_nuggets;           /* classes whose factor needed -lambda_min + eps */
  int64_t table_bytes;             /* device bytes of the plan's tables */
  int map_type;                    /* FLINTS_MAP_F64 or FLINTS_MAP_F32 */
} flints_plan_info_t;

int flints_plan_info(flints_plan_t plan, flints_plan_info_t *info);

typedef struct {
  int64_t bad_inputs;          /* targets with invalid angles */
  int64_t nugget_escalations;  /* factorisations that needed -lambda_min + eps */
  int64_t clamped_vars;        /* negative variances clamped to 0 */
  int64_t fp64_fallbacks;      /* FP32_IR points recomputed in FP64 */
  int64_t search_failures;     /* targets whose stencil was not found (NaN output) */
  int64_t table_range;         /* pair distances beyond the table (clamped) */
} flints_stats;

/* Counters accumulated since plan creation or the last reset: read on `stream`
 * (so they include all work enqueued on it before the call; work on other
 * streams counts once it has completed), and the call waits for `stream` only.
 * flints_plan_reset_stats enqueues the zeroing on `stream` (not for use inside a
 * captured graph). */
int flints_plan_stats(flints_plan_t plan, flints_stats *st, void *stream);
int flints_plan_reset_stats(flints_plan_t plan, void *stream);

/* Release a plan.  The caller must ensure no work using it is in flight. */
void flints_plan_destroy(flints_plan_t plan);

/*
 * Batched execution: many interpolation jobs (different plans -- N_side, K,
 * spin -- and target counts) in persistent fused launches.  Jobs are cut into
 * tiles of consecutive targets; FP64 jobs (FLINTS_VAR_PAPER) of one launch group
 * (system size n <= 16, <= 32, <= 48, <= 64 rows, n = K or 2K, and table size)
 * share one persistent launch whose blocks take tiles from a device queue, reload the job's
 * correlation table into LDS when the job changes, and run the same per-point
 * arithmetic as flints_interpolate (results are bit-identical to it); spin 0
 * and spin 2 jobs mix freely within a class.  Jobs with FP32_IR or MSE-variance
 * plans, and jobs whose system has more than 64 rows (spin 2 with K > 32, the LDS
 * elimination), run through the single-plan path in the same stream.  Batching is an
 * addition to the method: the paper interpolates one map at a time.
 */
typedef struct {
  flints_plan_t plan;        /* borrowed; must outlive the batch */
  const void *map;           /* as flints_interpolate */
  const double *theta, *phi; /* device double[n] */
  int64_t n;                 /* >= 0 */
  void *out, *var;           /* as flints_interpolate (var nullable) */
} flints_job_t;

typedef struct flints_batch_s *flints_batch_t;

enum {
  FLINTS_BATCH_AUTOTUNE = 1   /* choose tile size and waves per block by timing
                                 candidates on a sample of the batch at creation
                                 (this runs kernels that write the job outputs) */
};

/*
 * Build a batch from njobs (1 <= njobs <= 65536) job descriptors (host array,
 * copied; the device arrays they point to are borrowed).  Allocates the device
 * job table, tile lists and queue counters; with FLINTS_BATCH_AUTOTUNE also
 * synchronises the device.  Returns NULL on error.
 */
flints_batch_t flints_batch_create(const flints_job_t *jobs, int njobs, int flags);

/* Enqueue the whole batch on stream (replays the captured graph if one exists). */
int flints_batch_run(flints_batch_t batch, void *stream);

/*
 * Capture the launch sequence of flints_batch_run into a HIP graph (queue
 * counters are cleared by a kernel, not a memset, so replays are exact); later
 * flints_batch_run calls launch the graph.  stream must not be capturing.
 */
int flints_batch_capture(flints_batch_t batch, void *stream);

typedef struct {
  int njobs;
  int64_t points;            /* total targets */
  int fused_jobs;            /* jobs on the persistent launches */
  int classes;               /* persistent launch groups used per run */
  /* per launch group g = 6 * engine + bucket: engine by rows n <= 16, 32, 48,
   * 64; bucket (row-group engines only; the tile engines, n > 32, read their
   * tables through the caches and use bucket 0) by correlation-table size
   * <= 16, 36, 57, 77, 98 KB, larger */
  int tiles[24];
  int tile_points[24];       /* targets per tile (0 = group unused); a tile is
                                taken by one block (row-group engines) or one
                                wave (tile engines) */
  int waves_per_block[24];
  int captured;              /* 1 if runs replay a graph */
} flints_batch_info_t;

int flints_batch_info(flints_batch_t batch, flints_batch_info_t *info);

/* Release a batch (its graph, tile lists and counters; not the jobs' arrays).
 * The caller must ensure no run of it is in flight. */
void flints_batch_destroy(flints_batch_t batch);

/* Message of the last failure on the calling thread ("" if none). */
const char *flints_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* FLINTS_H */
