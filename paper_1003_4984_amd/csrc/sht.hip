// Lensing pipeline on the device (paper Sec. 3.1): spin-s synthesis of RING maps
// from harmonic coefficients -- the unlensed T, Q + iU and the deflection
// d = grad(phi) as a spin-1 field -- and the displacement of every pixel centre
// to n' = cos|d| n + sin|d| d/|d| in vector form (no special case at the poles).
//
// Synthesis, F(n) = sum_{l,m} a_lm sY_lm(n) with
//   sY_lm = (-1)^s sqrt((2l+1)/4pi) e^{i m phi} d^l_{m,-s}(theta)   (App. A).
// The stored coefficients (m >= 0) are scaled per spin to a = f_l (e + i b),
// with e and b each of a real-type field (e_{l,-m} = (-1)^m conj(e_lm)):
//   spin 0: e = T_lm, f = 1                  -> F = T
//   spin 1: e = phi_lm, f = -sqrt(l(l+1))    -> F = d_theta + i d_phi (grad phi)
//   spin 2: e = E_lm, b = B_lm, f = -1       -> F = Q + i U
// With d^l_{-m,-s} = (-1)^{m+s} d^l_{m,s} the negative orders fold onto m > 0:
//   F(theta, phi) = sum_{m>=0} X_m(theta) e^{i m phi} + sum_{m>0} Z_m(theta) e^{-i m phi},
//   X_m = (-1)^s sum_l N_l f_l (e + i b)_lm d^l_{m,-s},
//   Z_m = sum_l N_l f_l conj(e - i b)_lm d^l_{m,s},        N_l = sqrt((2l+1)/4pi)
// (spin 0, b = 0: Z_m = conj X_m and F is real).
//
// Stage 1 (k_sht_rings, one thread per north ring and order m): d^l_{m,+-s}
// advanced by the three-term recurrence in l from the closed form at
// l0 = max(m, s), in scaled arithmetic (mantissa x 2^E) so that seeds such as
// sin^m(theta/2), which underflow near the poles, stay exact.  The mirror ring
// pi - theta uses d^l_{m,s'}(pi - t) = (-1)^{l+m} d^l_{m,-s'}(t) on the same
// recurrence.  The block's threads share m, so the recurrence coefficients and
// the scaled coefficients of a chunk of l are computed once per block into LDS.
// Stage 2 (per ring of n pixels, phi_j = phi_0 + 2 pi j / n): the orders are
// folded modulo n, G_q = sum_{k = q mod n} C_k e^{i k phi_0}, and
// F_j = sum_q G_q e^{2 pi i q j / n} is one inverse DFT of length n: radix-2
// Stockham passes when n is a power of two (the belt rings at power-of-two
// N_side), otherwise Bluestein's chirp-z form q j = (q^2 + j^2 - (j - q)^2)/2, a
// circular convolution of power-of-two length M >= 2n - 1.  Rings of equal
// transform length are batched into one set of passes; the passes run in
// global memory only until each row has split into independent transforms of
// at most 2048 points, which then finish in LDS.
#include "plan.h"
#include "healpix_ring.h"
#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <type_traits>
#include <vector>

namespace flints {

namespace {

constexpr double SHT_PI = 3.14159265358979323846;
constexpr int SHT_TPB = 256;    // threads (north rings) per block of stage 1
constexpr int SHT_CH = 256;     // l values per LDS chunk
constexpr int SCALE_BITS = 480; // rescaling step of the scaled recurrence

struct cplx {
  double re, im;
};

__device__ inline cplx cmul(cplx a, cplx b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
__device__ inline cplx cadd(cplx a, cplx b) { return {a.re + b.re, a.im + b.im}; }
__device__ inline cplx csub(cplx a, cplx b) { return {a.re - b.re, a.im - b.im}; }

// e^{i pi num / den} for integers (num reduced modulo 2 den first, exactly).
__device__ inline cplx expi_pi_ratio(int64_t num, int64_t den) {
  int64_t r = num % (2 * den);
  if (r < 0) r += 2 * den;
  double s, c;
  sincos(SHT_PI * (double)r / (double)den, &s, &c);
  return {c, s};
}

// Scaled Wigner d: value = cur * 2^E (E <= 0, a multiple of SCALE_BITS), sf = 2^E.
struct ScaledD {
  double prev, cur;
  int E;
  double sf;
};

// d^{l0}_{m, sp}(theta), l0 = max(m, |sp|), from its closed form through its
// logarithm (lc = log cos(theta/2), ls = log sin(theta/2)).
__device__ inline void seed_d(int m, int sp, double lc, double ls, ScaledD &st) {
  const int s = sp < 0 ? -sp : sp;
  double lg, sign;
  if (m >= s) {
    // d^m_{m,sp} = (-1)^{m-sp} sqrt((2m)! / ((m+sp)! (m-sp)!)) c^{m+sp} s^{m-sp}
    lg = 0.5 * (lgamma(2.0 * m + 1.0) - lgamma((double)(m + sp) + 1.0) - lgamma((double)(m - sp) + 1.0)) +
         (double)(m + sp) * lc + (double)(m - sp) * ls;
    sign = ((m - sp) & 1) ? -1.0 : 1.0;
  } else if (sp > 0) {
    // d^s_{m,s} = sqrt((2s)! / ((s+m)! (s-m)!)) c^{s+m} s^{s-m}
    lg = 0.5 * (lgamma(2.0 * s + 1.0) - lgamma((double)(s + m) + 1.0) - lgamma((double)(s - m) + 1.0)) +
         (double)(s + m) * lc + (double)(s - m) * ls;
    sign = 1.0;
  } else {
    // d^s_{m,-s} = (-1)^{m+s} sqrt((2s)! / ((s-m)! (s+m)!)) c^{s-m} s^{s+m}
    lg = 0.5 * (lgamma(2.0 * s + 1.0) - lgamma((double)(s - m) + 1.0) - lgamma((double)(s + m) + 1.0)) +
         (double)(s - m) * lc + (double)(s + m) * ls;
    sign = ((m + s) & 1) ? -1.0 : 1.0;
  }
  const double l2 = lg * 1.4426950408889634;   // log2 |d| <= 0
  const int E = SCALE_BITS * (int)floor(l2 / SCALE_BITS);
  st.E = E;
  st.cur = sign * exp2(l2 - (double)E);
  st.prev = 0.0;
  st.sf = exp2((double)E);
}

// One recurrence step with precomputed coefficients:
// d^{l+1} = a d^l - cb d^{l-1}; mantissas rescaled past 2^SCALE_BITS.
__device__ inline void step_d(double a, double cb, ScaledD &st) {
  const double next = a * st.cur - cb * st.prev;
  st.prev = st.cur;
  st.cur = next;
  if (st.E < 0 && fabs(next) > 0x1p480) {
    st.prev *= 0x1p-480;
    st.cur *= 0x1p-480;
    st.E += SCALE_BITS;
    st.sf = exp2((double)st.E);
  }
}

// The same step for a lane whose scale is 2^0 (no rescaling can be due).
__device__ inline void step_plain(double a, double cb, ScaledD &st) {
  const double next = a * st.cur - cb * st.prev;
  st.prev = st.cur;
  st.cur = next;
}

// Stage 1.  X, Z: [ring 1..4N-1][m 0..lmax] (Z unused for spin 0).
template <int S>
__global__ __launch_bounds__(SHT_TPB) void k_sht_rings(int64_t N, int lmax, const double *__restrict__ elm,
                                                       const double *__restrict__ blm, cplx *__restrict__ X,
                                                       cplx *__restrict__ Z) {
  __shared__ double sc1[SHT_CH], sc0[SHT_CH], scb[SHT_CH];
  __shared__ cplx sap[SHT_CH], sam[SHT_CH];
  const int m = blockIdx.y;
  const int npair = (int)(2 * N);
  const int p = blockIdx.x * SHT_TPB + threadIdx.x;
  const bool live = p < npair;
  const int rn = live ? p + 1 : 1;
  const Ring R = ring_geom(N, rn);
  const double x = R.z;
  const double omz = R.s * R.s / (1.0 + R.z);   // 1 - z without cancellation
  const double lc = log(sqrt(0.5 * (1.0 + R.z))), ls = log(sqrt(0.5 * omz));
  const double inv4pi = 1.0 / (4.0 * SHT_PI);
  const int l0 = m > S ? m : S;
  const int W = lmax + 1;
  const int64_t abase = (int64_t)m * (2 * lmax + 3 - m) / 2 - m;   // index of (l, m) is abase + l

  ScaledD dp, dm;
  seed_d(m, S, lc, ls, dp);
  if (S != 0) seed_d(m, -S, lc, ls, dm);
  cplx s1 = {0, 0}, s2 = {0, 0}, s3 = {0, 0}, s4 = {0, 0};   // spin 0: s1 even l, s3 odd l

  for (int lb = l0; lb <= lmax; lb += SHT_CH) {
    __syncthreads();
    {
      const int l = lb + (int)threadIdx.x;
      if (l <= lmax) {
        const double lf = l, l1 = l + 1.0, mf = m, Sf = S;
        double c1, c0, cb;
        if (l == 0) {
          c1 = 1.0; c0 = 0.0; cb = 0.0;   // d^1_00 = cos theta
        } else {
          const double den = lf * sqrt((l1 * l1 - mf * mf) * (l1 * l1 - Sf * Sf));
          c1 = (2.0 * lf + 1.0) * lf * l1 / den;
          c0 = (2.0 * lf + 1.0) * mf * Sf / den;
          cb = l1 * sqrt((lf * lf - mf * mf) * (lf * lf - Sf * Sf)) / den;
        }
        double f = sqrt((2.0 * lf + 1.0) * inv4pi);
        if (S == 1) f *= -sqrt(lf * l1);
        if (S == 2) f = -f;
        const int64_t ai = abase + l;
        // real-type fields: the m = 0 coefficients are real (imaginary parts ignored)
        const cplx e = {elm[2 * ai], m == 0 ? 0.0 : elm[2 * ai + 1]};
        const cplx b = (S != 0 && blm) ? cplx{blm[2 * ai], m == 0 ? 0.0 : blm[2 * ai + 1]} : cplx{0.0, 0.0};
        sc1[threadIdx.x] = c1;
        sc0[threadIdx.x] = c0;
        scb[threadIdx.x] = cb;
        sap[threadIdx.x] = {f * (e.re - b.im), f * (e.im + b.re)};      // f (e + i b)
        sam[threadIdx.x] = {f * (e.re + b.im), -f * (e.im - b.re)};     // f conj(e - i b)
      }
    }
    __syncthreads();
    const int cnt = min(SHT_CH, lmax - lb + 1);
    // Once every lane of the wave has left the scaled range (E = 0, 2^E = 1)
    // the chunk runs the plain recurrence: no scale factor, no rescaling test.
    const bool scaled = __any(live && (dp.E < 0 || (S != 0 && dm.E < 0)));
    auto chunk = [&](auto checked) {
      constexpr bool CHK = decltype(checked)::value;
      for (int t = 0; t < cnt; ++t) {
        const int l = lb + t;
        const cplx ap = sap[t];
        const double vp = CHK ? dp.cur * dp.sf : dp.cur;
        if (S == 0) {
          if (l & 1) { s3.re += vp * ap.re; s3.im += vp * ap.im; }
          else       { s1.re += vp * ap.re; s1.im += vp * ap.im; }
          if (CHK) step_d(sc1[t] * x, scb[t], dp);
          else step_plain(sc1[t] * x, scb[t], dp);
        } else {
          const cplx am = sam[t];
          const double vm = CHK ? dm.cur * dm.sf : dm.cur;
          const double pvp = (l & 1) ? -vp : vp, pvm = (l & 1) ? -vm : vm;
          s1.re += vm * ap.re;  s1.im += vm * ap.im;
          s2.re += vp * am.re;  s2.im += vp * am.im;
          s3.re += pvp * ap.re; s3.im += pvp * ap.im;
          s4.re += pvm * am.re; s4.im += pvm * am.im;
          const double c1x = sc1[t] * x, c0 = sc0[t], cb = scb[t];
          if (CHK) {
            step_d(c1x - c0, cb, dp);
            step_d(c1x + c0, cb, dm);
          } else {
            step_plain(c1x - c0, cb, dp);
            step_plain(c1x + c0, cb, dm);
          }
        }
      }
    };
    if (live) {
      if (scaled) chunk(std::true_type{});
      else chunk(std::false_type{});
    }
  }
  if (!live) return;
  const int rs = (int)(4 * N) - rn;
  const double sgnM = (m & 1) ? -1.0 : 1.0;
  if (S == 0) {
    // X(north) = even + odd; X(south) = (-1)^m (even - odd)
    X[(int64_t)rn * W + m] = cadd(s1, s3);
    if (rs != rn) {
      const cplx d = csub(s1, s3);
      X[(int64_t)rs * W + m] = {sgnM * d.re, sgnM * d.im};
    }
  } else {
    // north: X = (-1)^S s1, Z = s2; south: X = (-1)^(S+m) s3, Z = (-1)^m s4
    const double sgnS = (S & 1) ? -1.0 : 1.0;
    X[(int64_t)rn * W + m] = {sgnS * s1.re, sgnS * s1.im};
    Z[(int64_t)rn * W + m] = s2;
    if (rs != rn) {
      X[(int64_t)rs * W + m] = {sgnS * sgnM * s3.re, sgnS * sgnM * s3.im};
      Z[(int64_t)rs * W + m] = {sgnM * s4.re, sgnM * s4.im};
    }
  }
}

// Per ring of a batch: ring number, pixel count n, and the offsets of its
// length-M slot and (Bluestein) of the chirp spectrum for its n.
struct RingJob {
  int32_t ring, n;
  int64_t slot;
  int64_t bspec;
};

// Stage 2a: folded orders a_q = G_q (times the chirp c_q = e^{i pi q^2/n} for
// Bluestein), zero for n <= q < M.  e^{i k phi_0} with phi_0 = pi/n or 0 is
// e^{i pi kmin/n} (-1)^t along the aliases k = kmin + t n.
template <int S>
__global__ void k_fold(int64_t N, int lmax, const cplx *__restrict__ X, const cplx *__restrict__ Z,
                       const RingJob *__restrict__ jobs, int njobs, int M, int chirp, cplx *__restrict__ A) {
  const int jb = blockIdx.y;
  if (jb >= njobs) return;
  const RingJob J = jobs[jb];
  const Ring R = ring_geom(N, J.ring);
  const int W = lmax + 1;
  const bool half = R.phi0 != 0.0;
  const cplx *Xr = X + (int64_t)J.ring * W;
  const cplx *Zr = (S == 0 ? X : Z) + (int64_t)J.ring * W;
  for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < M; q += gridDim.x * blockDim.x) {
    cplx acc = {0.0, 0.0};
    if (q < J.n) {
      const int n = J.n;
      const int64_t kmin = q - (int64_t)n * ((q + lmax) / n);
      double sg = 1.0;
      for (int64_t k = kmin; k <= lmax; k += n) {
        cplx c;
        if (k >= 0) {
          c = Xr[k];
        } else {
          c = Zr[-k];
          if (S == 0) c.im = -c.im;   // Z_m = conj X_m
        }
        acc.re += sg * c.re;
        acc.im += sg * c.im;
        if (half) sg = -sg;
      }
      if (half) acc = cmul(acc, expi_pi_ratio(kmin, n));
      if (chirp) acc = cmul(acc, expi_pi_ratio((int64_t)q * q, n));
    }
    A[J.slot + q] = acc;
  }
}

// Chirp b_k = e^{-i pi k^2 / n} on a circle of length M (k and M - k), zero
// elsewhere; one row per distinct n of a Bluestein group.
__global__ void k_chirp(const int32_t *__restrict__ ns, int nn, int M, cplx *__restrict__ B) {
  const int r = blockIdx.y;
  if (r >= nn) return;
  const int n = ns[r];
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < M; k += gridDim.x * blockDim.x) {
    cplx v = {0.0, 0.0};
    const int kk = k < n ? k : (k > M - n ? M - k : -1);
    if (kk >= 0) {
      const cplx c = expi_pi_ratio((int64_t)kk * kk, n);
      v = {c.re, -c.im};
    }
    B[(int64_t)r * M + k] = v;
  }
}

// Twiddles W[t] = e^{-2 pi i t / M}, t < M / 2.
__global__ void k_roots(int M, cplx *__restrict__ Wt) {
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < M / 2; t += gridDim.x * blockDim.x) {
    const cplx c = expi_pi_ratio(2 * (int64_t)t, M);
    Wt[t] = {c.re, -c.im};
  }
}

// One radix-2 Stockham pass over `rows` transforms of length M: half length l
// of the current sub-transforms, stride m (l m = M / 2).  `inverse` takes the
// conjugate twiddles (e^{+2 pi i / M}); no normalisation.
__global__ void k_stockham(const cplx *__restrict__ in, cplx *__restrict__ out, int64_t rows, int M, int l, int m,
                           const cplx *__restrict__ Wt, int inverse) {
  const int64_t half = M / 2;
  const int64_t total = rows * half;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t row = t / half;
    const int i = (int)(t - row * half);
    const int j = i / m, k = i - j * m;
    const cplx *xr = in + row * M;
    cplx *yr = out + row * M;
    const cplx c0 = xr[k + j * m], c1 = xr[k + j * m + l * m];
    cplx w = Wt[j * m];
    if (inverse) w.im = -w.im;
    yr[k + 2 * j * m] = cadd(c0, c1);
    yr[k + 2 * j * m + m] = cmul(w, csub(c0, c1));
  }
}

// The remaining passes of a length-M transform once the Stockham stride has
// reached m0 = M / MS: each residue class r mod m0 of a row is then an
// independent length-MS transform (every butterfly of a pass with stride
// m >= m0 joins elements of one class), so the block for (r, row) gathers
// x[r + m0 t], t < MS, into LDS, runs the passes with strides 1 .. MS/2 there
// (the same butterflies and twiddles W_M^{j m} as the global passes) and
// writes the class back in place.
constexpr int FFT_LDS_N = 2048;   // sub-transform length held in LDS (2 x 32 KB)
constexpr int FFT_LDS_TPB = 256;

// Blocks go to the 8 XCDs round robin, so block b is mapped to row 8 q' + b % 8
// and residue q % m0 (q = b / 8, q' = q / m0): the m0 blocks of one row, which
// read interleaved words of the same lines, run on one XCD and share its L2.
__global__ __launch_bounds__(FFT_LDS_TPB) void k_fft_lds(cplx *__restrict__ data, int64_t rows, int M, int MS,
                                                        int m0, const cplx *__restrict__ Wt, int inverse) {
  extern __shared__ cplx sm[];
  cplx *a = sm, *b = sm + MS;
  const int64_t q = blockIdx.x / 8;
  const int r = (int)(q % m0);
  const int64_t rw = (q / m0) * 8 + blockIdx.x % 8;
  if (rw >= rows) return;
  cplx *row = data + rw * M + r;
  for (int t = threadIdx.x; t < MS; t += blockDim.x) a[t] = row[(int64_t)m0 * t];
  __syncthreads();
  for (int l = MS / 2, mm = 1; l >= 1; l >>= 1, mm <<= 1) {
    for (int i = threadIdx.x; i < MS / 2; i += blockDim.x) {
      const int j = i / mm, k = i - j * mm;
      const cplx c0 = a[k + j * mm], c1 = a[k + j * mm + l * mm];
      cplx w = Wt[(int64_t)j * mm * m0];
      if (inverse) w.im = -w.im;
      b[k + 2 * j * mm] = cadd(c0, c1);
      b[k + 2 * j * mm + mm] = cmul(w, csub(c0, c1));
    }
    __syncthreads();
    cplx *t = a;
    a = b;
    b = t;
  }
  for (int t = threadIdx.x; t < MS; t += blockDim.x) row[(int64_t)m0 * t] = a[t];
}

// A[slot] *= B[its chirp spectrum].
__global__ void k_spec_mul(const RingJob *__restrict__ jobs, int njobs, int M, cplx *__restrict__ A,
                           const cplx *__restrict__ B) {
  const int jb = blockIdx.y;
  if (jb >= njobs) return;
  const RingJob J = jobs[jb];
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < M; k += gridDim.x * blockDim.x)
    A[J.slot + k] = cmul(A[J.slot + k], B[J.bspec + k]);
}

// F_j for j < n into the map: the transform output itself (direct), or
// c_j conv_j / M (Bluestein).  Real part into plane 0; the imaginary part into
// plane 1 for spin > 0.
__global__ void k_store(const RingJob *__restrict__ jobs, int njobs, int64_t N, int M, int chirp,
                        const cplx *__restrict__ A, double *__restrict__ map, int64_t npix, int two_planes) {
  const int jb = blockIdx.y;
  if (jb >= njobs) return;
  const RingJob J = jobs[jb];
  const Ring R = ring_geom(N, J.ring);
  const double scale = chirp ? 1.0 / (double)M : 1.0;
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < J.n; j += gridDim.x * blockDim.x) {
    cplx v = A[J.slot + j];
    if (chirp) v = cmul(v, expi_pi_ratio((int64_t)j * j, J.n));
    map[R.first + j] = v.re * scale;
    if (two_planes) map[npix + R.first + j] = v.im * scale;
  }
}

// Displaced pixel centres, n' = cos|d| n + sin|d| (d_theta e_theta + d_phi e_phi) / |d|.
__global__ void k_remap(int64_t N, int64_t npix, const double *__restrict__ defl, double *__restrict__ theta,
                        double *__restrict__ phi) {
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < npix;
       p += (int64_t)gridDim.x * blockDim.x) {
    const Ring R = ring_geom(N, pix_ring(N, p));
    const double ph = R.phi0 + (double)(p - R.first) * R.dphi;
    double sp, cp;
    sincos(ph, &sp, &cp);
    const double dt = defl[p], dph = defl[npix + p];
    const double d = sqrt(dt * dt + dph * dph);
    double sd, cd;
    sincos(d, &sd, &cd);
    const double f = d > 0.0 ? sd / d : 1.0;
    const double nx = R.s * cp, ny = R.s * sp, nz = R.z;   // n
    const double tx = R.z * cp, ty = R.z * sp, tz = -R.s;  // e_theta
    const double px = -sp, py = cp;                        // e_phi
    const double x = cd * nx + f * (dt * tx + dph * px);
    const double y = cd * ny + f * (dt * ty + dph * py);
    const double z = cd * nz + f * (dt * tz);
    theta[p] = atan2(sqrt(x * x + y * y), z);
    double a = atan2(y, x);
    if (a < 0.0) a += 2.0 * SHT_PI;
    phi[p] = a;
  }
}

int next_pow2(int v) {
  int m = 1;
  while (m < v) m <<= 1;
  return m;
}

// Stream-ordered workspace from the library's pool, freed on scope exit.
struct PoolBuf {
  void *p = nullptr;
  hipStream_t s;
  explicit PoolBuf(hipStream_t st) : s(st) {}
  bool alloc(size_t bytes) {
    hipMemPool_t pool = workspace_pool();
    const hipError_t e = pool ? hipMallocFromPoolAsync(&p, bytes, pool, s) : hipMallocAsync(&p, bytes, s);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      p = nullptr;
      return false;
    }
    return true;
  }
  ~PoolBuf() {
    if (p) (void)hipFreeAsync(p, s);
  }
};

unsigned grid1d(int64_t work, int tb, int64_t cap) {
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>((work + tb - 1) / tb, cap));
}

}  // namespace

// Ring groups of one N_side on one device: rings of equal transform length
// (direct or Bluestein), with their device job tables.  Built once per
// (device, N_side) with synchronous copies and kept for the process lifetime
// (a few dozen bytes per ring).
struct SynthGroup {
  int M, chirp;
  int64_t rowsA, rowsB;
  const RingJob *djobs;
  const int32_t *dns;
};

static int ring_groups(int64_t N, std::vector<SynthGroup> &out) {
  static std::mutex mu;
  static std::map<std::pair<int, int64_t>, std::vector<SynthGroup>> cache;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) {
    set_error("hipGetDevice failed");
    return FLINTS_EDEVICE;
  }
  std::lock_guard<std::mutex> g(mu);
  auto it = cache.find({dev, N});
  if (it != cache.end()) {
    out = it->second;
    return FLINTS_OK;
  }
  const int nring = (int)(4 * N - 1);
  std::map<std::pair<int, int>, std::vector<int>> groups;   // (M, chirp) -> rings
  for (int r = 1; r <= nring; ++r) {
    const int n = ring_geom(N, r).n;
    const bool pow2 = (n & (n - 1)) == 0;
    groups[{pow2 ? n : next_pow2(2 * n - 1), pow2 ? 0 : 1}].push_back(r);
  }
  std::vector<RingJob> jobs;
  std::vector<int32_t> ns;
  std::vector<SynthGroup> gl;
  std::vector<std::pair<size_t, size_t>> offs;   // first job, first n of each group
  for (auto &g2 : groups) {
    const int M = g2.first.first, chirp = g2.first.second;
    std::map<int, int> nidx;
    const size_t j0 = jobs.size(), n0 = ns.size();
    for (size_t i = 0; i < g2.second.size(); ++i) {
      const int n = ring_geom(N, g2.second[i]).n;
      if (chirp && !nidx.count(n)) {
        nidx[n] = (int)(ns.size() - n0);
        ns.push_back(n);
      }
      jobs.push_back({g2.second[i], n, (int64_t)i * M, chirp ? (int64_t)nidx[n] * M : 0});
    }
    gl.push_back({M, chirp, (int64_t)(jobs.size() - j0), (int64_t)(ns.size() - n0), nullptr, nullptr});
    offs.push_back({j0, n0});
  }
  const size_t jb = sizeof(RingJob) * jobs.size(), nb = sizeof(int32_t) * std::max<size_t>(ns.size(), 1);
  char *d = nullptr;
  if (hipMalloc((void **)&d, jb + nb) != hipSuccess) {
    (void)hipGetLastError();
    set_error("allocation of the ring tables failed");
    return FLINTS_ENOMEM;
  }
  if (hipMemcpy(d, jobs.data(), jb, hipMemcpyHostToDevice) != hipSuccess ||
      (!ns.empty() && hipMemcpy(d + jb, ns.data(), sizeof(int32_t) * ns.size(), hipMemcpyHostToDevice) != hipSuccess)) {
    (void)hipFree(d);
    set_error("upload of the ring tables failed");
    return FLINTS_EDEVICE;
  }
  for (size_t i = 0; i < gl.size(); ++i) {
    gl[i].djobs = (const RingJob *)d + offs[i].first;
    gl[i].dns = (const int32_t *)(d + jb) + offs[i].second;
  }
  cache[{dev, N}] = gl;
  out = gl;
  return FLINTS_OK;
}

int launch_synthesize(int64_t N, int lmax, int spin, const double *elm, const double *blm, double *map,
                      hipStream_t s) {
  hipFuncSetAttribute((const void *)k_fft_lds, hipFuncAttributeMaxDynamicSharedMemorySize,
                      2 * FFT_LDS_N * (int)sizeof(cplx));
  std::vector<SynthGroup> groups;
  const int rc = ring_groups(N, groups);
  if (rc != FLINTS_OK) return rc;
  const int nring = (int)(4 * N - 1);
  const int W = lmax + 1;
  const int64_t npix = 12 * N * N;
  PoolBuf xz(s);
  const size_t rowsXZ = (size_t)(nring + 1) * W;
  if (!xz.alloc(sizeof(cplx) * rowsXZ * (spin == 0 ? 1 : 2))) {
    set_error("workspace allocation for the synthesis failed");
    return FLINTS_ENOMEM;
  }
  cplx *X = (cplx *)xz.p, *Z = spin == 0 ? nullptr : X + rowsXZ;
  {
    const dim3 grid((unsigned)((2 * N + SHT_TPB - 1) / SHT_TPB), (unsigned)W);
    if (spin == 0) hipLaunchKernelGGL(k_sht_rings<0>, grid, dim3(SHT_TPB), 0, s, N, lmax, elm, blm, X, Z);
    else if (spin == 1) hipLaunchKernelGGL(k_sht_rings<1>, grid, dim3(SHT_TPB), 0, s, N, lmax, elm, blm, X, Z);
    else hipLaunchKernelGGL(k_sht_rings<2>, grid, dim3(SHT_TPB), 0, s, N, lmax, elm, blm, X, Z);
  }
  const int tb = 256;
  for (const SynthGroup &g : groups) {
    const int M = g.M, chirp = g.chirp;
    const int64_t rowsA = g.rowsA, rowsB = g.rowsB;
    PoolBuf buf(s);
    if (!buf.alloc(sizeof(cplx) * ((size_t)(2 * rowsA + 2 * rowsB) * M + std::max(M / 2, 1)))) {
      set_error("workspace allocation for the ring transforms failed");
      return FLINTS_ENOMEM;
    }
    cplx *A = (cplx *)buf.p, *A2 = A + rowsA * M, *B = A2 + rowsA * M, *B2 = B + rowsB * M;
    cplx *Wt = B2 + rowsB * M;
    const int nj = (int)rowsA;
    const unsigned gx = grid1d(M, tb, 64);
    hipLaunchKernelGGL(k_roots, dim3(grid1d(M / 2, tb, 256)), dim3(tb), 0, s, M, Wt);
    if (spin == 0) hipLaunchKernelGGL(k_fold<0>, dim3(gx, nj), dim3(tb), 0, s, N, lmax, X, Z, g.djobs, nj, M, chirp, A);
    else hipLaunchKernelGGL(k_fold<1>, dim3(gx, nj), dim3(tb), 0, s, N, lmax, X, Z, g.djobs, nj, M, chirp, A);
    // global radix-2 passes while the stride is below m0, then the rest in LDS
    const int MS = std::min(M, FFT_LDS_N), m0 = M / MS;
    auto fft = [&](cplx *&src, cplx *&dst, int64_t rows, int inverse) {
      const unsigned blocks = grid1d(rows * (M / 2), tb, 65536);
      for (int l = M / 2, m = 1; m < m0; l >>= 1, m <<= 1) {
        hipLaunchKernelGGL(k_stockham, dim3(blocks), dim3(tb), 0, s, src, dst, rows, M, l, m, Wt, inverse);
        std::swap(src, dst);
      }
      const int64_t nblk = ((rows + 7) / 8) * 8 * m0;
      hipLaunchKernelGGL(k_fft_lds, dim3((unsigned)nblk), dim3(FFT_LDS_TPB), 2 * MS * sizeof(cplx), s, src, rows,
                         M, MS, m0, Wt, inverse);
    };
    cplx *a = A, *a2 = A2;
    if (chirp) {
      cplx *b = B, *b2 = B2;
      hipLaunchKernelGGL(k_chirp, dim3(gx, (unsigned)rowsB), dim3(tb), 0, s, g.dns, (int)rowsB, M, B);
      fft(a, a2, rowsA, 0);
      fft(b, b2, rowsB, 0);
      hipLaunchKernelGGL(k_spec_mul, dim3(gx, nj), dim3(tb), 0, s, g.djobs, nj, M, a, b);
    }
    fft(a, a2, rowsA, 1);
    hipLaunchKernelGGL(k_store, dim3(gx, nj), dim3(tb), 0, s, g.djobs, nj, N, M, chirp, a, map, npix,
                       spin != 0 ? 1 : 0);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
      set_error(std::string("synthesis kernel launch failed: ") + hipGetErrorString(e));
      return FLINTS_EDEVICE;
    }
  }
  return FLINTS_OK;
}

int launch_lensed_directions(int64_t N, const double *defl, double *theta, double *phi, hipStream_t s) {
  const int64_t npix = 12 * N * N;
  hipLaunchKernelGGL(k_remap, dim3(grid1d(npix, 256, 65536)), dim3(256), 0, s, N, npix, defl, theta, phi);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    set_error(std::string("displacement kernel launch failed: ") + hipGetErrorString(e));
    return FLINTS_EDEVICE;
  }
  return FLINTS_OK;
}

}  // namespace flints
