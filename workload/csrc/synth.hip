// Input generation only (not part of the interpolation library): the Legendre
// stage of a spin-s HEALPix synthesis on the GPU.
//
// For every ring r (colatitude theta_r) and order m >= 0 it accumulates
//   A[m][r] = sum_l coef[l][m] (d^l_{m,-s} + d^l_{m,s})(theta_r)
//   B[m][r] = sum_l coef[l][m] (d^l_{m,-s} - d^l_{m,s})(theta_r)
// (complex coef, double precision) with the three-term l-recurrence of the
// Wigner d functions, started at l0 = max(m, s) from the closed-form seed and run
// in scaled arithmetic (value = mantissa * 2^E) so seeds that underflow double
// precision near the poles stay exact.  One thread per (ring, m).
#include <hip/hip_runtime.h>
#include <math.h>

struct DState {
  double prev, cur;
  int E;
};

__device__ inline void seed(int m, int mp, double lc, double ls, DState &st) {
  const int s = mp < 0 ? -mp : mp;
  double logv, sign;
  if (m >= s) {
    // d^m_{m,mp} = (-1)^{m-mp} sqrt(C(2m, m+mp)) c^{m+mp} s^{m-mp}
    logv = 0.5 * (lgamma(2.0 * m + 1.0) - lgamma((double)(m + mp) + 1.0) - lgamma((double)(m - mp) + 1.0)) +
           (double)(m + mp) * lc + (double)(m - mp) * ls;
    sign = ((m - mp) & 1) ? -1.0 : 1.0;
  } else if (mp >= 0) {
    // d^s_{m,s} = sqrt(C(2s, s+m)) c^{s+m} s^{s-m}
    logv = 0.5 * (lgamma(2.0 * s + 1.0) - lgamma((double)(s + m) + 1.0) - lgamma((double)(s - m) + 1.0)) +
           (double)(s + m) * lc + (double)(s - m) * ls;
    sign = 1.0;
  } else {
    // d^s_{m,-s} = (-1)^{m+s} sqrt(C(2s, s-m)) c^{s-m} s^{s+m}
    logv = 0.5 * (lgamma(2.0 * s + 1.0) - lgamma((double)(s - m) + 1.0) - lgamma((double)(s + m) + 1.0)) +
           (double)(s - m) * lc + (double)(s + m) * ls;
    sign = ((m + s) & 1) ? -1.0 : 1.0;
  }
  const double l2 = logv * 1.4426950408889634;  // log2
  const double E = floor(l2);
  st.E = (int)E;
  st.cur = sign * exp2(l2 - E);
  st.prev = 0.0;
}

// advance d^L -> d^{L+1}
__device__ inline void step(int L, int m, int mp, double x, DState &st) {
  double nw;
  if (L == 0) {
    nw = x * st.cur;  // only reached for m = mp = 0: d^1_00 = cos(theta)
  } else {
    const double dm = (double)m, dmp = (double)mp, dl = (double)L;
    const double a1 = (2.0 * dl + 1.0) * (dl * (dl + 1.0) * x - dm * dmp);
    const double c1 = (dl + 1.0) * sqrt(fmax((dl * dl - dm * dm) * (dl * dl - dmp * dmp), 0.0));
    const double den = dl * sqrt(((dl + 1.0) * (dl + 1.0) - dm * dm) * ((dl + 1.0) * (dl + 1.0) - dmp * dmp));
    nw = (a1 * st.cur - c1 * st.prev) / den;
  }
  st.prev = st.cur;
  st.cur = nw;
  if (fabs(nw) > 0x1p200) {
    st.cur *= 0x1p-200;
    st.prev *= 0x1p-200;
    st.E += 200;
  }
}

extern "C" __global__ void k_wigner_sums(const double *__restrict__ coef, int lmax, int s,
                                         const double *__restrict__ theta, int R,
                                         double *__restrict__ A, double *__restrict__ B) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  const int m = blockIdx.y;
  if (r >= R || m > lmax) return;
  const double th = theta[r];
  const double x = cos(th);
  const double lc = log(cos(0.5 * th));
  const double ls = log(sin(0.5 * th));
  const int l0 = m > s ? m : s;
  DState dm, dp;
  seed(m, -s, lc, ls, dm);
  seed(m, s, lc, ls, dp);
  double ar = 0.0, ai = 0.0, br = 0.0, bi = 0.0;
  const size_t stride = (size_t)(lmax + 1) * 2;
  for (int l = l0; l <= lmax; ++l) {
    if (l > l0) {
      step(l - 1, m, -s, x, dm);
      if (s != 0) step(l - 1, m, s, x, dp);
      else dp = dm;
    }
    const double vm = ldexp(dm.cur, dm.E);
    const double vp = (s != 0) ? ldexp(dp.cur, dp.E) : vm;
    const double cr = coef[(size_t)l * stride + 2 * m];
    const double ci = coef[(size_t)l * stride + 2 * m + 1];
    const double sp = vm + vp, sm = vm - vp;
    ar += cr * sp; ai += ci * sp;
    br += cr * sm; bi += ci * sm;
  }
  const size_t o = ((size_t)m * R + r) * 2;
  A[o] = ar; A[o + 1] = ai;
  if (B) { B[o] = br; B[o + 1] = bi; }
}

// Host launcher: returns 0 or the HIP error code.
extern "C" int synth_wigner_sums(const double *coef, int lmax, int s, const double *theta, int R,
                                 double *A, double *B, void *stream) {
  if (R <= 0 || lmax < 0) return 0;
  (void)hipGetLastError();   // an earlier call's error is not this launch's
  const int threads = 128;
  dim3 grid((R + threads - 1) / threads, lmax + 1, 1);
  hipLaunchKernelGGL(k_wigner_sums, grid, dim3(threads), 0, (hipStream_t)stream, coef, lmax, s,
                     theta, R, A, B);
  return (int)hipGetLastError();
}
