// Machine-peak probe for the roofline figures: FP64 vector FMA rate, FP64
// matrix-core (MFMA 16x16x4) rate and device-to-device copy bandwidth, each
// timed with HIP events (best of three after a warm-up).  Prints one JSON line.
// A stand-alone program; the interpolation library does not use it.
#include <hip/hip_runtime.h>
#include <algorithm>
#include <cstdio>

typedef double dbl4 __attribute__((ext_vector_type(4)));

constexpr int ITERS = 4096;
constexpr int CHAINS = 16;

#define CHECK(x)                                                                  \
  do {                                                                            \
    hipError_t e_ = (x);                                                          \
    if (e_ != hipSuccess) {                                                       \
      std::fprintf(stderr, "%s failed: %s\n", #x, hipGetErrorString(e_));         \
      return 1;                                                                   \
    }                                                                             \
  } while (0)

// CHAINS independent FMA chains per lane: ITERS * CHAINS v_fma_f64 per lane.
__global__ void k_fma64(double *out, double s, double c) {
  double a[CHAINS];
#pragma unroll
  for (int i = 0; i < CHAINS; ++i) a[i] = threadIdx.x * 1e-3 + i;
  for (int it = 0; it < ITERS; ++it) {
#pragma unroll
    for (int i = 0; i < CHAINS; ++i) a[i] = fma(a[i], s, c);
  }
  double t = 0.0;
#pragma unroll
  for (int i = 0; i < CHAINS; ++i) t += a[i];
  out[(size_t)blockIdx.x * blockDim.x + threadIdx.x] = t;
}

// Four independent accumulators per wave: ITERS v_mfma_f64_16x16x4f64 per wave
// (2 * 16 * 16 * 4 flops each).
__global__ void k_mfma64(double *out, double s) {
  dbl4 c0 = {0.0, 0.0, 0.0, 0.0}, c1 = c0, c2 = c0, c3 = c0;
  const double a = threadIdx.x * 1e-3, b = s;
  for (int it = 0; it < ITERS / 4; ++it) {
    c0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c0, 0, 0, 0);
    c1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c1, 0, 0, 0);
    c2 = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c2, 0, 0, 0);
    c3 = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c3, 0, 0, 0);
  }
  out[(size_t)blockIdx.x * blockDim.x + threadIdx.x] = c0[0] + c1[1] + c2[2] + c3[3];
}

// Grid-stride copy of n 16-byte elements.
__global__ void k_copy(const double2 *__restrict__ src, double2 *__restrict__ dst, size_t n) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) dst[i] = src[i];
}

template <typename F>
static float best_ms(F launch) {
  hipEvent_t e0, e1;
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);
  launch();   // warm-up
  float best = 1e30f;
  for (int r = 0; r < 3; ++r) {
    (void)hipEventRecord(e0, nullptr);
    launch();
    (void)hipEventRecord(e1, nullptr);
    (void)hipEventSynchronize(e1);
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    best = std::min(best, ms);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return best;
}

int main() {
  int dev = 0, ncu = 0, clk = 0;
  CHECK(hipGetDevice(&dev));
  CHECK(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
  CHECK(hipDeviceGetAttribute(&clk, hipDeviceAttributeClockRate, dev));
  const int threads = 256;            // 4 waves per block
  const int blocks = ncu * 8;         // 32 waves per CU, 8 per SIMD
  const size_t nthr = (size_t)blocks * threads;
  double *out = nullptr;
  CHECK(hipMalloc(&out, nthr * sizeof(double)));

  const float ms_fma = best_ms([&] { hipLaunchKernelGGL(k_fma64, dim3(blocks), dim3(threads), 0, nullptr, out, 0.999999, 1e-9); });
  CHECK(hipGetLastError());
  const double fma_tf = 2.0 * CHAINS * ITERS * (double)nthr / (ms_fma * 1e-3) / 1e12;

  const float ms_mfma = best_ms([&] { hipLaunchKernelGGL(k_mfma64, dim3(blocks), dim3(threads), 0, nullptr, out, 0.999999); });
  CHECK(hipGetLastError());
  const double waves = (double)nthr / 64.0;
  const double mfma_tf = 2048.0 * ITERS * waves / (ms_mfma * 1e-3) / 1e12;

  const size_t bytes = size_t(2) << 30;   // 2 GiB read + 2 GiB written
  const size_t n = bytes / sizeof(double2);
  double2 *src = nullptr, *dst = nullptr;
  CHECK(hipMalloc(&src, bytes));
  CHECK(hipMalloc(&dst, bytes));
  CHECK(hipMemset(src, 0, bytes));
  const int cblocks = ncu * 16;
  const float ms_copy = best_ms([&] { hipLaunchKernelGGL(k_copy, dim3(cblocks), dim3(256), 0, nullptr, src, dst, n); });
  CHECK(hipGetLastError());
  const double copy_gbs = 2.0 * (double)bytes / (ms_copy * 1e-3) / 1e9;
  CHECK(hipDeviceSynchronize());

  std::printf("{\"cus\": %d, \"clock_mhz\": %.0f, \"fp64_vector_fma_tflops\": %.2f, "
              "\"fp64_mfma_16x16x4_tflops\": %.2f, \"copy_gb_per_s\": %.0f, "
              "\"fma_ms\": %.3f, \"mfma_ms\": %.3f, \"copy_ms\": %.3f, \"copy_bytes_each_way\": %zu}\n",
              ncu, clk / 1e3, fma_tf, mfma_tf, copy_gbs, ms_fma, ms_mfma, ms_copy, bytes);
  (void)hipFree(src);
  (void)hipFree(dst);
  (void)hipFree(out);
  return 0;
}
