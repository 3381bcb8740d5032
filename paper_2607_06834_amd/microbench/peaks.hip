// Measured ceilings of one MI355X: FP64 MFMA 16x16x4, FP64 vector FMA, both
// issued together from the same waves, and a device-to-device streaming copy.
// Prints one JSON object.  Every kernel runs a fixed number of iterations and
// writes its accumulators so that no work is optimised away.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>

using v4d = double __attribute__((ext_vector_type(4)));

#define CK(x)                                                              \
  do {                                                                     \
    hipError_t e_ = (x);                                                   \
    if (e_ != hipSuccess) {                                                \
      std::fprintf(stderr, "%s: %s\n", #x, hipGetErrorString(e_));        \
      std::exit(1);                                                        \
    }                                                                      \
  } while (0)

constexpr int kIter = 4096;

__global__ __launch_bounds__(256) void k_mfma(double *out, double seed) {
  const double a = seed + threadIdx.x * 1e-3, b = seed - threadIdx.x * 1e-3;
  v4d c[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) c[k] = v4d{0.0, 0.0, 0.0, 0.0};
  for (int it = 0; it < kIter; ++it) {
#pragma unroll
    for (int k = 0; k < 8; ++k) c[k] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c[k], 0, 0, 0);
  }
  double s = 0.0;
#pragma unroll
  for (int k = 0; k < 8; ++k) s += c[k][0] + c[k][1] + c[k][2] + c[k][3];
  out[blockIdx.x * 256 + threadIdx.x] = s;
}

__global__ __launch_bounds__(256) void k_valu(double *out, double seed) {
  double x[8];
  const double m = 1.0 + 1e-12 * threadIdx.x, ad = seed * 1e-9;
#pragma unroll
  for (int k = 0; k < 8; ++k) x[k] = seed + k;
  for (int it = 0; it < kIter; ++it) {
#pragma unroll
    for (int k = 0; k < 8; ++k) x[k] = __builtin_fma(x[k], m, ad);
  }
  double s = 0.0;
#pragma unroll
  for (int k = 0; k < 8; ++k) s += x[k];
  out[blockIdx.x * 256 + threadIdx.x] = s;
}

// MFMA and vector FMA chains interleaved in the same wave.
__global__ __launch_bounds__(256) void k_both(double *out, double seed) {
  const double a = seed + threadIdx.x * 1e-3, b = seed - threadIdx.x * 1e-3;
  v4d c[8];
  double x[8];
  const double m = 1.0 + 1e-12 * threadIdx.x, ad = seed * 1e-9;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    c[k] = v4d{0.0, 0.0, 0.0, 0.0};
    x[k] = seed + k;
  }
  for (int it = 0; it < kIter; ++it) {
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      c[k] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c[k], 0, 0, 0);
#pragma unroll
      for (int r = 0; r < 4; ++r) x[(k + r) & 7] = __builtin_fma(x[(k + r) & 7], m, ad);
    }
  }
  double s = 0.0;
#pragma unroll
  for (int k = 0; k < 8; ++k) s += c[k][0] + c[k][1] + c[k][2] + c[k][3] + x[k];
  out[blockIdx.x * 256 + threadIdx.x] = s;
}

__global__ __launch_bounds__(256) void k_copy(const double2 *__restrict__ src, double2 *__restrict__ dst,
                                              size_t n) {
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256)
    dst[i] = src[i];
}

template <typename F>
float time_ms(F f, int reps) {
  hipEvent_t a, b;
  CK(hipEventCreate(&a));
  CK(hipEventCreate(&b));
  f();
  CK(hipDeviceSynchronize());
  CK(hipEventRecord(a));
  for (int r = 0; r < reps; ++r) f();
  CK(hipEventRecord(b));
  CK(hipEventSynchronize(b));
  float ms = 0.f;
  CK(hipEventElapsedTime(&ms, a, b));
  return ms / reps;
}

int main() {
  hipDeviceProp_t prop;
  CK(hipGetDeviceProperties(&prop, 0));
  const int cus = prop.multiProcessorCount;
  const int blocks = cus * 8;                 // 8 blocks x 4 waves per CU
  double *out;
  CK(hipMalloc(&out, (size_t)blocks * 256 * sizeof(double)));
  const double waves = (double)blocks * 4;
  const double mfma_flops = waves * kIter * 8 * (16.0 * 16 * 4 * 2);
  const double valu_flops = (double)blocks * 256 * kIter * 8 * 2.0;
  const double both_valu = (double)blocks * 256 * kIter * 8 * 4 * 2.0;
  const float t_mfma = time_ms([&] { hipLaunchKernelGGL(k_mfma, dim3(blocks), dim3(256), 0, 0, out, 1.0); }, 5);
  const float t_valu = time_ms([&] { hipLaunchKernelGGL(k_valu, dim3(blocks), dim3(256), 0, 0, out, 1.0); }, 5);
  const float t_both = time_ms([&] { hipLaunchKernelGGL(k_both, dim3(blocks), dim3(256), 0, 0, out, 1.0); }, 5);
  const size_t nbytes = (size_t)1 << 31;      // 2 GiB each way
  double2 *src, *dst;
  CK(hipMalloc(&src, nbytes));
  CK(hipMalloc(&dst, nbytes));
  CK(hipMemset(src, 0, nbytes));
  const size_t n2 = nbytes / sizeof(double2);
  const float t_copy = time_ms([&] {
    hipLaunchKernelGGL(k_copy, dim3(cus * 32), dim3(256), 0, 0, src, dst, n2);
  }, 5);
  std::printf("{\"cus\": %d, \"clock_mhz\": %d, "
              "\"mfma_f64_tflops\": %.2f, \"valu_f64_tflops\": %.2f, "
              "\"mfma_plus_valu_tflops\": %.2f, \"mfma_part_tflops\": %.2f, "
              "\"copy_gbs\": %.1f}\n",
              cus, prop.clockRate / 1000, mfma_flops / (t_mfma * 1e-3) / 1e12,
              valu_flops / (t_valu * 1e-3) / 1e12,
              (mfma_flops + both_valu) / (t_both * 1e-3) / 1e12,
              mfma_flops / (t_both * 1e-3) / 1e12, 2.0 * nbytes / (t_copy * 1e-3) / 1e9);
  CK(hipFree(src));
  CK(hipFree(dst));
  CK(hipFree(out));
  return 0;
}
