// Measured ceilings of the device (diagnostics for the roofline report):
// register-resident matrix-core loops and an HBM triad far larger than the
// 256 MB Infinity Cache.
#include "gemm.h"

namespace fr {

template <typename T, int CH>
__global__ __launch_bounds__(256) void mfma_loop_kernel(int iters, T seed, double *sink) {
  typedef typename Mma<T>::acc_t acc_t;
  const int lane = threadIdx.x & 63;
  T a = seed + (T)(lane * 1e-3), b = seed - (T)(lane * 1e-3);
  acc_t acc[CH];
#pragma unroll
  for (int c = 0; c < CH; ++c) acc[c] = acc_t{0, 0, 0, 0};
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int c = 0; c < CH; ++c) acc[c] = Mma<T>::run(a, b, acc[c]);
  }
  double s = 0;
#pragma unroll
  for (int c = 0; c < CH; ++c) s += (double)(acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3]);
  if (s == 12345.678) sink[0] = s;  // never true for the seeds used; keeps the loop live
}

// One double per thread over a grid that covers the arrays: on MI355X this
// form streams faster (6.2 TB/s) than a grid-stride loop over 32-byte
// elements (5.2-5.5 TB/s), and nontemporal hints only slow it.
__global__ __launch_bounds__(256) void triad_kernel(const double *__restrict__ b,
                                                    const double *__restrict__ c,
                                                    double *__restrict__ a, double s, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) a[i] = b[i] + s * c[i];
}

// kind 0: HBM triad GB/s; 1: FP64 MFMA TFLOP/s; 2: FP32 MFMA TFLOP/s
hipError_t measure_ceiling(int kind, double *value, hipStream_t s) {
  hipEvent_t e0, e1;
  hipError_t err;
  if ((err = hipEventCreate(&e0)) != hipSuccess) return err;
  if ((err = hipEventCreate(&e1)) != hipSuccess) return err;
  float ms = 0;
  if (kind == 0) {
    const int64_t n = (int64_t)1 << 28;  // 256 Mi doubles = 2 GiB per array
    double *a = nullptr, *b = nullptr, *c = nullptr;
    if ((err = hipMalloc(&a, n * sizeof(double))) != hipSuccess) return err;
    if ((err = hipMalloc(&b, n * sizeof(double))) != hipSuccess) { hipFree(a); return err; }
    if ((err = hipMalloc(&c, n * sizeof(double))) != hipSuccess) { hipFree(a); hipFree(b); return err; }
    hipMemsetAsync(b, 0, n * sizeof(double), s);
    hipMemsetAsync(c, 0, n * sizeof(double), s);
    const unsigned grid = (unsigned)(n / 256);
    for (int w = 0; w < 2; ++w) triad_kernel<<<grid, 256, 0, s>>>(b, c, a, 0.5, n);
    hipEventRecord(e0, s);
    const int reps = 10;
    for (int w = 0; w < reps; ++w) triad_kernel<<<grid, 256, 0, s>>>(b, c, a, 0.5, n);
    hipEventRecord(e1, s);
    hipEventSynchronize(e1);
    hipEventElapsedTime(&ms, e0, e1);
    *value = 3.0 * n * sizeof(double) * reps / (ms * 1e-3) / 1e9;
    hipFree(a); hipFree(b); hipFree(c);
  } else {
    double *sink = nullptr;
    if ((err = hipMalloc(&sink, 8)) != hipSuccess) return err;
    const int iters = 4096, CH = 8;
    const unsigned grid = 256 * 8;  // 8 workgroups (32 waves) per CU
    auto run = [&](int reps) {
      for (int w = 0; w < reps; ++w) {
        if (kind == 1) mfma_loop_kernel<double, CH><<<grid, 256, 0, s>>>(iters, 1.0, sink);
        else mfma_loop_kernel<float, CH><<<grid, 256, 0, s>>>(iters, 1.0f, sink);
      }
    };
    run(1);
    hipEventRecord(e0, s);
    run(3);
    hipEventRecord(e1, s);
    hipEventSynchronize(e1);
    hipEventElapsedTime(&ms, e0, e1);
    const double flops = 3.0 * grid * 4 * (double)iters * CH * 16 * 16 * 4 * 2;
    *value = flops / (ms * 1e-3) / 1e12;
    hipFree(sink);
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  return hipGetLastError();
}

}  // namespace fr
