// Issue-rate probe of the gfx950 vector ALU, for the roofline of the pair
// kernel.  Not part of the ordering: bench.py loads this small separate
// library (liblingam_probe.so) to measure, on the machine it runs on,
//   * FP32 fused multiply-add lane operations per second (v_fma_f32; the
//     library is built with packed FP32 instruction selection switched off,
//     so this is the unpacked rate the pair kernel's arithmetic runs at),
//   * v_exp_f32 lane operations per second,
//   * evaluation-shaped work per second: 7 FP32 FMAs + 2 v_exp_f32 per unit,
//     all independent, i.e. the instruction mix of one pair evaluation
//     without its loads.
// Every kernel keeps eight independent dependency chains per lane and enough
// waves per SIMD that issue, not latency, bounds it; results are written out
// so that nothing is removed as dead code.
#include <hip/hip_runtime.h>

#include <stdint.h>

namespace {

constexpr int kThreads = 256;
constexpr int kUnroll = 16;

__global__ __launch_bounds__(kThreads) void k_probe_fma(float* out, int iters, float a, float b) {
  const int gid = blockIdx.x * kThreads + threadIdx.x;
  float x[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) x[k] = 1e-3f * (float)(gid + k);
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
#pragma unroll
      for (int k = 0; k < 8; ++k) x[k] = fmaf(x[k], a, b);
    }
  }
  float s = 0.f;
#pragma unroll
  for (int k = 0; k < 8; ++k) s += x[k];
  out[gid] = s;
}

__global__ __launch_bounds__(kThreads) void k_probe_exp(float* out, int iters) {
  const int gid = blockIdx.x * kThreads + threadIdx.x;
  float x[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) x[k] = 1e-3f * (float)((gid + k) & 1023);
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
#pragma unroll
      for (int k = 0; k < 8; ++k) x[k] = __builtin_amdgcn_exp2f(-x[k]);  // stays in (0, 1]
    }
  }
  float s = 0.f;
#pragma unroll
  for (int k = 0; k < 8; ++k) s += x[k];
  out[gid] = s;
}

// The evaluation mix: each pass of the inner loop does 7 FMAs on each of 8
// chains and 2 exp2 on each of 8 other chains, i.e. 8 units of 7 FMAs + 2
// exp2 (the pair kernel's 7 VALU + 2 transcendentals per evaluation).
__global__ __launch_bounds__(kThreads) void k_probe_mix(float* out, int iters, float a, float b) {
  const int gid = blockIdx.x * kThreads + threadIdx.x;
  float f[8], e[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    f[k] = 1e-3f * (float)(gid + k);
    e[k] = 1e-3f * (float)((gid + 3 * k) & 1023);
  }
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int u = 0; u < kUnroll / 8; ++u) {
#pragma unroll
      for (int r = 0; r < 7; ++r) {
#pragma unroll
        for (int k = 0; k < 8; ++k) f[k] = fmaf(f[k], a, b);
      }
#pragma unroll
      for (int r = 0; r < 2; ++r) {
#pragma unroll
        for (int k = 0; k < 8; ++k) e[k] = __builtin_amdgcn_exp2f(-e[k]);
      }
    }
  }
  float s = 0.f;
#pragma unroll
  for (int k = 0; k < 8; ++k) s += f[k] + e[k];
  out[gid] = s;
}

}  // namespace

extern "C" {

/*
 * Measures the three rates above on the current device and writes them to
 * the host array out[3]: FP32 FMA lane-ops/s, v_exp_f32 lane-ops/s, and
 * evaluation-shaped units/s (7 FMA + 2 exp2 each).  Allocates a small device
 * buffer (measurement only).
 * Returns 0 on success, a HIP error code otherwise.
 */
int lingam_probe_rates(double* out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return (int)e;
  int cu = 0;
  e = hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return (int)e;
  const int blocks = cu * 16;  // 4096 threads per CU: 16 waves per SIMD
  const int iters = 2048;
  float* buf = nullptr;
  e = hipMalloc(&buf, sizeof(float) * (size_t)blocks * kThreads);
  if (e != hipSuccess) return (int)e;
  hipEvent_t t0, t1;
  (void)hipEventCreate(&t0);
  (void)hipEventCreate(&t1);
  const double lanes = (double)blocks * kThreads * iters;
  double ms[3] = {0, 0, 0};
  for (int which = 0; which < 3; ++which) {
    for (int rep = 0; rep < 2; ++rep) {  // the first launch warms up
      (void)hipEventRecord(t0, nullptr);
      if (which == 0)
        hipLaunchKernelGGL(k_probe_fma, dim3(blocks), dim3(kThreads), 0, nullptr, buf, iters,
                           0.999f, 1e-4f);
      else if (which == 1)
        hipLaunchKernelGGL(k_probe_exp, dim3(blocks), dim3(kThreads), 0, nullptr, buf, iters);
      else
        hipLaunchKernelGGL(k_probe_mix, dim3(blocks), dim3(kThreads), 0, nullptr, buf, iters,
                           0.999f, 1e-4f);
      (void)hipEventRecord(t1, nullptr);
      e = hipEventSynchronize(t1);
      if (e != hipSuccess) break;
      float f = 0.f;
      (void)hipEventElapsedTime(&f, t0, t1);
      ms[which] = f;
    }
    if (e != hipSuccess) break;
  }
  (void)hipEventDestroy(t0);
  (void)hipEventDestroy(t1);
  (void)hipFree(buf);
  if (e != hipSuccess) return (int)e;
  out[0] = lanes * kUnroll * 8 / (ms[0] * 1e-3);
  out[1] = lanes * kUnroll * 8 / (ms[1] * 1e-3);
  out[2] = lanes * (kUnroll / 8) * 8 / (ms[2] * 1e-3);
  return 0;
}

}  // extern "C"
