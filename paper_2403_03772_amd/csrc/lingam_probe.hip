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
//
// A second probe prices the two ways of separating the phases of an ordering
// step (pair moments, selection, residual update), which depend on each other
// across the whole device: a kernel boundary, or a grid-wide barrier inside
// one persistent kernel.  See lingam_probe_sync.
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

// One workgroup-sized step of no work: each workgroup bumps a counter of its
// own, so consecutive launches touch the same memory as a real step would.
__global__ __launch_bounds__(kThreads) void k_probe_touch(unsigned* cnt) {
  if (threadIdx.x == 0) cnt[blockIdx.x] += 1u;
}

// `rounds` grid-wide barriers in one launch (all workgroups co-resident: the
// host launches it cooperatively).  In a barrier each workgroup bumps its own
// counter (the phase's work) and arrives; its wave 0 then waits, polling
// without a cache invalidate, and takes one device-scope acquire at the end.
//   kGroups == 1: every workgroup adds to one arrival count (device scope,
//                 release) and waits for rounds-so-far x workgroups;
//   kGroups == 8: workgroup b arrives on the count of group b mod 8 (the
//                 compute die it is dispatched to; the eight counts lie in
//                 different 256-byte blocks), and the group's last arrival
//                 adds one to the top count, which the waits poll.
// Arrival counts only grow, so no reset is needed between rounds.  A wait
// gives up after `spin_limit` polls and counts that in `*late`, so the
// kernel ends whatever happens.
template <int kGroups>
__global__ __launch_bounds__(kThreads) void k_probe_barrier(unsigned* bar, unsigned* cnt,
                                                            int rounds, int spin_limit,
                                                            unsigned* late) {
  unsigned* top = bar;
  const int grp = (int)(blockIdx.x % kGroups);
  unsigned* sub = bar + 64 * (1 + grp);
  const unsigned ng = gridDim.x < (unsigned)kGroups ? gridDim.x : (unsigned)kGroups;
  const unsigned in_grp = (gridDim.x - (unsigned)grp + kGroups - 1) / kGroups;
  for (int r = 1; r <= rounds; ++r) {
    __syncthreads();
    if (threadIdx.x == 0) {
      cnt[blockIdx.x] += 1u;
      if (kGroups == 1) {
        __hip_atomic_fetch_add(top, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      } else {
        const unsigned got =
            __hip_atomic_fetch_add(sub, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT) + 1u;
        if (got == (unsigned)r * in_grp)
          __hip_atomic_fetch_add(top, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      }
      const unsigned target = (unsigned)r * (kGroups == 1 ? gridDim.x : ng);
      for (int s = 0;
           __hip_atomic_load(top, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target; ++s) {
        if (s == spin_limit) {
          atomicAdd(late, 1u);
          break;
        }
        __builtin_amdgcn_s_sleep(1);
      }
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    __syncthreads();
  }
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

/*
 * Prices a phase boundary of the ordering step on the current device, each
 * figure over `rounds` boundaries:
 *   out[0]  microseconds per launch boundary in a replayed HIP graph of
 *           dependent launches of a kernel of no work, over a grid of 4
 *           workgroups of 256 threads per compute unit (what the step's small
 *           kernels launch),
 *   out[1]  the same launches made one by one on a stream,
 *   out[2]  microseconds per grid-wide barrier inside one cooperative launch
 *           of the same grid, one arrival count,
 *   out[3]  the same with arrivals gathered in 8 groups first,
 *   out[4]  the same over 1 workgroup per compute unit,
 *   out[5]  the grid of out[0] - out[3] (workgroups),
 *   out[6]  barrier waits that gave up at their poll limit (0 when every
 *           workgroup was resident and the barriers worked).
 * Allocates small device buffers and a stream of default priority
 * (measurement only).  Returns 0 on success, a HIP error code otherwise
 * (hipErrorNotSupported without cooperative launches).
 */
int lingam_probe_sync(int rounds, double* out) {
  if (rounds < 1) return (int)hipErrorInvalidValue;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return (int)e;
  int cu = 0, coop = 0, per_cu1 = 0, per_cu8 = 0;
  e = hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return (int)e;
  e = hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev);
  if (e != hipSuccess) return (int)e;
  if (!coop) return (int)hipErrorNotSupported;
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu1, k_probe_barrier<1>, kThreads, 0);
  if (e != hipSuccess) return (int)e;
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu8, k_probe_barrier<8>, kThreads, 0);
  if (e != hipSuccess) return (int)e;
  int per_cu = per_cu1 < per_cu8 ? per_cu1 : per_cu8;
  per_cu = per_cu < 4 ? per_cu : 4;
  const int grid = cu * per_cu;
  if (grid < 1) return (int)hipErrorInvalidConfiguration;
  // a poll is a device-scope load and a short sleep: milliseconds per wait at most
  const int spin_limit = 5000;
  constexpr int kBar = 64 * 9;  // top count, then 8 group counts 256 bytes apart
  unsigned* buf = nullptr;      // [0, kBar) counts, [kBar] late waits, then per-workgroup
  e = hipMalloc(&buf, sizeof(unsigned) * (size_t)(kBar + 1 + grid));
  if (e != hipSuccess) return (int)e;
  unsigned *bar = buf, *late = buf + kBar, *cnt = buf + kBar + 1;
  hipStream_t st = nullptr;
  hipGraph_t g = nullptr;
  hipGraphExec_t ge = nullptr;
  hipEvent_t t0 = nullptr, t1 = nullptr;
  float ms[5] = {0, 0, 0, 0, 0};
  unsigned late_h = 0;
  do {
    if ((e = hipMemset(buf, 0, sizeof(unsigned) * (size_t)(kBar + 1 + grid))) != hipSuccess) break;
    if ((e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking)) != hipSuccess) break;
    if ((e = hipEventCreate(&t0)) != hipSuccess) break;
    if ((e = hipEventCreate(&t1)) != hipSuccess) break;
    // graph of `rounds` launches
    if ((e = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal)) != hipSuccess) break;
    for (int i = 0; i < rounds; ++i)
      hipLaunchKernelGGL(k_probe_touch, dim3(grid), dim3(kThreads), 0, st, cnt);
    if ((e = hipStreamEndCapture(st, &g)) != hipSuccess) break;
    if ((e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0)) != hipSuccess) break;
    for (int rep = 0; rep < 2 && e == hipSuccess; ++rep) {  // the first replay warms up
      (void)hipEventRecord(t0, st);
      e = hipGraphLaunch(ge, st);
      (void)hipEventRecord(t1, st);
      if (e == hipSuccess) e = hipEventSynchronize(t1);
      if (e == hipSuccess) e = hipEventElapsedTime(&ms[0], t0, t1);
    }
    if (e != hipSuccess) break;
    // the same launches one by one
    for (int rep = 0; rep < 2 && e == hipSuccess; ++rep) {
      (void)hipEventRecord(t0, st);
      for (int i = 0; i < rounds; ++i)
        hipLaunchKernelGGL(k_probe_touch, dim3(grid), dim3(kThreads), 0, st, cnt);
      (void)hipEventRecord(t1, st);
      e = hipGetLastError();
      if (e == hipSuccess) e = hipEventSynchronize(t1);
      if (e == hipSuccess) e = hipEventElapsedTime(&ms[1], t0, t1);
    }
    if (e != hipSuccess) break;
    // cooperative launches passing `rounds` barriers
    int rr = rounds, sl = spin_limit;
    void* args[] = {&bar, &cnt, &rr, &sl, &late};
    for (int which = 2; which < 5 && e == hipSuccess; ++which) {
      const void* fn =
          which == 2 ? (const void*)k_probe_barrier<1> : (const void*)k_probe_barrier<8>;
      const int gw = which == 4 ? cu : grid;
      for (int rep = 0; rep < 2 && e == hipSuccess; ++rep) {
        e = hipMemsetAsync(bar, 0, sizeof(unsigned) * kBar, st);  // counts restart at 0
        if (e != hipSuccess) break;
        (void)hipEventRecord(t0, st);
        e = hipLaunchCooperativeKernel(fn, dim3(gw), dim3(kThreads), args, 0, st);
        (void)hipEventRecord(t1, st);
        if (e == hipSuccess) e = hipEventSynchronize(t1);
        if (e == hipSuccess) e = hipEventElapsedTime(&ms[which], t0, t1);
      }
    }
    if (e != hipSuccess) break;
    e = hipMemcpy(&late_h, late, sizeof(unsigned), hipMemcpyDeviceToHost);
  } while (false);
  if (ge) (void)hipGraphExecDestroy(ge);
  if (g) (void)hipGraphDestroy(g);
  if (t0) (void)hipEventDestroy(t0);
  if (t1) (void)hipEventDestroy(t1);
  if (st) (void)hipStreamDestroy(st);
  (void)hipFree(buf);
  if (e != hipSuccess) return (int)e;
  for (int k = 0; k < 5; ++k) out[k] = ms[k] * 1e3 / rounds;
  out[5] = grid;
  out[6] = late_h;
  return 0;
}

}  // extern "C"
