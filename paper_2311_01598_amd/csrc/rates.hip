// rates.hip -- issue-rate and bandwidth probes that back the roofline peaks.
//
// Each probe runs long chains of one instruction kind with 8 independent
// chains per lane (enough ILP to hide latency) over a grid that fills every
// CU several times, and reports lane-operations per second.  The copy probe
// streams a buffer far larger than the 256 MB last-level cache.
#include "plan.h"
#include "modarith.h"

namespace ks {

constexpr int kIters = 4096;
constexpr int kChains = 8;

// Each chain step is one instruction written as inline asm (arithmetic
// only) so the compiler can neither fold the recurrence nor change the
// instruction; kind 5 is the library's lazy Shoup butterfly for reference.
template <int KIND>
__global__ __launch_bounds__(256) void k_probe(uint32_t *sink, uint32_t seed) {
  uint32_t a[kChains];
  uint64_t acc[kChains];
  double f[kChains];
  const uint32_t b = seed | 1u;
  const double fb = 0.999999, fc = 1e-7;
#pragma unroll
  for (int c = 0; c < kChains; c++) {
    a[c] = threadIdx.x * 2654435761u + c * 97u + seed;
    acc[c] = a[c];
    f[c] = (double)a[c] * 1e-9;
  }
  for (int it = 0; it < kIters; it++) {
#pragma unroll
    for (int c = 0; c < kChains; c++) {
      if constexpr (KIND == 0) asm volatile("v_add_u32 %0, %0, %1" : "+v"(a[c]) : "v"(b));
      if constexpr (KIND == 1) asm volatile("v_mul_lo_u32 %0, %0, %1" : "+v"(a[c]) : "v"(b));
      if constexpr (KIND == 2) asm volatile("v_mul_hi_u32 %0, %0, %1" : "+v"(a[c]) : "v"(b));
      if constexpr (KIND == 3) {
        uint64_t carry;
        asm volatile("v_mad_u64_u32 %0, %1, %2, %3, %0" : "+v"(acc[c]), "=s"(carry) : "v"(a[c]), "v"(b));
      }
      if constexpr (KIND == 4) asm volatile("v_fma_f64 %0, %0, %1, %2" : "+v"(f[c]) : "v"(fb), "v"(fc));
      if constexpr (KIND == 5) {
        if (c & 1) continue;  // four independent butterfly chains on pairs (a[c], a[c+1])
        bfly_ct(a[c], a[c + 1], b, b ^ 0x5bd1e995u, 0x3fffc001u);
      }
    }
  }
  uint32_t r = 0;
#pragma unroll
  for (int c = 0; c < kChains; c++) r ^= a[c] ^ (uint32_t)acc[c] ^ (uint32_t)(acc[c] >> 32) ^ (uint32_t)f[c];
  if (r == 0x12345678u) sink[threadIdx.x] = r;  // keeps the chains live
}

__global__ __launch_bounds__(256) void k_copy(const uint4 *__restrict__ src, uint4 *__restrict__ dst, size_t n) {
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) dst[i] = src[i];
}

}  // namespace ks

using namespace ks;

extern "C" ks_status_t ks_device_rates(double *out, void *stream) {
  if (!out) return KS_ERR_INVALID_ARG;
  hipStream_t st = (hipStream_t)stream;
  hipDeviceProp_t prop;
  int dev;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return KS_ERR_DEVICE;
  const uint32_t blocks = (uint32_t)prop.multiProcessorCount * 16;
  uint32_t *sink = nullptr;
  if (hipMalloc(&sink, 4096) != hipSuccess) return KS_ERR_NOMEM;
  hipEvent_t e0, e1;
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);
  ks_status_t status = KS_OK;
  auto timed = [&](auto launch) -> double {
    launch();  // warm-up
    (void)hipEventRecord(e0, st);
    launch();
    (void)hipEventRecord(e1, st);
    (void)hipEventSynchronize(e1);
    float ms = 0;
    (void)hipEventElapsedTime(&ms, e0, e1);
    return ms * 1e-3;
  };
  const double lane_ops = (double)blocks * 256 * kIters * kChains;
  out[0] = lane_ops / timed([&] { hipLaunchKernelGGL(k_probe<0>, dim3(blocks), dim3(256), 0, st, sink, 3u); });
  out[1] = lane_ops / timed([&] { hipLaunchKernelGGL(k_probe<1>, dim3(blocks), dim3(256), 0, st, sink, 3u); });
  out[2] = lane_ops / timed([&] { hipLaunchKernelGGL(k_probe<2>, dim3(blocks), dim3(256), 0, st, sink, 3u); });
  out[3] = lane_ops / timed([&] { hipLaunchKernelGGL(k_probe<3>, dim3(blocks), dim3(256), 0, st, sink, 3u); });
  out[4] = lane_ops / timed([&] { hipLaunchKernelGGL(k_probe<4>, dim3(blocks), dim3(256), 0, st, sink, 3u); });
  out[6] = lane_ops / 2 / timed([&] { hipLaunchKernelGGL(k_probe<5>, dim3(blocks), dim3(256), 0, st, sink, 3u); });
  const size_t bytes = (size_t)1 << 30;  // 1 GiB each way
  void *a = nullptr, *b = nullptr;
  if (hipMalloc(&a, bytes) != hipSuccess || hipMalloc(&b, bytes) != hipSuccess) {
    status = KS_ERR_NOMEM;
    out[5] = 0;
  } else {
    (void)hipMemsetAsync(a, 1, bytes, st);
    const size_t n = bytes / sizeof(uint4);
    out[5] = 2.0 * bytes / timed([&] {
      hipLaunchKernelGGL(k_copy, dim3(blocks * 4), dim3(256), 0, st, (const uint4 *)a, (uint4 *)b, n);
    });
  }
  if (hipGetLastError() != hipSuccess) status = KS_ERR_DEVICE;
  (void)hipStreamSynchronize(st);
  if (a) (void)hipFree(a);
  if (b) (void)hipFree(b);
  (void)hipFree(sink);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return status;
}
