// Achievable HBM bandwidth on this device: streaming read, write and copy
// kernels over a buffer far larger than the caches, timed with HIP events.
// The measured figures are the practical ceiling that the HBM-bound passes
// are compared against beside the datasheet peak.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/vie.h"

namespace {

constexpr int PT = 256;

// Sum of every 16-byte word (kept live by one store per workgroup).
__global__ __launch_bounds__(PT) void k_probe_read(const float4* __restrict__ a, int64_t n,
                                                   float* __restrict__ out) {
  float acc = 0.f;
  for (int64_t i = (int64_t)blockIdx.x * PT + threadIdx.x; i < n; i += (int64_t)gridDim.x * PT) {
    const float4 v = a[i];
    acc += (v.x + v.y) + (v.z + v.w);
  }
  for (int m = 32; m >= 1; m >>= 1) acc += __shfl_xor(acc, m);
  if ((threadIdx.x & 63) == 0) out[blockIdx.x * (PT / 64) + (threadIdx.x >> 6)] = acc;
}

__global__ __launch_bounds__(PT) void k_probe_write(float4* __restrict__ a, int64_t n, float v) {
  for (int64_t i = (int64_t)blockIdx.x * PT + threadIdx.x; i < n; i += (int64_t)gridDim.x * PT)
    a[i] = make_float4(v, v, v, v);
}

__global__ __launch_bounds__(PT) void k_probe_copy(const float4* __restrict__ a,
                                                   float4* __restrict__ b, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * PT + threadIdx.x; i < n; i += (int64_t)gridDim.x * PT)
    b[i] = a[i];
}

}  // namespace

extern "C" int vie_hbm_probe(int64_t bytes, int32_t reps, double* gbps) {
  if (!gbps || reps < 1 || bytes < (1 << 20) || bytes > ((int64_t)64 << 30)) return VIE_EINVAL;
  const int64_t n = bytes / 16;
  float4 *a = nullptr, *b = nullptr;
  float* part = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int grid = 0;
  {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
      return VIE_EDEVICE;
    grid = cus * 16;  // 16 workgroups per CU, grid-stride over the buffer
  }
  int rc = VIE_OK;
  if (hipMalloc(&a, n * 16) != hipSuccess || hipMalloc(&b, n * 16) != hipSuccess ||
      hipMalloc(&part, (size_t)grid * (PT / 64) * sizeof(float)) != hipSuccess) {
    rc = VIE_ENOMEM;
  } else if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    rc = VIE_EDEVICE;
  } else {
    k_probe_write<<<grid, PT>>>(a, n, 1.0f);
    k_probe_write<<<grid, PT>>>(b, n, 2.0f);
    for (int kind = 0; kind < 3 && rc == VIE_OK; ++kind) {
      for (int r = -1; r < reps; ++r) {  // r = -1: untimed warm-up
        if (r == 0) (void)hipEventRecord(e0, nullptr);
        if (kind == 0) k_probe_read<<<grid, PT>>>(a, n, part);
        if (kind == 1) k_probe_write<<<grid, PT>>>(b, n, 3.0f);
        if (kind == 2) k_probe_copy<<<grid, PT>>>(a, b, n);
      }
      (void)hipEventRecord(e1, nullptr);
      float ms = 0.f;
      if (hipGetLastError() != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
          hipEventElapsedTime(&ms, e0, e1) != hipSuccess || !(ms > 0)) {
        rc = VIE_EDEVICE;
        break;
      }
      const double moved = (double)n * 16 * (kind == 2 ? 2 : 1) * reps;
      gbps[kind] = moved / (ms * 1e-3) / 1e9;
    }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (a) (void)hipFree(a);
  if (b) (void)hipFree(b);
  if (part) (void)hipFree(part);
  return rc;
}
