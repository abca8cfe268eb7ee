// Diagnostics beside the seeding path: a streaming copy (to calibrate the HBM byte counters of the
// profiler against a known size) and a random 128-byte line gather (the rate at which this GPU
// serves independent random line accesses, the ceiling the seeding kernels are compared with).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>

#include "mbw_internal.h"
#include "../../include/mbw.h"

namespace {

__global__ void k_probe_copy(const uint4 *__restrict__ a, uint4 *__restrict__ b, uint64_t n) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) b[i] = a[i];
}

__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// eight lanes fetch one random 128-byte line (16 bytes each); the next line depends on the data
__global__ void k_probe_gather(const uint4 *__restrict__ buf, uint64_t nlines, int iters, uint64_t *__restrict__ out) {
  const uint64_t tid = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  const int q = threadIdx.x & 7;
  uint64_t h = mix64(tid >> 3);
  for (int it = 0; it < iters; ++it) {
    const uint64_t line = h % nlines;
    const uint4 v = buf[line * 8 + q];
    uint32_t x = v.x ^ v.y ^ v.z ^ v.w;
    x ^= __shfl_xor(x, 1, 8);
    x ^= __shfl_xor(x, 2, 8);
    x ^= __shfl_xor(x, 4, 8);
    h = mix64(h ^ x);
  }
  out[tid] = h;
}

}  // namespace

#define TRY(call) MBW_HIP_TRY(call)

extern "C" int mbw_probe_copy(int device, uint64_t bytes, float *ms) {
  if (!ms || bytes < 4096) { mbw_set_error("bad probe arguments"); return MBW_E_INVAL; }
  TRY(hipSetDevice(device));
  const uint64_t n = bytes / 16;
  uint4 *a = nullptr, *b = nullptr;
  TRY(hipMalloc((void **)&a, n * 16));
  if (hipMalloc((void **)&b, n * 16) != hipSuccess) { (void)hipFree(a); mbw_set_error("hipMalloc failed"); return MBW_E_NOMEM; }
  hipEvent_t e0, e1;
  int rc = [&]() -> int {
    TRY(hipMemset(a, 1, n * 16));
    TRY(hipEventCreate(&e0));
    TRY(hipEventCreate(&e1));
    k_probe_copy<<<8192, 256>>>(a, b, n);   // warm
    TRY(hipEventRecord(e0));
    k_probe_copy<<<8192, 256>>>(a, b, n);
    TRY(hipEventRecord(e1));
    TRY(hipEventSynchronize(e1));
    TRY(hipEventElapsedTime(ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return 0;
  }();
  (void)hipFree(a);
  (void)hipFree(b);
  return rc;
}

extern "C" int mbw_probe_gather(int device, uint64_t bytes, int iters, double *lines_per_s, float *ms) {
  if (!lines_per_s || !ms || bytes < (1u << 20) || iters < 1) { mbw_set_error("bad probe arguments"); return MBW_E_INVAL; }
  TRY(hipSetDevice(device));
  const uint64_t nlines = bytes / 128;
  const int grid = 16384, block = 256;
  uint4 *buf = nullptr;
  uint64_t *out = nullptr;
  TRY(hipMalloc((void **)&buf, nlines * 128));
  if (hipMalloc((void **)&out, (uint64_t)grid * block * 8) != hipSuccess) { (void)hipFree(buf); mbw_set_error("hipMalloc failed"); return MBW_E_NOMEM; }
  hipEvent_t e0, e1;
  int rc = [&]() -> int {
    TRY(hipMemset(buf, 0x5a, nlines * 128));
    TRY(hipEventCreate(&e0));
    TRY(hipEventCreate(&e1));
    k_probe_gather<<<grid, block>>>(buf, nlines, iters, out);   // warm
    TRY(hipEventRecord(e0));
    k_probe_gather<<<grid, block>>>(buf, nlines, iters, out);
    TRY(hipEventRecord(e1));
    TRY(hipEventSynchronize(e1));
    TRY(hipEventElapsedTime(ms, e0, e1));
    *lines_per_s = (double)grid * block / 8 * iters / (*ms * 1e-3);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return 0;
  }();
  (void)hipFree(buf);
  (void)hipFree(out);
  return rc;
}
