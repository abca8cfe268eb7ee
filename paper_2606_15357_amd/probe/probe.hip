// Measurement helpers beside the seeding library (built into libmbw_probe.so, not libmbw.so): a
// streaming copy (to calibrate the HBM byte counters of the profiler against a known size) and a
// random 128-byte line gather (the rate at which this GPU serves independent random line accesses,
// the ceiling the seeding kernels are compared with).
//
// C ABI (status 0 on success, -1 bad argument, -2 out of memory, -3 HIP error; message from
// mbwprobe_last_error()):
//   int mbwprobe_copy(int device, uint64_t bytes, float *ms)
//       streams `bytes` bytes (>= 4096) from one buffer to another once; *ms = kernel time.
//   int mbwprobe_gather(int device, uint64_t bytes, int iters, int waves_per_simd, double *lines_per_s,
//                       float *ms)
//       every lane follows four chains of random 128-byte lines (16 bytes read per line) over the
//       largest power-of-two number of lines that fits in `bytes` (>= 1 MiB), `iters` dependent
//       fetches per chain; *lines_per_s = random lines served per second.  waves_per_simd 0: 8,192
//       blocks of 256 threads (as many waves as the CUs hold); 1..8: that many blocks per CU, i.e.
//       that many waves per SIMD, each lane taking 8192 / (blocks) times `iters` fetches per chain so
//       that every setting makes the same number of fetches.
// Both allocate and free their own device memory.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <string>

namespace {

__global__ void k_probe_copy(const uint4 *__restrict__ a, uint4 *__restrict__ b, uint64_t n) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) b[i] = a[i];
}

// Every lane follows four independent chains of random 128-byte lines (16 bytes read per line, one
// lane per line, as the seeding kernels do); the next line of a chain depends on the data read, so
// nothing can be prefetched, and the line index is a 32-bit LCG step masked to a power of two.
__global__ void k_probe_gather(const uint4 *__restrict__ buf, uint32_t mask, int iters, uint64_t *__restrict__ out) {
  const uint64_t tid = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  uint32_t h0 = (uint32_t)(tid * 0x9E3779B1u) ^ 0x1234567u, h1 = h0 * 0x85EBCA6Bu + 1u, h2 = h1 * 0xC2B2AE35u + 7u,
           h3 = h2 * 0x27D4EB2Fu + 13u;
  for (int it = 0; it < iters; ++it) {
    const uint4 a = buf[(uint64_t)(h0 & mask) * 8], b = buf[(uint64_t)(h1 & mask) * 8 + 1],
                c = buf[(uint64_t)(h2 & mask) * 8 + 2], d = buf[(uint64_t)(h3 & mask) * 8 + 3];
    h0 = h0 * 1664525u + 1013904223u + a.x;
    h1 = h1 * 1664525u + 1013904223u + b.y;
    h2 = h2 * 1664525u + 1013904223u + c.z;
    h3 = h3 * 1664525u + 1013904223u + d.w;
  }
  out[tid] = (uint64_t)(h0 ^ h1) << 32 | (h2 ^ h3);
}

}  // namespace

static thread_local std::string g_probe_err;
static void set_error(const std::string &m) { g_probe_err = m; }
extern "C" const char *mbwprobe_last_error(void) { return g_probe_err.c_str(); }

#define TRY(call)                                                                          \
  do {                                                                                     \
    hipError_t e_ = (call);                                                                \
    if (e_ != hipSuccess) {                                                                \
      set_error(std::string(#call) + ": " + hipGetErrorString(e_));                        \
      return e_ == hipErrorOutOfMemory ? -2 : -3;                                          \
    }                                                                                      \
  } while (0)

extern "C" int mbwprobe_copy(int device, uint64_t bytes, float *ms) {
  if (!ms || bytes < 4096) { set_error("bad probe arguments"); return -1; }
  TRY(hipSetDevice(device));
  const uint64_t n = bytes / 16;
  uint4 *a = nullptr, *b = nullptr;
  TRY(hipMalloc((void **)&a, n * 16));
  if (hipMalloc((void **)&b, n * 16) != hipSuccess) { (void)hipFree(a); set_error("hipMalloc failed"); return -2; }
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

extern "C" int mbwprobe_gather(int device, uint64_t bytes, int iters, int waves_per_simd, double *lines_per_s,
                               float *ms) {
  if (!lines_per_s || !ms || bytes < (1u << 20) || iters < 1 || waves_per_simd < 0 || waves_per_simd > 8) {
    set_error("bad probe arguments");
    return -1;
  }
  TRY(hipSetDevice(device));
  uint64_t nlines = 1;                                   // a power of two, at most bytes / 128 and 2^32
  while (nlines * 2 <= bytes / 128 && nlines < (1ull << 32)) nlines *= 2;
  const uint32_t mask = (uint32_t)(nlines - 1);
  const int block = 256;
  int grid = 8192;
  if (waves_per_simd > 0) {
    int n_cu = 0;
    TRY(hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, device));
    grid = std::max(1, n_cu) * waves_per_simd;
    const int64_t it = (int64_t)iters * 8192 / grid;
    if (it > (1 << 24)) { set_error("bad probe arguments"); return -1; }
    iters = (int)std::max<int64_t>(1, it);
  }
  uint4 *buf = nullptr;
  uint64_t *out = nullptr;
  TRY(hipMalloc((void **)&buf, nlines * 128));
  if (hipMalloc((void **)&out, (uint64_t)grid * block * 8) != hipSuccess) { (void)hipFree(buf); set_error("hipMalloc failed"); return -2; }
  hipEvent_t e0, e1;
  int rc = [&]() -> int {
    TRY(hipMemset(buf, 0x5a, nlines * 128));
    TRY(hipEventCreate(&e0));
    TRY(hipEventCreate(&e1));
    k_probe_gather<<<grid, block>>>(buf, mask, iters, out);   // warm
    TRY(hipEventRecord(e0));
    k_probe_gather<<<grid, block>>>(buf, mask, iters, out);
    TRY(hipEventRecord(e1));
    TRY(hipEventSynchronize(e1));
    TRY(hipEventElapsedTime(ms, e0, e1));
    *lines_per_s = (double)grid * block * 4 * iters / (*ms * 1e-3);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return 0;
  }();
  (void)hipFree(buf);
  (void)hipFree(out);
  return rc;
}
