// Read-bandwidth probe: the rate at which the memory level holding a buffer
// serves float4 reads to every CU, streamed (coalesced, each byte once per
// pass) or gathered (one float4 per lane at a pseudo-random index per pass,
// the access of the gridded field's corner loads).  The buffer's size picks
// the level: a few MiB stay in each XCD's L2, some hundred MiB in the MALL,
// GiBs come from HBM.  Used to state the serving level's peak next to the
// gridded trace's achieved bandwidth.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "radiotrace_probe.h"
#include "rt_params.hpp"

namespace rt {
namespace {

// 'never' is 0 at every launch; the compiler cannot know it, so the sums stay live.
// The buffer is read 'reps' times over within one launch, so that a buffer
// small enough for the L2 is timed over more than the launch latency.
__global__ void __launch_bounds__(256) probe_stream_kernel(float4* __restrict__ buf, uint64_t n,
                                                           int32_t reps, int32_t never) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  float acc = 0.0f;
  for (int r = 0; r < reps; ++r) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
      const float4 v = buf[i];
      acc += v.x + v.y + v.z + v.w;
    }
  }
  const uint64_t i0 = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (never && i0 < n) buf[i0] = make_float4(acc, 0, 0, 0);
}

// n a power of two; every lane reads 'reads' float4 at a hashed index.
__global__ void __launch_bounds__(256) probe_gather_kernel(float4* __restrict__ buf, uint64_t n,
                                                           int32_t reads, uint32_t salt,
                                                           int32_t never) {
  const uint64_t tid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  uint32_t h = (uint32_t)tid * 2654435761u ^ salt;
  float acc = 0.0f;
  for (int r = 0; r < reads; ++r) {
    h ^= h << 13;
    h ^= h >> 17;
    h ^= h << 5;
    const float4 v = buf[(uint64_t)h & (n - 1)];
    acc += v.x + v.y + v.z + v.w;
  }
  if (never) buf[tid & (n - 1)] = make_float4(acc, 0, 0, 0);
}

}  // namespace
}  // namespace rt

#define PROBE_TRY(expr)                                                       \
  do {                                                                        \
    hipError_t e_ = (expr);                                                   \
    if (e_ != hipSuccess) {                                                   \
      rt::set_last_error("%s: %s", #expr, hipGetErrorString(e_));             \
      if (b) hipEventDestroy(b);                                              \
      if (e) hipEventDestroy(e);                                              \
      return RT_ERR_DEVICE;                                                   \
    }                                                                         \
  } while (0)

extern "C" rt_status rt_probe_read_bandwidth(void* buffer, size_t bytes, int32_t pattern,
                                             int32_t passes, void* stream, double* gb_per_s) {
  using namespace rt;
  if (!buffer || !gb_per_s || passes < 1 || bytes < 4096 || bytes % 16 != 0) {
    set_last_error("probe: buffer, gb_per_s, passes >= 1 and bytes >= 4096 (a multiple of 16)");
    return RT_ERR_INVALID_ARG;
  }
  const uint64_t n = bytes / 16;
  if (pattern == RT_PROBE_GATHER && (n & (n - 1)) != 0) {
    set_last_error("probe: a gather needs a power-of-two number of float4 elements");
    return RT_ERR_INVALID_ARG;
  }
  if (pattern != RT_PROBE_STREAM && pattern != RT_PROBE_GATHER) {
    set_last_error("probe: unknown pattern %d", pattern);
    return RT_ERR_INVALID_ARG;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipEvent_t b = nullptr, e = nullptr;
  int dev = 0, ncu = 0;
  PROBE_TRY(hipGetDevice(&dev));
  PROBE_TRY(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
  PROBE_TRY(hipEventCreate(&b));
  PROBE_TRY(hipEventCreate(&e));
  float4* buf = static_cast<float4*>(buffer);
  // streaming: enough blocks to fill the chip, each thread a grid-stride
  // loop; gather: 8 blocks per CU, every lane 64 reads per pass
  const unsigned blocks = (unsigned)ncu * 8u;
  const int reads = 64;
  // a streamed pass reads at least 512 MiB
  const int reps_stream = (int)std::max<uint64_t>(1, (512ull << 20) / bytes);
  double bytes_per_pass = 0.0;
  for (int p = 0; p <= passes; ++p) {  // pass 0 warms the level up, untimed
    if (p == 1) PROBE_TRY(hipEventRecord(b, s));
    if (pattern == RT_PROBE_STREAM) {
      const unsigned g = (unsigned)std::min<uint64_t>((n + 255) / 256, (uint64_t)blocks * 4);
      hipLaunchKernelGGL(probe_stream_kernel, dim3(g), dim3(256), 0, s, buf, n, reps_stream, 0);
      bytes_per_pass = (double)bytes * reps_stream;
    } else {
      hipLaunchKernelGGL(probe_gather_kernel, dim3(blocks), dim3(256), 0, s, buf, n, reads,
                         (uint32_t)(0x9e3779b9u * (uint32_t)(p + 1)), 0);
      bytes_per_pass = (double)blocks * 256.0 * reads * 16.0;
    }
    PROBE_TRY(hipGetLastError());
  }
  PROBE_TRY(hipEventRecord(e, s));
  PROBE_TRY(hipEventSynchronize(e));
  float ms = 0.0f;
  PROBE_TRY(hipEventElapsedTime(&ms, b, e));
  hipEventDestroy(b);
  hipEventDestroy(e);
  *gb_per_s = bytes_per_pass * passes / (ms * 1e-3) / 1e9;
  return RT_OK;
}
