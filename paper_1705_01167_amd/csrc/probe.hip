// Random-gather bandwidth probe: the access pattern of the band search
// without the search.  Groups of 8 lanes read whole 128-byte lines (16 bytes
// per lane) at hashed random line indices of a large buffer; each group keeps
// `depth` independent lines in flight per step.  The achieved line rate times
// 128 bytes is the achievable HBM gather bandwidth that the search kernels
// are compared against.
#include "cddt_common.h"

namespace cddt {
namespace {

__device__ __forceinline__ uint32_t mix32(uint32_t x) {
  // integer finaliser (xorshift-multiply) for well-spread line indices
  x ^= x >> 16;
  x *= 0x7feb352dU;
  x ^= x >> 15;
  x *= 0x846ca68bU;
  x ^= x >> 16;
  return x;
}

template <int Depth>
__global__ __launch_bounds__(256) void k_probe(const int4* __restrict__ buf, uint64_t n_lines, int32_t steps,
                                               uint32_t seed, int32_t* __restrict__ sink) {
  const int lane = threadIdx.x & 63, sub = lane & 7;
  const uint32_t group = (blockIdx.x * blockDim.x + threadIdx.x) >> 3;
  int32_t acc = 0;
  for (int32_t s = 0; s < steps; ++s) {
    int4 v[Depth];
#pragma unroll
    for (int d = 0; d < Depth; ++d) {
      const uint32_t h = mix32(group * 0x9e3779b9U ^ (uint32_t)(s * Depth + d) * 0x85ebca6bU ^ seed);
      const uint64_t line = ((uint64_t)h * n_lines) >> 32;  // uniform in [0, n_lines)
      v[d] = buf[line * 8 + sub];
    }
#pragma unroll
    for (int d = 0; d < Depth; ++d) acc += v[d].x ^ v[d].y ^ v[d].z ^ v[d].w;
  }
  sink[blockIdx.x * blockDim.x + threadIdx.x] = acc;
}

}  // namespace
}  // namespace cddt

using namespace cddt;

extern "C" {

// Measurement helper (not part of the method): buf is a device buffer of
// `bytes` bytes (multiple of 128, at least 128); sink is device int32[blocks*256].
// Launches blocks x 256 threads, each 8-lane group reading steps*depth random
// 128-byte lines (depth in {1, 2, 4, 8}).  Asynchronous.
cddt_status cddt_probe_gather(const void* buf, int64_t bytes, int32_t blocks, int32_t steps, int32_t depth,
                              uint32_t seed, int32_t* sink, void* stream) {
  if (!buf || !sink || bytes < 128 || (bytes & 127) || blocks < 1 || steps < 1)
    return fail(CDDT_EINVAL, "cddt_probe_gather: bad argument");
  if ((uint64_t)bytes / 128 > 0xffffffffull) return fail(CDDT_EINVAL, "cddt_probe_gather: buffer too large");
  const uint64_t lines = (uint64_t)bytes / 128;
  hipStream_t st = (hipStream_t)stream;
  const int4* b = (const int4*)buf;
  switch (depth) {
    case 1: hipLaunchKernelGGL(k_probe<1>, dim3(blocks), dim3(256), 0, st, b, lines, steps, seed, sink); break;
    case 2: hipLaunchKernelGGL(k_probe<2>, dim3(blocks), dim3(256), 0, st, b, lines, steps, seed, sink); break;
    case 4: hipLaunchKernelGGL(k_probe<4>, dim3(blocks), dim3(256), 0, st, b, lines, steps, seed, sink); break;
    case 8: hipLaunchKernelGGL(k_probe<8>, dim3(blocks), dim3(256), 0, st, b, lines, steps, seed, sink); break;
    default: return fail(CDDT_EINVAL, "cddt_probe_gather: depth must be 1, 2, 4 or 8");
  }
  CDDT_HIP(hipGetLastError());
  return CDDT_OK;
}

}  // extern "C"
