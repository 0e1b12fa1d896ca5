// Plain query kernels: one lane per ray (cast) and one wave per particle
// (beam-model weight).  The per-ray and per-particle arithmetic lives in
// query_device.h and is shared with the persistent batched kernel.
#include "query_device.h"

namespace cddt {
namespace {

constexpr int kCastThreads = 256;
constexpr int kWeightThreads = 256;  // 4 particles (waves) per block
constexpr int kCastK = 0;            // search strategy (band_search): one lane per search
constexpr int kWeightK = 0;

// One wave takes 64 consecutive rays at a time (lane = ray); the loop bound is
// the same for every lane of a wave so the cooperative search stays converged.
// Maps without a bucket index only (those with one go to k_cast_tiles), so
// never 16-bit lines.
// ticks (nullable): per ray, the device wall-clock ticks its wave spent from
// loading the ray to its result.
__global__ __launch_bounds__(kCastThreads) void k_cast(MapDev m, const float* __restrict__ x,
                                                       const float* __restrict__ y,
                                                       const float* __restrict__ th, int64_t n,
                                                       int32_t max_range, int32_t* __restrict__ out,
                                                       int32_t* __restrict__ ticks) {
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t waves = (int64_t)gridDim.x * (kCastThreads / kWave);
  const int64_t chunks = (n + kWave - 1) / kWave;
  for (int64_t c = (int64_t)blockIdx.x * (kCastThreads / kWave) + (threadIdx.x >> 6); c < chunks; c += waves) {
    const uint64_t t0 = ticks ? wall_clock64() : 0;
    const int64_t i = c * kWave + lane;
    const bool active = i < n;
    const float xi = active ? ldg(x + i) : 0.0f, yi = active ? ldg(y + i) : 0.0f, ti = active ? ldg(th + i) : 0.0f;
    const int32_t r = wave_cast<kCastK, false>(m, active, xi, yi, ti, max_range);
    if (active) {
      stg(out + i, r);
      if (ticks) stg(ticks + i, (int32_t)(wall_clock64() - t0));
    }
  }
}

// Casts on maps with a bucket index: kCastQ * 64 rays per wave through
// the search queue (half-line first pass, deferred full searches).
constexpr int kCastQ = 8;
template <bool Z>
__global__ __launch_bounds__(kCastThreads) void k_cast_tiles(MapDev m, const float* __restrict__ x,
                                                             const float* __restrict__ y,
                                                             const float* __restrict__ th, int64_t n,
                                                             int32_t max_range, int32_t* __restrict__ out,
                                                             int32_t* __restrict__ ticks) {
  __shared__ int2 jobs[kCastThreads / kWave][kCastQ * kWave];
  __shared__ int32_t codes[kCastThreads / kWave][kCastQ * kWave];
  __shared__ int32_t later[kCastThreads / kWave][kCastQ * kWave];
  const int wave = threadIdx.x >> 6;
  const int64_t per = (int64_t)kCastQ * kWave;
  const int64_t tiles = (n + per - 1) / per;
  const int64_t waves = (int64_t)gridDim.x * (kCastThreads / kWave);
  for (int64_t t = (int64_t)blockIdx.x * (kCastThreads / kWave) + wave; t < tiles; t += waves)
    wave_cast_tile<kCastQ, Z>(m, x, y, th, n, t * per, max_range, out, jobs[wave], codes[wave], later[wave], ticks);
}

// Q particles per wave through the phased tile routine (ray layouts of <= 64 rays).
constexpr int kWeightQ = 4;
constexpr int64_t kTileMinParticles = 1 << 17;
template <bool Z>
__global__ __launch_bounds__(kWeightThreads) void k_weight_tiles(FilterDev f) {
  __shared__ int2 jobs[kWeightThreads / kWave][kWeightQ * kWave];
  __shared__ int32_t codes[kWeightThreads / kWave][kWeightQ * kWave];
  __shared__ int32_t later[kWeightThreads / kWave][kWeightQ * kWave];
  const int wave = threadIdx.x >> 6;
  const int64_t p0 = ((int64_t)blockIdx.x * (kWeightThreads / kWave) + wave) * kWeightQ;
  if (p0 >= f.n_particles) return;  // whole wave leaves together
  const int32_t cnt = (int32_t)min((int64_t)kWeightQ, f.n_particles - p0);
  wave_tile_logw<kWeightQ, false, Z>(f, p0, cnt, jobs[wave], codes[wave], later[wave]);
}

template <bool Z>
__global__ __launch_bounds__(kWeightThreads) void k_weight(FilterDev f) {
  const int64_t p = (int64_t)blockIdx.x * (kWeightThreads / kWave) + (threadIdx.x >> 6);
  if (p >= f.n_particles) return;  // whole wave leaves together
  float lw = wave_particle_logw<kWeightK, Z>(f.map, ldg(f.px + p), ldg(f.py + p), ldg(f.pth + p), f.offsets, f.obs,
                                          f.n_rays, f.pair_offset,
                                f.table, f.max_range, f.ranges ? f.ranges + p * f.n_rays : nullptr);
  if ((threadIdx.x & 63) == 0) stg(f.logw + p, lw);
}

}  // namespace

cddt_status launch_cast(const MapDev& m, const float* x, const float* y, const float* th, int64_t n,
                        int32_t max_range, int32_t* out, hipStream_t st, int32_t* ticks) {
  if (n == 0) return CDDT_OK;
  if (m.bk) {
    const int64_t tiles = (n + (int64_t)kCastQ * kWave - 1) / ((int64_t)kCastQ * kWave);
    int64_t tb = (tiles + kCastThreads / kWave - 1) / (kCastThreads / kWave);
    if (tb > (1 << 16)) tb = 1 << 16;
    if (m.zp16)
      hipLaunchKernelGGL(k_cast_tiles<true>, dim3((unsigned)tb), dim3(kCastThreads), 0, st, m, x, y, th, n,
                         max_range, out, ticks);
    else
      hipLaunchKernelGGL(k_cast_tiles<false>, dim3((unsigned)tb), dim3(kCastThreads), 0, st, m, x, y, th, n,
                         max_range, out, ticks);
    CDDT_HIP(hipGetLastError());
    return CDDT_OK;
  }
  int64_t blocks = (n + kCastThreads - 1) / kCastThreads;
  if (blocks > (1 << 16)) blocks = 1 << 16;
  hipLaunchKernelGGL(k_cast, dim3((unsigned)blocks), dim3(kCastThreads), 0, st, m, x, y, th, n, max_range, out,
                     ticks);
  CDDT_HIP(hipGetLastError());
  return CDDT_OK;
}

cddt_status launch_weight(const FilterDev& f, hipStream_t st) {
  if (f.n_particles == 0) return CDDT_OK;
  const int per_block = kWeightThreads / kWave;
  // tiles of Q particles per wave only when there are enough particles to fill the chip
  if (f.n_rays <= kWave && f.n_particles >= kTileMinParticles) {
    const int64_t blocks = (f.n_particles + per_block * kWeightQ - 1) / (per_block * kWeightQ);
    if (blocks > 0x7fffffffLL) return fail(CDDT_EINVAL, "too many particles for one launch");
    if (f.map.zp16)
      hipLaunchKernelGGL(k_weight_tiles<true>, dim3((unsigned)blocks), dim3(kWeightThreads), 0, st, f);
    else
      hipLaunchKernelGGL(k_weight_tiles<false>, dim3((unsigned)blocks), dim3(kWeightThreads), 0, st, f);
  } else {
    const int64_t blocks = (f.n_particles + per_block - 1) / per_block;
    if (blocks > 0x7fffffffLL) return fail(CDDT_EINVAL, "too many particles for one launch");
    if (f.map.zp16)
      hipLaunchKernelGGL(k_weight<true>, dim3((unsigned)blocks), dim3(kWeightThreads), 0, st, f);
    else
      hipLaunchKernelGGL(k_weight<false>, dim3((unsigned)blocks), dim3(kWeightThreads), 0, st, f);
  }
  CDDT_HIP(hipGetLastError());
  return CDDT_OK;
}

}  // namespace cddt
