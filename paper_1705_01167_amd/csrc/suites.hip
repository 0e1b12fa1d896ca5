// Measurement helpers for the paper's query-time suites (Sec. VI: casts from
// a uniformly spaced grid of states and from uniformly random states, timed
// per query) and its dense lookup-table comparator (Sec. II-III: the range of
// every discrete state stored in a 3-D table).
//
// cddt_cast_timed runs the same kernels as cddt_cast and also records, per
// ray, the device wall-clock ticks its wave spent on it.  The table holds, for
// every bin k and cell (i, j), the cast from the cell centre at the bin's
// centre angle, computed by this library's own cast (so from grid states the
// table and the CDDT agree exactly); a table lookup rounds the query to its
// cell and bin.
#include <algorithm>

#include "cddt_common.h"
#include "query_device.h"

namespace cddt {
namespace {

constexpr int kLutThreads = 256;

// One lane per state (bin k, row j, cell i), k slowest; the cast of a lane's
// state is computed by the one-lane-per-search routine, so every lane of a
// wave calls it together.
template <bool Z>
__global__ __launch_bounds__(kLutThreads) void k_lut_build(MapDev m, int32_t max_range, uint16_t* __restrict__ lut,
                                                           int64_t states) {
  const int64_t cells = (int64_t)m.w * m.h;
  const int64_t stride = (int64_t)gridDim.x * kLutThreads;
  const int64_t lanes = (states + kWave - 1) / kWave * kWave;  // every lane of a wave runs the loop alike
  for (int64_t s = (int64_t)blockIdx.x * kLutThreads + threadIdx.x; s < lanes; s += stride) {
    const bool active = s < states;
    const int64_t k = active ? s / cells : 0;
    const int64_t c = active ? s - k * cells : 0;
    const int32_t j = (int32_t)(c / m.w), i = (int32_t)(c - (int64_t)j * m.w);
    // bin centre angle 2 pi k / n in double, rounded to float (as the oracle's table)
    const float th = (float)(2.0 * M_PI * (double)k / (double)m.n);
    const int32_t r = wave_cast<0, Z>(m, active, (float)i + 0.5f, (float)j + 0.5f, th, max_range);
    if (active) stg(lut + s, (uint16_t)r);
  }
}

// Table lookup: the same guards and bin as a cast, then the stored cast of
// the query's cell and bin.
__global__ __launch_bounds__(kLutThreads) void k_lut_cast(const uint16_t* __restrict__ lut, int32_t w, int32_t h,
                                                          int32_t n, float k_scale, const float* __restrict__ x,
                                                          const float* __restrict__ y,
                                                          const float* __restrict__ th, int64_t count,
                                                          int32_t* __restrict__ out, int32_t* __restrict__ ticks) {
  const int64_t stride = (int64_t)gridDim.x * kLutThreads;
  for (int64_t q = (int64_t)blockIdx.x * kLutThreads + threadIdx.x; q < count; q += stride) {
    const uint64_t t0 = ticks ? wall_clock64() : 0;
    const float xi = ldg(x + q), yi = ldg(y + q), ti = ldg(th + q);
    int32_t r = 0;
    if (fabsf(ti) < 1e6f && xi >= 0.0f && xi < (float)w && yi >= 0.0f && yi < (float)h) {
      const int32_t i = quantize16(xi) >> 16, j = quantize16(yi) >> 16;
      const int32_t k = theta_bin(ti, k_scale, n);
      r = ldg(lut + ((int64_t)k * h + j) * w + i);
    }
    stg(out + q, r);
    if (ticks) stg(ticks + q, (int32_t)(wall_clock64() - t0));
  }
}

}  // namespace
}  // namespace cddt

using namespace cddt;

extern "C" {

int32_t cddt_device_clock_khz(void) {
  int dev = 0, khz = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess) return 0;
  return khz;
}

cddt_status cddt_cast_timed(cddt_map m, const float* x, const float* y, const float* theta, int64_t n,
                            int32_t max_range, int32_t* ranges_out, int32_t* ticks_out, void* stream) {
  if (!m) return fail(CDDT_EINVAL, "cddt_cast_timed: map is NULL");
  if (n < 0) return fail(CDDT_EINVAL, "cddt_cast_timed: n < 0");
  if (max_range < 0 || max_range > 65535) return fail(CDDT_EINVAL, "cddt_cast_timed: max_range must be in 0..65535");
  if (n > 0 && (!x || !y || !theta || !ranges_out || !ticks_out))
    return fail(CDDT_EINVAL, "cddt_cast_timed: NULL array");
  return launch_cast(m->dev(), x, y, theta, n, max_range, ranges_out, (hipStream_t)stream, ticks_out);
}

cddt_status cddt_lut_build(cddt_map m, int32_t max_range, uint16_t* lut, void* stream) {
  if (!m || !lut) return fail(CDDT_EINVAL, "cddt_lut_build: NULL argument");
  if (max_range < 0 || max_range > 65535) return fail(CDDT_EINVAL, "cddt_lut_build: max_range must be in 0..65535");
  const MapDev d = m->dev();
  const int64_t states = (int64_t)d.n * d.w * d.h;
  const int64_t blocks = std::min<int64_t>((states + kLutThreads - 1) / kLutThreads, 1 << 16);
  if (d.zp16)
    hipLaunchKernelGGL(k_lut_build<true>, dim3((unsigned)blocks), dim3(kLutThreads), 0, (hipStream_t)stream, d,
                       max_range, lut, states);
  else
    hipLaunchKernelGGL(k_lut_build<false>, dim3((unsigned)blocks), dim3(kLutThreads), 0, (hipStream_t)stream, d,
                       max_range, lut, states);
  CDDT_HIP(hipGetLastError());
  return CDDT_OK;
}

cddt_status cddt_lut_cast(const uint16_t* lut, int32_t width, int32_t height, int32_t theta_bins, const float* x,
                          const float* y, const float* theta, int64_t n, int32_t* ranges_out, int32_t* ticks_out,
                          void* stream) {
  if (!lut || width < 1 || height < 1 || width > kMaxSide || height > kMaxSide)
    return fail(CDDT_EINVAL, "cddt_lut_cast: bad table or map size");
  if (theta_bins < 2 || theta_bins > kMaxBins || (theta_bins & 1))
    return fail(CDDT_EINVAL, "cddt_lut_cast: theta_bins must be even, 2..8192");
  if (n < 0) return fail(CDDT_EINVAL, "cddt_lut_cast: n < 0");
  if (n == 0) return CDDT_OK;
  if (!x || !y || !theta || !ranges_out) return fail(CDDT_EINVAL, "cddt_lut_cast: NULL array");
  const float k_scale = (float)((double)theta_bins / (2.0 * M_PI));
  const int64_t blocks = std::min<int64_t>((n + kLutThreads - 1) / kLutThreads, 1 << 16);
  hipLaunchKernelGGL(k_lut_cast, dim3((unsigned)blocks), dim3(kLutThreads), 0, (hipStream_t)stream, lut, width,
                     height, theta_bins, k_scale, x, y, theta, n, ranges_out, ticks_out);
  CDDT_HIP(hipGetLastError());
  return CDDT_OK;
}

}  // extern "C"
