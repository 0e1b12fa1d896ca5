// Measurement helpers for the paper's query-time suites (Sec. VI: casts from
// a uniformly spaced grid of states and from uniformly random states, timed
// per query) and two of its comparators (Sec. II-III): the dense lookup table
// (the range of every discrete state stored in a 3-D table) and a cell-by-cell
// walk along the exact ray (the family of Bresenham's line; here the exact
// traversal of Amanatides and Woo).
//
// cddt_cast_timed runs the same kernels as cddt_cast and also records, per
// ray, the device wall-clock ticks its wave spent on it.  The table holds, for
// every bin k and cell (i, j), the cast from the cell centre at the bin's
// centre angle, computed by this library's own cast (so from grid states the
// table and the CDDT agree exactly); a table lookup rounds the query to its
// cell and bin.
#include <algorithm>

#include "cddt_common.h"
#include "det_math.h"
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

// Cell walk: from the query position along (cos theta, sin theta) (theta not
// binned; sin and cos from det_math.h), stepping from cell to cell in the
// order the exact ray enters them (ties step in y), the range is the entry
// distance into the first occupied cell, rounded half up and capped at
// max_range, or max_range when the ray leaves the map first; the cast's
// guards give 0 (including a query in an occupied cell).  In double, every
// operation as written.
__device__ int32_t march_one(const uint8_t* __restrict__ occ, int32_t w, int32_t h, float x, float y, float th,
                             int32_t max_range) {
  if (!(fabsf(th) < 1e6f) || !(x >= 0.0f && x < (float)w && y >= 0.0f && y < (float)h)) return 0;
  const double px = (double)x, py = (double)y;
  int32_t i = (int32_t)floor(px), j = (int32_t)floor(py);
  if (ldg(occ + (size_t)j * w + i) != 0) return 0;
  double dy, dx;
  sin_cos((double)th, dy, dx);
  const int32_t si = dx > 0.0 ? 1 : -1, sj = dy > 0.0 ? 1 : -1;
  const double inf = __builtin_huge_val();
  double tmx = inf, tdx = inf, tmy = inf, tdy = inf;
  if (dx != 0.0) {
    tmx = ((double)(dx > 0.0 ? i + 1 : i) - px) / dx;
    tdx = fabs(1.0 / dx);
  }
  if (dy != 0.0) {
    tmy = ((double)(dy > 0.0 ? j + 1 : j) - py) / dy;
    tdy = fabs(1.0 / dy);
  }
  const double limit = (double)max_range + 0.5;  // entries at or beyond round to max_range or more
  for (;;) {
    double t;
    if (tmx < tmy) {
      t = tmx;
      i += si;
      tmx += tdx;
    } else {
      t = tmy;
      j += sj;
      tmy += tdy;
    }
    if (t >= limit || i < 0 || i >= w || j < 0 || j >= h) return max_range;
    if (ldg(occ + (size_t)j * w + i) != 0) return (int32_t)floor(t + 0.5);
  }
}

__global__ __launch_bounds__(kLutThreads) void k_march_cast(const uint8_t* __restrict__ occ, int32_t w, int32_t h,
                                                            const float* __restrict__ x, const float* __restrict__ y,
                                                            const float* __restrict__ th, int64_t count,
                                                            int32_t max_range, int32_t* __restrict__ out,
                                                            int32_t* __restrict__ ticks) {
  const int64_t stride = (int64_t)gridDim.x * kLutThreads;
  for (int64_t q = (int64_t)blockIdx.x * kLutThreads + threadIdx.x; q < count; q += stride) {
    const uint64_t t0 = ticks ? wall_clock64() : 0;
    const int32_t r = march_one(occ, w, h, ldg(x + q), ldg(y + q), ldg(th + q), max_range);
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

cddt_status cddt_march_cast(cddt_map m, const float* x, const float* y, const float* theta, int64_t n,
                            int32_t max_range, int32_t* ranges_out, int32_t* ticks_out, void* stream) {
  if (!m) return fail(CDDT_EINVAL, "cddt_march_cast: map is NULL");
  if (n < 0) return fail(CDDT_EINVAL, "cddt_march_cast: n < 0");
  if (max_range < 0 || max_range > 65535) return fail(CDDT_EINVAL, "cddt_march_cast: max_range must be in 0..65535");
  if (n == 0) return CDDT_OK;
  if (!x || !y || !theta || !ranges_out) return fail(CDDT_EINVAL, "cddt_march_cast: NULL array");
  const int64_t blocks = std::min<int64_t>((n + kLutThreads - 1) / kLutThreads, 1 << 16);
  hipLaunchKernelGGL(k_march_cast, dim3((unsigned)blocks), dim3(kLutThreads), 0, (hipStream_t)stream, m->d_occ, m->w,
                     m->h, x, y, theta, n, max_range, ranges_out, ticks_out);
  CDDT_HIP(hipGetLastError());
  return CDDT_OK;
}

}  // extern "C"
