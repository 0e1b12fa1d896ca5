// Device-side types and helpers of libcddt: the per-map and per-filter
// descriptors that kernels take by value, and the edge-cell test.
#pragma once

#include <hip/hip_runtime.h>

#include <climits>
#include <cstdint>

namespace cddt {

// One stored slice: direction (2^30 fixed point), the offset that turns a
// lateral band number into a global band index, and the bucket origin (the
// lowest along-slice projection of the map rectangle, Q16).
struct SliceDev {
  int32_t c, s;
  int32_t row_off;  // global band = row_off + (lateral projection >> 46)
  int32_t zlo;
};

// Everything a query needs about one map, passed by value to kernels.
struct MapDev {
  const uint8_t* occ;        // W*H grid, row-major, nonzero = occupied
  const SliceDev* slices;    // n/2 entries
  const int32_t* hdr;        // per band: a 128-byte header node (band_layout.h)
  const int32_t* zeros;      // band regions: keys (Q16, ascending) and sample levels
  const int32_t* bk;         // bucket index lines (nullptr: no bucket index)
  int32_t w, h, n, half;
  float k_scale;             // (float)(n / (2 pi))
  int32_t bshift;            // bucket width 2^bshift in Q16 units
  int32_t nbk;               // buckets per band
  int32_t zp16;              // bucket lines hold 16-bit zero points (1/8-cell bins)
};

// One filter of a batched step (device copy of cddt_filter plus its map).
struct FilterDev {
  MapDev map;
  const float* px;
  const float* py;
  const float* pth;
  const float* offsets;
  const int32_t* obs;
  const float* table;
  float* logw;
  int32_t* ranges;
  int64_t n_particles;
  int32_t n_rays, pair_offset, max_range, pad;
};

constexpr int kWave = 64;

// Edge-map test of cell (i, j) (Sec. IV-C): occupied, and at least one of its
// 8 neighbours is free or off the map.  With `full` every occupied cell counts.
__device__ __forceinline__ bool edge_cell(const uint8_t* __restrict__ occ, int w, int h, int i, int j, int full) {
  if (occ[(size_t)j * w + i] == 0) return false;
  if (full) return true;
  for (int dj = -1; dj <= 1; ++dj) {
    const int b = j + dj;
    if (b < 0 || b >= h) return true;  // off-map neighbour counts as free
    for (int di = -1; di <= 1; ++di) {
      const int a = i + di;
      if (a < 0 || a >= w) return true;
      if (occ[(size_t)b * w + a] == 0) return true;
    }
  }
  return false;
}
constexpr int kMaxSide = 16384;
constexpr int kMaxBins = 8192;
constexpr int kMaxRays = 1024;
// Bucket index line: [0] last key before the bucket (INT_MIN: none), [1] first
// key after it (INT_MAX: none), [2..31] its keys ascending, INT_MAX padded; all
// relative to the slice's zlo.  An overflowing bucket holds kBucketOverflow
// in [0] and zlo in [1].
constexpr int kBucketKeys = 30;
// With 16-bit zero points a line holds [0] the previous key's bin centre,
// [1] the next key's bin centre (both relative to zlo, INT_MIN / INT_MAX for
// none) and [2..31] 60 bin indices relative to the bucket's first bin, two per
// word (low half first), ascending, padded with 0xffff.
constexpr int kBucketKeys16 = 60;
constexpr int kBinShift = 13;  // 1/8 cell in Q16
constexpr int32_t kBucketOverflow = INT_MIN + 1;
constexpr int kBucketLog2Default = 7;
// Bytes of device memory holding the persistent batched kernel's tile counters.
constexpr size_t kBatchCounterBytes = 2048;

}  // namespace cddt
