// Storage layout of one band ("CDDT bin") of zero points.
//
// Header node (kNodeInts = 32 ints = 128 bytes, one per band):
//   [0] start  offset of the band's region in the zero-point array (multiple of 32)
//   [1] len    number of zero points in the band
//   [2] cap    key capacity (multiple of 32; len <= cap)
//   [3..31]    the band's top search level: its first kTopEntries entries
// Region at `start` (all pieces multiples of 32 ints, so every 32-entry line
// is one aligned 128-byte line):
//   keys       cap slots, the band's zero points ascending in [0, len)
//   level 1    every 32nd key           (stored only if the band can need it)
//   level 2    every 1024th key, ...
// Level t holds ceil(len / 32^t) entries, entry j being key j * 32^t.  The top
// level T is the first one with at most kTopEntries entries; it lives in the
// header node (T = 0 puts the keys themselves there), so a search reads the
// header line and then one line at each level T-1, ..., 0.  Unused slots of the
// last line of every level and of the header are INT_MAX, which no zero point
// reaches (|Z| < 2^31 - 2^28 for maps up to 16384 cells a side), so a search can
// scan whole lines without bounds checks.
#pragma once

#include <hip/hip_runtime.h>

#include <climits>
#include <cstdint>

namespace cddt {

constexpr int kNodeInts = 32;
constexpr int kHeaderWords = 3;
constexpr int kTopEntries = kNodeInts - kHeaderWords;  // 29
constexpr int kLineInts = 32;
constexpr int kLineShift = 5;

__host__ __device__ __forceinline__ uint32_t round_line(uint64_t v) {
  return (uint32_t)((v + kLineInts - 1) & ~(uint64_t)(kLineInts - 1));
}

// Entries at level t for a band of `len` keys: ceil(len / 32^t).
__host__ __device__ __forceinline__ int32_t level_count(int32_t len, int t) {
  for (; t > 0; --t) len = (len + kLineInts - 1) >> kLineShift;
  return len;
}

// Top level of a band of `len` keys.
__host__ __device__ __forceinline__ int top_level(int32_t len) {
  int t = 0;
  while (len > kTopEntries) {
    len = (len + kLineInts - 1) >> kLineShift;
    ++t;
  }
  return t;
}

// Slots reserved for stored level t >= 1 of a band with key capacity cap.
// Level t is stored when a band that fills its capacity would need it, i.e.
// when level t lies below the top level of a full band.
__host__ __device__ __forceinline__ uint32_t level_slots(uint32_t cap, int t) {
  return t < top_level((int32_t)cap) ? round_line((uint64_t)level_count((int32_t)cap, t)) : 0u;
}

// Offset of level t of the band starting at `start` with key capacity `cap`.
__host__ __device__ __forceinline__ uint32_t level_base(uint32_t start, uint32_t cap, int t) {
  if (t == 0) return start;
  uint32_t b = start + cap;
  for (int u = 1; u < t; ++u) b += level_slots(cap, u);
  return b;
}

// Total slots of a band region with key capacity `cap`.
__host__ __device__ __forceinline__ uint64_t region_slots(uint32_t cap) {
  uint64_t s = cap;
  const int tmax = top_level((int32_t)cap);
  for (int t = 1; t < tmax; ++t) s += level_slots(cap, t);
  return s;
}

// Key capacity for a band of `len` keys: room for updates unless static.
__host__ __device__ __forceinline__ uint32_t key_capacity(uint32_t len, bool no_slack) {
  return round_line((uint64_t)len + (no_slack ? 0u : 8u + (len >> 3)));
}

// Sample levels and header top level of a band whose region starts at
// `start` with capacity `cap`, from its len sorted keys at src (the region
// itself, or a copy in LDS); all 64 lanes of the calling wave take part.
__device__ __forceinline__ void band_levels(int32_t* __restrict__ hdr_node, int32_t* __restrict__ zeros,
                                            uint32_t start, int32_t len, uint32_t cap, const int32_t* src) {
  const int lane = threadIdx.x & 63;
  const int T = top_level(len);
  for (int t = 1; t < T; ++t) {
    const int32_t nt = level_count(len, t);
    int32_t* lv = zeros + level_base(start, cap, t);
    for (int32_t k = lane; k < (int32_t)round_line((uint64_t)nt); k += 64)
      lv[k] = k < nt ? src[(int64_t)k << (kLineShift * t)] : INT_MAX;
  }
  const int32_t nT = level_count(len, T);
  if (lane >= kHeaderWords && lane < kNodeInts) {
    const int32_t u = lane - kHeaderWords;
    hdr_node[lane] = u < nT ? src[(int64_t)u << (kLineShift * T)] : INT_MAX;
  }
}

// Padding, sample levels and header top level of one band from its sorted
// keys in place; all 64 lanes of the calling wave take part.  Used after
// construction and after an update changes the band in place.
__device__ inline void finalize_band(int32_t* __restrict__ hdr_node, int32_t* __restrict__ zeros) {
  const int lane = threadIdx.x & 63;
  const uint32_t start = (uint32_t)hdr_node[0];
  const int32_t len = hdr_node[1];
  const uint32_t cap = (uint32_t)hdr_node[2];
  for (int32_t k = len + lane; k < (int32_t)round_line((uint64_t)len); k += 64) zeros[start + k] = INT_MAX;
  band_levels(hdr_node, zeros, start, len, cap, zeros + start);
}

}  // namespace cddt
