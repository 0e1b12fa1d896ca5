// Bucket index lines of one band, written by one wave (the line format is in
// device_types.h).  Used by the full fill after a build and by the band edits
// of an incremental update, which rewrite only the lines an edit can change.
//
// first[b], b = 0..nbk, is the index of the band's first key at or after the
// start of bucket b (len when there is none): one pass over the keys in order
// lets key k claim the buckets after its predecessor's bucket up to its own.
// A bucket's line then follows from first[b] and first[b + 1].  The keys may
// sit in LDS or in global memory; first[] and the marks live in LDS.
#pragma once

#include <hip/hip_runtime.h>

#include <climits>
#include <cstdint>

#include "band_layout.h"
#include "device_types.h"

namespace cddt {

// Orders the calling wave's memory operations for its other lanes.  A wave's
// LDS operations are performed in order, so no wait is needed; the fence
// keeps the compiler from moving accesses across it.
__device__ __forceinline__ void wave_fence() { __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront"); }

// Buckets per band are at most (16384 sqrt(2) cells) / 2^4 + 1 = 1449: the
// longest slice extent of the largest map at the narrowest bucket width.
constexpr int kFillMaxBuckets = 1456;

// The slice of a band: the last s with row_start[s] <= band (row_start rises
// from row_start[0] = 0).  A 64-ary search by the whole wave, one candidate
// per lane and the ballot's count as the answer: two dependent loads instead
// of log2(half).  `band` is the same on every lane.
static_assert(kMaxBins / 2 <= 64 * 64, "two levels of 64 candidates cover every slice count");
__device__ __forceinline__ int32_t band_slice(const int32_t* __restrict__ row_start, int32_t half, uint32_t band) {
  const int lane = threadIdx.x & 63;
  const int32_t stride = (half + 63) >> 6;
  int32_t s = lane * stride;
  uint64_t m = __ballot(s < half && (uint32_t)row_start[s] <= band);
  int32_t lo = (__popcll(m) - 1) * stride;
  if (stride > 1) {
    s = lo + lane;
    m = __ballot(lane < stride && s < half && (uint32_t)row_start[s] <= band);
    lo += __popcll(m) - 1;
  }
  return lo;
}

// Bucket of key z, nbk for keys past the last bucket (z >= zlo, so the
// difference fits 32 unsigned bits).
__device__ __forceinline__ int32_t bucket_of(int32_t z, int32_t zlo, int32_t shift, int32_t nbk) {
  return (int32_t)min(((uint32_t)z - (uint32_t)zlo) >> shift, (uint32_t)nbk);
}

// first[0..nbk] of keys[0, len) (keys ascending, all >= zlo).
__device__ __forceinline__ void bucket_firsts(const int32_t* keys, int32_t len, int32_t zlo, int32_t shift,
                                              int32_t nbk, int32_t* first) {
  const int lane = threadIdx.x & 63;
  for (int32_t b = lane; b <= nbk; b += 64) first[b] = len;
  wave_fence();
  for (int32_t k0 = 0; k0 < len; k0 += 64) {
    const int32_t k = k0 + lane;
    if (k < len) {
      const int32_t bk_k = bucket_of(keys[k], zlo, shift, nbk);
      const int32_t bk_p = k > 0 ? bucket_of(keys[k - 1], zlo, shift, nbk) : -1;
      for (int32_t b = bk_p + 1; b <= bk_k; ++b) first[b] = k;  // key k is the first at or after bucket b
    }
  }
  wave_fence();
}

// first[0..nbk] of keys[0, len) in LDS, 16-byte aligned: each lane takes four
// consecutive keys.
__device__ __forceinline__ void bucket_firsts4(const int32_t* keys, int32_t len, int32_t zlo, int32_t shift,
                                               int32_t nbk, int32_t* first) {
  const int lane = threadIdx.x & 63;
  for (int32_t b = lane; b <= nbk; b += 64) first[b] = len;
  wave_fence();
  for (int32_t k0 = 4 * lane; k0 < len; k0 += 256) {
    const int4 v = *reinterpret_cast<const int4*>(keys + k0);
    int32_t bp = k0 > 0 ? bucket_of(keys[k0 - 1], zlo, shift, nbk) : -1;
    const int32_t kv[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      if (k0 + c < len) {
        const int32_t bk = bucket_of(kv[c], zlo, shift, nbk);
        for (int32_t b = bp + 1; b <= bk; ++b) first[b] = k0 + c;
        bp = bk;
      }
    }
  }
  wave_fence();
}

// Marks the buckets whose line inserting or removing zero point z can change
// (first[] of the edited keys): z's bucket and, on each side, the empty
// buckets up to and including the first one that holds a key (they carry z as
// their next or previous key).  Called by the lanes that hold a record.
__device__ __forceinline__ void mark_around(int32_t z, int32_t zlo, int32_t shift, int32_t nbk,
                                            const int32_t* first, uint8_t* mark) {
  const int32_t bz = (int32_t)min(max(((int64_t)z - zlo) >> shift, (int64_t)0), (int64_t)nbk - 1);
  mark[bz] = 1;
  for (int32_t b = bz - 1; b >= 0; --b) {
    mark[b] = 1;
    if (first[b] < first[b + 1]) break;
  }
  for (int32_t b = bz + 1; b < nbk; ++b) {
    mark[b] = 1;
    if (first[b] < first[b + 1]) break;
  }
}

// Entry j of bucket b's line, from the band's keys (the line format is in
// device_types.h); i0, i1 = first[b], first[b + 1].
__device__ __forceinline__ int32_t line_entry(const int32_t* keys, int32_t len, int32_t zlo, int32_t shift,
                                              int32_t b, int32_t i0, int32_t i1, int j, int zp16) {
  const int32_t n_in = i1 - i0;
  if (n_in > (zp16 ? kBucketKeys16 : kBucketKeys)) return j == 0 ? kBucketOverflow : (j == 1 ? zlo : 0);
  if (j < 2) {  // the previous and the next key (16-bit lines: their bin centres)
    const bool ok = j == 0 ? i0 > 0 : i1 < len;
    const int32_t none = j == 0 ? INT_MIN : INT_MAX;
    if (!ok) return none;
    const int32_t z = keys[j == 0 ? i0 - 1 : i1] - zlo;
    return zp16 ? (z >> kBinShift) * 8192 + 4096 : z;
  }
  if (!zp16) return j - 2 < n_in ? keys[i0 + j - 2] - zlo : INT_MAX;
  // two bins per word, relative to the bucket's first bin, low half first
  const int32_t base = b << (shift - kBinShift);
  const int k = 2 * (j - 2);
  const int32_t lo = k < n_in ? ((keys[i0 + k] - zlo) >> kBinShift) - base : 0xffff;
  const int32_t hi = k + 1 < n_in ? ((keys[i0 + k + 1] - zlo) >> kBinShift) - base : 0xffff;
  return (int32_t)(((uint32_t)hi << 16) | (uint32_t)lo);
}

// One lane per bucket: writes the line of every bucket (mark null) or of every
// marked one.  Gather: every entry of a line is loaded before its stores (the
// loads of all lanes in flight together; for keys in global memory);
// otherwise a line is built and stored 16 bytes at a time (fewer registers).
// first_old (nullable) holds first[] of the band before an edit; the return
// value is this lane's share of the change of the overflowing-bucket count.
template <bool Gather>
__device__ __forceinline__ int write_bucket_lines(const int32_t* keys, int32_t len, int32_t zlo, int32_t shift,
                                                  int32_t nbk, const int32_t* first, const uint8_t* mark,
                                                  const int32_t* first_old, int32_t* __restrict__ lines, int zp16) {
  const int lane = threadIdx.x & 63;
  const int cap_keys = zp16 ? kBucketKeys16 : kBucketKeys;
  int over_delta = 0;
  for (int32_t b0 = 0; b0 < nbk; b0 += 64) {
    const int32_t b = b0 + lane;
    if (b >= nbk || (mark && !mark[b])) continue;
    const int32_t i0 = first[b], i1 = first[b + 1];
    int4* line = reinterpret_cast<int4*>(lines + (int64_t)b * kLineInts);
    if constexpr (Gather) {
      int32_t e[kLineInts];
#pragma unroll
      for (int j = 0; j < kLineInts; ++j) e[j] = line_entry(keys, len, zlo, shift, b, i0, i1, j, zp16);
#pragma unroll
      for (int q = 0; q < kLineInts / 4; ++q) line[q] = make_int4(e[4 * q], e[4 * q + 1], e[4 * q + 2], e[4 * q + 3]);
    } else {
#pragma unroll
      for (int q = 0; q < kLineInts / 4; ++q)
        line[q] = make_int4(line_entry(keys, len, zlo, shift, b, i0, i1, 4 * q, zp16),
                            line_entry(keys, len, zlo, shift, b, i0, i1, 4 * q + 1, zp16),
                            line_entry(keys, len, zlo, shift, b, i0, i1, 4 * q + 2, zp16),
                            line_entry(keys, len, zlo, shift, b, i0, i1, 4 * q + 3, zp16));
    }
    const int old_over = first_old ? (first_old[b + 1] - first_old[b] > cap_keys ? 1 : 0) : 0;
    over_delta += (i1 - i0 > cap_keys ? 1 : 0) - old_over;
  }
  return over_delta;
}

// Half a wave per bucket, for keys in LDS: the buckets set in `mask` (bit i:
// bucket b0 + i) are written two at a time, lanes 0-31 one line and lanes
// 32-63 the next, lane j writing entry j (one 128-byte store per half).
// old_n(b) is the bucket's key count before the edit.  The return value is
// this lane's share of the change of the overflowing-bucket count.
template <class OldN>
__device__ __forceinline__ int write_lines_halves(const int32_t* keys, int32_t len, int32_t zlo, int32_t shift,
                                                  int32_t b0, uint64_t mask, const int32_t* first,
                                                  int32_t* __restrict__ lines, int zp16, OldN old_n) {
  const int lane = threadIdx.x & 63, j = lane & 31;
  const int cap_keys = zp16 ? kBucketKeys16 : kBucketKeys;
  int over_delta = 0;
  while (mask) {
    const int ba = __builtin_ctzll(mask);
    mask &= mask - 1;
    const int bb = mask ? __builtin_ctzll(mask) : -1;
    if (mask) mask &= mask - 1;
    const int bo = lane < 32 ? ba : bb;
    if (bo >= 0) {
      const int32_t b = b0 + bo;
      const int32_t i0 = first[b], i1 = first[b + 1];
      lines[(int64_t)b * kLineInts + j] = line_entry(keys, len, zlo, shift, b, i0, i1, j, zp16);
      if (j == 0) over_delta += (i1 - i0 > cap_keys ? 1 : 0) - (old_n(b) > cap_keys ? 1 : 0);
    }
  }
  return over_delta;
}

}  // namespace cddt
