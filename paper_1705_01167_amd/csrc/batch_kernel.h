// The persistent batched kernel: every wave repeatedly takes the next tile
// index from the 64-bit device counter of its part of the tiles, finds its
// filter (from the tile map when the caller provides one, else by binary
// search over the prefix sums of tile counts) and computes the tile's particle
// weights with the same per-particle routine as the plain kernel.
#pragma once

#include "query_device.h"

namespace cddt {
namespace {

// Tiles are split into kTileParts contiguous parts, one counter each, 256
// bytes apart: blocks are dispatched to the 8 XCDs in turn, so block b starts
// on part b % 8, and the device-scope increments of one launch spread over
// eight addresses instead of queueing on one.  A wave whose part is used up
// reads all eight counters at once and moves on to the next part that still
// has tiles; it leaves when none has.
constexpr int kTileParts = 8;
constexpr int kCounterStride = 32;  // 64-bit words between counters
static_assert(kTileParts * kCounterStride * sizeof(unsigned long long) == kBatchCounterBytes, "counter block size");

__global__ void k_reset_counter(unsigned long long* counter) {
  if (threadIdx.x < kTileParts) counter[threadIdx.x * kCounterStride] = 0ull;
}

__device__ __forceinline__ uint64_t uniform_u64(uint64_t v) {
  uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  return ((uint64_t)hi << 32) | lo;
}

// Search modes (the tuning's search_mode): 0 one lane per search, one particle
// per wave at a time; 1..5 eight lanes per search with that many searches per
// group in flight; 6 / 7 / 8 one lane per search with the searches of 4 / 8 /
// 16 particles queued in LDS and drained together, one search per lane per
// round; 9 / 10 the same with 8 / 16 particles and two searches per lane per
// round (ray layouts of <= 64 rays; longer layouts fall back to mode 0).
constexpr int kModeTile4 = 6, kModeTile8 = 7, kModeTile16 = 8, kModeTile8x2 = 9, kModeTile16x2 = 10;
__host__ __device__ constexpr int tile_q(int mode) {
  return (mode == kModeTile4) ? 4
         : (mode == kModeTile8 || mode == kModeTile8x2) ? 8
         : (mode == kModeTile16 || mode == kModeTile16x2) ? 16
                                                          : 0;
}
__host__ __device__ constexpr bool tile_x2(int mode) { return mode == kModeTile8x2 || mode == kModeTile16x2; }

constexpr int kMaxBatchThreads = 512;

// Dynamic LDS of one block: per wave and queued particle slot, a search job
// (int2, whose first word later holds the packed result), the lane's result
// code (int32) and, for the one-search-per-lane modes, a slot of the queue of
// searches left for the full pass (int32).
__host__ __device__ constexpr size_t tile_lds_bytes(int mode, int waves) {
  return (size_t)waves * tile_q(mode) * kWave *
         (sizeof(int2) + sizeof(int32_t) + (tile_x2(mode) ? 0 : sizeof(int32_t)));
}

// Z: instantiated for batches that hold a map with 16-bit zero points in its
// bucket lines (the plain instantiation has no code for them).
// tilemap (nullable): per tile {filter, first particle, end particle, 0}; a
// tile may be empty (first == end).  Without it tile t of filter f covers
// particles [t ppt, (t + 1) ppt) of f (the last tile clipped).
template <int Mode, bool Z>
__global__ __launch_bounds__(kMaxBatchThreads) void k_batch(const FilterDev* __restrict__ filters, const int64_t* __restrict__ prefix,
                        const int4* __restrict__ tilemap, int32_t n_filters, int64_t total_tiles, int32_t ppt,
                        unsigned long long* __restrict__ counter) {
  extern __shared__ int2 smem_jobs[];
  constexpr int Q = tile_q(Mode);
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  int2* jobs = smem_jobs + wave * Q * kWave;
  int32_t* codes = reinterpret_cast<int32_t*>(smem_jobs + nw * Q * kWave) + wave * Q * kWave;
  int32_t* later = reinterpret_cast<int32_t*>(smem_jobs + nw * Q * kWave) + (nw + wave) * Q * kWave;
  int part = (int)(blockIdx.x % kTileParts);
  // Tickets: lane 0 claims the next ticket of its part while the current tile
  // runs, so the atomic's round trip overlaps the tile's own loads.  Every
  // claimed ticket is used: in range it is the next tile, out of range it
  // moves the wave to the next part.
  auto claim = [&](int pt) {
    unsigned long long v = 0;
    if (lane == 0) v = atomicAdd(counter + pt * kCounterStride, 1ull);
    return v;
  };
  unsigned long long ticket = claim(part);
  for (;;) {
    const uint64_t part_lo = (uint64_t)total_tiles * part / kTileParts;
    const uint64_t part_hi = (uint64_t)total_tiles * (part + 1) / kTileParts;
    const uint64_t t = uniform_u64(ticket) + part_lo;  // lane 0's ticket (the first active lane)
    if (t >= part_hi) {
      // This part is used up.  Read every part's counter at once (lane k reads
      // part k) and move to the next part in turn that still has tiles; leave
      // when none has.  Counters only grow, so a part seen used up stays used
      // up, and every tile is still handed out by exactly one claim.
      bool left = false;
      if (lane < kTileParts) {
        const uint64_t lo = (uint64_t)total_tiles * lane / kTileParts;
        const uint64_t hi = (uint64_t)total_tiles * (lane + 1) / kTileParts;
        const unsigned long long c =
            __hip_atomic_load(counter + lane * kCounterStride, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        left = c < hi - lo;
      }
      const uint32_t have = (uint32_t)__ballot(left) & ((1u << kTileParts) - 1u);
      if (have == 0) break;
      // the first part with tiles at or after part + 1, cyclically
      const uint32_t rot = ((have >> (part + 1)) | (have << (kTileParts - part - 1))) & ((1u << kTileParts) - 1u);
      part = (part + 1 + __builtin_ctz(rot)) % kTileParts;
      ticket = claim(part);
      continue;
    }
    ticket = claim(part);
    // the tile's filter and particles: one load from the tile map, or
    // prefix[lo] <= t < prefix[hi]; by scalar loads, which wait on their own
    // counter, not behind the ticket claim and other vector loads in flight
    // (both arrays are written before the launch, so the scalar cache is current)
    int32_t lo = 0;
    int64_t p0, p1;
    if (tilemap) {
      const __attribute__((address_space(4))) int32_t* stm =
          (const __attribute__((address_space(4))) int32_t*)tilemap;
      lo = stm[4 * t];
      p0 = stm[4 * t + 1];
      p1 = stm[4 * t + 2];
      if (p0 >= p1) continue;  // an empty tile
    } else {
      const __attribute__((address_space(4))) int64_t* sprefix =
          (const __attribute__((address_space(4))) int64_t*)prefix;
      int32_t hi = n_filters;
      while (hi - lo > 1) {
        int32_t mid = (lo + hi) >> 1;
        if ((uint64_t)sprefix[mid] <= t)
          lo = mid;
        else
          hi = mid;
      }
      p0 = (int64_t)(t - (uint64_t)sprefix[lo]) * ppt;
      p1 = -1;
    }
    const FilterDev f = filters[lo];
    if (p1 < 0) p1 = p0 + ppt < f.n_particles ? p0 + ppt : f.n_particles;
    if constexpr (Q > 0) {
      if (f.n_rays <= kWave) {
        for (int64_t p = p0; p < p1; p += Q)
          wave_tile_logw<Q, tile_x2(Mode), Z>(f, p, (int32_t)min((int64_t)Q, p1 - p), jobs, codes, later);
        continue;
      }
    }
    constexpr int K = Q > 0 ? 0 : Mode;
    for (int64_t p = p0; p < p1; ++p) {
      float lw = wave_particle_logw<K, Z>(f.map, ldg(f.px + p), ldg(f.py + p), ldg(f.pth + p), f.offsets, f.obs,
                                       f.n_rays, f.pair_offset, f.table, f.max_range,
                                       f.ranges ? f.ranges + p * f.n_rays : nullptr);
      if (lane == 0) stg(f.logw + p, lw);
    }
  }
}

}  // namespace
}  // namespace cddt
