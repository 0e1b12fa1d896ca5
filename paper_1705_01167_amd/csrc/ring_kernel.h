// The resident serving kernel: one launch that admits requests while it runs.
//
// Host threads write each request into a slot of a ring in fine-grained
// (uncached) pinned host memory: its inputs, its filter descriptor and the
// global numbers of its tiles (tile t of the service belongs to the slot
// tilemap[t & mask]).  Publishing a request raises the host's count of
// published tiles.  Block 0's first wave is the watcher: it mirrors that
// count into device memory, so that the other waves wait on device memory
// instead of all reading host memory.  Every other wave takes the next tile
// ticket from a device counter, sleeps until its tile is published, computes
// the tile with the batched kernel's per-tile routine, and counts it done for
// its request; the wave that finishes a request's last tile clears the count
// and writes the request's completion word back into host memory.
//
// Exit: the watcher leaves when the host asks the kernel to drain, or when no
// tile has been published for `watch_ticks` of the constant wall clock, and
// then tells every wave to leave (the top bit of the device copy of the
// count); a worker also leaves by itself after `idle_ticks` without work.  A wave may leave holding an unpublished ticket;
// the host gives requests that an ended kernel left unfinished new tile
// numbers before the next launch.
//
// Ordering.  Every word the host writes (inputs, descriptors, tile map, the
// published count) and every log-weight and completion word the kernel writes
// lives in pinned host memory and is read and written by system-coherent
// loads and stores (relaxed atomics at system scope), which bypass the L2:
// a load returns the host's current value and a store is performed at the
// host once it is acknowledged.  So no cache needs flushing or invalidating:
// a wave reads a slot only after it has seen the published count cover its
// tile (a branch on the loaded value), waits for its log-weight stores to be
// acknowledged before counting its tile done, and the request's last wave
// writes the completion word after seeing every tile counted.  Acquire and
// release fences at system scope would write back and invalidate the L2 on
// every poll and every tile.
#pragma once

#include "batch_kernel.h"

namespace cddt {

// Control words in pinned host memory (one 64-byte line).
struct RingCtl {
  int64_t pub;    // tiles published so far (written by the host, release)
  int32_t drain;  // the host asks the kernel to leave
  int32_t pad[13];
};
static_assert(sizeof(RingCtl) == 64, "one line");

// One request slot in pinned host memory, written before its tiles are published.
struct RingSlot {
  FilterDev f;      // inputs and log-weights point into the slot's region of the pinned arena
  int64_t t_begin;  // global number of the request's first tile
  int32_t n_tiles;
  int32_t ppt;      // particles per tile of this request
  int64_t id;       // the completion word receives id + 1
  int64_t pad2;
};
static_assert(sizeof(RingSlot) % 64 == 0, "slots stay line-aligned");

// Device-side counters, 256 bytes apart.
struct RingDev {
  unsigned long long claim;  // next tile ticket
  unsigned long long pad0[31];
  unsigned long long dpub;   // the watcher's copy of RingCtl::pub; kRingLeave set as the watcher leaves
  unsigned long long pad1[31];
};
constexpr unsigned long long kRingLeave = 1ull << 63;

namespace {

// Before a launch: tickets start at `base`, nothing published past it yet,
// no drain, every slot's tile count zero.
__global__ void k_ring_reset(RingDev* rd, unsigned long long base, uint32_t* tiles_done, int32_t n_slots) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) {
    rd->claim = base;
    rd->dpub = base;
  }
  for (int k = i; k < n_slots; k += gridDim.x * blockDim.x) tiles_done[k] = 0u;
}

constexpr int kRingSlotWords = (int)(sizeof(RingSlot) / 4);
static_assert(kRingSlotWords <= kWave, "a slot is read by one load per lane");

// The slot of a published tile, read word by word across the wave's lanes
// (vector loads of uncached host memory) and gathered into uniform registers.
__device__ __forceinline__ RingSlot load_ring_slot(const RingSlot* p, int lane) {
  const uint32_t* src = reinterpret_cast<const uint32_t*>(p);
  const uint32_t v = lane < kRingSlotWords ? ldx<true>(src + lane) : 0u;
  union {
    RingSlot s;
    uint32_t w[kRingSlotWords];
  } u;
#pragma unroll
  for (int k = 0; k < kRingSlotWords; ++k) u.w[k] = (uint32_t)__builtin_amdgcn_readlane((int32_t)v, k);
  return u.s;
}

// Wait until every load and store this wave has issued is complete (stores
// acknowledged); the signal fences keep the compiler from moving memory
// operations across the wait.
__device__ __forceinline__ void wait_all_memory() {
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_s_waitcnt(0);
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

__device__ __forceinline__ unsigned long long lane0_u64(unsigned long long v) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int32_t)(uint32_t)v);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int32_t)(uint32_t)(v >> 32));
  return ((unsigned long long)hi << 32) | lo;
}

__device__ __forceinline__ void ring_watch(RingCtl* ctl, RingDev* rd, uint64_t watch_ticks) {
  const int lane = threadIdx.x & (kWave - 1);
  unsigned long long last = 0;
  uint64_t since = wall_clock64();
  for (;;) {
    unsigned long long p = 0;
    int32_t drain = 0;
    if (lane == 0) {
      p = (unsigned long long)__hip_atomic_load(&ctl->pub, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
      drain = __hip_atomic_load(&ctl->drain, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    }
    p = lane0_u64(p);
    drain = __builtin_amdgcn_readfirstlane(drain);
    const uint64_t now = wall_clock64();
    if (p > last) {
      if (lane == 0) __hip_atomic_store(&rd->dpub, p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      last = p;
      since = now;
    } else if (now - since > watch_ticks) {
      drain = 1;
    }
    if (drain) {
      if (lane == 0) __hip_atomic_store(&rd->dpub, last | kRingLeave, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return;
    }
    __builtin_amdgcn_s_sleep(4);
  }
}

// Mode: the batched kernel's search mode (0, or a queued mode 6..8).
template <int Mode, bool Z>
__global__ __launch_bounds__(kMaxBatchThreads) void k_resident(RingCtl* ctl, const RingSlot* __restrict__ slots,
                                                               const int32_t* __restrict__ tilemap, int64_t mask,
                                                               int64_t* done, RingDev* rd,
                                                               uint32_t* __restrict__ tiles_done, int32_t n_slots,
                                                               uint64_t idle_ticks, uint64_t watch_ticks) {
  extern __shared__ int2 smem_jobs[];
  constexpr int Q = tile_q(Mode);
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  if (blockIdx.x == 0) {
    if (wave == 0) ring_watch(ctl, rd, watch_ticks);
    return;
  }
  int2* jobs = smem_jobs + wave * Q * kWave;
  int32_t* codes = reinterpret_cast<int32_t*>(smem_jobs + nw * Q * kWave) + wave * Q * kWave;
  int32_t* later = reinterpret_cast<int32_t*>(smem_jobs + nw * Q * kWave) + (nw + wave) * Q * kWave;
  auto claim = [&]() {
    unsigned long long v = 0;
    if (lane == 0) v = atomicAdd(&rd->claim, 1ull);
    return lane0_u64(v);
  };
  unsigned long long t = claim();
  for (;;) {
    // wait, sleeping, until tile t is published (or leave); a wave whose
    // ticket lies far beyond the published count sleeps longer between polls
    const uint64_t since = wall_clock64();
    for (;;) {
      unsigned long long p = 0;
      if (lane == 0) p = __hip_atomic_load(&rd->dpub, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      p = lane0_u64(p);
      if (p & kRingLeave) return;
      if (t < p) break;
      if (wall_clock64() - since > idle_ticks) return;
      const uint64_t gap = t - p;
      for (uint64_t k = 0; k <= (gap >> 7) && k < 8; ++k) __builtin_amdgcn_s_sleep(16);
    }
    const int32_t slot =
        __builtin_amdgcn_readfirstlane(lane == 0 ? ldx<true>(tilemap + (int64_t)(t & (uint64_t)mask)) : 0);
    if ((uint32_t)slot >= (uint32_t)n_slots) {  // never written: not a tile of any request
      t = claim();
      continue;
    }
    const RingSlot s = load_ring_slot(slots + slot, lane);
    const FilterDev& f = s.f;
    if (t < (uint64_t)s.t_begin || t >= (uint64_t)s.t_begin + (uint64_t)s.n_tiles) {
      // a tile number the host has since given to another request: skip it
      // (its request, if unfinished, is given new tiles when this launch ends)
      t = claim();
      continue;
    }
    const int64_t p0 = (int64_t)(t - (uint64_t)s.t_begin) * s.ppt;
    const int64_t p1 = p0 + s.ppt < f.n_particles ? p0 + s.ppt : f.n_particles;
    bool queued = false;
    if constexpr (Q > 0) {
      if (f.n_rays <= kWave) {
        for (int64_t p = p0; p < p1; p += Q)
          wave_tile_logw<Q, false, Z, true>(f, p, (int32_t)min((int64_t)Q, p1 - p), jobs, codes, later);
        queued = true;
      }
    }
    if (!queued) {
      for (int64_t p = p0; p < p1; ++p) {
        const float lw =
            wave_particle_logw<0, Z, true>(f.map, ldx<true>(f.px + p), ldx<true>(f.py + p), ldx<true>(f.pth + p),
                                           f.offsets, f.obs, f.n_rays, f.pair_offset, f.table, f.max_range, nullptr);
        if (lane == 0) stx<true>(f.logw + p, lw);
      }
    }
    // this tile's log-weight stores are acknowledged (performed at the host)
    // before the tile counts as done
    wait_all_memory();
    uint32_t before = 0;
    if (lane == 0) before = __hip_atomic_fetch_add(tiles_done + slot, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    before = (uint32_t)__builtin_amdgcn_readfirstlane((int32_t)before);
    if (before + 1 == (uint32_t)s.n_tiles && lane == 0) {
      // the request's last tile: every other tile was counted after its stores
      __hip_atomic_store(tiles_done + slot, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      wait_all_memory();
      __hip_atomic_store(done + slot, s.id + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    }
    t = claim();
  }
}

}  // namespace
}  // namespace cddt
