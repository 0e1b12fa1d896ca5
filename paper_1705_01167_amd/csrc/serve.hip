// Continuous-batching server over resident CDDT maps.
//
// Requests (one robot: its particles and one scan on one resident map) are
// queued by host threads.  A scheduler thread owns `n_lanes` lanes; each lane
// has its own stream, a device arena of budget_bytes / n_lanes and pinned host
// staging.  Whenever a lane is idle, the scheduler admits queued requests in
// arrival order while the lane's arena and batch size allow, packs their
// inputs and filter descriptors into the staging buffer, and issues a staging
// kernel that pulls them into the arena and one persistent batched launch
// (the same kernel as cddt_plan_run), which writes the log-weights straight
// into the lane's pinned output buffer, followed by an event: a batch uses no
// copy engine, only its lane's kernel queue.  Up to n_lanes
// batches are in flight at once, so requests that arrive while others run are
// admitted as lanes and memory free up and their work overlaps on the device.
// A batch's requests complete when its event has fired: their log-weights are
// taken from the pinned buffer and their completion time is stamped on the
// host clock.
//
// Results are bit-identical to running each request alone: every particle's
// weight is computed by the same per-particle routine, in a fixed order.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "cddt_common.h"
#include "ring_kernel.h"

namespace cddt {
namespace {

using Clock = std::chrono::steady_clock;

struct ServedMap {
  cddt_map map;
  float* d_offsets;
  int32_t n_rays;
  int32_t pair;
  const float* table;
  int32_t max_range;
};

struct Request {
  int64_t id;
  int32_t map;
  int32_t n;
  std::vector<float> poses;   // px[n], py[n], pth[n]
  std::vector<int32_t> obs;
  std::vector<float> logw;
  size_t bytes;
  double submit_t = 0, done_t = 0;
  bool done = false;
};

struct TimesSlot {
  int64_t id = -1;
  double submit = 0, done = 0;
};
constexpr size_t kTimesRing = 1 << 16;
constexpr double kSpinSeconds = 200e-6;  // idle polling before the scheduler blocks

constexpr size_t kAlign = 256;
// Lanes are streams, and HIP maps a process's streams onto four hardware
// queues by default: more lanes would share queues (and wait on each other).
constexpr int32_t kMaxLanes = 4;
size_t align_up(size_t v) { return (v + kAlign - 1) & ~(kAlign - 1); }

// Copy a lane's packed inputs from pinned host memory into its device arena.
__global__ void k_stage_in(const uint4* __restrict__ src, uint4* __restrict__ dst, size_t n16) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += (size_t)gridDim.x * blockDim.x)
    dst[i] = src[i];
}

struct Lane {
  hipStream_t stream = nullptr;
  hipEvent_t start = nullptr;  // before the input copy
  hipEvent_t done = nullptr;   // after the batch kernel
  char* d_arena = nullptr;   // device: [descriptors][prefix][counter][inputs...]
  char* h_in = nullptr;      // pinned staging of the same layout (inputs part)
  const char* h_in_dev = nullptr;  // h_in as the device addresses it
  float* h_out = nullptr;    // pinned log-weights, written by the batch kernel
  float* h_out_dev = nullptr;  // h_out as the device addresses it
  size_t arena = 0;
  std::vector<Request*> batch;
  std::vector<size_t> out_off;  // per request: float offset of its log-weights in h_out
  size_t out_floats = 0;
  size_t bytes = 0;
  bool busy = false;
};

// Resident mode: the ring in pinned, fine-grained host memory (host and
// device addresses), the device counters, and the host's bookkeeping.
struct Pending {
  Request* r;
  int32_t slot;  // >= 0: the inputs are already in this slot
};
struct Resident {
  RingCtl* ctl = nullptr;
  RingSlot* slots = nullptr;
  int32_t* tilemap = nullptr;
  int64_t* done = nullptr;
  char* arena = nullptr;
  RingCtl* ctl_d = nullptr;
  RingSlot* slots_d = nullptr;
  int32_t* tilemap_d = nullptr;
  int64_t* done_d = nullptr;
  char* arena_d = nullptr;
  RingDev* rd = nullptr;          // device
  uint32_t* tiles_done = nullptr;  // device, one count per slot
  int32_t n_slots = 0;
  size_t slot_bytes = 0;
  int64_t tiles = 0;  // tile map entries (a power of two)
  int64_t busy_tiles = 0;  // waves of the resident grid: more tiles than this in the ring count as busy
  hipStream_t stream = nullptr;
  hipEvent_t ev_start = nullptr, ev_end = nullptr;
  bool running = false, drain_asked = false;
  int64_t pub = 0;  // tiles published (host copy of ctl->pub)
  std::vector<int32_t> free_slots;
  std::vector<Request*> owner;          // request in each slot
  // id of the request published in each slot, -1 when none: set under the
  // lock by publication, cleared only by the driver, read by the driver's
  // unlocked scan of completion words
  std::unique_ptr<std::atomic<int64_t>[]> pub_id;
  std::vector<int64_t> t_begin;         // host copy of each slot's first tile
  std::vector<int32_t> inflight;        // published slots, not finished
  std::vector<int32_t> where;           // index of each slot in inflight (-1: not there)
  std::deque<Pending> pending;
  std::deque<std::pair<int64_t, int32_t>> order;  // (first tile, slot) in publication order, pruned lazily
  uint64_t idle_ticks = 0, watch_ticks = 0;  // of the device's constant wall clock
};

}  // namespace
}  // namespace cddt

struct cddt_server_s {
  std::vector<cddt::ServedMap> maps;
  cddt_server_config cfg{};
  int32_t cus = 0;
  int device = 0;
  bool zp16 = false;  // some map has 16-bit zero points
  std::vector<cddt::Lane> lanes;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<cddt::Request*> queue;
  std::unordered_map<int64_t, cddt::Request*> live;
  // submit/done times of the most recent completions, slot id % kTimesRing
  std::vector<cddt::TimesSlot> times = std::vector<cddt::TimesSlot>(cddt::kTimesRing);
  std::thread sched;
  bool stop = false;
  int64_t next_id = 0;
  cddt_server_stats stats{};
  int64_t bytes_in_flight = 0;
  cddt::Clock::time_point t0;
  double busy_since = -1.0;
  std::string error;
  std::unique_ptr<cddt::Resident> res;  // resident mode
  double now() const { return std::chrono::duration<double>(cddt::Clock::now() - t0).count(); }
};

namespace cddt {
namespace {

size_t request_bytes(const cddt_server_s* s, int32_t map, int32_t n) {
  const ServedMap& m = s->maps[map];
  // poses + log-weights + observations + descriptor + prefix entry, each padded
  return align_up((size_t)n * 12) + align_up((size_t)n * 4) + align_up((size_t)m.n_rays * 4) + sizeof(FilterDev) +
         sizeof(int64_t);
}

// Pack a lane's admitted batch into its staging buffer and launch it.  Runs
// on the scheduler thread without the lock: the lane and the requests in its
// batch belong to the scheduler until they are marked done.  The kernel's tile
// counter is cleared by the same host-to-device copy that carries the inputs.
cddt_status launch_lane(const cddt_server_s* s, Lane& L) {
  const size_t nb = L.batch.size();
  const size_t desc_bytes = align_up(sizeof(FilterDev) * nb);
  const size_t prefix_bytes = align_up(sizeof(int64_t) * (nb + 1));
  const size_t counter_off = desc_bytes + prefix_bytes;
  size_t off = counter_off + kBatchCounterBytes;
  FilterDev* fd = (FilterDev*)L.h_in;
  int64_t* prefix = (int64_t*)(L.h_in + desc_bytes);
  std::memset(L.h_in + counter_off, 0, kBatchCounterBytes);
  prefix[0] = 0;
  L.out_off.assign(nb, 0);
  size_t out_floats = 0;
  const int64_t ppt = s->cfg.tuning.particles_per_tile;
  for (size_t k = 0; k < nb; ++k) {
    const Request* r = L.batch[k];
    const ServedMap& m = s->maps[r->map];
    const size_t n = (size_t)r->n;
    std::memcpy(L.h_in + off, r->poses.data(), n * 12);
    const char* dp = L.d_arena + off;
    off += align_up(n * 12);
    std::memcpy(L.h_in + off, r->obs.data(), (size_t)m.n_rays * 4);
    const int32_t* dobs = (const int32_t*)(L.d_arena + off);
    off += align_up((size_t)m.n_rays * 4);
    FilterDev d{};
    d.map = m.map->dev();
    d.px = (const float*)dp;
    d.py = (const float*)dp + n;
    d.pth = (const float*)dp + 2 * n;
    d.offsets = m.d_offsets;
    d.obs = dobs;
    d.table = m.table;
    d.ranges = nullptr;
    d.n_particles = (int64_t)n;
    d.n_rays = m.n_rays;
    d.pair_offset = m.pair;
    d.max_range = m.max_range;
    L.out_off[k] = out_floats;
    out_floats += align_up(n * 4) / 4;
    fd[k] = d;
    prefix[k + 1] = prefix[k] + ((int64_t)n + ppt - 1) / ppt;
  }
  const size_t in_bytes = off;
  for (size_t k = 0; k < nb; ++k) fd[k].logw = L.h_out_dev + L.out_off[k];
  L.out_floats = out_floats;
  CDDT_HIP(hipEventRecord(L.start, L.stream));
  // the inputs are pulled from pinned memory by a kernel, so that all of a
  // batch's device work runs on the lane's one queue
  const size_t n16 = in_bytes / 16;  // in_bytes is a multiple of kAlign
  const unsigned blocks = (unsigned)std::min<size_t>((n16 + 255) / 256, 1024);
  hipLaunchKernelGGL(k_stage_in, dim3(blocks), dim3(256), 0, L.stream, (const uint4*)L.h_in_dev, (uint4*)L.d_arena,
                     n16);
  CDDT_TRY(launch_batch((const FilterDev*)L.d_arena, (const int64_t*)(L.d_arena + desc_bytes), (int32_t)nb,
                        prefix[nb], s->cfg.tuning, (unsigned long long*)(L.d_arena + counter_off), s->cus,
                        L.stream, s->zp16, /*counter_zeroed=*/true));
  CDDT_HIP(hipEventRecord(L.done, L.stream));
  return CDDT_OK;
}

// Lock held.  Report NaN weights for a batch that could not run.
void fail_batch(cddt_server_s* s, Lane& L) {
  const double t = s->now();
  for (Request* r : L.batch) {
    r->logw.assign((size_t)r->n, __builtin_nanf(""));
    r->done = true;
    r->done_t = t;
    s->times[(size_t)r->id % kTimesRing] = {r->id, r->submit_t, t};
  }
  L.batch.clear();
  s->cv_done.notify_all();
}

// The scheduler alternates between work done without the lock (event polls,
// copying results out of pinned memory, packing and enqueueing batches) and
// short critical sections that publish completions and take queued requests,
// so submitters are never held up by HIP calls.
void scheduler(cddt_server_s* s) {
  (void)hipSetDevice(s->device);
  std::vector<char> finished(s->lanes.size()), failed(s->lanes.size()), launched(s->lanes.size());
  std::vector<hipError_t> status(s->lanes.size());
  std::vector<double> device_s(s->lanes.size());
  bool any_busy = false;
  double idle_since = -1.0;
  for (;;) {
    // 1. unlocked: poll in-flight lanes, copy finished results into their requests
    for (size_t l = 0; l < s->lanes.size(); ++l) {
      Lane& L = s->lanes[l];
      finished[l] = 0;
      if (!L.busy) continue;
      status[l] = hipEventQuery(L.done);
      if (status[l] == hipErrorNotReady) continue;
      finished[l] = 1;
      if (status[l] != hipSuccess) continue;
      float ms = 0.f;
      device_s[l] = hipEventElapsedTime(&ms, L.start, L.done) == hipSuccess ? 1e-3 * ms : 0.0;
      for (size_t k = 0; k < L.batch.size(); ++k) {
        Request* r = L.batch[k];
        r->logw.assign(L.h_out + L.out_off[k], L.h_out + L.out_off[k] + r->n);
        r->poses.clear();
        r->poses.shrink_to_fit();
      }
    }
    // 2. locked: publish completions, admit queued requests into idle lanes
    bool any_new = false;
    {
      std::lock_guard<std::mutex> g(s->mu);
      const double t = s->now();
      bool notify = false;
      for (size_t l = 0; l < s->lanes.size(); ++l) {
        Lane& L = s->lanes[l];
        if (!finished[l]) continue;
        s->bytes_in_flight -= (int64_t)L.bytes;
        L.bytes = 0;
        L.busy = false;
        if (status[l] != hipSuccess) {
          s->error = hipGetErrorString(status[l]);
          fail_batch(s, L);
          continue;
        }
        s->stats.device_seconds += device_s[l];
        s->stats.max_batch_seconds = std::max(s->stats.max_batch_seconds, device_s[l]);
        for (Request* r : L.batch) {
          r->done_t = t;
          r->done = true;
          s->times[(size_t)r->id % kTimesRing] = {r->id, r->submit_t, t};
          s->stats.completed++;
          s->stats.rays += (int64_t)r->n * s->maps[r->map].n_rays;
        }
        L.batch.clear();
        notify = true;
      }
      if (notify) s->cv_done.notify_all();
      for (size_t l = 0; l < s->lanes.size(); ++l) {
        Lane& L = s->lanes[l];
        launched[l] = 0;
        if (L.busy || s->queue.empty()) continue;
        size_t used = 0;
        while (!s->queue.empty() && (int32_t)L.batch.size() < s->cfg.max_batch) {
          Request* r = s->queue.front();
          if (used + r->bytes > L.arena) break;
          used += r->bytes;
          L.batch.push_back(r);
          s->queue.pop_front();
        }
        if (L.batch.empty()) continue;
        L.bytes = used;
        L.busy = true;
        launched[l] = 1;
        any_new = true;
        s->stats.batches++;
        s->bytes_in_flight += (int64_t)used;
        s->stats.peak_bytes = std::max<int64_t>(s->stats.peak_bytes, s->bytes_in_flight);
      }
      any_busy = false;
      for (const Lane& L : s->lanes) any_busy |= L.busy;
      if (any_busy && s->busy_since < 0) s->busy_since = t;
      if (!any_busy && s->busy_since >= 0) {
        s->stats.busy_seconds += t - s->busy_since;
        s->busy_since = -1.0;
      }
    }
    // 3. unlocked: pack and enqueue the new batches
    if (any_new) {
      for (size_t l = 0; l < s->lanes.size(); ++l) {
        if (!launched[l]) continue;
        Lane& L = s->lanes[l];
        if (launch_lane(s, L) == CDDT_OK) continue;
        const std::string err = cddt_last_error();
        std::lock_guard<std::mutex> g(s->mu);
        s->error = err;
        s->bytes_in_flight -= (int64_t)L.bytes;
        L.bytes = 0;
        L.busy = false;
        fail_batch(s, L);
      }
      continue;  // poll again at once: completions may already be waiting
    }
    // 4. wait for arrivals or for in-flight batches to finish.  While work is in
    // flight, or shortly after it, the thread polls (yielding the core between
    // polls) rather than sleeping, since a timed sleep or a wake-up costs tens
    // of microseconds of latency; an idle server blocks on the condition.
    if (any_busy) {
      idle_since = -1.0;
      std::this_thread::yield();
      continue;
    }
    std::unique_lock<std::mutex> lk(s->mu);
    if (s->stop) break;
    if (!s->queue.empty()) continue;
    const double t = s->now();
    if (idle_since < 0) idle_since = t;
    if (t - idle_since < kSpinSeconds) {
      lk.unlock();
      std::this_thread::yield();
      continue;
    }
    s->cv_work.wait(lk, [&] { return s->stop || !s->queue.empty(); });
    idle_since = -1.0;
  }
}

void destroy_lanes(cddt_server_s* s) {
  for (Lane& L : s->lanes) {
    if (L.start) (void)hipEventDestroy(L.start);
    if (L.done) (void)hipEventDestroy(L.done);
    if (L.stream) (void)hipStreamDestroy(L.stream);
    if (L.d_arena) (void)hipFree(L.d_arena);
    if (L.h_in) (void)hipHostFree(L.h_in);
    if (L.h_out) (void)hipHostFree(L.h_out);
  }
  s->lanes.clear();
  for (auto& m : s->maps)
    if (m.d_offsets) (void)hipFree(m.d_offsets);
  s->maps.clear();
}

// ---------------------------------------------------------------------------
// Resident mode
// ---------------------------------------------------------------------------
// The server leaves the kernel on the device this long after its last request
// finished (then asks it to drain); the kernel's own limits are far longer and
// only matter if the host stops answering.
constexpr double kResidentIdleSeconds = 1e-3;
constexpr double kWatchSeconds = 1.0, kWorkerIdleSeconds = 2.0;
// Tile size factor while the ring is busy (see ring_publish).
constexpr int64_t kBusyTileFactor = 4;

// Bytes a request takes in a slot: poses, observations, log-weights.
size_t slot_need(const cddt_server_s* s, int32_t map, int32_t n) {
  return align_up((size_t)n * 12) + align_up((size_t)s->maps[map].n_rays * 4) + align_up((size_t)n * 4);
}

// Copy a request's inputs into slot `sl` (host side of the pinned arena).
void ring_fill(cddt_server_s* s, int32_t sl, int32_t map, int32_t n, const float* px, const float* py,
               const float* pth, const int32_t* obs) {
  Resident& R = *s->res;
  char* b = R.arena + (size_t)sl * R.slot_bytes;
  std::memcpy(b, px, 4 * (size_t)n);
  std::memcpy(b + 4 * (size_t)n, py, 4 * (size_t)n);
  std::memcpy(b + 8 * (size_t)n, pth, 4 * (size_t)n);
  std::memcpy(b + align_up((size_t)n * 12), obs, 4 * (size_t)s->maps[map].n_rays);
}

// Lock held.  Give the request in slot `sl` the next tile numbers, write its
// descriptor and tile map entries, and publish.  False when the tile map has
// no room yet (the oldest request in flight still holds numbers that would
// be reused).
bool ring_publish(cddt_server_s* s, int32_t sl) {
  Resident& R = *s->res;
  Request* r = R.owner[sl];
  while (!R.order.empty()) {  // drop finished or renumbered entries from the front
    const auto& e = R.order.front();
    if (R.where[e.second] >= 0 && R.t_begin[e.second] == e.first) break;
    R.order.pop_front();
  }
  const int64_t oldest = R.order.empty() ? R.pub : R.order.front().first;
  // Tiles of the tuning's size while the ring holds fewer tiles than the
  // kernel has waves (latency: a request spreads over many waves); larger
  // tiles beyond that (throughput: fewer per-tile host-memory round trips).
  const int64_t base = s->cfg.tuning.particles_per_tile;
  const int64_t ppt = R.pub - oldest < R.busy_tiles ? base : std::min<int64_t>(base * kBusyTileFactor, 256);
  const int64_t nt = ((int64_t)r->n + ppt - 1) / ppt;
  if (R.pub + nt - oldest > R.tiles) return false;
  const ServedMap& m = s->maps[r->map];
  const size_t n = (size_t)r->n;
  char* b = R.arena_d + (size_t)sl * R.slot_bytes;
  RingSlot slot{};
  FilterDev& d = slot.f;
  d.map = m.map->dev();
  d.px = (const float*)b;
  d.py = (const float*)b + n;
  d.pth = (const float*)b + 2 * n;
  d.obs = (const int32_t*)(b + align_up(n * 12));
  d.logw = (float*)(b + align_up(n * 12) + align_up((size_t)m.n_rays * 4));
  d.offsets = m.d_offsets;
  d.table = m.table;
  d.ranges = nullptr;
  d.n_particles = (int64_t)n;
  d.n_rays = m.n_rays;
  d.pair_offset = m.pair;
  d.max_range = m.max_range;
  slot.t_begin = R.pub;
  slot.n_tiles = (int32_t)nt;
  slot.ppt = (int32_t)ppt;
  slot.id = r->id;
  std::memcpy(&R.slots[sl], &slot, sizeof(RingSlot));
  for (int64_t k = 0; k < nt; ++k) R.tilemap[(R.pub + k) & (R.tiles - 1)] = sl;
  __atomic_store_n(&R.done[sl], (int64_t)0, __ATOMIC_RELAXED);
  R.t_begin[sl] = R.pub;
  R.order.emplace_back(R.pub, sl);
  if (R.where[sl] < 0) {
    R.where[sl] = (int32_t)R.inflight.size();
    R.inflight.push_back(sl);
  }
  R.pub += nt;
  __atomic_store_n(&R.ctl->pub, R.pub, __ATOMIC_RELEASE);
  R.pub_id[sl].store(r->id, std::memory_order_release);
  return true;
}

// Lock held.  Publish waiting requests while slots and tile numbers allow.
void ring_admit(cddt_server_s* s) {
  Resident& R = *s->res;
  while (!R.pending.empty()) {
    Pending& pd = R.pending.front();
    if (pd.slot < 0) {
      if (R.free_slots.empty()) return;
      pd.slot = R.free_slots.back();
      R.free_slots.pop_back();
      Request* r = pd.r;
      R.owner[pd.slot] = r;
      const size_t n = (size_t)r->n;
      ring_fill(s, pd.slot, r->map, r->n, r->poses.data(), r->poses.data() + n, r->poses.data() + 2 * n,
                r->obs.data());
      r->poses.clear();
      r->poses.shrink_to_fit();
      s->bytes_in_flight += (int64_t)R.slot_bytes;
      s->stats.peak_bytes = std::max<int64_t>(s->stats.peak_bytes, s->bytes_in_flight);
    }
    if (!ring_publish(s, pd.slot)) return;
    R.pending.pop_front();
  }
}

// Lock held.  Finish the request in slot `sl` (results already copied out,
// or NaN when `ok` is false).
void ring_finish(cddt_server_s* s, int32_t sl, double t, bool ok = true) {
  Resident& R = *s->res;
  Request* r = R.owner[sl];
  r->done_t = t;
  r->done = true;
  s->times[(size_t)r->id % kTimesRing] = {r->id, r->submit_t, t};
  if (ok) {
    s->stats.completed++;
    s->stats.rays += (int64_t)r->n * s->maps[r->map].n_rays;
  }
  R.owner[sl] = nullptr;
  R.pub_id[sl].store(-1, std::memory_order_relaxed);
  const int32_t i = R.where[sl];
  R.inflight[i] = R.inflight.back();
  R.where[R.inflight[i]] = i;
  R.inflight.pop_back();
  R.where[sl] = -1;
  R.free_slots.push_back(sl);
  s->bytes_in_flight -= (int64_t)R.slot_bytes;
}

template <int Mode>
void ring_launch_mode(cddt_server_s* s, unsigned blocks, unsigned threads, size_t lds) {
  Resident& R = *s->res;
  if (s->zp16)
    hipLaunchKernelGGL((k_resident<Mode, true>), dim3(blocks), dim3(threads), lds, R.stream, R.ctl_d, R.slots_d,
                       R.tilemap_d, R.tiles - 1, R.done_d, R.rd, R.tiles_done, R.n_slots, R.idle_ticks,
                       R.watch_ticks);
  else
    hipLaunchKernelGGL((k_resident<Mode, false>), dim3(blocks), dim3(threads), lds, R.stream, R.ctl_d, R.slots_d,
                       R.tilemap_d, R.tiles - 1, R.done_d, R.rd, R.tiles_done, R.n_slots, R.idle_ticks,
                       R.watch_ticks);
}

// Launch the resident kernel with tickets from `base` (nothing below it is
// left to do), after clearing its counters, between two events.
cddt_status ring_launch(cddt_server_s* s, int64_t base) {
  Resident& R = *s->res;
  const cddt_tuning& t = s->cfg.tuning;
  hipLaunchKernelGGL(k_ring_reset, dim3(std::max(1, std::min(64, (R.n_slots + 255) / 256))), dim3(256), 0,
                     R.stream, R.rd, (unsigned long long)base, R.tiles_done, R.n_slots);
  CDDT_HIP(hipGetLastError());
  CDDT_HIP(hipEventRecord(R.ev_start, R.stream));
  const unsigned blocks = (unsigned)(s->cus * t.blocks_per_cu + 1);  // block 0 watches
  const unsigned threads = (unsigned)(kWave * t.waves_per_block);
  const size_t lds = tile_lds_bytes(t.search_mode, t.waves_per_block);
  switch (t.search_mode) {
    case 0: ring_launch_mode<0>(s, blocks, threads, lds); break;
    case 6: ring_launch_mode<6>(s, blocks, threads, lds); break;
    case 7: ring_launch_mode<7>(s, blocks, threads, lds); break;
    case 8: ring_launch_mode<8>(s, blocks, threads, lds); break;
    default: return fail(CDDT_EINVAL, "resident server: search mode must be 0, 6, 7 or 8");
  }
  CDDT_HIP(hipGetLastError());
  CDDT_HIP(hipEventRecord(R.ev_end, R.stream));
  return CDDT_OK;
}

// Lock held.  The kernel has ended: renumber every request still in flight
// (the ended kernel may have dropped some of its tiles), fail them all if it
// ended in error.
void ring_after_end(cddt_server_s* s, hipError_t st) {
  Resident& R = *s->res;
  R.running = false;
  R.drain_asked = false;
  __atomic_store_n(&R.ctl->drain, 0, __ATOMIC_RELEASE);
  float ms = 0.f;
  if (st == hipSuccess && hipEventElapsedTime(&ms, R.ev_start, R.ev_end) == hipSuccess) {
    s->stats.device_seconds += 1e-3 * ms;
    s->stats.max_batch_seconds = std::max(s->stats.max_batch_seconds, 1e-3 * ms);
  }
  if (st != hipSuccess) {
    s->error = hipGetErrorString(st);
    const double t = s->now();
    while (!R.inflight.empty()) {
      const int32_t sl = R.inflight.back();
      Request* r = R.owner[sl];
      r->logw.assign((size_t)r->n, __builtin_nanf(""));
      ring_finish(s, sl, t, false);
    }
    s->cv_done.notify_all();
    return;
  }
  R.order.clear();
  const std::vector<int32_t> again = R.inflight;
  for (int32_t sl : again) (void)ring_publish(s, sl);  // the map is sized for every slot at once
}

void ring_driver(cddt_server_s* s) {
  (void)hipSetDevice(s->device);
  Resident& R = *s->res;
  std::vector<int32_t> finished;
  double idle_since = -1.0, last_query = -1.0, last_locked = -1.0;
  int64_t seen_pub = -1;
  for (;;) {
    // 1. unlocked: completion words of every published slot, results out of
    // the pinned arena (a published slot keeps its request until this thread
    // finishes it, so its owner is stable here)
    finished.clear();
    for (int32_t sl = 0; sl < R.n_slots; ++sl) {
      const int64_t id = R.pub_id[sl].load(std::memory_order_acquire);
      if (id < 0 || __atomic_load_n(&R.done[sl], __ATOMIC_ACQUIRE) != id + 1) continue;
      Request* r = R.owner[sl];
      const ServedMap& m = s->maps[r->map];
      const float* lw = (const float*)(R.arena + (size_t)sl * R.slot_bytes + align_up((size_t)r->n * 12) +
                                       align_up((size_t)m.n_rays * 4));
      r->logw.assign(lw, lw + r->n);
      finished.push_back(sl);
    }
    // the kernel's end: looked for while it drains, otherwise every 50 us (a
    // runtime call costs microseconds; the kernel only ends on its own if the
    // host stopped answering for a second)
    hipError_t ended = hipErrorNotReady;
    const double tq = s->now();
    if (R.running && (R.drain_asked || tq - last_query > 50e-6)) {
      ended = hipEventQuery(R.ev_end);
      last_query = tq;
    }
    // 2. locked: publish completions, relaunch or drain.  Taken when a request
    // finished, the kernel ended or a new one was published, and otherwise at
    // most every 20 us (for the idle and stop checks), so that submissions do
    // not queue behind this thread for the lock.
    bool launch = false, busy = false, stop = false;
    int64_t base = 0;
    const int64_t pub_now = __atomic_load_n(&R.ctl->pub, __ATOMIC_ACQUIRE);
    if (finished.empty() && ended == hipErrorNotReady && pub_now == seen_pub && tq - last_locked < 20e-6) {
      std::this_thread::yield();
      continue;
    }
    seen_pub = pub_now;
    last_locked = tq;
    {
      std::lock_guard<std::mutex> g(s->mu);
      const double t = s->now();
      for (int32_t sl : finished) ring_finish(s, sl, t);
      if (!finished.empty()) s->cv_done.notify_all();
      if (ended != hipErrorNotReady && R.running) ring_after_end(s, ended);
      ring_admit(s);
      stop = s->stop;
      busy = !R.inflight.empty() || !R.pending.empty();
      if (busy && s->busy_since < 0) s->busy_since = t;
      if (!busy && s->busy_since >= 0) {
        s->stats.busy_seconds += t - s->busy_since;
        s->busy_since = -1.0;
      }
      if (!R.running && !R.inflight.empty() && !stop) {
        // every tile below the oldest first tile in flight is finished or dropped
        base = R.pub;
        for (int32_t sl : R.inflight) base = std::min(base, R.t_begin[sl]);
        R.running = true;
        launch = true;
        s->stats.batches++;
      }
      if (R.running && !R.drain_asked) {
        if (busy && !stop) {
          idle_since = -1.0;
        } else {
          if (idle_since < 0) idle_since = t;
          if (stop || t - idle_since > kResidentIdleSeconds) {
            __atomic_store_n(&R.ctl->drain, 1, __ATOMIC_RELEASE);
            R.drain_asked = true;
          }
        }
      }
      if (stop && !R.running) break;
    }
    if (launch && ring_launch(s, base) != CDDT_OK) {
      std::lock_guard<std::mutex> g(s->mu);
      ring_after_end(s, hipErrorLaunchFailure);
      continue;
    }
    // 3. spin while a kernel is on the device or work waits; block when idle
    if (R.running || busy) {
      std::this_thread::yield();
      continue;
    }
    std::unique_lock<std::mutex> lk(s->mu);
    s->cv_work.wait(lk, [&] { return s->stop || !R.pending.empty() || !R.inflight.empty(); });
  }
  (void)hipStreamSynchronize(R.stream);
}

// Submission in resident mode: a free slot is filled without the lock and
// published at once; otherwise the request waits with its own copy.
cddt_status ring_submit(cddt_server_s* s, int32_t map_index, const float* px_h, const float* py_h,
                        const float* ptheta_h, int32_t n_particles, const int32_t* obs_h, double arrival,
                        int64_t* id_h) {
  Resident& R = *s->res;
  if (slot_need(s, map_index, n_particles) > R.slot_bytes) {
    std::lock_guard<std::mutex> g(s->mu);
    s->stats.rejected++;
    return fail(CDDT_EBUSY, "server: request larger than a ring slot (budget_bytes / max_batch)");
  }
  Request* r = new Request();
  r->map = map_index;
  r->n = n_particles;
  r->bytes = R.slot_bytes;
  int32_t sl = -1;
  {
    std::lock_guard<std::mutex> g(s->mu);
    if (s->stop) {
      s->stats.rejected++;
      delete r;
      return fail(CDDT_EBUSY, "server: closing");
    }
    r->id = s->next_id++;
    r->submit_t = arrival >= 0.0 ? arrival : s->now();
    s->live[r->id] = r;
    s->stats.submitted++;
    *id_h = r->id;
    if (n_particles == 0) {  // nothing to compute
      r->done = true;
      r->done_t = s->now();
      s->times[(size_t)r->id % kTimesRing] = {r->id, r->submit_t, r->done_t};
      s->stats.completed++;
      s->cv_done.notify_all();
      return CDDT_OK;
    }
    if (R.pending.empty() && !R.free_slots.empty()) {
      sl = R.free_slots.back();
      R.free_slots.pop_back();
      R.owner[sl] = r;
      s->bytes_in_flight += (int64_t)R.slot_bytes;
      s->stats.peak_bytes = std::max<int64_t>(s->stats.peak_bytes, s->bytes_in_flight);
    }
  }
  if (sl >= 0) {
    ring_fill(s, sl, map_index, n_particles, px_h, py_h, ptheta_h, obs_h);
    std::lock_guard<std::mutex> g(s->mu);
    if (!R.pending.empty() || !ring_publish(s, sl)) R.pending.push_back({r, sl});
  } else {
    r->poses.resize((size_t)n_particles * 3);
    std::memcpy(r->poses.data(), px_h, 4 * (size_t)n_particles);
    std::memcpy(r->poses.data() + n_particles, py_h, 4 * (size_t)n_particles);
    std::memcpy(r->poses.data() + 2 * (size_t)n_particles, ptheta_h, 4 * (size_t)n_particles);
    r->obs.assign(obs_h, obs_h + s->maps[map_index].n_rays);
    std::lock_guard<std::mutex> g(s->mu);
    R.pending.push_back({r, -1});
    ring_admit(s);
  }
  s->cv_work.notify_one();
  return CDDT_OK;
}

void destroy_resident(cddt_server_s* s) {
  if (!s->res) return;
  Resident& R = *s->res;
  if (R.ev_start) (void)hipEventDestroy(R.ev_start);
  if (R.ev_end) (void)hipEventDestroy(R.ev_end);
  if (R.stream) (void)hipStreamDestroy(R.stream);
  if (R.rd) (void)hipFree(R.rd);
  if (R.tiles_done) (void)hipFree(R.tiles_done);
  for (void* p : {(void*)R.ctl, (void*)R.slots, (void*)R.tilemap, (void*)R.done, (void*)R.arena})
    if (p) (void)hipHostFree(p);
  for (Pending& pd : R.pending) {
    if (s->live.erase(pd.r->id) == 0) continue;
    delete pd.r;
  }
  R.pending.clear();
  s->res.reset();
}

// Allocate the ring for `c` (resident mode).  Errors as cddt_server_create.
cddt_status create_resident(cddt_server_s* s, const cddt_server_config& c) {
  s->res.reset(new Resident());
  Resident& R = *s->res;
  R.n_slots = c.max_batch;
  R.slot_bytes = (size_t)(c.budget_bytes / c.max_batch) & ~(kAlign - 1);
  if (R.slot_bytes < 3 * kAlign + (size_t)4 * c.max_rays)
    return fail(CDDT_EINVAL, "cddt_server_create: budget_bytes / max_batch too small for one request");
  const int64_t max_n = (int64_t)(R.slot_bytes / 16);
  const int64_t per_slot = (max_n + c.tuning.particles_per_tile - 1) / c.tuning.particles_per_tile;
  R.tiles = 1;
  while (R.tiles < (int64_t)R.n_slots * per_slot) R.tiles *= 2;
  R.busy_tiles = (int64_t)s->cus * c.tuning.blocks_per_cu * c.tuning.waves_per_block;
  if (R.tiles > ((int64_t)1 << 28)) return fail(CDDT_EINVAL, "cddt_server_create: ring tile map too large");
  // the kernel's own exit limits in ticks of the device's constant wall clock
  int khz = 0;
  if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, s->device) != hipSuccess || khz <= 0)
    return fail(CDDT_EDEVICE, "cddt_server_create: cannot query the device's wall clock rate");
  R.watch_ticks = (uint64_t)(kWatchSeconds * 1e3 * khz);
  R.idle_ticks = (uint64_t)(kWorkerIdleSeconds * 1e3 * khz);
  const unsigned fl = hipHostMallocCoherent | hipHostMallocMapped;
  auto pin = [&](void** h, void** d, size_t bytes) {
    return hipHostMalloc(h, bytes, fl) == hipSuccess && hipHostGetDevicePointer(d, *h, 0) == hipSuccess;
  };
  if (!pin((void**)&R.ctl, (void**)&R.ctl_d, sizeof(RingCtl)) ||
      !pin((void**)&R.slots, (void**)&R.slots_d, sizeof(RingSlot) * (size_t)R.n_slots) ||
      !pin((void**)&R.tilemap, (void**)&R.tilemap_d, 4 * (size_t)R.tiles) ||
      !pin((void**)&R.done, (void**)&R.done_d, 8 * (size_t)R.n_slots) ||
      !pin((void**)&R.arena, (void**)&R.arena_d, R.slot_bytes * (size_t)R.n_slots) ||
      hipMalloc(&R.rd, sizeof(RingDev)) != hipSuccess || hipMalloc(&R.tiles_done, 4 * (size_t)R.n_slots) != hipSuccess ||
      hipStreamCreateWithFlags(&R.stream, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreate(&R.ev_start) != hipSuccess || hipEventCreate(&R.ev_end) != hipSuccess)
    return fail(CDDT_ENOMEM, "cddt_server_create: ring allocation failed");
  std::memset(R.ctl, 0, sizeof(RingCtl));
  std::memset(R.tilemap, 0xff, 4 * (size_t)R.tiles);  // -1: no slot
  std::memset(R.done, 0, 8 * (size_t)R.n_slots);
  R.owner.assign(R.n_slots, nullptr);
  R.pub_id.reset(new std::atomic<int64_t>[R.n_slots]);
  for (int32_t k = 0; k < R.n_slots; ++k) R.pub_id[k].store(-1, std::memory_order_relaxed);
  R.t_begin.assign(R.n_slots, 0);
  R.where.assign(R.n_slots, -1);
  for (int32_t k = R.n_slots - 1; k >= 0; --k) R.free_slots.push_back(k);
  return CDDT_OK;
}

}  // namespace
}  // namespace cddt

namespace cddt {
namespace {
cddt_status submit_one(cddt_server_s* s, int32_t map_index, const float* px_h, const float* py_h,
                       const float* ptheta_h, int32_t n_particles, const int32_t* obs_h, double arrival,
                       int64_t* id_h);
}  // namespace
}  // namespace cddt

using namespace cddt;

extern "C" {

cddt_status cddt_server_create(const cddt_map* maps_h, int32_t n_maps, const float* const* offsets_h,
                               const int32_t* n_rays_h, const float* const* log_tables, const int32_t* max_range_h,
                               const cddt_server_config* config_h, cddt_server* out_h) {
  if (!out_h) return fail(CDDT_EINVAL, "cddt_server_create: out_h is NULL");
  *out_h = nullptr;
  if (!maps_h || !offsets_h || !n_rays_h || !log_tables || !max_range_h || !config_h || n_maps < 1)
    return fail(CDDT_EINVAL, "cddt_server_create: NULL argument or no maps");
  const cddt_server_config& c = *config_h;
  if (c.n_lanes < 1 || c.n_lanes > kMaxLanes)
    return fail(CDDT_EINVAL, "cddt_server_create: n_lanes must be in 1..4");
  if (c.resident != 0 && c.resident != 1) return fail(CDDT_EINVAL, "cddt_server_create: resident must be 0 or 1");
  if (c.resident && c.n_lanes != 1) return fail(CDDT_EINVAL, "cddt_server_create: resident mode takes n_lanes = 1");
  if (c.resident && c.tuning.search_mode != 0 && (c.tuning.search_mode < 6 || c.tuning.search_mode > 8))
    return fail(CDDT_EINVAL, "cddt_server_create: resident mode takes search modes 0, 6, 7 and 8");
  if (c.max_batch < 1 || c.max_batch > (c.resident ? 65536 : 4096))
    return fail(CDDT_EINVAL, "cddt_server_create: max_batch in 1..4096 (resident: 1..65536)");
  if (c.max_rays < 1 || c.max_rays > kMaxRays) return fail(CDDT_EINVAL, "cddt_server_create: max_rays in 1..1024");
  if (c.budget_bytes < (int64_t)c.n_lanes * 4096) return fail(CDDT_EINVAL, "cddt_server_create: budget too small");
  CDDT_TRY(check_tuning(c.tuning));
  for (int32_t i = 0; i < n_maps; ++i) {
    if (!maps_h[i] || !offsets_h[i] || !log_tables[i]) return fail(CDDT_EINVAL, "cddt_server_create: NULL map entry");
    if (n_rays_h[i] < 1 || n_rays_h[i] > c.max_rays) return fail(CDDT_EINVAL, "cddt_server_create: bad n_rays");
    if (max_range_h[i] < 0 || max_range_h[i] > 65535) return fail(CDDT_EINVAL, "cddt_server_create: bad max_range");
  }
  cddt_server_s* s = new cddt_server_s();
  s->cfg = c;
  s->cus = cddt_device_cus();
  (void)hipGetDevice(&s->device);
  s->t0 = Clock::now();
  auto bail = [&](const std::string& msg) {
    destroy_lanes(s);
    delete s;
    return fail(CDDT_EDEVICE, msg);
  };
  for (int32_t i = 0; i < n_maps; ++i) {
    ServedMap m{};
    m.map = maps_h[i];
    s->zp16 = s->zp16 || (m.map->flags & CDDT_FLAG_ZP16) != 0;
    m.n_rays = n_rays_h[i];
    m.pair = cddt_pair_offset(offsets_h[i], n_rays_h[i]);
    m.table = log_tables[i];
    m.max_range = max_range_h[i];
    if (hipMalloc(&m.d_offsets, 4 * (size_t)m.n_rays) != hipSuccess) return bail("cddt_server_create: hipMalloc");
    s->maps.push_back(m);
    if (hipMemcpy(m.d_offsets, offsets_h[i], 4 * (size_t)m.n_rays, hipMemcpyHostToDevice) != hipSuccess)
      return bail("cddt_server_create: offsets upload");
  }
  if (c.resident) {
    const cddt_status st = create_resident(s, c);
    if (st != CDDT_OK) {
      const std::string msg = cddt_last_error();
      destroy_resident(s);
      destroy_lanes(s);
      delete s;
      return fail(st, msg);
    }
    s->sched = std::thread(ring_driver, s);
    *out_h = s;
    return CDDT_OK;
  }
  const size_t arena = (size_t)(c.budget_bytes / c.n_lanes);
  s->lanes.resize(c.n_lanes);
  for (Lane& L : s->lanes) {
    L.arena = arena;
    const size_t fixed = align_up(sizeof(FilterDev) * c.max_batch) + align_up(sizeof(int64_t) * (c.max_batch + 1)) +
                         kBatchCounterBytes;
    if (hipStreamCreateWithFlags(&L.stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreate(&L.start) != hipSuccess || hipEventCreate(&L.done) != hipSuccess ||
        hipMalloc(&L.d_arena, fixed + arena) != hipSuccess ||
        hipHostMalloc((void**)&L.h_in, fixed + arena, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void**)&L.h_out, arena, hipHostMallocDefault) != hipSuccess ||
        hipHostGetDevicePointer((void**)&L.h_in_dev, L.h_in, 0) != hipSuccess ||
        hipHostGetDevicePointer((void**)&L.h_out_dev, L.h_out, 0) != hipSuccess)
      return bail("cddt_server_create: lane allocation failed");
  }
  s->sched = std::thread(scheduler, s);
  *out_h = s;
  return CDDT_OK;
}

cddt_status cddt_server_submit(cddt_server s, int32_t map_index, const float* px_h, const float* py_h,
                               const float* ptheta_h, int32_t n_particles, const int32_t* obs_h, int64_t* id_h) {
  if (!s || !id_h) return fail(CDDT_EINVAL, "cddt_server_submit: NULL argument");
  if (map_index < 0 || map_index >= (int32_t)s->maps.size()) return fail(CDDT_EINVAL, "cddt_server_submit: bad map");
  if (n_particles < 0 || (n_particles > 0 && (!px_h || !py_h || !ptheta_h)) || !obs_h)
    return fail(CDDT_EINVAL, "cddt_server_submit: bad particle or observation arrays");
  return submit_one(s, map_index, px_h, py_h, ptheta_h, n_particles, obs_h, -1.0, id_h);
}

cddt_status cddt_server_replay_threads(cddt_server s, int32_t n_threads, int32_t n, const int32_t* map_h,
                                       const int32_t* count_h, const float* const* px_h,
                                       const float* const* py_h, const float* const* ptheta_h,
                                       const int32_t* const* obs_h, const double* at_h, int64_t* ids_h) {
  if (!s || n < 0 || (n > 0 && (!map_h || !count_h || !px_h || !py_h || !ptheta_h || !obs_h || !at_h || !ids_h)))
    return fail(CDDT_EINVAL, "cddt_server_replay: NULL argument");
  if (n_threads < 1 || n_threads > 16) return fail(CDDT_EINVAL, "cddt_server_replay: n_threads must be in 1..16");
  for (int32_t i = 0; i < n; ++i) {  // validate everything before the first submission
    if (map_h[i] < 0 || map_h[i] >= (int32_t)s->maps.size()) return fail(CDDT_EINVAL, "cddt_server_replay: bad map");
    if (count_h[i] < 0 || (count_h[i] > 0 && (!px_h[i] || !py_h[i] || !ptheta_h[i])) || !obs_h[i])
      return fail(CDDT_EINVAL, "cddt_server_replay: bad particle or observation arrays");
    if (at_h[i] < 0.0 || (i > 0 && at_h[i] < at_h[i - 1]))
      return fail(CDDT_EINVAL, "cddt_server_replay: offsets must be non-negative and not decrease");
  }
  const double t0 = s->now();
  auto share = [&](int32_t k) {
    for (int32_t i = k; i < n; i += n_threads) {
      const double at = t0 + at_h[i];
      while (s->now() < at) {
      }
      ids_h[i] = -1;
      submit_one(s, map_h[i], px_h[i], py_h[i], ptheta_h[i], count_h[i], obs_h[i], at, &ids_h[i]);
    }
  };
  std::vector<std::thread> others;
  for (int32_t k = 1; k < n_threads; ++k) others.emplace_back(share, k);
  share(0);
  for (auto& th : others) th.join();
  return CDDT_OK;
}

cddt_status cddt_server_replay(cddt_server s, int32_t n, const int32_t* map_h, const int32_t* count_h,
                               const float* const* px_h, const float* const* py_h, const float* const* ptheta_h,
                               const int32_t* const* obs_h, const double* at_h, int64_t* ids_h) {
  return cddt_server_replay_threads(s, 1, n, map_h, count_h, px_h, py_h, ptheta_h, obs_h, at_h, ids_h);
}

}  // extern "C"

namespace cddt {
namespace {
cddt_status submit_one(cddt_server_s* s, int32_t map_index, const float* px_h, const float* py_h,
                       const float* ptheta_h, int32_t n_particles, const int32_t* obs_h, double arrival,
                       int64_t* id_h) {
  if (s->res) return ring_submit(s, map_index, px_h, py_h, ptheta_h, n_particles, obs_h, arrival, id_h);
  const size_t bytes = request_bytes(s, map_index, n_particles);
  Request* r = new Request();
  r->map = map_index;
  r->n = n_particles;
  r->bytes = bytes;
  r->poses.resize((size_t)n_particles * 3);
  std::memcpy(r->poses.data(), px_h, 4 * (size_t)n_particles);
  std::memcpy(r->poses.data() + n_particles, py_h, 4 * (size_t)n_particles);
  std::memcpy(r->poses.data() + 2 * (size_t)n_particles, ptheta_h, 4 * (size_t)n_particles);
  r->obs.assign(obs_h, obs_h + s->maps[map_index].n_rays);
  {
    std::lock_guard<std::mutex> g(s->mu);
    if (bytes > s->lanes[0].arena || s->stop) {
      s->stats.rejected++;
      delete r;
      return fail(CDDT_EBUSY, "server: request larger than a lane's share of the budget");
    }
    r->id = s->next_id++;
    r->submit_t = arrival >= 0.0 ? arrival : s->now();
    s->live[r->id] = r;
    s->queue.push_back(r);
    s->stats.submitted++;
    *id_h = r->id;
  }
  s->cv_work.notify_one();
  return CDDT_OK;
}
}  // namespace
}  // namespace cddt

extern "C" {

cddt_status cddt_server_poll(cddt_server s, int64_t id, float* logw_h, int32_t* done_h) {
  if (!s || !done_h) return fail(CDDT_EINVAL, "cddt_server_poll: NULL argument");
  std::lock_guard<std::mutex> g(s->mu);
  auto it = s->live.find(id);
  if (it == s->live.end()) return fail(CDDT_EINVAL, "cddt_server_poll: unknown or already collected request");
  Request* r = it->second;
  *done_h = r->done ? 1 : 0;
  if (r->done) {
    if (logw_h) std::memcpy(logw_h, r->logw.data(), 4 * r->logw.size());
    s->live.erase(it);
    delete r;
  }
  return CDDT_OK;
}

cddt_status cddt_server_wait(cddt_server s, int64_t id, float* logw_h) {
  if (!s) return fail(CDDT_EINVAL, "cddt_server_wait: NULL server");
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->live.find(id);
  if (it == s->live.end()) return fail(CDDT_EINVAL, "cddt_server_wait: unknown or already collected request");
  Request* r = it->second;
  s->cv_done.wait(lk, [&] { return r->done; });
  if (logw_h) std::memcpy(logw_h, r->logw.data(), 4 * r->logw.size());
  s->live.erase(id);
  delete r;
  return CDDT_OK;
}

cddt_status cddt_server_times(cddt_server s, int64_t id, double* submit_h, double* done_h) {
  if (!s || !submit_h || !done_h) return fail(CDDT_EINVAL, "cddt_server_times: NULL argument");
  std::lock_guard<std::mutex> g(s->mu);
  const cddt::TimesSlot& t = s->times[(size_t)(id < 0 ? 0 : id) % cddt::kTimesRing];
  if (id < 0 || t.id != id)
    return fail(CDDT_EINVAL, "cddt_server_times: request not finished, or one of the oldest completions");
  *submit_h = t.submit;
  *done_h = t.done;
  return CDDT_OK;
}

cddt_status cddt_server_stats_get(cddt_server s, cddt_server_stats* out_h) {
  if (!s || !out_h) return fail(CDDT_EINVAL, "cddt_server_stats_get: NULL argument");
  std::lock_guard<std::mutex> g(s->mu);
  *out_h = s->stats;
  if (s->busy_since >= 0) out_h->busy_seconds += s->now() - s->busy_since;
  return CDDT_OK;
}

double cddt_server_now(cddt_server s) { return s ? s->now() : 0.0; }

cddt_status cddt_server_destroy(cddt_server s) {
  if (!s) return CDDT_OK;
  {
    std::lock_guard<std::mutex> g(s->mu);
    s->stop = true;
    for (Request* r : s->queue) {  // never admitted: dropped
      s->live.erase(r->id);
      delete r;
    }
    s->queue.clear();
  }
  s->cv_work.notify_all();
  if (s->sched.joinable()) s->sched.join();
  destroy_resident(s);
  for (auto& kv : s->live) delete kv.second;
  s->live.clear();
  destroy_lanes(s);
  delete s;
  return CDDT_OK;
}

}  // extern "C"
