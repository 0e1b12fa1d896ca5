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
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "cddt_common.h"

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
  if (c.max_batch < 1 || c.max_batch > 4096) return fail(CDDT_EINVAL, "cddt_server_create: max_batch in 1..4096");
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

cddt_status cddt_server_replay(cddt_server s, int32_t n, const int32_t* map_h, const int32_t* count_h,
                               const float* const* px_h, const float* const* py_h, const float* const* ptheta_h,
                               const int32_t* const* obs_h, const double* at_h, int64_t* ids_h) {
  if (!s || n < 0 || (n > 0 && (!map_h || !count_h || !px_h || !py_h || !ptheta_h || !obs_h || !at_h || !ids_h)))
    return fail(CDDT_EINVAL, "cddt_server_replay: NULL argument");
  for (int32_t i = 0; i < n; ++i) {  // validate everything before the first submission
    if (map_h[i] < 0 || map_h[i] >= (int32_t)s->maps.size()) return fail(CDDT_EINVAL, "cddt_server_replay: bad map");
    if (count_h[i] < 0 || (count_h[i] > 0 && (!px_h[i] || !py_h[i] || !ptheta_h[i])) || !obs_h[i])
      return fail(CDDT_EINVAL, "cddt_server_replay: bad particle or observation arrays");
    if (at_h[i] < 0.0 || (i > 0 && at_h[i] < at_h[i - 1]))
      return fail(CDDT_EINVAL, "cddt_server_replay: offsets must be non-negative and not decrease");
  }
  const double t0 = s->now();
  for (int32_t i = 0; i < n; ++i) {
    const double at = t0 + at_h[i];
    while (s->now() < at) {
    }
    ids_h[i] = -1;
    submit_one(s, map_h[i], px_h[i], py_h[i], ptheta_h[i], count_h[i], obs_h[i], at, &ids_h[i]);
  }
  return CDDT_OK;
}

}  // extern "C"

namespace cddt {
namespace {
cddt_status submit_one(cddt_server_s* s, int32_t map_index, const float* px_h, const float* py_h,
                       const float* ptheta_h, int32_t n_particles, const int32_t* obs_h, double arrival,
                       int64_t* id_h) {
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
  for (auto& kv : s->live) delete kv.second;
  s->live.clear();
  destroy_lanes(s);
  delete s;
  return CDDT_OK;
}

}  // extern "C"
