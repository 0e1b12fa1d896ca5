// Many particle filters in one persistent launch.
//
// A plan holds a device table of filter descriptors (map, particles, rays,
// observations, table, outputs) and the prefix sums of their tile counts.
// The persistent grid has blocks_per_cu blocks per compute unit; every wave
// repeatedly takes the next tile index from one of eight 64-bit device
// counters (one per contiguous part of the tiles), finds
// its filter in the plan's tile map (one load) and computes the tile's
// particle weights with the same per-particle routine as the plain kernel, so
// the results are identical bit for bit.  A wave leaves when every part's
// counter has passed the part's last tile, so the grid always drains.
//
// Each run is two kernel launches (counter reset, persistent kernel) and
// nothing else, so a run can be captured into a hipGraph and replayed.
#include <algorithm>

#include "batch_kernel.h"

struct cddt_plan_s {
  std::vector<cddt_filter> filters;
  std::vector<cddt::FilterDev> fdev;
  std::vector<uint64_t> gen;  // each filter's map generation when fdev was taken
  std::vector<int64_t> prefix;  // n_filters + 1 tile offsets for the current tuning
  cddt::FilterDev* d_filters = nullptr;
  int64_t* d_prefix = nullptr;
  int4* d_tilemap = nullptr;  // per tile {filter, first particle, end particle, 0}; one entry per particle
  unsigned long long* d_counter = nullptr;
  cddt_tuning tuning{};
  int64_t total_tiles = 0;
  int32_t cus = 0;
  bool zp16 = false;  // some filter's map has 16-bit zero points
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  // particle-filter step (motion, weights, resampling)
  int64_t total_particles = 0;
  int64_t* d_ppre = nullptr;   // n_filters + 1 particle offsets
  float* d_stage = nullptr;    // 3 * total_particles pose scratch for resampling
  int32_t* d_idx = nullptr;    // total_particles source indices
  const float* mcl_odom = nullptr;
  const uint32_t* mcl_u = nullptr;
  const float* mcl_noise = nullptr;
  // resampling segments (built with the scratch on first use)
  std::vector<void*> seg_mem;
  cddt::ResampleSegs segs{};
};

namespace cddt {

// Counter reset plus one persistent launch over the tiles of n_filters filters.
cddt_status launch_batch(const FilterDev* d_filters, const int64_t* d_prefix, int32_t n_filters,
                         int64_t total_tiles, const cddt_tuning& t, unsigned long long* d_counter, int32_t cus,
                         hipStream_t st, bool zp16, bool counter_zeroed, const int4* d_tilemap) {
  if (!counter_zeroed) hipLaunchKernelGGL(k_reset_counter, dim3(1), dim3(64), 0, st, d_counter);
  if (total_tiles > 0) {
    // no more blocks than tiles need (small batches): every wave claims at least once per part
    const int64_t need = (total_tiles + t.waves_per_block - 1) / t.waves_per_block;
    const unsigned blocks = (unsigned)std::max<int64_t>(1, std::min<int64_t>((int64_t)cus * t.blocks_per_cu, need));
    const unsigned threads = (unsigned)(kWave * t.waves_per_block);
    const int32_t ppt = t.particles_per_tile;
    const size_t lds = tile_lds_bytes(t.search_mode, t.waves_per_block);
    switch (t.search_mode) {
#define CDDT_BATCH_K(KK)                                                                                        \
  case KK:                                                                                                      \
    if (zp16)                                                                                                   \
      hipLaunchKernelGGL((k_batch<KK, true>), dim3(blocks), dim3(threads), lds, st, d_filters, d_prefix,        \
                         d_tilemap, n_filters, total_tiles, ppt, d_counter);                                               \
    else                                                                                                        \
      hipLaunchKernelGGL((k_batch<KK, false>), dim3(blocks), dim3(threads), lds, st, d_filters, d_prefix,       \
                         d_tilemap, n_filters, total_tiles, ppt, d_counter);                                               \
    break;
      CDDT_BATCH_K(1)
      CDDT_BATCH_K(2)
      CDDT_BATCH_K(3)
      CDDT_BATCH_K(4)
      CDDT_BATCH_K(5)
      CDDT_BATCH_K(0)
      CDDT_BATCH_K(6)
      CDDT_BATCH_K(7)
      CDDT_BATCH_K(8)
      CDDT_BATCH_K(9)
      CDDT_BATCH_K(10)
#undef CDDT_BATCH_K
      default:
        return fail(CDDT_EINVAL, "tuning: search_mode must be in 0..10");
    }
  }
  CDDT_HIP(hipGetLastError());
  return CDDT_OK;
}

cddt_status check_tuning(const cddt_tuning& t) {
  if (t.particles_per_tile < 1 || t.particles_per_tile > 256)
    return fail(CDDT_EINVAL, "tuning: particles_per_tile must be in 1..256");
  if (t.waves_per_block < 1 || t.waves_per_block * kWave > kMaxBatchThreads)
    return fail(CDDT_EINVAL, "tuning: waves_per_block must be in 1..8");
  if (t.blocks_per_cu < 1 || t.blocks_per_cu > 32) return fail(CDDT_EINVAL, "tuning: blocks_per_cu must be in 1..32");
  if (t.search_mode < 0 || t.search_mode > 10) return fail(CDDT_EINVAL, "tuning: search_mode must be in 0..10");
  if (tile_lds_bytes(t.search_mode, t.waves_per_block) > 65536)
    return fail(CDDT_EINVAL, "tuning: the search queue of this mode and block size exceeds 64 KiB of LDS");
  return CDDT_OK;
}

cddt_tuning default_tuning() {
  cddt_tuning t{};
  t.particles_per_tile = 4;
  t.waves_per_block = 4;
  t.blocks_per_cu = 8;
  t.search_mode = kModeTile16;
  return t;
}

namespace {

// The tile map of a tuning: tiles of ppt particles (the last of a filter
// clipped), in filter order.  (Cutting the launch's last tiles into smaller
// pieces, so that waves end closer together, measured slower: a tile's fixed
// costs outweigh the shorter tail.)
std::vector<int4> build_tilemap(const std::vector<cddt_filter>& filters, const cddt_tuning& t) {
  const int64_t ppt = t.particles_per_tile;
  std::vector<int4> tm;
  for (size_t f = 0; f < filters.size(); ++f)
    for (int64_t p = 0; p < filters[f].n_particles; p += ppt)
      tm.push_back(make_int4((int32_t)f, (int32_t)p, (int32_t)std::min(p + ppt, filters[f].n_particles), 0));
  return tm;
}

// Recompute the tile prefix sums and the tile map for the plan's tuning and
// upload them (blocking).  The kernel takes its tiles from the map.
cddt_status apply_tuning(cddt_plan_s* p, const cddt_tuning& t, hipStream_t st) {
  CDDT_TRY(check_tuning(t));
  const int64_t ppt = t.particles_per_tile;
  p->prefix.assign(p->filters.size() + 1, 0);
  for (size_t f = 0; f < p->filters.size(); ++f)
    p->prefix[f + 1] = p->prefix[f] + (p->filters[f].n_particles + ppt - 1) / ppt;
  const std::vector<int4> tm = build_tilemap(p->filters, t);
  p->total_tiles = (int64_t)tm.size();  // = prefix.back()
  CDDT_HIP(hipMemcpyAsync(p->d_prefix, p->prefix.data(), sizeof(int64_t) * p->prefix.size(), hipMemcpyHostToDevice,
                          st));
  if (!tm.empty())
    CDDT_HIP(hipMemcpyAsync(p->d_tilemap, tm.data(), sizeof(int4) * tm.size(), hipMemcpyHostToDevice, st));
  CDDT_HIP(hipStreamSynchronize(st));
  p->tuning = t;
  return CDDT_OK;
}

// A map whose structure was re-laid since the plan took its descriptor (an
// update that rebuilt it) has new band arrays: take the descriptors again and
// upload them in stream order before the next launch or graph replay, which
// read them from d_filters.
cddt_status refresh_descriptors(cddt_plan_s* p, hipStream_t st) {
  bool stale = false;
  for (size_t f = 0; f < p->filters.size(); ++f) {
    if (p->filters[f].map->generation == p->gen[f]) continue;
    p->fdev[f] = filter_dev(p->filters[f]);
    p->gen[f] = p->filters[f].map->generation;
    stale = true;
  }
  if (stale)
    CDDT_HIP(hipMemcpyAsync(p->d_filters, p->fdev.data(), sizeof(FilterDev) * p->fdev.size(), hipMemcpyHostToDevice,
                            st));
  return CDDT_OK;
}

cddt_status launch_plan(cddt_plan_s* p, hipStream_t st) {
  return launch_batch(p->d_filters, p->d_prefix, (int32_t)p->filters.size(), p->total_tiles, p->tuning,
                      p->d_counter, p->cus, st, p->zp16, /*counter_zeroed=*/false, p->d_tilemap);
}

void drop_graph(cddt_plan_s* p);

cddt_status launch_mcl(cddt_plan_s* p, hipStream_t st) {
  const int32_t nf = (int32_t)p->filters.size();
  if (p->total_particles == 0) return launch_plan(p, st);
  CDDT_TRY(launch_motion_many(p->d_filters, p->d_ppre, nf, p->total_particles, p->mcl_odom, p->mcl_noise, st));
  CDDT_TRY(launch_plan(p, st));
  return launch_resample_many(p->d_filters, p->d_ppre, p->mcl_u, p->d_stage, p->d_idx, p->segs, st);
}

template <class Body>
cddt_status capture_into(cddt_plan_s* p, hipStream_t st, Body body) {
  drop_graph(p);
  CDDT_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
  cddt_status s = body();
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(st, &g);
  if (s != CDDT_OK) {
    if (g) (void)hipGraphDestroy(g);
    return s;
  }
  if (e != hipSuccess) return fail(CDDT_EDEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
  p->graph = g;
  CDDT_HIP(hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0));
  return CDDT_OK;
}

void drop_graph(cddt_plan_s* p) {
  if (p->exec) (void)hipGraphExecDestroy(p->exec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  p->exec = nullptr;
  p->graph = nullptr;
}

}  // namespace
}  // namespace cddt

using namespace cddt;

extern "C" {

cddt_status cddt_plan_create(const cddt_filter* filters_h, int32_t n_filters, const cddt_tuning* tuning_h,
                             void* stream, cddt_plan* out_h) {
  if (!out_h) return fail(CDDT_EINVAL, "cddt_plan_create: out_h is NULL");
  *out_h = nullptr;
  if (!filters_h || n_filters < 1 || n_filters > 65536)
    return fail(CDDT_EINVAL, "cddt_plan_create: need 1..65536 filters");
  for (int32_t f = 0; f < n_filters; ++f) CDDT_TRY(validate_filter(filters_h[f], "cddt_plan_create"));
  cddt_tuning t = tuning_h ? *tuning_h : cached_tuning(filters_h, n_filters);
  CDDT_TRY(check_tuning(t));
  hipStream_t st = (hipStream_t)stream;
  cddt_plan_s* p = new cddt_plan_s();
  p->filters.assign(filters_h, filters_h + n_filters);
  for (auto& f : p->filters) {
    p->fdev.push_back(filter_dev(f));
    p->gen.push_back(f.map->generation);
  }
  for (auto& f : p->fdev) p->zp16 = p->zp16 || f.map.zp16;
  p->cus = cddt_device_cus();
  if (p->cus <= 0) {
    delete p;
    return fail(CDDT_EDEVICE, "cddt_plan_create: cannot query the device");
  }
  std::vector<int64_t> ppre(n_filters + 1, 0);
  for (int32_t f = 0; f < n_filters; ++f) ppre[f + 1] = ppre[f] + p->filters[f].n_particles;
  p->total_particles = ppre.back();
  auto bail = [&](const std::string& msg) {
    if (p->d_filters) (void)hipFree(p->d_filters);
    if (p->d_prefix) (void)hipFree(p->d_prefix);
    if (p->d_tilemap) (void)hipFree(p->d_tilemap);
    if (p->d_counter) (void)hipFree(p->d_counter);
    if (p->d_ppre) (void)hipFree(p->d_ppre);
    delete p;
    return fail(CDDT_EDEVICE, msg);
  };
  if (hipMalloc(&p->d_filters, sizeof(FilterDev) * n_filters) != hipSuccess ||
      hipMalloc(&p->d_prefix, sizeof(int64_t) * (n_filters + 1)) != hipSuccess ||
      hipMalloc(&p->d_tilemap, sizeof(int4) * (size_t)std::max<int64_t>(1, p->total_particles)) != hipSuccess ||
      hipMalloc(&p->d_counter, kBatchCounterBytes) != hipSuccess ||
      hipMalloc(&p->d_ppre, sizeof(int64_t) * (n_filters + 1)) != hipSuccess)
    return bail("cddt_plan_create: hipMalloc failed");
  if (hipMemcpyAsync(p->d_filters, p->fdev.data(), sizeof(FilterDev) * n_filters, hipMemcpyHostToDevice, st) !=
          hipSuccess ||
      hipMemcpyAsync(p->d_ppre, ppre.data(), sizeof(int64_t) * ppre.size(), hipMemcpyHostToDevice, st) != hipSuccess)
    return bail("cddt_plan_create: descriptor upload failed");
  cddt_status s = apply_tuning(p, t, st);
  if (s != CDDT_OK) return bail(cddt_last_error());
  *out_h = p;
  return CDDT_OK;
}

cddt_status cddt_plan_set_tuning(cddt_plan p, const cddt_tuning* tuning_h) {
  if (!p || !tuning_h) return fail(CDDT_EINVAL, "cddt_plan_set_tuning: NULL argument");
  CDDT_TRY(check_tuning(*tuning_h));
  drop_graph(p);
  return apply_tuning(p, *tuning_h, nullptr);
}

cddt_status cddt_plan_get_tuning(cddt_plan p, cddt_tuning* tuning_h) {
  if (!p || !tuning_h) return fail(CDDT_EINVAL, "cddt_plan_get_tuning: NULL argument");
  *tuning_h = p->tuning;
  return CDDT_OK;
}

cddt_status cddt_plan_run(cddt_plan p, void* stream) {
  if (!p) return fail(CDDT_EINVAL, "cddt_plan_run: plan is NULL");
  CDDT_TRY(refresh_descriptors(p, (hipStream_t)stream));
  return launch_plan(p, (hipStream_t)stream);
}

cddt_status cddt_plan_capture(cddt_plan p, void* stream) {
  if (!p) return fail(CDDT_EINVAL, "cddt_plan_capture: plan is NULL");
  if (!stream) return fail(CDDT_EINVAL, "cddt_plan_capture: capture needs a non-default stream");
  hipStream_t st = (hipStream_t)stream;
  CDDT_TRY(refresh_descriptors(p, st));
  return capture_into(p, st, [&] { return launch_plan(p, st); });
}

cddt_status cddt_plan_set_mcl(cddt_plan p, const float* odom, const uint32_t* u, const float* noise) {
  if (!p || !odom || !u || !noise) return fail(CDDT_EINVAL, "cddt_plan_set_mcl: NULL argument");
  for (const auto& f : p->filters)
    if (f.n_particles > kMaxResample)
      return fail(CDDT_EINVAL, "cddt_plan_set_mcl: resampling takes at most 2^20 particles per filter");
  if (!p->d_stage && p->total_particles > 0) {
    // segments of kResampleSegment particles per filter
    std::vector<int32_t> seg_f, seg_lo, fseg(p->filters.size() + 1, 0);
    for (size_t f = 0; f < p->filters.size(); ++f) {
      for (int64_t lo = 0; lo < p->filters[f].n_particles; lo += kResampleSegment) {
        seg_f.push_back((int32_t)f);
        seg_lo.push_back((int32_t)lo);
      }
      fseg[f + 1] = (int32_t)seg_f.size();
    }
    const size_t ns = seg_f.size();
    void* mem[9] = {};
    const size_t bytes[9] = {sizeof(float) * 3 * (size_t)p->total_particles, sizeof(int32_t) * (size_t)p->total_particles,
                             4 * ns, 4 * ns, 4 * fseg.size(), 4 * ns, 4 * ns, 8 * ns, 4 * ns};
    bool ok = true;
    for (int k = 0; k < 9 && ok; ++k) ok = hipMalloc(&mem[k], bytes[k]) == hipSuccess;
    if (ok)
      ok = hipMemcpy(mem[2], seg_f.data(), bytes[2], hipMemcpyHostToDevice) == hipSuccess &&
           hipMemcpy(mem[3], seg_lo.data(), bytes[3], hipMemcpyHostToDevice) == hipSuccess &&
           hipMemcpy(mem[4], fseg.data(), bytes[4], hipMemcpyHostToDevice) == hipSuccess;
    if (!ok) {
      for (void* q : mem)
        if (q) (void)hipFree(q);
      return fail(CDDT_ENOMEM, "cddt_plan_set_mcl: scratch allocation failed");
    }
    p->d_stage = (float*)mem[0];
    p->d_idx = (int32_t*)mem[1];
    p->seg_mem.assign(mem + 2, mem + 9);
    p->segs.seg_f = (const int32_t*)mem[2];
    p->segs.seg_lo = (const int32_t*)mem[3];
    p->segs.fseg = (const int32_t*)mem[4];
    p->segs.seg_max = (float*)mem[5];
    p->segs.seg_any = (int32_t*)mem[6];
    p->segs.seg_sum = (unsigned long long*)mem[7];
    p->segs.seg_mmax = (int32_t*)mem[8];
    p->segs.nseg = (int32_t)ns;
  }
  drop_graph(p);  // a captured step would keep the old pointers
  p->mcl_odom = odom;
  p->mcl_u = u;
  p->mcl_noise = noise;
  return CDDT_OK;
}

cddt_status cddt_plan_run_mcl(cddt_plan p, void* stream) {
  if (!p) return fail(CDDT_EINVAL, "cddt_plan_run_mcl: plan is NULL");
  if (!p->mcl_odom) return fail(CDDT_EINVAL, "cddt_plan_run_mcl: call cddt_plan_set_mcl first");
  CDDT_TRY(refresh_descriptors(p, (hipStream_t)stream));
  return launch_mcl(p, (hipStream_t)stream);
}

cddt_status cddt_plan_capture_mcl(cddt_plan p, void* stream) {
  if (!p) return fail(CDDT_EINVAL, "cddt_plan_capture_mcl: plan is NULL");
  if (!stream) return fail(CDDT_EINVAL, "cddt_plan_capture_mcl: capture needs a non-default stream");
  if (!p->mcl_odom) return fail(CDDT_EINVAL, "cddt_plan_capture_mcl: call cddt_plan_set_mcl first");
  hipStream_t st = (hipStream_t)stream;
  CDDT_TRY(refresh_descriptors(p, st));
  return capture_into(p, st, [&] { return launch_mcl(p, st); });
}

cddt_status cddt_plan_replay(cddt_plan p, void* stream) {
  if (!p) return fail(CDDT_EINVAL, "cddt_plan_replay: plan is NULL");
  if (!p->exec) return fail(CDDT_EINVAL, "cddt_plan_replay: no captured graph");
  CDDT_TRY(refresh_descriptors(p, (hipStream_t)stream));
  CDDT_HIP(hipGraphLaunch(p->exec, (hipStream_t)stream));
  return CDDT_OK;
}

cddt_status cddt_plan_time(cddt_plan p, const cddt_tuning* tuning_h, int32_t reps, void* stream, float* ms_h) {
  if (!p || !ms_h || reps < 1) return fail(CDDT_EINVAL, "cddt_plan_time: bad argument");
  hipStream_t st = (hipStream_t)stream;
  cddt_tuning keep = p->tuning;
  CDDT_TRY(refresh_descriptors(p, st));
  if (tuning_h) CDDT_TRY(apply_tuning(p, *tuning_h, st));
  hipEvent_t a, b;
  CDDT_HIP(hipEventCreate(&a));
  CDDT_HIP(hipEventCreate(&b));
  cddt_status s = launch_plan(p, st);  // warm-up
  if (s == CDDT_OK) {
    (void)hipEventRecord(a, st);
    for (int32_t r = 0; r < reps && s == CDDT_OK; ++r) s = launch_plan(p, st);
    (void)hipEventRecord(b, st);
    (void)hipEventSynchronize(b);
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, a, b);
    *ms_h = ms / reps;
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  if (tuning_h) CDDT_TRY(apply_tuning(p, keep, st));
  return s;
}

cddt_status cddt_plan_run_plain(cddt_plan p, void* stream) {
  if (!p) return fail(CDDT_EINVAL, "cddt_plan_run_plain: plan is NULL");
  CDDT_TRY(refresh_descriptors(p, (hipStream_t)stream));
  for (auto& f : p->fdev) CDDT_TRY(launch_weight(f, (hipStream_t)stream));
  return CDDT_OK;
}

cddt_status cddt_plan_destroy(cddt_plan p) {
  if (!p) return CDDT_OK;
  (void)hipDeviceSynchronize();
  drop_graph(p);
  if (p->d_filters) (void)hipFree(p->d_filters);
  if (p->d_prefix) (void)hipFree(p->d_prefix);
  if (p->d_tilemap) (void)hipFree(p->d_tilemap);
  if (p->d_counter) (void)hipFree(p->d_counter);
  if (p->d_ppre) (void)hipFree(p->d_ppre);
  if (p->d_stage) (void)hipFree(p->d_stage);
  if (p->d_idx) (void)hipFree(p->d_idx);
  for (void* q : p->seg_mem) (void)hipFree(q);
  delete p;
  return CDDT_OK;
}

}  // extern "C"
