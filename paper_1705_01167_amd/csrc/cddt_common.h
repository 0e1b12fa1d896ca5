// Internal declarations shared by the libcddt translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "cddt.h"

#include "device_types.h"

namespace cddt {

// ---------------------------------------------------------------------------
// Error reporting
// ---------------------------------------------------------------------------
void set_error(const std::string& msg);
cddt_status fail(cddt_status code, const std::string& msg);

#define CDDT_HIP(call)                                                              \
  do {                                                                              \
    hipError_t e_ = (call);                                                         \
    if (e_ != hipSuccess)                                                           \
      return ::cddt::fail(CDDT_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

#define CDDT_TRY(expr)                 \
  do {                                 \
    cddt_status s_ = (expr);           \
    if (s_ != CDDT_OK) return s_;      \
  } while (0)

// ---------------------------------------------------------------------------
// Device memory through the caller's allocator (or hipMalloc)
// ---------------------------------------------------------------------------
struct Allocator {
  cddt_allocator cb{};
  bool custom = false;
  cddt_status alloc(void** p, size_t bytes, const char* what);
  void release(void* p);
};

// Growable device scratch owned by a map.
struct Scratch {
  void* ptr = nullptr;
  size_t bytes = 0;
};
cddt_status ensure(Allocator& a, Scratch& s, size_t bytes, const char* what);

}  // namespace cddt

// Host-side state of a map.
struct cddt_map_s {
  int32_t w = 0, h = 0, n = 0, half = 0;
  uint32_t flags = 0;
  cddt::Allocator alloc;
  float k_scale = 0.f;
  std::vector<int32_t> c, s, row_min, nrows, row_base, zlo;
  int64_t rows = 0;
  uint8_t* d_occ = nullptr;
  cddt::SliceDev* d_slices = nullptr;
  int32_t* d_hdr = nullptr;      // rows * kNodeInts header nodes
  int32_t* d_zeros = nullptr;    // band regions
  int64_t capacity = 0, zero_points = 0, edge_cells = 0, max_row_len = 0, rebuilds = 0;
  bool stats_stale = false;  // max_row_len not recomputed since the last update
  // bumped whenever the band arrays are (re)allocated (build_structure):
  // device descriptors taken before then hold freed pointers
  uint64_t generation = 0;
  // spare area at the end of the zero-point array, for bands that outgrow
  // their region during updates: [capacity - spare, capacity); cursor on device
  unsigned long long* d_spare = nullptr;
  int64_t spare_end = 0;
  int64_t device_bytes = 0;
  // bucket index (CDDT_FLAG_BUCKETS): rows * nbk lines of 128 bytes
  int32_t blog2 = 0, nbk = 0;
  int32_t* d_bk = nullptr;
  int32_t* d_row_start = nullptr;          // half + 1 global band offsets
  unsigned long long* d_bk_over = nullptr;  // overflowing buckets (device counter)
  int64_t bucket_overflow = 0;
  // update scratch (grown on demand, released with the map)
  cddt::Scratch upd_ops, upd_changed, upd_cand, upd_edits, upd_rec, upd_rowcnt;
  cddt::Scratch upd_slot, upd_touched, upd_grp, upd_tiles;
  bool upd_rowcnt_clear = false;  // upd_rowcnt holds zeros for every band
  void* upd_host = nullptr;       // pinned staging of a chunk's ops and counters (hipHostMalloc)
  cddt::MapDev dev() const {
    cddt::MapDev m;
    m.occ = d_occ;
    m.slices = d_slices;
    m.hdr = d_hdr;
    m.zeros = d_zeros;
    m.bk = d_bk;
    m.w = w;
    m.h = h;
    m.n = n;
    m.half = half;
    m.k_scale = k_scale;
    m.bshift = d_bk ? 16 + blog2 : 0;
    m.nbk = nbk;
    m.zp16 = d_bk && (flags & CDDT_FLAG_ZP16) ? 1 : 0;
    return m;
  }
};

namespace cddt {
// build.hip.  build_structure also fills the bucket index when the map has
// one; fill_buckets writes every band's bucket lines and the overflow count,
// and blocks.  (An incremental update rewrites its edited bands' lines itself.)
cddt_status build_structure(cddt_map_s* m, hipStream_t st);
cddt_status fill_buckets(cddt_map_s* m, hipStream_t st);
void free_structure(cddt_map_s* m);
cddt_status refresh_stats(cddt_map_s* m, hipStream_t st);
// Band layout from per-band lengths cnt[rows] (reset to 0 on return): header
// words {start, len, cap} of every band in hdr, with or without slack; the
// total slots, total length and longest band come back.  Blocks.
cddt_status layout_bands(cddt_map_s* m, uint32_t* cnt, int32_t* hdr, bool no_slack, uint64_t* total_cap,
                         uint64_t* total_len, uint64_t* max_len, hipStream_t st);
// Sample levels, padding and header top levels of every band (keys in place).
cddt_status finalize_bands(int32_t* hdr, int32_t* zeros, int64_t rows, hipStream_t st);
// prune.hip: PCDDT pruning of a freshly built static structure.  Blocks.
cddt_status prune_structure(cddt_map_s* m, hipStream_t st);
// query.hip
// ticks (nullable): per ray, device wall-clock ticks of its wave from load to result.
cddt_status launch_cast(const MapDev& m, const float* x, const float* y, const float* th, int64_t n,
                        int32_t max_range, int32_t* out, hipStream_t st, int32_t* ticks = nullptr);
cddt_status launch_weight(const FilterDev& f, hipStream_t st);
// batch.hip.  d_counter: kBatchCounterBytes of device memory (the per-part
// tile counters); counter_zeroed: the caller has already cleared all of it in
// stream order; d_tilemap (nullable): per tile {filter, first particle, end
// particle, 0}, total_tiles entries; else tile t of a filter is its t-th run
// of ppt particles, the filter found by searching d_prefix.
cddt_status launch_batch(const FilterDev* d_filters, const int64_t* d_prefix, int32_t n_filters,
                         int64_t total_tiles, const cddt_tuning& t, unsigned long long* d_counter, int32_t cus,
                         hipStream_t st, bool zp16, bool counter_zeroed = false, const int4* d_tilemap = nullptr);
cddt_status check_tuning(const cddt_tuning& t);
// mcl.hip: motion of every particle of every filter (particle offsets d_pre,
// n_filters + 1 entries), and one resampling workgroup per filter.
constexpr int64_t kMaxResample = int64_t(1) << 20;
cddt_status launch_motion_many(const FilterDev* d_filters, const int64_t* d_pre, int32_t nf, int64_t total,
                               const float* d_odom, const float* d_noise, hipStream_t st);
// Segmented resampling of many filters: segment g covers particles
// [seg_lo[g], seg_lo[g] + kResampleSegment) of filter seg_f[g]; filter f owns
// segments fseg[f] .. fseg[f+1]-1.  The per-segment arrays are scratch.
constexpr int32_t kResampleSegment = 4096;
struct ResampleSegs {
  const int32_t* seg_f;
  const int32_t* seg_lo;
  const int32_t* fseg;
  float* seg_max;
  int32_t* seg_any;
  unsigned long long* seg_sum;
  int32_t* seg_mmax;
  int32_t nseg;
};
cddt_status launch_resample_many(const FilterDev* d_filters, const int64_t* d_pre, const uint32_t* d_u,
                                 float* d_stage, int32_t* d_idx, const ResampleSegs& segs, hipStream_t st);
cddt_tuning default_tuning();
// onecall.hip: the autotuned tuning recorded for this filter set, else default_tuning().
cddt_tuning cached_tuning(const cddt_filter* filters_h, int32_t n_filters);
// api.hip
FilterDev filter_dev(const cddt_filter& f);
cddt_status validate_filter(const cddt_filter& f, const char* who);
// update.hip
cddt_status apply_update(cddt_map_s* m, const int32_t* xs, const int32_t* ys, const uint8_t* vals,
                         int64_t n_ops, hipStream_t st);
}  // namespace cddt
