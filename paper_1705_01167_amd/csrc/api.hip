// C ABI entry points: validation, per-slice tables, allocation, export.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>

#include "band_layout.h"
#include "cddt_common.h"

namespace cddt {

namespace {
thread_local std::string g_error = "no error";
}

void set_error(const std::string& msg) { g_error = msg; }

cddt_status fail(cddt_status code, const std::string& msg) {
  g_error = msg;
  return code;
}

cddt_status Allocator::alloc(void** p, size_t bytes, const char* what) {
  *p = nullptr;
  if (bytes == 0) bytes = 16;
  if (custom) {
    *p = cb.alloc(bytes, cb.ctx);
    if (!*p) return fail(CDDT_ENOMEM, std::string("allocator callback failed for ") + what);
    return CDDT_OK;
  }
  hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) {
    *p = nullptr;
    (void)hipGetLastError();
    return fail(CDDT_ENOMEM, std::string("hipMalloc failed for ") + what + " (" + std::to_string(bytes) +
                                 " bytes): " + hipGetErrorString(e));
  }
  return CDDT_OK;
}

void Allocator::release(void* p) {
  if (!p) return;
  if (custom)
    cb.free(p, cb.ctx);
  else
    (void)hipFree(p);
}

cddt_status ensure(Allocator& a, Scratch& s, size_t bytes, const char* what) {
  if (s.bytes >= bytes && s.ptr) return CDDT_OK;
  if (s.ptr) a.release(s.ptr);
  s.ptr = nullptr;
  s.bytes = 0;
  size_t want = std::max<size_t>(bytes, 256);
  want = want + want / 4;
  CDDT_TRY(a.alloc(&s.ptr, want, what));
  s.bytes = want;
  return CDDT_OK;
}

namespace {

void release_scratch(cddt_map_s* m) {
  for (Scratch* s : {&m->upd_ops, &m->upd_changed, &m->upd_cand, &m->upd_edits, &m->upd_rec, &m->upd_rowcnt,
                     &m->upd_slot, &m->upd_touched, &m->upd_grp, &m->upd_tiles}) {
    if (s->ptr) m->alloc.release(s->ptr);
    s->ptr = nullptr;
    s->bytes = 0;
  }
  if (m->upd_host) (void)hipHostFree(m->upd_host);
  m->upd_host = nullptr;
  m->upd_rowcnt_clear = false;
}

void release_all(cddt_map_s* m) {
  free_structure(m);
  release_scratch(m);
  if (m->d_occ) m->alloc.release(m->d_occ);
  if (m->d_slices) m->alloc.release(m->d_slices);
  if (m->d_bk) m->alloc.release(m->d_bk);
  if (m->d_row_start) m->alloc.release(m->d_row_start);
  if (m->d_bk_over) m->alloc.release(m->d_bk_over);
  if (m->d_spare) m->alloc.release(m->d_spare);
  m->d_spare = nullptr;
  m->d_occ = nullptr;
  m->d_slices = nullptr;
  m->d_bk = nullptr;
  m->d_row_start = nullptr;
  m->d_bk_over = nullptr;
}

// Direction table, band ranges and band offsets of every stored slice.
void slice_tables(cddt_map_s* m) {
  const int half = m->half;
  m->c.assign(half, 0);
  m->s.assign(half, 0);
  m->row_min.assign(half, 0);
  m->nrows.assign(half, 0);
  m->row_base.assign(half, 0);
  m->zlo.assign(half, 0);
  int64_t base = 0, nbk = 1;
  for (int k = 0; k < half; ++k) {
    const double a = 2.0 * M_PI * k / m->n;
    const int64_t c = std::llround(std::cos(a) * 1073741824.0);
    const int64_t s = std::llround(std::sin(a) * 1073741824.0);
    int64_t lo = INT64_MAX, hi = INT64_MIN;
    const int64_t xs[2] = {0, m->w}, ys[2] = {0, m->h};
    for (int64_t X : xs)
      for (int64_t Y : ys) {
        const int64_t v = (Y * c - X * s) >> 30;
        lo = std::min(lo, v);
        hi = std::max(hi, v);
      }
    m->c[k] = (int32_t)c;
    m->s[k] = (int32_t)s;
    m->row_min[k] = (int32_t)lo;
    m->nrows[k] = (int32_t)(hi - lo + 1);
    m->row_base[k] = (int32_t)base;
    base += hi - lo + 1;
    // along-slice range of the map rectangle in Q16, with the query's rounding
    const int64_t wc = ((int64_t)m->w << 16) * c, hs = ((int64_t)m->h << 16) * s;
    const int64_t zlo = (std::min<int64_t>(0, wc) + std::min<int64_t>(0, hs)) >> 30;
    const int64_t zhi = (std::max<int64_t>(0, wc) + std::max<int64_t>(0, hs)) >> 30;
    m->zlo[k] = (int32_t)zlo;
    if (m->blog2) nbk = std::max<int64_t>(nbk, ((zhi - zlo) >> (16 + m->blog2)) + 1);
  }
  m->rows = base;
  m->nbk = m->blog2 ? (int32_t)nbk : 0;
  m->k_scale = (float)((double)m->n / (2.0 * M_PI));
}

}  // namespace
}  // namespace cddt

using namespace cddt;

// The message is only built on failure: a valid filter costs no host allocation.
static cddt_status check_filter(const cddt_filter& f, const char* who) {
  const char* why = nullptr;
  if (!f.map)
    why = ": map is NULL";
  else if (f.n_particles < 0)
    why = ": n_particles < 0";
  else if (f.n_rays < 1 || f.n_rays > kMaxRays)
    why = ": n_rays must be in 1..1024";
  else if (f.pair_offset < 0 || f.pair_offset >= f.n_rays)
    why = ": pair_offset must be in 0..n_rays-1";
  else if (f.max_range < 0 || f.max_range > 65535)
    why = ": max_range must be in 0..65535";
  else if (!f.ray_offsets || !f.obs_ranges || !f.log_table)
    why = ": NULL ray/obs/table array";
  else if (f.n_particles > 0 && (!f.px || !f.py || !f.ptheta || !f.logw_out))
    why = ": NULL particle array";
  return why ? fail(CDDT_EINVAL, std::string(who) + why) : CDDT_OK;
}

namespace cddt {
FilterDev filter_dev(const cddt_filter& f) {
  FilterDev d;
  d.map = f.map->dev();
  d.px = f.px;
  d.py = f.py;
  d.pth = f.ptheta;
  d.offsets = f.ray_offsets;
  d.obs = f.obs_ranges;
  d.table = f.log_table;
  d.logw = f.logw_out;
  d.ranges = f.ranges_out;
  d.n_particles = f.n_particles;
  d.n_rays = f.n_rays;
  d.pair_offset = f.pair_offset;
  d.max_range = f.max_range;
  d.pad = 0;
  return d;
}
cddt_status validate_filter(const cddt_filter& f, const char* who) { return check_filter(f, who); }
}  // namespace cddt

extern "C" {

const char* cddt_last_error(void) { return g_error.c_str(); }

int32_t cddt_device_cus(void) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  return cus;
}

cddt_status cddt_create(const uint8_t* occ, int32_t width, int32_t height, int32_t theta_bins, uint32_t flags,
                        const cddt_allocator* alloc, void* stream, cddt_map* out_h) {
  if (!out_h) return fail(CDDT_EINVAL, "cddt_create: out_h is NULL");
  *out_h = nullptr;
  if (!occ) return fail(CDDT_EINVAL, "cddt_create: occ is NULL");
  if (width < 1 || height < 1 || width > kMaxSide || height > kMaxSide)
    return fail(CDDT_EINVAL, "cddt_create: width and height must be in 1..16384");
  if (theta_bins < 2 || theta_bins > kMaxBins || (theta_bins & 1))
    return fail(CDDT_EINVAL, "cddt_create: theta_bins must be even and in 2..8192");
  if (flags & ~(uint32_t)(CDDT_FLAG_FULL_MAP | CDDT_FLAG_STATIC | CDDT_FLAG_BUCKETS | CDDT_FLAG_ZP16 | CDDT_FLAG_PRUNE |
                         CDDT_BUCKET_LOG2(15)))
    return fail(CDDT_EINVAL, "cddt_create: unknown flag bits");
  if ((flags & CDDT_FLAG_ZP16) && !(flags & CDDT_FLAG_BUCKETS))
    return fail(CDDT_EINVAL, "cddt_create: 16-bit zero points need CDDT_FLAG_BUCKETS");
  if ((flags & CDDT_FLAG_PRUNE) && !(flags & CDDT_FLAG_STATIC))
    return fail(CDDT_EINVAL, "cddt_create: CDDT_FLAG_PRUNE needs CDDT_FLAG_STATIC");
  if ((flags & CDDT_FLAG_PRUNE) && (flags & CDDT_FLAG_ZP16))
    return fail(CDDT_EINVAL, "cddt_create: CDDT_FLAG_PRUNE and CDDT_FLAG_ZP16 are not combined");
  int32_t blog2 = (int32_t)((flags >> 8) & 15u);
  if (!(flags & CDDT_FLAG_BUCKETS) && blog2)
    return fail(CDDT_EINVAL, "cddt_create: a bucket width needs CDDT_FLAG_BUCKETS");
  if (flags & CDDT_FLAG_BUCKETS) {
    if (blog2 == 0) blog2 = kBucketLog2Default;
    if (blog2 < 4 || blog2 > 10) return fail(CDDT_EINVAL, "cddt_create: bucket width must be 2^4..2^10 cells");
  }
  if (alloc && (!alloc->alloc || !alloc->free))
    return fail(CDDT_EINVAL, "cddt_create: allocator needs both alloc and free");
  hipStream_t st = (hipStream_t)stream;
  cddt_map_s* m = new cddt_map_s();
  m->w = width;
  m->h = height;
  m->n = theta_bins;
  m->half = theta_bins / 2;
  m->flags = flags;
  m->blog2 = blog2;
  if (alloc) {
    m->alloc.cb = *alloc;
    m->alloc.custom = true;
  }
  slice_tables(m);
  auto bail = [&](cddt_status s) {
    std::string msg = g_error;
    (void)hipStreamSynchronize(st);
    release_all(m);
    delete m;
    g_error = msg;
    return s;
  };
  cddt_status s;
  const size_t cells = (size_t)width * height;
  if ((s = m->alloc.alloc((void**)&m->d_occ, cells, "occupancy grid")) != CDDT_OK) return bail(s);
  if ((s = m->alloc.alloc((void**)&m->d_slices, sizeof(SliceDev) * m->half, "slice table")) != CDDT_OK)
    return bail(s);
  std::vector<SliceDev> sl(m->half);
  for (int k = 0; k < m->half; ++k) sl[k] = SliceDev{m->c[k], m->s[k], m->row_base[k] - m->row_min[k], m->zlo[k]};
  std::vector<int32_t> row_start(m->half + 1);
  for (int k = 0; k < m->half; ++k) row_start[k] = m->row_base[k];
  row_start[m->half] = (int32_t)m->rows;
  if (m->blog2) {
    const size_t lines = (size_t)m->rows * (size_t)m->nbk;
    if ((s = m->alloc.alloc((void**)&m->d_bk, lines * 128, "bucket index")) != CDDT_OK) return bail(s);
    if ((s = m->alloc.alloc((void**)&m->d_row_start, 4 * row_start.size(), "slice band offsets")) != CDDT_OK)
      return bail(s);
    if ((s = m->alloc.alloc((void**)&m->d_bk_over, 8, "bucket counter")) != CDDT_OK) return bail(s);
  }
  hipError_t e = hipMemcpyAsync(m->d_occ, occ, cells, hipMemcpyDeviceToDevice, st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(m->d_slices, sl.data(), sizeof(SliceDev) * m->half, hipMemcpyHostToDevice, st);
  if (e == hipSuccess && m->d_row_start)
    e = hipMemcpyAsync(m->d_row_start, row_start.data(), 4 * row_start.size(), hipMemcpyHostToDevice, st);
  if (e != hipSuccess) return bail(fail(CDDT_EDEVICE, std::string("cddt_create: copy failed: ") + hipGetErrorString(e)));
  if ((s = build_structure(m, st)) != CDDT_OK) return bail(s);
  *out_h = m;
  return CDDT_OK;
}

cddt_status cddt_destroy(cddt_map m) {
  if (!m) return CDDT_OK;
  (void)hipDeviceSynchronize();
  release_all(m);
  delete m;
  return CDDT_OK;
}

cddt_status cddt_cast(cddt_map m, const float* x, const float* y, const float* theta, int64_t n, int32_t max_range,
                      int32_t* ranges_out, void* stream) {
  if (!m) return fail(CDDT_EINVAL, "cddt_cast: map is NULL");
  if (n < 0) return fail(CDDT_EINVAL, "cddt_cast: n < 0");
  if (max_range < 0 || max_range > 65535) return fail(CDDT_EINVAL, "cddt_cast: max_range must be in 0..65535");
  if (n > 0 && (!x || !y || !theta || !ranges_out)) return fail(CDDT_EINVAL, "cddt_cast: NULL array");
  return launch_cast(m->dev(), x, y, theta, n, max_range, ranges_out, (hipStream_t)stream);
}

cddt_status cddt_weight(cddt_map m, const float* px, const float* py, const float* ptheta, int64_t n_particles,
                        const float* ray_offsets, int32_t n_rays, int32_t pair_offset, const int32_t* obs_ranges,
                        const float* log_table, int32_t max_range, float* logw_out, int32_t* ranges_out,
                        void* stream) {
  cddt_filter f{};
  f.map = m;
  f.px = px;
  f.py = py;
  f.ptheta = ptheta;
  f.n_particles = n_particles;
  f.ray_offsets = ray_offsets;
  f.n_rays = n_rays;
  f.pair_offset = pair_offset;
  f.obs_ranges = obs_ranges;
  f.log_table = log_table;
  f.max_range = max_range;
  f.logw_out = logw_out;
  f.ranges_out = ranges_out;
  CDDT_TRY(check_filter(f, "cddt_weight"));
  return launch_weight(filter_dev(f), (hipStream_t)stream);
}

int32_t cddt_pair_offset(const float* offsets_h, int32_t n_rays) {
  if (!offsets_h || n_rays < 2) return 0;
  int32_t best = 0, best_n = 0;
  for (int32_t p = 1; p < n_rays; ++p) {
    int32_t cnt = 0;
    for (int32_t r = 0; r + p < n_rays; ++r) {
      double d = (double)offsets_h[r + p] - (double)offsets_h[r];
      if (std::fabs(std::fabs(d) - M_PI) < 1e-4) ++cnt;
    }
    if (cnt > best_n) {
      best_n = cnt;
      best = p;
    }
  }
  return best;
}

cddt_status cddt_info(cddt_map m, cddt_stats* out_h) {
  if (!m || !out_h) return fail(CDDT_EINVAL, "cddt_info: NULL argument");
  if (m->stats_stale) {  // the longest band after updates: one reduction over the band headers
    CDDT_TRY(refresh_stats(m, nullptr));
    m->stats_stale = false;
  }
  cddt_stats s{};
  s.width = m->w;
  s.height = m->h;
  s.theta_bins = m->n;
  s.slices = m->half;
  s.flags = m->flags;
  s.rows = m->rows;
  s.edge_cells = m->edge_cells;
  s.zero_points = m->zero_points;
  s.capacity = m->capacity;
  s.max_row_len = m->max_row_len;
  s.bucket_lines = m->d_bk ? m->rows * m->nbk : 0;
  s.bucket_overflow = m->d_bk ? m->bucket_overflow : 0;
  s.bucket_log2 = m->d_bk ? m->blog2 : 0;
  s.device_bytes = (int64_t)m->w * m->h + (int64_t)sizeof(SliceDev) * m->half + m->rows * kNodeInts * 4 +
                   m->capacity * 4 + s.bucket_lines * 128 + (m->d_bk ? 4 * (m->half + 1) + 8 : 0);
  s.rebuilds = m->rebuilds;
  *out_h = s;
  return CDDT_OK;
}

cddt_status cddt_slice_table(cddt_map m, int32_t* c_h, int32_t* s_h, int32_t* row_min_h, int32_t* nrows_h,
                             float* k_scale_h) {
  if (!m) return fail(CDDT_EINVAL, "cddt_slice_table: map is NULL");
  for (int k = 0; k < m->half; ++k) {
    if (c_h) c_h[k] = m->c[k];
    if (s_h) s_h[k] = m->s[k];
    if (row_min_h) row_min_h[k] = m->row_min[k];
    if (nrows_h) nrows_h[k] = m->nrows[k];
  }
  if (k_scale_h) *k_scale_h = m->k_scale;
  return CDDT_OK;
}

cddt_status cddt_export(cddt_map m, int64_t* row_start_h, int32_t* row_len_h, int32_t* zeros_h) {
  if (!m) return fail(CDDT_EINVAL, "cddt_export: map is NULL");
  CDDT_HIP(hipDeviceSynchronize());
  std::vector<int32_t> hdr((size_t)m->rows * kNodeInts);
  CDDT_HIP(hipMemcpy(hdr.data(), m->d_hdr, 4 * hdr.size(), hipMemcpyDeviceToHost));
  int64_t total = 0;
  for (int64_t r = 0; r < m->rows; ++r) total += hdr[r * kNodeInts + 1];
  if (total != m->zero_points) return fail(CDDT_EINTERNAL, "cddt_export: band lengths do not add up");
  std::vector<int32_t> z;
  if (zeros_h && m->capacity) {
    z.resize((size_t)m->capacity);
    CDDT_HIP(hipMemcpy(z.data(), m->d_zeros, 4 * (size_t)m->capacity, hipMemcpyDeviceToHost));
  }
  int64_t o = 0;
  for (int64_t r = 0; r < m->rows; ++r) {
    const uint32_t start = (uint32_t)hdr[r * kNodeInts];
    const int32_t len = hdr[r * kNodeInts + 1];
    if (row_start_h) row_start_h[r] = o;
    if (row_len_h) row_len_h[r] = len;
    if (zeros_h && len) std::memcpy(zeros_h + o, z.data() + start, 4 * (size_t)len);
    o += len;
  }
  if (row_start_h) row_start_h[m->rows] = o;
  return CDDT_OK;
}

cddt_status cddt_export_grid(cddt_map m, uint8_t* occ_h) {
  if (!m || !occ_h) return fail(CDDT_EINVAL, "cddt_export_grid: NULL argument");
  CDDT_HIP(hipDeviceSynchronize());
  CDDT_HIP(hipMemcpy(occ_h, m->d_occ, (size_t)m->w * m->h, hipMemcpyDeviceToHost));
  return CDDT_OK;
}

cddt_status cddt_export_buckets(cddt_map m, int32_t* lines_h, int64_t n_ints) {
  if (!m || !lines_h) return fail(CDDT_EINVAL, "cddt_export_buckets: NULL argument");
  if (!m->d_bk) return fail(CDDT_EINVAL, "cddt_export_buckets: the map has no bucket index");
  const int64_t want = m->rows * (int64_t)m->nbk * kLineInts;
  if (n_ints != want)
    return fail(CDDT_EINVAL, "cddt_export_buckets: n_ints must be " + std::to_string(want));
  CDDT_HIP(hipDeviceSynchronize());
  CDDT_HIP(hipMemcpy(lines_h, m->d_bk, 4 * (size_t)want, hipMemcpyDeviceToHost));
  return CDDT_OK;
}

cddt_status cddt_update(cddt_map m, const int32_t* xs_h, const int32_t* ys_h, const uint8_t* values_h,
                        int64_t n_ops, void* stream) {
  if (!m) return fail(CDDT_EINVAL, "cddt_update: map is NULL");
  if (n_ops < 0) return fail(CDDT_EINVAL, "cddt_update: n_ops < 0");
  if (n_ops == 0) return CDDT_OK;
  if (!xs_h || !ys_h || !values_h) return fail(CDDT_EINVAL, "cddt_update: NULL array");
  for (int64_t k = 0; k < n_ops; ++k)
    if (xs_h[k] < 0 || ys_h[k] < 0 || xs_h[k] >= m->w || ys_h[k] >= m->h)
      return fail(CDDT_EINVAL, "cddt_update: op " + std::to_string(k) + " is off the map");
  return apply_update(m, xs_h, ys_h, values_h, n_ops, (hipStream_t)stream);
}

}  // extern "C"
