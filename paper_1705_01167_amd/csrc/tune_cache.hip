// Tunings of the persistent batched launch found by the autotuner, kept in
// the library per filter set, so that a plan or a one-call launch created
// without a tuning uses them.
#include <algorithm>
#include <cmath>
#include <mutex>
#include <unordered_map>

#include "cddt_common.h"

namespace cddt {
namespace {

// Tuning cache: signature of a filter set -> tuning.  The signature covers
// what the best tuning depends on: device, filter count, the particle total
// to the nearest power of two, the set of theta bin counts and the set of
// structure layouts (bucket width, 16-bit lines, pruning).
std::mutex g_tune_mu;
std::unordered_map<uint64_t, cddt_tuning> g_tune;

inline void fnv(uint64_t& h, uint64_t v) {
  for (int k = 0; k < 8; ++k) {
    h ^= (v >> (8 * k)) & 0xffu;
    h *= 1099511628211ull;
  }
}

uint64_t signature_of(const cddt_filter* fs, int32_t n) {
  uint64_t bins[kMaxBins / 2 / 64] = {};  // one bit per possible slice count
  uint64_t layouts[2] = {};               // one bit per (bucket width, zp16, prune)
  int64_t total = 0;
  for (int32_t f = 0; f < n; ++f) {
    const cddt_map_s* m = fs[f].map;
    const int32_t half = m->half - 1;
    bins[half >> 6] |= 1ull << (half & 63);
    const uint32_t lay = (uint32_t)(m->d_bk ? m->blog2 : 0) * 4u + ((m->flags & CDDT_FLAG_ZP16) ? 2u : 0u) +
                         ((m->flags & CDDT_FLAG_PRUNE) ? 1u : 0u);
    layouts[lay >> 6] |= 1ull << (lay & 63);
    total += fs[f].n_particles;
  }
  int dev = 0;
  (void)hipGetDevice(&dev);
  uint64_t h = 1469598103934665603ull;
  fnv(h, (uint64_t)dev);
  fnv(h, (uint64_t)n);
  fnv(h, (uint64_t)std::llround(std::log2((double)std::max<int64_t>(1, total))));
  for (uint64_t w : bins) fnv(h, w);
  for (uint64_t w : layouts) fnv(h, w);
  return h;
}

}  // namespace

// The autotuned tuning of this filter set, else the library default.
cddt_tuning cached_tuning(const cddt_filter* filters_h, int32_t n_filters) {
  const uint64_t key = signature_of(filters_h, n_filters);
  std::lock_guard<std::mutex> g(g_tune_mu);
  auto it = g_tune.find(key);
  return it != g_tune.end() ? it->second : default_tuning();
}

}  // namespace cddt

using namespace cddt;

extern "C" {

cddt_status cddt_tuning_cache_put(const cddt_filter* filters_h, int32_t n_filters, const cddt_tuning* tuning_h) {
  if (!filters_h || !tuning_h || n_filters < 1) return fail(CDDT_EINVAL, "cddt_tuning_cache_put: bad argument");
  for (int32_t f = 0; f < n_filters; ++f) CDDT_TRY(validate_filter(filters_h[f], "cddt_tuning_cache_put"));
  CDDT_TRY(check_tuning(*tuning_h));
  const uint64_t key = signature_of(filters_h, n_filters);
  std::lock_guard<std::mutex> g(g_tune_mu);
  g_tune[key] = *tuning_h;
  return CDDT_OK;
}

cddt_status cddt_tuning_cache_get(const cddt_filter* filters_h, int32_t n_filters, cddt_tuning* tuning_h,
                                  int32_t* found_h) {
  if (!filters_h || !tuning_h || n_filters < 1) return fail(CDDT_EINVAL, "cddt_tuning_cache_get: bad argument");
  for (int32_t f = 0; f < n_filters; ++f) CDDT_TRY(validate_filter(filters_h[f], "cddt_tuning_cache_get"));
  const uint64_t key = signature_of(filters_h, n_filters);
  std::lock_guard<std::mutex> g(g_tune_mu);
  auto it = g_tune.find(key);
  if (found_h) *found_h = it != g_tune.end() ? 1 : 0;
  *tuning_h = it != g_tune.end() ? it->second : default_tuning();
  return CDDT_OK;
}

}  // extern "C"
