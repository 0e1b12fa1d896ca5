// Many filters in one persistent launch, called without a plan object.
//
// The filter descriptors and the prefix sums of their tile counts reach the
// device as kernel arguments: a short kernel per chunk of kPutChunk filters
// writes them into a workspace (and the first one clears the tile counters),
// then the persistent kernel of batch.hip runs over them.  A call is thus
// kernel launches only: no host-to-device copy, no synchronisation, and no
// allocation once the workspace holds enough filters, so a call can be
// recorded into a hipGraph, whose kernel nodes keep the descriptors of the
// capture by value.
//
// The workspace belongs to the (device, stream) pair of the call, so calls
// on one stream are ordered and calls on different streams do not share it.
// The variant for callers that cannot allocate takes its workspace from a
// fixed device array instead (one copy per device, shared by every call).
#include <algorithm>
#include <map>
#include <mutex>
#include <utility>

#include "batch_kernel.h"

namespace cddt {
namespace {

constexpr int kPutChunk = 20;
struct PutChunk {
  FilterDev f[kPutChunk];
  int64_t prefix[kPutChunk];  // prefix[base + i + 1] for i < count
  int32_t base, count;
  int32_t first;  // also write prefix[0] = 0 and clear the tile counters
  int32_t pad;
};
static_assert(sizeof(PutChunk) <= 4000, "kernel arguments stay under 4 KB");
static_assert(sizeof(FilterDev) % 8 == 0, "descriptors copy as 64-bit words");
constexpr int kPutThreads = 256;
constexpr int kWordsPerFilter = (int)(sizeof(FilterDev) / 8);

__global__ __launch_bounds__(kPutThreads) void k_put_filters(PutChunk c, FilterDev* __restrict__ filters,
                                                             int64_t* __restrict__ prefix,
                                                             unsigned long long* __restrict__ counter) {
  const uint64_t* src = reinterpret_cast<const uint64_t*>(&c.f[0]);
  uint64_t* dst = reinterpret_cast<uint64_t*>(filters + c.base);
  for (int w = threadIdx.x; w < c.count * kWordsPerFilter; w += kPutThreads) dst[w] = src[w];
  if (threadIdx.x < c.count) prefix[c.base + threadIdx.x + 1] = c.prefix[threadIdx.x];
  if (c.first) {
    if (threadIdx.x == 0) prefix[0] = 0;
    if (threadIdx.x < kTileParts) counter[threadIdx.x * kCounterStride] = 0ull;
  }
}

// A workspace: tile counters, n + 1 prefix sums and n descriptors in one block.
struct Workspace {
  void* mem = nullptr;
  int32_t cap = 0;
};
constexpr size_t workspace_bytes(int32_t cap) {
  return kBatchCounterBytes + sizeof(int64_t) * (size_t)(cap + 1 + 1) + sizeof(FilterDev) * (size_t)cap;
}
struct Parts {
  unsigned long long* counter;
  int64_t* prefix;
  FilterDev* filters;
};
Parts carve(void* mem, int32_t cap) {
  Parts p;
  char* b = static_cast<char*>(mem);
  p.counter = reinterpret_cast<unsigned long long*>(b);
  p.prefix = reinterpret_cast<int64_t*>(b + kBatchCounterBytes);
  // descriptors start on a 16-byte boundary after cap + 1 prefix words
  p.filters = reinterpret_cast<FilterDev*>(b + kBatchCounterBytes + sizeof(int64_t) * (size_t)((cap + 1 + 1) & ~1));
  return p;
}

std::mutex g_ws_mu;
std::map<std::pair<int, hipStream_t>, Workspace> g_ws;

// Workspace of cddt_batch_weight_noalloc: at most kNoAllocFilters filters
// (about 170 KiB), held by every device the library runs on until the
// process ends.  Host code reaches it only through the address that
// hipGetSymbolAddress returns for the current device (g_scratch_ptr).
constexpr int32_t kNoAllocFilters = 1024;
constexpr size_t kNoAllocBytes = workspace_bytes(kNoAllocFilters);
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// The device address of `scratch` on device `dev` (current), taken once.
cddt_status scratch_address(int dev, void** out) {
  if (dev < 0 || dev >= kMaxDevices) return fail(CDDT_EDEVICE, "cddt_batch_weight_noalloc: device index out of range");
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    CDDT_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(CDDT_EDEVICE, "cddt_batch_weight_noalloc: no device address for the workspace");
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return CDDT_OK;
}

// Host side of one call: check, take descriptors, upload by kernel
// arguments into `parts`, launch.  `cus` compute units.
cddt_status enqueue_batch(const cddt_filter* filters_h, int32_t n, const cddt_tuning& t, const Parts& parts,
                          int32_t cus, hipStream_t st) {
  const int64_t ppt = t.particles_per_tile;
  bool zp16 = false;
  int64_t total = 0;
  PutChunk c{};
  for (int32_t base = 0; base < n; base += kPutChunk) {
    c = PutChunk{};
    c.base = base;
    c.count = std::min(kPutChunk, n - base);
    c.first = base == 0 ? 1 : 0;
    for (int32_t i = 0; i < c.count; ++i) {
      const cddt_filter& f = filters_h[base + i];
      c.f[i] = filter_dev(f);
      zp16 = zp16 || c.f[i].map.zp16;
      total += (f.n_particles + ppt - 1) / ppt;
      c.prefix[i] = total;
    }
    hipLaunchKernelGGL(k_put_filters, dim3(1), dim3(kPutThreads), 0, st, c, parts.filters, parts.prefix,
                       parts.counter);
    CDDT_HIP(hipGetLastError());
  }
  return launch_batch(parts.filters, parts.prefix, n, total, t, parts.counter, cus, st, zp16,
                      /*counter_zeroed=*/true);
}

cddt_status check_call(const cddt_filter* filters_h, int32_t n, const cddt_tuning* tuning_h, const char* who,
                       cddt_tuning* t) {
  if (!filters_h || n < 1 || n > 65536) return fail(CDDT_EINVAL, std::string(who) + ": need 1..65536 filters");
  for (int32_t f = 0; f < n; ++f) CDDT_TRY(validate_filter(filters_h[f], who));
  *t = tuning_h ? *tuning_h : cached_tuning(filters_h, n);
  return check_tuning(*t);
}

}  // namespace
}  // namespace cddt

using namespace cddt;

extern "C" {

cddt_status cddt_batch_weight(const cddt_filter* filters_h, int32_t n_filters, const cddt_tuning* tuning_h,
                              void* stream) {
  cddt_tuning t;
  CDDT_TRY(check_call(filters_h, n_filters, tuning_h, "cddt_batch_weight", &t));
  hipStream_t st = (hipStream_t)stream;
  int dev = 0;
  CDDT_HIP(hipGetDevice(&dev));
  const int32_t cus = cddt_device_cus();
  if (cus <= 0) return fail(CDDT_EDEVICE, "cddt_batch_weight: cannot query the device");
  // held while enqueueing, so calls from several threads on one stream do not
  // interleave their descriptor uploads
  std::lock_guard<std::mutex> g(g_ws_mu);
  Workspace& ws = g_ws[{dev, st}];
  if (ws.cap < n_filters) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    CDDT_HIP(hipStreamIsCapturing(st, &cs));
    if (cs != hipStreamCaptureStatusNone)
      return fail(CDDT_EINVAL,
                  "cddt_batch_weight: the stream's workspace must first grow to this many filters in a call "
                  "outside graph capture");
    int32_t cap = 64;
    while (cap < n_filters) cap *= 2;
    void* mem = nullptr;
    if (hipMalloc(&mem, workspace_bytes(cap)) != hipSuccess)
      return fail(CDDT_ENOMEM, "cddt_batch_weight: workspace allocation failed");
    if (ws.mem) {
      // the previous workspace may still be read by work queued on the stream
      if (hipStreamSynchronize(st) != hipSuccess) {
        (void)hipFree(mem);
        return fail(CDDT_EDEVICE, "cddt_batch_weight: stream synchronisation failed");
      }
      (void)hipFree(ws.mem);
    }
    ws.mem = mem;
    ws.cap = cap;
  }
  return enqueue_batch(filters_h, n_filters, t, carve(ws.mem, ws.cap), cus, st);
}

cddt_status cddt_batch_weight_noalloc(const cddt_filter* filters_h, int32_t n_filters, const cddt_tuning* tuning_h,
                                      void* stream) {
  if (n_filters > kNoAllocFilters)
    return fail(CDDT_EINVAL, "cddt_batch_weight_noalloc: at most 1024 filters (the fixed workspace's size)");
  cddt_tuning t;
  CDDT_TRY(check_call(filters_h, n_filters, tuning_h, "cddt_batch_weight_noalloc", &t));
  int dev = 0;
  CDDT_HIP(hipGetDevice(&dev));
  void* ws = nullptr;
  CDDT_TRY(scratch_address(dev, &ws));
  const int32_t cus = cddt_device_cus();
  if (cus <= 0) return fail(CDDT_EDEVICE, "cddt_batch_weight_noalloc: cannot query the device");
  std::lock_guard<std::mutex> g(g_scratch_mu);
  return enqueue_batch(filters_h, n_filters, t, carve(ws, kNoAllocFilters), cus, (hipStream_t)stream);
}

}  // extern "C"
