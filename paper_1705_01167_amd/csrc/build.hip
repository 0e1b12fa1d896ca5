// CDDT construction on the GPU (Sec. IV-A: edge map by erosion, projection of
// every edge cell into every stored slice, one sorted zero-point list per band).
//
// Pipeline (one stream):
//   k_edges    (x2)  8-neighbour erosion test per cell; a count pass, then a
//                    compaction pass (wave ballots, one atomic per block of
//                    4096 cells).
//   k_project  (count) per (slice, edge cell): the bands its rotated square
//                    covers; atomic per-band counters.
//   scan             per-band region = key capacity (length + slack, whole
//                    128-byte lines) + sample levels; exclusive scan gives each
//                    band's start (3-phase block scan, 64-bit totals).
//   k_project  (fill) scatter each zero point into its bands through per-band
//                    cursors (order inside a band is arbitrary here).
//   k_sort_small     one wave per band: bands of <= 64 sorted in registers
//                    (bitonic over lanes); longer bands are queued.
//   k_sort_large     persistent blocks take queued bands; bitonic network in
//                    LDS (<= 16384 values) or in place in global memory.
//   k_finalize       one wave per band: sample levels and the header node's
//                    top level (band_layout.h).
// Each band ends as the ascending multiset of its zero points, which is unique,
// so the result does not depend on atomic ordering.
#include <algorithm>
#include <climits>

#include "band_layout.h"
#include "bucket_lines.h"
#include "cddt_common.h"

namespace cddt {
namespace {

constexpr int kScanThreads = 1024;
constexpr int kScanItems = 4;
constexpr int kScanTile = kScanThreads * kScanItems;
constexpr int kLdsSortCap = 16384;

// Small device scalars used during a build.
struct BuildCounters {
  uint32_t edges;
  uint32_t big;
  uint64_t total_cap;
  uint64_t total_len;
  uint64_t max_len;
};

// Edge cells are packed as i | j << 16 (both < 2^14).  A block covers
// kEdgeThreads * kEdgeSweeps consecutive cells: it counts its edge cells
// (wave ballots summed in LDS), takes its place in the list with one atomic
// and, in the write pass, sweeps its cells again to store them.  The list
// order is arbitrary; the build does not depend on it.
constexpr int kEdgeThreads = 256;
constexpr int kEdgeSweeps = 16;
__global__ __launch_bounds__(kEdgeThreads) void k_edges(const uint8_t* __restrict__ occ, int w, int h, int full,
                                                        uint32_t* __restrict__ list, BuildCounters* ctr, int write) {
  __shared__ uint32_t wave_cnt[kEdgeThreads / 64];
  __shared__ uint32_t block_base;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t cells = (int64_t)w * h;
  const int64_t first = (int64_t)blockIdx.x * (kEdgeThreads * kEdgeSweeps);
  auto test = [&](int k, int& i, int& j) {
    const int64_t idx = first + (int64_t)k * kEdgeThreads + threadIdx.x;
    if (idx >= cells) return false;
    j = (int)(idx / w);
    i = (int)(idx - (int64_t)j * w);
    return edge_cell(occ, w, h, i, j, full);
  };
  uint32_t mine = 0;
  for (int k = 0; k < kEdgeSweeps; ++k) {
    int i = 0, j = 0;
    mine += (uint32_t)__popcll(__ballot(test(k, i, j)));
  }
  if (lane == 0) wave_cnt[wave] = mine;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t total = 0;
    for (int q = 0; q < kEdgeThreads / 64; ++q) total += wave_cnt[q];
    block_base = total ? atomicAdd(&ctr->edges, total) : 0u;
  }
  __syncthreads();
  if (!write) return;
  uint32_t off = block_base;
  for (int q = 0; q < wave; ++q) off += wave_cnt[q];
  for (int k = 0; k < kEdgeSweeps; ++k) {
    int i = 0, j = 0;
    const bool e = test(k, i, j);
    const uint64_t mask = __ballot(e);
    if (e) list[off + (uint32_t)__popcll(mask & ((1ull << lane) - 1ull))] = (uint32_t)i | ((uint32_t)j << 16);
    off += (uint32_t)__popcll(mask);
  }
}

// Per (slice = blockIdx.y, edge cell): count (fill == 0) or scatter (fill == 1).
__global__ void k_project(const SliceDev* __restrict__ slices, const uint32_t* __restrict__ cells,
                          uint32_t n_cells, uint32_t* __restrict__ cnt,
                          const int32_t* __restrict__ hdr, int32_t* __restrict__ zeros, int fill) {
  uint32_t e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n_cells) return;
  const SliceDev sl = slices[blockIdx.y];
  const uint32_t packed = cells[e];
  const int64_t i2 = 2 * (int64_t)(packed & 0xffffu) + 1;
  const int64_t j2 = 2 * (int64_t)(packed >> 16) + 1;
  const int64_t yc = j2 * sl.c - i2 * sl.s;
  const int64_t hs = (int64_t)abs(sl.c) + (int64_t)abs(sl.s);
  const int32_t lo = (int32_t)((yc - hs) >> 31);
  const int32_t hi = (int32_t)((yc + hs - 1) >> 31);
  const int32_t z = (int32_t)((i2 * sl.c + j2 * sl.s) >> 15);
  for (int32_t r = lo; r <= hi; ++r) {
    const int32_t row = sl.row_off + r;
    if (!fill) {
      atomicAdd(&cnt[row], 1u);
    } else {
      uint32_t pos = atomicAdd(&cnt[row], 1u);
      zeros[(uint32_t)hdr[(int64_t)row * kNodeInts] + pos] = z;
    }
  }
}

// Bucket index fill after a build: one wave per band, every line of the band
// (bucket_lines.h).
constexpr int kFillThreads = 256;
// LDS words of one wave's tables: first[0..nbk].
__host__ __device__ constexpr int32_t fill_wave_words(int32_t nbk) { return nbk + 1; }
static_assert((kFillThreads / 64) * fill_wave_words(kFillMaxBuckets) * 4 <= 65536, "fill tables fit in LDS");

__global__ __launch_bounds__(kFillThreads) void k_bucket_fill(const int32_t* __restrict__ hdr,
                                                              const int32_t* __restrict__ zeros,
                                                              const SliceDev* __restrict__ slices,
                                                              const int32_t* __restrict__ row_start, int32_t half,
                                                              int32_t shift, int32_t nbk, int32_t* __restrict__ bk,
                                                              uint64_t n_bands, unsigned long long* __restrict__ over,
                                                              int zp16) {
  extern __shared__ int32_t fill_lds[];
  int32_t* first = fill_lds + (threadIdx.x >> 6) * fill_wave_words(nbk);
  const uint64_t n_waves = ((uint64_t)gridDim.x * blockDim.x) >> 6;
  int over_n = 0;
  for (uint64_t band = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; band < n_bands; band += n_waves) {
    const int32_t zlo = slices[band_slice(row_start, half, (uint32_t)band)].zlo;
    const int32_t* node = hdr + (int64_t)band * kNodeInts;
    const int32_t* keys = zeros + (uint32_t)node[0];
    const int32_t len = node[1];
    bucket_firsts(keys, len, zlo, shift, nbk, first);
    int32_t* lines = bk + (int64_t)band * nbk * kLineInts;
    over_n += write_bucket_lines<true>(keys, len, zlo, shift, nbk, first, nullptr, nullptr, lines, zp16);
    wave_fence();  // first[] is rewritten for the wave's next band
  }
  if (over_n != 0) atomicAdd(over, (unsigned long long)over_n);
}

__device__ __forceinline__ uint64_t region_of(uint32_t len, int no_slack) {
  return region_slots(key_capacity(len, no_slack != 0));
}

// Inclusive scan of one value per thread across the block (uint64).
__device__ uint64_t block_inclusive_scan(uint64_t v, uint64_t* wave_tot) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    uint64_t t = __shfl_up(v, o);
    if (lane >= o) v += t;
  }
  if (lane == 63) wave_tot[wid] = v;
  __syncthreads();
  if (wid == 0) {
    uint64_t t = lane < nw ? wave_tot[lane] : 0;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      uint64_t u = __shfl_up(t, o);
      if (lane >= o) t += u;
    }
    if (lane < nw) wave_tot[lane] = t;
  }
  __syncthreads();
  if (wid > 0) v += wave_tot[wid - 1];
  __syncthreads();
  return v;
}

__global__ __launch_bounds__(kScanThreads) void k_tile_sum(const uint32_t* __restrict__ cnt, int64_t n,
                                                           int no_slack, uint64_t* __restrict__ tile_sum) {
  __shared__ uint64_t wt[kScanThreads / 64];
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  uint64_t s = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k)
    if (base + k < n) {
      s += region_of(cnt[base + k], no_slack);
    }
  uint64_t inc = block_inclusive_scan(s, wt);
  if (threadIdx.x == blockDim.x - 1) tile_sum[blockIdx.x] = inc;
}

// Single block: exclusive scan of the tile sums, total capacity into ctr.
__global__ __launch_bounds__(kScanThreads) void k_scan_tiles(uint64_t* __restrict__ tile_sum, int64_t ntiles,
                                                             BuildCounters* ctr) {
  __shared__ uint64_t wt[kScanThreads / 64];
  __shared__ uint64_t carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int64_t b = 0; b < ntiles; b += kScanThreads) {
    int64_t t = b + threadIdx.x;
    uint64_t v = t < ntiles ? tile_sum[t] : 0;
    uint64_t inc = block_inclusive_scan(v, wt);
    uint64_t c = carry;
    if (t < ntiles) tile_sum[t] = c + inc - v;
    __syncthreads();
    if (threadIdx.x == blockDim.x - 1) carry = c + inc;
    __syncthreads();
  }
  if (threadIdx.x == 0) ctr->total_cap = carry;
}

// Band starts and capacities; cnt is reset to 0 to serve as the fill cursor.
__global__ __launch_bounds__(kScanThreads) void k_scan_apply(uint32_t* __restrict__ cnt, int64_t n, int no_slack,
                                                             const uint64_t* __restrict__ tile_off,
                                                             int32_t* __restrict__ hdr,
                                                             BuildCounters* ctr) {
  __shared__ uint64_t wt[kScanThreads / 64];
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  uint32_t len[kScanItems];
  uint64_t s = 0, lsum = 0;
  uint32_t lmax = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    len[k] = base + k < n ? cnt[base + k] : 0u;
    s += base + k < n ? region_of(len[k], no_slack) : 0u;
    lsum += len[k];
    lmax = len[k] > lmax ? len[k] : lmax;
  }
  uint64_t off = block_inclusive_scan(s, wt) - s + tile_off[blockIdx.x];
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    if (base + k < n) {
      int32_t* h = hdr + (base + k) * kNodeInts;
      h[0] = (int32_t)(uint32_t)off;
      h[1] = (int32_t)len[k];
      h[2] = (int32_t)key_capacity(len[k], no_slack != 0);
      cnt[base + k] = 0;
      off += region_of(len[k], no_slack);
    }
  }
  // block totals of lengths and max length: one atomic per wave
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    lsum += __shfl_xor(lsum, o);
    uint32_t t = __shfl_xor(lmax, o);
    lmax = t > lmax ? t : lmax;
  }
  if ((threadIdx.x & 63) == 0) {
    if (lsum) atomicAdd((unsigned long long*)&ctr->total_len, (unsigned long long)lsum);
    if (lmax) atomicMax((unsigned long long*)&ctr->max_len, (unsigned long long)lmax);
  }
}

// Bitonic sort of one value per lane across a wave (ascending).
__device__ __forceinline__ int32_t wave_bitonic(int32_t v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int k = 2; k <= 64; k <<= 1) {
#pragma unroll
    for (int j = k >> 1; j > 0; j >>= 1) {
      int32_t p = __shfl_xor(v, j);
      bool asc = (lane & k) == 0;
      bool low = (lane & j) == 0;
      v = (low == asc) ? min(v, p) : max(v, p);
    }
  }
  return v;
}

__global__ void k_sort_small(const int32_t* __restrict__ hdr, int32_t* __restrict__ zeros, int64_t nrows,
                             uint32_t* __restrict__ big_list, BuildCounters* ctr) {
  const int64_t row = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (row >= nrows) return;
  const int lane = threadIdx.x & 63;
  const int2 hd = make_int2(hdr[row * kNodeInts], hdr[row * kNodeInts + 1]);
  if (hd.y <= 1) return;
  if (hd.y > 64) {
    if (lane == 0) big_list[atomicAdd(&ctr->big, 1u)] = (uint32_t)row;
    return;
  }
  int32_t* z = zeros + (uint32_t)hd.x;
  int32_t v = lane < hd.y ? z[lane] : INT_MAX;
  v = wave_bitonic(v);
  if (lane < hd.y) z[lane] = v;
}

// Sorting network over a[0, len) with every comparator ascending (min to the
// lower index); indices >= len behave as +infinity and are never touched.
template <typename Ptr>
__device__ void block_sort_network(Ptr a, int32_t len) {
  int32_t p2 = 1;
  while (p2 < len) p2 <<= 1;
  for (int32_t k = 2; k <= p2; k <<= 1) {
    for (int32_t j = k >> 1; j > 0; j >>= 1) {
      const bool flip = j == (k >> 1);
      for (int32_t t = threadIdx.x; t < (p2 >> 1); t += blockDim.x) {
        // t-th pair: insert a zero bit at position log2(j)
        int32_t lo = ((t & ~(j - 1)) << 1) | (t & (j - 1));
        int32_t hi = flip ? (lo ^ (k - 1)) : (lo | j);
        if (hi < len) {
          int32_t x = a[lo], y = a[hi];
          if (y < x) {
            a[lo] = y;
            a[hi] = x;
          }
        }
      }
      __syncthreads();
    }
  }
}

__global__ __launch_bounds__(256) void k_sort_large(const int32_t* __restrict__ hdr, int32_t* __restrict__ zeros,
                                                    const uint32_t* __restrict__ big_list,
                                                    const BuildCounters* ctr) {
  __shared__ int32_t buf[kLdsSortCap];
  const uint32_t nbig = ctr->big;
  for (uint32_t b = blockIdx.x; b < nbig; b += gridDim.x) {
    const int64_t row = big_list[b];
    const int2 hd = make_int2(hdr[row * kNodeInts], hdr[row * kNodeInts + 1]);
    int32_t* z = zeros + (uint32_t)hd.x;
    if (hd.y <= kLdsSortCap) {
      for (int32_t t = threadIdx.x; t < hd.y; t += blockDim.x) buf[t] = z[t];
      __syncthreads();
      block_sort_network(buf, hd.y);
      for (int32_t t = threadIdx.x; t < hd.y; t += blockDim.x) z[t] = buf[t];
    } else {
      block_sort_network(z, hd.y);
    }
    __syncthreads();
  }
}

__global__ void k_fill_u32(uint32_t* p, int64_t n, uint32_t v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// Sum and maximum of the band lengths (header word 1 of every node).
__global__ void k_len_stats(const int32_t* __restrict__ hdr, int64_t nrows, BuildCounters* ctr) {
  uint64_t sum = 0, mx = 0;
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < nrows; r += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t l = (uint32_t)hdr[r * kNodeInts + 1];
    sum += l;
    mx = l > mx ? l : mx;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    sum += __shfl_xor(sum, o);
    const uint64_t t = __shfl_xor(mx, o);
    mx = t > mx ? t : mx;
  }
  if ((threadIdx.x & 63) == 0) {
    if (sum) atomicAdd((unsigned long long*)&ctr->total_len, (unsigned long long)sum);
    if (mx) atomicMax((unsigned long long*)&ctr->max_len, (unsigned long long)mx);
  }
}

__global__ void k_finalize(int32_t* __restrict__ hdr, int32_t* __restrict__ zeros, int64_t nrows) {
  const int64_t row = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (row >= nrows) return;
  finalize_band(hdr + row * kNodeInts, zeros);
}

// RAII holder for build temporaries.
struct Temp {
  Allocator* a;
  void* p = nullptr;
  explicit Temp(Allocator* al) : a(al) {}
  ~Temp() {
    if (p) a->release(p);
  }
  cddt_status get(size_t bytes, const char* what) { return a->alloc(&p, bytes ? bytes : 16, what); }
};

unsigned grid_for(int64_t n, int threads) {
  int64_t b = (n + threads - 1) / threads;
  return (unsigned)(b < 1 ? 1 : b);
}

}  // namespace

void free_structure(cddt_map_s* m) {
  if (m->d_hdr) m->alloc.release(m->d_hdr);
  if (m->d_zeros) m->alloc.release(m->d_zeros);
  m->d_hdr = nullptr;
  m->d_zeros = nullptr;
}

// Exact zero-point total and longest band, from the header nodes.  Blocks.
cddt_status refresh_stats(cddt_map_s* m, hipStream_t st) {
  Temp ctr_t(&m->alloc);
  CDDT_TRY(ctr_t.get(sizeof(BuildCounters), "stats counters"));
  BuildCounters* ctr = (BuildCounters*)ctr_t.p;
  CDDT_HIP(hipMemsetAsync(ctr, 0, sizeof(BuildCounters), st));
  const int64_t blocks = std::min<int64_t>((m->rows + 255) / 256, 4096);
  hipLaunchKernelGGL(k_len_stats, dim3((unsigned)std::max<int64_t>(blocks, 1)), dim3(256), 0, st,
                     (const int32_t*)m->d_hdr, m->rows, ctr);
  CDDT_HIP(hipGetLastError());
  BuildCounters hc{};
  CDDT_HIP(hipMemcpyAsync(&hc, ctr, sizeof(hc), hipMemcpyDeviceToHost, st));
  CDDT_HIP(hipStreamSynchronize(st));
  m->zero_points = (int64_t)hc.total_len;
  m->max_row_len = (int64_t)hc.max_len;
  m->stats_stale = false;
  return CDDT_OK;
}

// Builds the header nodes and band regions from m->d_occ and m->d_slices.
// Blocks on `st`.
cddt_status build_structure(cddt_map_s* m, hipStream_t st) {
  free_structure(m);
  ++m->generation;
  const int64_t cells = (int64_t)m->w * m->h;
  const int64_t R = m->rows;
  Temp ctr_t(&m->alloc), edges_t(&m->alloc), cnt_t(&m->alloc), big_t(&m->alloc);
  CDDT_TRY(ctr_t.get(sizeof(BuildCounters), "build counters"));
  BuildCounters* ctr = (BuildCounters*)ctr_t.p;
  CDDT_HIP(hipMemsetAsync(ctr, 0, sizeof(BuildCounters), st));
  const int full = (m->flags & CDDT_FLAG_FULL_MAP) ? 1 : 0;
  const int no_slack = (m->flags & CDDT_FLAG_STATIC) ? 1 : 0;

  // 1. edge map: count, then compact
  const unsigned edge_blocks = grid_for(cells, kEdgeThreads * kEdgeSweeps);
  hipLaunchKernelGGL(k_edges, dim3(edge_blocks), dim3(kEdgeThreads), 0, st, m->d_occ, m->w, m->h, full,
                     (uint32_t*)nullptr, ctr, 0);
  CDDT_HIP(hipGetLastError());
  BuildCounters hc{};
  CDDT_HIP(hipMemcpyAsync(&hc, ctr, sizeof(hc), hipMemcpyDeviceToHost, st));
  CDDT_HIP(hipStreamSynchronize(st));
  const uint32_t n_edges = hc.edges;
  m->edge_cells = n_edges;
  CDDT_TRY(edges_t.get((size_t)n_edges * 4, "edge list"));
  CDDT_HIP(hipMemsetAsync(ctr, 0, sizeof(BuildCounters), st));
  if (n_edges)
    hipLaunchKernelGGL(k_edges, dim3(edge_blocks), dim3(kEdgeThreads), 0, st, m->d_occ, m->w, m->h, full,
                       (uint32_t*)edges_t.p, ctr, 1);

  // 2. per-band counts
  CDDT_TRY(cnt_t.get((size_t)R * 4, "band counters"));
  uint32_t* cnt = (uint32_t*)cnt_t.p;
  hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(R, 256) < 65536 ? grid_for(R, 256) : 65536), dim3(256), 0, st,
                     cnt, R, 0u);
  if (n_edges)
    hipLaunchKernelGGL(k_project, dim3(grid_for(n_edges, 256), m->half), dim3(256), 0, st, m->d_slices,
                       (const uint32_t*)edges_t.p, n_edges, cnt, (const int32_t*)nullptr, (int32_t*)nullptr, 0);
  CDDT_HIP(hipGetLastError());

  // 3. band layout
  CDDT_TRY(m->alloc.alloc((void**)&m->d_hdr, (size_t)R * kNodeInts * 4, "band header nodes"));
  uint64_t used = 0;
  CDDT_TRY(layout_bands(m, cnt, m->d_hdr, no_slack != 0, &used, &hc.total_len, &hc.max_len, st));

  // a spare area (1/8 of the regions, at least 64 Ki slots; none for static
  // maps) takes bands that outgrow their region during updates
  const uint64_t spare = no_slack ? 0 : (uint64_t)round_line(std::max<uint64_t>(used / 8, 65536));
  if (used + spare >= (1ull << 32)) {
    free_structure(m);
    return fail(CDDT_ENOMEM, "structure needs more than 2^32 zero-point slots");
  }
  m->capacity = (int64_t)(used + spare);
  m->spare_end = (int64_t)(used + spare);
  m->zero_points = (int64_t)hc.total_len;
  m->max_row_len = (int64_t)hc.max_len;
  if (!m->d_spare) CDDT_TRY(m->alloc.alloc((void**)&m->d_spare, 8, "spare cursor"));
  {
    const unsigned long long cursor = used;
    CDDT_HIP(hipMemcpyAsync(m->d_spare, &cursor, 8, hipMemcpyHostToDevice, st));
    CDDT_HIP(hipStreamSynchronize(st));  // the host value goes out of scope
  }

  // 4. fill, sort, finalize
  cddt_status st_alloc = m->alloc.alloc((void**)&m->d_zeros, (size_t)(m->capacity ? m->capacity : 1) * 4,
                                        "zero points");
  if (st_alloc != CDDT_OK) {
    free_structure(m);
    return st_alloc;
  }
  if (n_edges)
    hipLaunchKernelGGL(k_project, dim3(grid_for(n_edges, 256), m->half), dim3(256), 0, st, m->d_slices,
                       (const uint32_t*)edges_t.p, n_edges, cnt, (const int32_t*)m->d_hdr, m->d_zeros, 1);
  CDDT_TRY(big_t.get((size_t)R * 4, "long-band list"));
  hipLaunchKernelGGL(k_sort_small, dim3(grid_for(R, 4)), dim3(256), 0, st, (const int32_t*)m->d_hdr, m->d_zeros,
                     R, (uint32_t*)big_t.p, ctr);
  hipLaunchKernelGGL(k_sort_large, dim3(2048), dim3(256), 0, st, (const int32_t*)m->d_hdr, m->d_zeros,
                     (const uint32_t*)big_t.p, (const BuildCounters*)ctr);
  CDDT_TRY(finalize_bands(m->d_hdr, m->d_zeros, R, st));
  if (m->flags & CDDT_FLAG_PRUNE) CDDT_TRY(prune_structure(m, st));
  if (m->d_bk) return fill_buckets(m, st);
  return CDDT_OK;
}

cddt_status layout_bands(cddt_map_s* m, uint32_t* cnt, int32_t* hdr, bool no_slack, uint64_t* total_cap,
                         uint64_t* total_len, uint64_t* max_len, hipStream_t st) {
  const int64_t R = m->rows;
  Temp ctr_t(&m->alloc), tiles_t(&m->alloc);
  CDDT_TRY(ctr_t.get(sizeof(BuildCounters), "layout counters"));
  BuildCounters* ctr = (BuildCounters*)ctr_t.p;
  CDDT_HIP(hipMemsetAsync(ctr, 0, sizeof(BuildCounters), st));
  const int64_t ntiles = (R + kScanTile - 1) / kScanTile;
  CDDT_TRY(tiles_t.get((size_t)ntiles * 8, "scan tiles"));
  uint64_t* tiles = (uint64_t*)tiles_t.p;
  const int ns = no_slack ? 1 : 0;
  hipLaunchKernelGGL(k_tile_sum, dim3((unsigned)ntiles), dim3(kScanThreads), 0, st, cnt, R, ns, tiles);
  hipLaunchKernelGGL(k_scan_tiles, dim3(1), dim3(kScanThreads), 0, st, tiles, ntiles, ctr);
  hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)ntiles), dim3(kScanThreads), 0, st, cnt, R, ns,
                     (const uint64_t*)tiles, hdr, ctr);
  CDDT_HIP(hipGetLastError());
  BuildCounters hc{};
  CDDT_HIP(hipMemcpyAsync(&hc, ctr, sizeof(hc), hipMemcpyDeviceToHost, st));
  CDDT_HIP(hipStreamSynchronize(st));
  *total_cap = hc.total_cap;
  *total_len = hc.total_len;
  *max_len = hc.max_len;
  return CDDT_OK;
}

cddt_status finalize_bands(int32_t* hdr, int32_t* zeros, int64_t rows, hipStream_t st) {
  if (rows > 0) hipLaunchKernelGGL(k_finalize, dim3(grid_for(rows, 4)), dim3(256), 0, st, hdr, zeros, rows);
  CDDT_HIP(hipGetLastError());
  CDDT_HIP(hipStreamSynchronize(st));
  return CDDT_OK;
}

cddt_status fill_buckets(cddt_map_s* m, hipStream_t st) {
  const int64_t n_rows = m->rows;
  if (!m->d_bk || n_rows <= 0) return CDDT_OK;
  if (m->nbk > kFillMaxBuckets) return fail(CDDT_EINTERNAL, "bucket fill: more buckets per band than planned");
  CDDT_HIP(hipMemsetAsync(m->d_bk_over, 0, 8, st));
  const uint64_t blocks = std::min<uint64_t>(((uint64_t)n_rows + 3) / 4, 1u << 16);  // 4 bands per block
  const size_t lds = (size_t)(kFillThreads / 64) * fill_wave_words(m->nbk) * sizeof(int32_t);
  hipLaunchKernelGGL(k_bucket_fill, dim3((unsigned)std::max<uint64_t>(blocks, 1)), dim3(kFillThreads), lds, st,
                     (const int32_t*)m->d_hdr, (const int32_t*)m->d_zeros, (const SliceDev*)m->d_slices,
                     (const int32_t*)m->d_row_start, m->half, 16 + m->blog2, m->nbk, m->d_bk, (uint64_t)n_rows,
                     m->d_bk_over, (m->flags & CDDT_FLAG_ZP16) ? 1 : 0);
  CDDT_HIP(hipGetLastError());
  unsigned long long over = 0;
  CDDT_HIP(hipMemcpyAsync(&over, m->d_bk_over, 8, hipMemcpyDeviceToHost, st));
  CDDT_HIP(hipStreamSynchronize(st));
  m->bucket_overflow = (int64_t)over;
  return CDDT_OK;
}

}  // namespace cddt
