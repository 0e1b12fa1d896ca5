// PCDDT: pruning of a static CDDT (Sec. IV-C, pruning).  The paper casts from
// every state of the discrete configuration space and drops every zero point
// that no cast returns.  The states here are the centres of the free cells
// under every theta bin: both bins of a stored slice (theta and theta + pi)
// land a centre at the same band and projection, one returning the successor
// and the other the predecessor, so one band search per (free cell, slice)
// covers both.  Each band then keeps the distinct values that some state
// returned, ascending; casts from those states answer exactly as on the full
// structure, other queries may see past a dropped point.
//
//   k_prune_mark     one lane per (cell, slice): the band's ranks of the
//                    centre's projection (keys <= x, keys < x) by the band's
//                    search lines; marks the successor and predecessor slots.
//   k_prune_keep     one wave per band: a slot is kept when it starts its run
//                    of equal keys and some slot of the run is marked; counts.
//   layout           band starts for the kept lengths (no slack).
//   k_prune_compact  one wave per band: kept keys in order (ballot ranks).
//   finalize         sample levels and header top levels (band_layout.h).
#include <algorithm>
#include <climits>

#include "query_device.h"

namespace cddt {
namespace {

// Ranks of x among a band's keys: le = keys <= x, lt = keys < x; start and len
// of the band's key region.
__device__ __forceinline__ void band_ranks(const MapDev& m, int32_t row, int32_t x, uint32_t& start, int32_t& len,
                                           int32_t& le, int32_t& lt) {
  Line32 L = load_line(m.hdr + (int64_t)row * kNodeInts);
  start = (uint32_t)L.e[0];
  len = L.e[1];
  const uint32_t cap = (uint32_t)L.e[2];
  int32_t c, nxt, prv;
  scan_line<kHeaderWords>(L, x, INT_MAX, c, nxt, prv);
  for (int t = top_level(len) - 1; t >= 0 && c > 0; --t) {
    const int32_t blk = c - 1;
    L = load_line(m.zeros + level_base(start, cap, t) + (uint32_t)blk * kLineInts);
    int32_t lc;
    scan_line<0>(L, x, nxt, lc, nxt, prv);
    c = blk * kLineInts + lc;
  }
  le = c;
  lt = (c > 0 && prv == x) ? lower_bound_i32(m.zeros + start, c, x) : c;
}

// m: the map's band view (no bucket index).  mark: one byte per zero-point slot.
__global__ void k_prune_mark(MapDev m, uint8_t* __restrict__ mark) {
  const int64_t cell = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (cell >= (int64_t)m.w * m.h) return;
  if (ldg(m.occ + cell) != 0) return;  // casts from inside an obstacle return 0 without a search
  const int32_t i = (int32_t)(cell % m.w), j = (int32_t)(cell / m.w);
  const int32_t xf = (i << 16) + 0x8000, yf = (j << 16) + 0x8000;  // the cell centre, Q16
  const Landing l = land(m, (int32_t)blockIdx.y, xf, yf);
  uint32_t start;
  int32_t len, le, lt;
  band_ranks(m, l.row, l.xq, start, len, le, lt);
  if (le < len) mark[(uint64_t)start + (uint32_t)le] = 1;      // successor: first key > x
  if (lt > 0) mark[(uint64_t)start + (uint32_t)(lt - 1)] = 1;  // predecessor: last key < x
}

__global__ void k_prune_keep(const int32_t* __restrict__ hdr, const int32_t* __restrict__ zeros,
                             uint8_t* __restrict__ mark, int64_t nrows, uint32_t* __restrict__ cnt) {
  const int64_t row = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (row >= nrows) return;  // whole wave
  const int lane = threadIdx.x & 63;
  const uint32_t start = (uint32_t)hdr[row * kNodeInts];
  const int32_t len = hdr[row * kNodeInts + 1];
  uint32_t kept = 0;
  for (int32_t b = 0; b < len; b += 64) {
    const int32_t k = b + lane;
    bool keep = false;
    if (k < len) {
      const int32_t v = zeros[start + k];
      if (k == 0 || zeros[start + k - 1] != v) {  // first slot of its run of equal keys
        bool any = false;
        for (int32_t q = k; q < len && zeros[start + q] == v; ++q) any = any || (mark[start + q] & 1) != 0;
        keep = any;
      }
    }
    const uint64_t bal = __ballot(keep);
    // bit 1 = kept; bit 0, which other lanes read above, is left as it is
    if (keep) mark[start + k] = (uint8_t)(mark[start + k] | 2);
    kept += (uint32_t)__popcll(bal);
  }
  if (lane == 0) cnt[row] = kept;
}

__global__ void k_prune_compact(const int32_t* __restrict__ ohdr, const int32_t* __restrict__ ozeros,
                                const uint8_t* __restrict__ mark, int64_t nrows, const int32_t* __restrict__ nhdr,
                                int32_t* __restrict__ nzeros) {
  const int64_t row = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (row >= nrows) return;  // whole wave
  const int lane = threadIdx.x & 63;
  const uint32_t os = (uint32_t)ohdr[row * kNodeInts], ns = (uint32_t)nhdr[row * kNodeInts];
  const int32_t len = ohdr[row * kNodeInts + 1];
  uint32_t base = 0;
  for (int32_t b = 0; b < len; b += 64) {
    const int32_t k = b + lane;
    const bool keep = k < len && (mark[os + k] & 2) != 0;
    const uint64_t bal = __ballot(keep);
    if (keep) nzeros[ns + base + (uint32_t)__popcll(bal & ((1ull << lane) - 1ull))] = ozeros[os + k];
    base += (uint32_t)__popcll(bal);
  }
}

unsigned blocks_of(int64_t n, int per_block) {
  const int64_t b = (n + per_block - 1) / per_block;
  return (unsigned)(b < 1 ? 1 : b);
}

}  // namespace

cddt_status prune_structure(cddt_map_s* m, hipStream_t st) {
  const int64_t R = m->rows, cells = (int64_t)m->w * m->h;
  void *mark_p = nullptr, *cnt_p = nullptr, *hdr_p = nullptr, *zeros_p = nullptr;
  auto drop = [&]() {
    for (void* p : {mark_p, cnt_p, hdr_p, zeros_p})
      if (p) m->alloc.release(p);
  };
  cddt_status s = m->alloc.alloc(&mark_p, (size_t)std::max<int64_t>(m->capacity, 1), "prune marks");
  if (s == CDDT_OK) s = m->alloc.alloc(&cnt_p, (size_t)R * 4, "prune counts");
  if (s == CDDT_OK) s = m->alloc.alloc(&hdr_p, (size_t)R * kNodeInts * 4, "pruned header nodes");
  if (s != CDDT_OK) {
    drop();
    return s;
  }
  uint8_t* mark = (uint8_t*)mark_p;
  if (hipMemsetAsync(mark, 0, (size_t)std::max<int64_t>(m->capacity, 1), st) != hipSuccess) {
    drop();
    return fail(CDDT_EDEVICE, "prune: clearing the marks failed");
  }
  MapDev md = m->dev();
  md.bk = nullptr;  // the band view: absolute projections, search lines
  md.zp16 = 0;
  if (cells > 0) hipLaunchKernelGGL(k_prune_mark, dim3(blocks_of(cells, 256), m->half), dim3(256), 0, st, md, mark);
  hipLaunchKernelGGL(k_prune_keep, dim3(blocks_of(R, 4)), dim3(256), 0, st, (const int32_t*)m->d_hdr,
                     (const int32_t*)m->d_zeros, mark, R, (uint32_t*)cnt_p);
  if (hipGetLastError() != hipSuccess) {
    drop();
    return fail(CDDT_EDEVICE, "prune: mark or keep launch failed");
  }
  uint64_t used = 0, total_len = 0, max_len = 0;
  s = layout_bands(m, (uint32_t*)cnt_p, (int32_t*)hdr_p, true, &used, &total_len, &max_len, st);
  if (s == CDDT_OK) s = m->alloc.alloc(&zeros_p, (size_t)std::max<uint64_t>(used, 1) * 4, "pruned zero points");
  if (s != CDDT_OK) {
    drop();
    return s;
  }
  hipLaunchKernelGGL(k_prune_compact, dim3(blocks_of(R, 4)), dim3(256), 0, st, (const int32_t*)m->d_hdr,
                     (const int32_t*)m->d_zeros, (const uint8_t*)mark, R, (const int32_t*)hdr_p, (int32_t*)zeros_p);
  if (hipGetLastError() != hipSuccess) {
    drop();
    return fail(CDDT_EDEVICE, "prune: compaction launch failed");
  }
  s = finalize_bands((int32_t*)hdr_p, (int32_t*)zeros_p, R, st);  // blocks: the old structure is free after it
  if (s != CDDT_OK) {
    drop();
    return s;
  }
  free_structure(m);
  m->d_hdr = (int32_t*)hdr_p;
  m->d_zeros = (int32_t*)zeros_p;
  hdr_p = zeros_p = nullptr;
  m->capacity = (int64_t)used;
  m->spare_end = (int64_t)used;
  m->zero_points = (int64_t)total_len;
  m->max_row_len = (int64_t)max_len;
  drop();
  return CDDT_OK;
}

}  // namespace cddt
