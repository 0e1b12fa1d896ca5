// Incremental obstacle update on the GPU (Sec. IV-D, with the edge-map rule
// of Sec. IV-C applied to insertions as well as deletions).
//
// Ops are applied in chunks of at most kOpChunk, in order (a later chunk sees
// the result of an earlier one, so "last write wins" holds across chunks).
// Per chunk:
//   k_changed      op i is the last write to its cell within the chunk and
//                  changes the cell -> changed list {cell, value}
//   k_candidates   every in-map cell of the 3x3 block of a changed cell, owned
//                  by the lowest-index changed cell next to it (no duplicates),
//                  with its edge status on the old grid
//   k_apply        write the changed values into the grid
//   k_flips        candidates whose edge status differs on the new grid ->
//                  edits {cell, +1 insert / -1 remove}
//   k_records      per (edit, slice): one record per band the cell covers
//   k_group_count  per-band counters; the first record of a band registers it
//                  in the touched list
//   scan           offsets of each touched band's records
//   k_group_fill   records scattered into per-band groups
//   k_apply_bands  one wave per touched band: removes, then inserts, shifting
//                  keys inside the band's slack; the band's sample levels and
//                  header node are rewritten; a band without room raises the
//                  overflow flag and is left for the rebuild
// The host reads the flags once per chunk; an overflow re-lays the whole
// structure from the updated grid.
#include <algorithm>
#include <cstring>
#include <vector>

#include "band_layout.h"
#include "cddt_common.h"

namespace cddt {
namespace {

constexpr int kOpChunk = 4096;
constexpr int kThreads = 256;
constexpr int kScanThreads = 1024;
constexpr int kScanItems = 4;
constexpr int kScanTile = kScanThreads * kScanItems;

struct UpdCounters {
  uint32_t changed;
  uint32_t cand;
  uint32_t edits;
  uint32_t records;
  uint32_t touched;
  uint32_t overflow;
  uint32_t missing;   // a removal found no matching zero point (structure inconsistent)
  int32_t delta;      // change of the zero-point total when every record applies
};

__device__ __forceinline__ uint32_t pack_cell(int i, int j) { return (uint32_t)i | ((uint32_t)j << 16); }
__device__ __forceinline__ int cell_i(uint32_t p) { return (int)(p & 0xffffu); }
__device__ __forceinline__ int cell_j(uint32_t p) { return (int)(p >> 16); }

// Op i changes its cell when no later op writes the same cell and its value
// differs from the grid's.  The later ops are compared from LDS tiles.
constexpr int kTile = 1024;
__global__ void k_changed(const int32_t* __restrict__ xs, const int32_t* __restrict__ ys,
                          const uint8_t* __restrict__ vals, int32_t n, const uint8_t* __restrict__ occ, int w,
                          int2* __restrict__ changed, UpdCounters* ctr) {
  __shared__ uint32_t tile[kTile];
  const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  const bool live = i < n;
  const uint32_t key = live ? pack_cell(xs[i], ys[i]) : 0xffffffffu;
  bool later = false;
  for (int32_t t0 = blockIdx.x * blockDim.x; t0 < n; t0 += kTile) {  // ops before this block never matter
    __syncthreads();
    for (int32_t k = threadIdx.x; k < kTile; k += blockDim.x)
      tile[k] = t0 + k < n ? pack_cell(xs[t0 + k], ys[t0 + k]) : 0xfffffffeu;
    __syncthreads();
    const int32_t lim = min(kTile, n - t0);
    for (int32_t k = 0; k < lim; ++k) later |= (t0 + k > i) && tile[k] == key;
  }
  if (!live || later) return;  // a later op wins
  const int32_t x = xs[i], y = ys[i];
  const uint8_t v = vals[i] ? 1 : 0;
  const uint8_t cur = occ[(size_t)y * w + x] ? 1 : 0;
  if (v == cur) return;
  const uint32_t k = atomicAdd(&ctr->changed, 1u);
  changed[k] = make_int2((int32_t)pack_cell(x, y), v);
}

// Cell (i, j) next to changed cell k is a candidate unless an earlier changed
// cell is also next to it (the lowest-index changed neighbour owns it); the
// earlier changed cells are compared from LDS tiles.
__global__ void k_candidates(const int2* __restrict__ changed, const UpdCounters* ctr_in,
                             const uint8_t* __restrict__ occ, int w, int h, int full, int2* __restrict__ cand,
                             UpdCounters* ctr) {
  __shared__ uint32_t tile[kTile];
  const uint32_t nc = ctr_in->changed;
  const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  const bool live = t < nc * 9u;
  const uint32_t k = live ? t / 9u : 0u, o = live ? t - k * 9u : 0u;
  const uint32_t pk = live ? (uint32_t)changed[k].x : 0u;
  const int i = cell_i(pk) + (int)(o % 3u) - 1, j = cell_j(pk) + (int)(o / 3u) - 1;
  bool owned = false;
  const uint32_t k_max = (uint32_t)min((uint64_t)nc, ((uint64_t)blockIdx.x * blockDim.x + blockDim.x) / 9u + 1);
  for (uint32_t q0 = 0; q0 < k_max; q0 += kTile) {
    __syncthreads();
    for (uint32_t q = threadIdx.x; q < kTile; q += blockDim.x)
      tile[q] = q0 + q < nc ? (uint32_t)changed[q0 + q].x : 0u;
    __syncthreads();
    const uint32_t lim = min((uint32_t)kTile, k > q0 ? k - q0 : 0u);
    for (uint32_t q = 0; q < lim; ++q) {
      const uint32_t pq = tile[q];
      owned |= abs(cell_i(pq) - i) <= 1 && abs(cell_j(pq) - j) <= 1;
    }
  }
  if (!live || owned || i < 0 || j < 0 || i >= w || j >= h) return;
  const uint32_t slot = atomicAdd(&ctr->cand, 1u);
  cand[slot] = make_int2((int32_t)pack_cell(i, j), edge_cell(occ, w, h, i, j, full) ? 1 : 0);
}

__global__ void k_apply(const int2* __restrict__ changed, const UpdCounters* ctr, uint8_t* __restrict__ occ, int w) {
  const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= ctr->changed) return;
  const int2 c = changed[k];
  occ[(size_t)cell_j((uint32_t)c.x) * w + cell_i((uint32_t)c.x)] = (uint8_t)c.y;
}

__global__ void k_flips(const int2* __restrict__ cand, const UpdCounters* ctr_in, const uint8_t* __restrict__ occ,
                        int w, int h, int full, int2* __restrict__ edits, UpdCounters* ctr) {
  const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= ctr_in->cand) return;
  const int2 c = cand[k];
  const uint32_t p = (uint32_t)c.x;
  const int now = edge_cell(occ, w, h, cell_i(p), cell_j(p), full) ? 1 : 0;
  if (now == c.y) return;
  const uint32_t slot = atomicAdd(&ctr->edits, 1u);
  edits[slot] = make_int2(c.x, now ? 1 : -1);
}

// Records: row | remove-bit << 31, zero point, rank within the band.
struct Rec {
  uint32_t row;
  int32_t z;
};

__global__ void k_records(const SliceDev* __restrict__ slices, const int2* __restrict__ edits,
                          const UpdCounters* ctr_in, Rec* __restrict__ rec, UpdCounters* ctr) {
  const uint32_t e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ctr_in->edits) return;
  const SliceDev sl = slices[blockIdx.y];
  const int2 ed = edits[e];
  const uint32_t p = (uint32_t)ed.x;
  const int64_t i2 = 2 * (int64_t)cell_i(p) + 1, j2 = 2 * (int64_t)cell_j(p) + 1;
  const int64_t yc = j2 * sl.c - i2 * sl.s;
  const int64_t hs = (int64_t)abs(sl.c) + (int64_t)abs(sl.s);
  const int32_t lo = (int32_t)((yc - hs) >> 31), hi = (int32_t)((yc + hs - 1) >> 31);
  const int32_t z = (int32_t)((i2 * sl.c + j2 * sl.s) >> 15);
  const uint32_t rm = ed.y < 0 ? 0x80000000u : 0u;
  const uint32_t base = atomicAdd(&ctr->records, (uint32_t)(hi - lo + 1));
  // zero-point total change if every record applies (otherwise the structure is rebuilt)
  atomicAdd(&ctr->delta, rm ? -(hi - lo + 1) : (hi - lo + 1));
  for (int32_t r = lo; r <= hi; ++r) {
    Rec q;
    q.row = (uint32_t)(sl.row_off + r) | rm;
    q.z = z;
    rec[base + (uint32_t)(r - lo)] = q;
  }
}

__global__ void k_group_count(const Rec* __restrict__ rec, const UpdCounters* ctr_in, uint32_t* __restrict__ rowcnt,
                              uint32_t* __restrict__ row_slot, uint32_t* __restrict__ touched,
                              uint32_t* __restrict__ local, UpdCounters* ctr) {
  const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= ctr_in->records) return;
  const uint32_t row = rec[k].row & 0x7fffffffu;
  const uint32_t l = atomicAdd(&rowcnt[row], 1u);
  local[k] = l;
  if (l == 0) {
    const uint32_t s = atomicAdd(&ctr->touched, 1u);
    row_slot[row] = s;
    touched[s] = row;
  }
}

__global__ void k_touched_counts(const uint32_t* __restrict__ touched, const UpdCounters* ctr,
                                 const uint32_t* __restrict__ rowcnt, uint32_t* __restrict__ tcount) {
  const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= ctr->touched) return;
  tcount[k] = rowcnt[touched[k]];
}

// --- exclusive scan of tcount[0, *n) in place (n read on the device) ---------
__device__ uint32_t block_scan_incl(uint32_t v, uint32_t* wt) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    uint32_t t = __shfl_up(v, o);
    if (lane >= o) v += t;
  }
  if (lane == 63) wt[wid] = v;
  __syncthreads();
  if (wid == 0) {
    uint32_t t = lane < nw ? wt[lane] : 0u;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      uint32_t u = __shfl_up(t, o);
      if (lane >= o) t += u;
    }
    if (lane < nw) wt[lane] = t;
  }
  __syncthreads();
  if (wid > 0) v += wt[wid - 1];
  __syncthreads();
  return v;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_sum(const uint32_t* __restrict__ a, const UpdCounters* ctr,
                                                           uint32_t* __restrict__ tiles) {
  __shared__ uint32_t wt[kScanThreads / 64];
  const uint32_t n = ctr->touched;
  const uint32_t base = blockIdx.x * kScanTile + threadIdx.x * kScanItems;
  uint32_t s = 0;
#pragma unroll
  for (int q = 0; q < kScanItems; ++q)
    if (base + q < n) s += a[base + q];
  const uint32_t inc = block_scan_incl(s, wt);
  if (threadIdx.x == blockDim.x - 1) tiles[blockIdx.x] = inc;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_tiles(uint32_t* __restrict__ tiles, uint32_t ntiles) {
  __shared__ uint32_t wt[kScanThreads / 64];
  __shared__ uint32_t carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (uint32_t b = 0; b < ntiles; b += kScanThreads) {
    const uint32_t t = b + threadIdx.x;
    const uint32_t v = t < ntiles ? tiles[t] : 0u;
    const uint32_t inc = block_scan_incl(v, wt);
    const uint32_t c = carry;
    if (t < ntiles) tiles[t] = c + inc - v;
    __syncthreads();
    if (threadIdx.x == blockDim.x - 1) carry = c + inc;
    __syncthreads();
  }
}

__global__ __launch_bounds__(kScanThreads) void k_scan_apply(uint32_t* __restrict__ a, const UpdCounters* ctr,
                                                             const uint32_t* __restrict__ tiles) {
  __shared__ uint32_t wt[kScanThreads / 64];
  const uint32_t n = ctr->touched;
  const uint32_t base = blockIdx.x * kScanTile + threadIdx.x * kScanItems;
  uint32_t v[kScanItems];
  uint32_t s = 0;
#pragma unroll
  for (int q = 0; q < kScanItems; ++q) {
    v[q] = base + q < n ? a[base + q] : 0u;
    s += v[q];
  }
  uint32_t off = block_scan_incl(s, wt) - s + tiles[blockIdx.x];
#pragma unroll
  for (int q = 0; q < kScanItems; ++q)
    if (base + q < n) {
      a[base + q] = off;
      off += v[q];
    }
}

__global__ void k_group_fill(const Rec* __restrict__ rec, const UpdCounters* ctr,
                             const uint32_t* __restrict__ row_slot, const uint32_t* __restrict__ toff,
                             const uint32_t* __restrict__ local, Rec* __restrict__ grp) {
  const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= ctr->records) return;
  const Rec r = rec[k];
  grp[toff[row_slot[r.row & 0x7fffffffu]] + local[k]] = r;
}

// Shift keys[a, b) one slot right (towards b), last chunk first.
__device__ void shift_right(int32_t* keys, int32_t a, int32_t b) {
  const int lane = threadIdx.x & 63;
  for (int32_t e = b; e > a; e -= 64) {
    const int32_t s = max(a, e - 64);
    const int32_t i = s + lane;
    int32_t v = 0;
    if (i < e) v = keys[i];
    __threadfence_block();
    if (i < e) keys[i + 1] = v;
    __threadfence_block();
  }
}

// Shift keys[a, b) one slot left (towards a), first chunk first.
__device__ void shift_left(int32_t* keys, int32_t a, int32_t b) {
  const int lane = threadIdx.x & 63;
  for (int32_t s = a; s < b; s += 64) {
    const int32_t i = s + lane;
    int32_t v = 0;
    if (i < b) v = keys[i];
    __threadfence_block();
    if (i < b) keys[i - 1] = v;
    __threadfence_block();
  }
}

// Position in keys[0, len) of the first key >= z (lower) or > z (upper); every lane computes it.
__device__ int32_t bound(const int32_t* keys, int32_t len, int32_t z, bool upper) {
  int32_t lo = 0, cnt = len;
  while (cnt > 0) {
    const int32_t half = cnt >> 1;
    const int32_t v = keys[lo + half];
    if (upper ? v <= z : v < z) {
      lo += half + 1;
      cnt -= half + 1;
    } else {
      cnt = half;
    }
  }
  return lo;
}

// A band whose edits exceed its capacity moves to a new region taken from the
// spare area at the end of the zero-point array (1.5x its new length plus the
// usual slack); only when the spare area is used up is the overflow flagged
// (the host then re-lays the whole structure).
__global__ void k_apply_bands(int32_t* __restrict__ hdr, int32_t* __restrict__ zeros,
                              const uint32_t* __restrict__ touched, const uint32_t* __restrict__ toff,
                              uint32_t* __restrict__ rowcnt, const Rec* __restrict__ grp, UpdCounters* ctr,
                              unsigned long long* __restrict__ spare_cursor, uint64_t spare_end) {
  const uint32_t t = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (t >= ctr->touched) return;  // uniform per wave
  const int lane = threadIdx.x & 63;
  const uint32_t row = touched[t];
  const uint32_t cnt = rowcnt[row];
  const Rec* g = grp + toff[t];
  int32_t* node = hdr + (int64_t)row * kNodeInts;
  uint32_t start = (uint32_t)node[0];
  int32_t len = node[1];
  int32_t cap = node[2];
  int32_t ins = 0, rem = 0;
  for (uint32_t k = 0; k < cnt; ++k) (g[k].row & 0x80000000u) ? ++rem : ++ins;
  if (len - rem + ins > cap) {
    const uint32_t need = (uint32_t)(len + ins);
    const uint32_t ncap = key_capacity(need + (need >> 1), false);
    const uint64_t slots = region_slots(ncap);
    unsigned long long pos = 0;
    if (lane == 0 && spare_cursor) pos = atomicAdd(spare_cursor, (unsigned long long)slots);
    pos = __shfl(pos, 0);
    if (spare_cursor == nullptr || pos + slots > spare_end) {
      if (lane == 0) {
        atomicOr(&ctr->overflow, 1u);
        rowcnt[row] = 0;
      }
      return;
    }
    int32_t* nk = zeros + pos;
    for (int32_t k = lane; k < len; k += 64) nk[k] = zeros[start + k];
    __threadfence_block();
    if (lane == 0) {
      node[0] = (int32_t)pos;
      node[2] = (int32_t)ncap;
    }
    __threadfence_block();
    start = (uint32_t)pos;
    cap = (int32_t)ncap;
  }
  int32_t* keys = zeros + start;
  for (uint32_t k = 0; k < cnt; ++k) {  // removals first: every one must find its key
    if (!(g[k].row & 0x80000000u)) continue;
    const int32_t z = g[k].z;
    const int32_t pos = bound(keys, len, z, false);
    if (pos >= len || keys[pos] != z) {
      if (lane == 0) atomicOr(&ctr->missing, 1u);
      continue;
    }
    shift_left(keys, pos + 1, len);
    --len;
  }
  for (uint32_t k = 0; k < cnt; ++k) {
    if (g[k].row & 0x80000000u) continue;
    if (len >= cap) {  // only reachable if a removal above found no key
      if (lane == 0) atomicOr(&ctr->overflow, 1u);
      break;
    }
    const int32_t z = g[k].z;
    const int32_t pos = bound(keys, len, z, true);
    shift_right(keys, pos, len);
    if (lane == 0) keys[pos] = z;
    __threadfence_block();
    ++len;
  }
  if (lane == 0) {
    node[1] = len;
    rowcnt[row] = 0;
  }
  __threadfence_block();
  finalize_band(node, zeros);
}

unsigned blocks_for(uint64_t n, int threads) {
  uint64_t b = (n + threads - 1) / threads;
  return (unsigned)(b < 1 ? 1 : b);
}

}  // namespace

cddt_status apply_update(cddt_map_s* m, const int32_t* xs_h, const int32_t* ys_h, const uint8_t* vals_h,
                         int64_t n_ops, hipStream_t st) {
  const int full = (m->flags & CDDT_FLAG_FULL_MAP) ? 1 : 0;
  const int64_t R = m->rows;
  // band counters stay zero between updates (every touched band resets its own)
  CDDT_TRY(ensure(m->alloc, m->upd_rowcnt, (size_t)R * 4, "update band counters"));
  CDDT_TRY(ensure(m->alloc, m->upd_slot, (size_t)R * 4, "update band slots"));
  if (!m->upd_rowcnt_clear) {
    CDDT_HIP(hipMemsetAsync(m->upd_rowcnt.ptr, 0, m->upd_rowcnt.bytes, st));
    m->upd_rowcnt_clear = true;
  }
  CDDT_TRY(ensure(m->alloc, m->upd_misc, sizeof(UpdCounters), "update counters"));
  CDDT_TRY(ensure(m->alloc, m->upd_ops, (size_t)kOpChunk * 9, "update ops"));
  CDDT_TRY(ensure(m->alloc, m->upd_changed, (size_t)kOpChunk * sizeof(int2), "changed cells"));
  CDDT_TRY(ensure(m->alloc, m->upd_cand, (size_t)kOpChunk * 9 * sizeof(int2), "candidate cells"));
  CDDT_TRY(ensure(m->alloc, m->upd_edits, (size_t)kOpChunk * 9 * sizeof(int2), "edge flips"));
  UpdCounters* ctr = (UpdCounters*)m->upd_misc.ptr;
  std::vector<uint8_t> packed((size_t)kOpChunk * 9);
  // A pruned (PCDDT) structure depends on every free cell, not only on edge
  // flips: its grid takes the ops and the structure is rebuilt and pruned.
  const bool pruned = (m->flags & CDDT_FLAG_PRUNE) != 0;
  bool grid_changed = false;

  for (int64_t o0 = 0; o0 < n_ops; o0 += kOpChunk) {
    const int32_t n = (int32_t)std::min<int64_t>(kOpChunk, n_ops - o0);
    int32_t* d_xs = (int32_t*)m->upd_ops.ptr;
    int32_t* d_ys = d_xs + kOpChunk;
    uint8_t* d_vs = (uint8_t*)(d_ys + kOpChunk);
    std::memcpy(packed.data(), xs_h + o0, 4 * (size_t)n);
    std::memcpy(packed.data() + 4 * (size_t)kOpChunk, ys_h + o0, 4 * (size_t)n);
    std::memcpy(packed.data() + 8 * (size_t)kOpChunk, vals_h + o0, (size_t)n);
    CDDT_HIP(hipMemcpyAsync(d_xs, packed.data(), packed.size(), hipMemcpyHostToDevice, st));
    CDDT_HIP(hipMemsetAsync(ctr, 0, sizeof(UpdCounters), st));
    const int2* changed = (const int2*)m->upd_changed.ptr;
    const int2* cand = (const int2*)m->upd_cand.ptr;
    const int2* edits = (const int2*)m->upd_edits.ptr;
    hipLaunchKernelGGL(k_changed, dim3(blocks_for(n, kThreads)), dim3(kThreads), 0, st, d_xs, d_ys, d_vs, n,
                       m->d_occ, m->w, (int2*)changed, ctr);
    hipLaunchKernelGGL(k_candidates, dim3(blocks_for((uint64_t)n * 9, kThreads)), dim3(kThreads), 0, st, changed,
                       (const UpdCounters*)ctr, m->d_occ, m->w, m->h, full, (int2*)cand, ctr);
    hipLaunchKernelGGL(k_apply, dim3(blocks_for(n, kThreads)), dim3(kThreads), 0, st, changed,
                       (const UpdCounters*)ctr, m->d_occ, m->w);
    hipLaunchKernelGGL(k_flips, dim3(blocks_for((uint64_t)n * 9, kThreads)), dim3(kThreads), 0, st, cand,
                       (const UpdCounters*)ctr, m->d_occ, m->w, m->h, full, (int2*)edits, ctr);
    CDDT_HIP(hipGetLastError());
    UpdCounters hc{};
    CDDT_HIP(hipMemcpyAsync(&hc, ctr, sizeof(hc), hipMemcpyDeviceToHost, st));
    CDDT_HIP(hipStreamSynchronize(st));
    if (pruned) {
      grid_changed = grid_changed || hc.changed > 0;
      continue;
    }
    if (hc.edits == 0) continue;

    // band records, grouped per band
    const uint64_t max_rec = (uint64_t)hc.edits * m->half * 3;
    CDDT_TRY(ensure(m->alloc, m->upd_rec, max_rec * (sizeof(Rec) + 4), "update records"));
    CDDT_TRY(ensure(m->alloc, m->upd_grp, max_rec * sizeof(Rec), "grouped records"));
    CDDT_TRY(ensure(m->alloc, m->upd_touched, max_rec * 8, "touched bands"));
    const uint64_t ntiles = (max_rec + kScanTile - 1) / kScanTile;
    CDDT_TRY(ensure(m->alloc, m->upd_tiles, ntiles * 4, "update scan tiles"));
    Rec* rec = (Rec*)m->upd_rec.ptr;
    uint32_t* local = (uint32_t*)(rec + max_rec);
    uint32_t* touched = (uint32_t*)m->upd_touched.ptr;
    uint32_t* toff = touched + max_rec;
    uint32_t* rowcnt = (uint32_t*)m->upd_rowcnt.ptr;
    uint32_t* slot = (uint32_t*)m->upd_slot.ptr;
    hipLaunchKernelGGL(k_records, dim3(blocks_for(hc.edits, kThreads), m->half), dim3(kThreads), 0, st,
                       m->d_slices, edits, (const UpdCounters*)ctr, rec, ctr);
    hipLaunchKernelGGL(k_group_count, dim3(blocks_for(max_rec, kThreads)), dim3(kThreads), 0, st, rec,
                       (const UpdCounters*)ctr, rowcnt, slot, touched, local, ctr);
    hipLaunchKernelGGL(k_touched_counts, dim3(blocks_for(max_rec, kThreads)), dim3(kThreads), 0, st, touched,
                       (const UpdCounters*)ctr, rowcnt, toff);
    hipLaunchKernelGGL(k_scan_sum, dim3((unsigned)ntiles), dim3(kScanThreads), 0, st, toff, (const UpdCounters*)ctr,
                       (uint32_t*)m->upd_tiles.ptr);
    hipLaunchKernelGGL(k_scan_tiles, dim3(1), dim3(kScanThreads), 0, st, (uint32_t*)m->upd_tiles.ptr,
                       (uint32_t)ntiles);
    hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)ntiles), dim3(kScanThreads), 0, st, toff,
                       (const UpdCounters*)ctr, (const uint32_t*)m->upd_tiles.ptr);
    hipLaunchKernelGGL(k_group_fill, dim3(blocks_for(max_rec, kThreads)), dim3(kThreads), 0, st, rec,
                       (const UpdCounters*)ctr, slot, toff, local, (Rec*)m->upd_grp.ptr);
    hipLaunchKernelGGL(k_apply_bands, dim3(blocks_for(max_rec, 4)), dim3(kThreads), 0, st, m->d_hdr, m->d_zeros,
                       touched, toff, rowcnt, (const Rec*)m->upd_grp.ptr, ctr, m->d_spare,
                       (uint64_t)m->spare_end);
    CDDT_HIP(hipGetLastError());
    CDDT_HIP(hipMemcpyAsync(&hc, ctr, sizeof(hc), hipMemcpyDeviceToHost, st));
    CDDT_HIP(hipStreamSynchronize(st));
    if (hc.missing) {  // never expected: restore a consistent structure, then report
      CDDT_TRY(build_structure(m, st));
      ++m->rebuilds;
      return fail(CDDT_EINTERNAL, "cddt_update: a removed zero point was not in its band (structure rebuilt)");
    }
    if (hc.overflow) {  // some band ran out of slack: re-lay the structure from the new grid
      CDDT_TRY(build_structure(m, st));
      ++m->rebuilds;
    } else {
      m->zero_points += hc.delta;  // exact: every applied band reported its length change
      m->stats_stale = true;       // the longest band is recomputed when asked for
      // the buckets the edits can change, in the edited bands
      CDDT_TRY(fill_buckets(m, touched, (int64_t)hc.touched, st, toff, (const int2*)m->upd_grp.ptr, hc.records));
    }
  }
  if (grid_changed) {
    CDDT_TRY(build_structure(m, st));
    ++m->rebuilds;
  }
  return CDDT_OK;
}

}  // namespace cddt
