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
//   k_edit_bands   one wave per touched band: removes, then inserts, in an LDS
//                  copy of the band (long bands: in place); the band's keys,
//                  sample levels and header node are rewritten, moving to the
//                  spare area when it outgrows its slack, and so are the
//                  bucket lines the edits can change; a band without room
//                  raises the overflow flag and is left for the rebuild
// The host reads the flags once per chunk; an overflow re-lays the whole
// structure from the updated grid.
#include <algorithm>
#include <cstring>
#include <vector>

#include "band_layout.h"
#include "bucket_lines.h"
#include "cddt_common.h"

namespace cddt {
namespace {

constexpr int kOpChunk = 4096;
constexpr int kThreads = 256;
constexpr int kScanThreads = 1024;
constexpr int kScanItems = 4;
constexpr int kScanTile = kScanThreads * kScanItems;
constexpr unsigned kEditBlocks = 16384;   // band-edit launch: waves take touched bands in turn
constexpr unsigned kStrideBlocks = 2048;  // record-sized launches: threads take records in turn
// A chunk's device staging: xs, ys (int32) and values (uint8), kOpChunk each,
// then the counters.
constexpr size_t kCounterOffset = (size_t)kOpChunk * 9;
// Bytes per record of the record, grouping and touched-band arrays.
constexpr uint64_t kRecordBytes = 8 + 4 + 2 + 8 + 12;
// Record arrays up to this size are allocated for the chunk's worst case, so
// that the host need not wait for the count of edge flips.
constexpr uint64_t kNoWaitBytes = 256ull << 20;

struct UpdCounters {
  uint32_t changed;
  uint32_t cand;
  uint32_t edits;
  uint32_t records;
  uint32_t touched;
  uint32_t overflow;
  uint32_t missing;   // a removal found no matching zero point (structure inconsistent)
  int32_t delta;      // change of the zero-point total when every record applies
  int32_t bk_over;    // change of the overflowing-bucket count
};
constexpr size_t kStageBytes = kCounterOffset + sizeof(UpdCounters);

__device__ __forceinline__ uint32_t pack_cell(int i, int j) { return (uint32_t)i | ((uint32_t)j << 16); }
__device__ __forceinline__ int cell_i(uint32_t p) { return (int)(p & 0xffffu); }
__device__ __forceinline__ int cell_j(uint32_t p) { return (int)(p >> 16); }

// Inclusive sum over the block of every thread's v (blockDim.x a multiple of 64).
__device__ __forceinline__ uint32_t block_scan_incl(uint32_t v, uint32_t* wt) {
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


// Cell tables in LDS: open addressing with linear probing, key = packed cell,
// value = the largest op or changed-cell index stored for it.  The table has
// twice as many slots as a chunk has ops, so a probe always ends.  Every block
// builds the table of the whole chunk and then answers for its own items.
constexpr int kHashLog2 = 13;
constexpr int kHashSlots = 1 << kHashLog2;
static_assert(kHashSlots >= 2 * kOpChunk, "cell table load factor at most 1/2");
constexpr uint32_t kEmptyCell = 0xffffffffu;  // no packed cell of a map (cells < 16384 a side)

__device__ __forceinline__ uint32_t cell_slot(uint32_t key) { return (key * 2654435761u) >> (32 - kHashLog2); }

__device__ __forceinline__ void table_clear(uint32_t* hk, int32_t* hv) {
  for (int s = threadIdx.x; s < kHashSlots; s += blockDim.x) {
    hk[s] = kEmptyCell;
    hv[s] = -1;
  }
}

__device__ __forceinline__ void table_put_max(uint32_t* hk, int32_t* hv, uint32_t key, int32_t v) {
  for (uint32_t h = cell_slot(key);; h = (h + 1) & (kHashSlots - 1)) {
    const uint32_t prev = atomicCAS(&hk[h], kEmptyCell, key);
    if (prev == kEmptyCell || prev == key) {
      atomicMax(&hv[h], v);
      return;
    }
  }
}

// The value stored for key, -1 when absent.
__device__ __forceinline__ int32_t table_get(const uint32_t* hk, const int32_t* hv, uint32_t key) {
  for (uint32_t h = cell_slot(key);; h = (h + 1) & (kHashSlots - 1)) {
    const uint32_t k = hk[h];
    if (k == key) return hv[h];
    if (k == kEmptyCell) return -1;
  }
}

// Op i changes its cell when it is the chunk's last op on that cell and its
// value differs from the grid's.
__global__ __launch_bounds__(kThreads) void k_changed(const int32_t* __restrict__ xs, const int32_t* __restrict__ ys,
                                                      const uint8_t* __restrict__ vals, int32_t n,
                                                      const uint8_t* __restrict__ occ, int w,
                                                      int2* __restrict__ changed, UpdCounters* ctr) {
  __shared__ uint32_t hk[kHashSlots];
  __shared__ int32_t hv[kHashSlots];
  table_clear(hk, hv);
  __syncthreads();
  for (int32_t k = threadIdx.x; k < n; k += blockDim.x) table_put_max(hk, hv, pack_cell(xs[k], ys[k]), k);
  __syncthreads();
  const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int32_t x = xs[i], y = ys[i];
  if (table_get(hk, hv, pack_cell(x, y)) != i) return;  // a later op wins
  const uint8_t v = vals[i] ? 1 : 0;
  const uint8_t cur = occ[(size_t)y * w + x] ? 1 : 0;
  if (v == cur) return;
  const uint32_t k = atomicAdd(&ctr->changed, 1u);
  changed[k] = make_int2((int32_t)pack_cell(x, y), v);
}

// Cell (i, j) next to changed cell k is a candidate unless a changed cell
// with a lower index is also next to it (the lowest-index changed neighbour
// owns it): the changed cells (each cell at most once) go into the table with
// their indices, and the candidate looks up its 3x3 block.
__global__ __launch_bounds__(kThreads) void k_candidates(const int2* __restrict__ changed,
                                                         const UpdCounters* ctr_in, const uint8_t* __restrict__ occ,
                                                         int w, int h, int full, int2* __restrict__ cand,
                                                         UpdCounters* ctr) {
  __shared__ uint32_t hk[kHashSlots];
  __shared__ int32_t hv[kHashSlots];
  const uint32_t nc = ctr_in->changed;
  table_clear(hk, hv);
  __syncthreads();
  for (uint32_t k = threadIdx.x; k < nc; k += blockDim.x) table_put_max(hk, hv, (uint32_t)changed[k].x, (int32_t)k);
  __syncthreads();
  const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nc * 9u) return;
  const uint32_t k = t / 9u, o = t - k * 9u;
  const uint32_t pk = (uint32_t)changed[k].x;
  const int i = cell_i(pk) + (int)(o % 3u) - 1, j = cell_j(pk) + (int)(o / 3u) - 1;
  if (i < 0 || j < 0 || i >= w || j >= h) return;
  for (int b = max(j - 1, 0); b <= min(j + 1, h - 1); ++b)
    for (int a = max(i - 1, 0); a <= min(i + 1, w - 1); ++a) {
      const int32_t q = table_get(hk, hv, pack_cell(a, b));
      if (q >= 0 && (uint32_t)q < k) return;
    }
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

// One thread per (edit, slice): one record per band the cell covers.  The
// block's records take one range of the record array (one atomic per block).
__global__ __launch_bounds__(kThreads) void k_records(const SliceDev* __restrict__ slices,
                                                      const int2* __restrict__ edits, const UpdCounters* ctr_in,
                                                      Rec* __restrict__ rec, uint16_t* __restrict__ rslice,
                                                      UpdCounters* ctr) {
  __shared__ uint32_t wt[kThreads / 64];
  __shared__ uint32_t base;
  const uint32_t e = blockIdx.x * blockDim.x + threadIdx.x;
  const bool live = e < ctr_in->edits;
  const SliceDev sl = slices[blockIdx.y];
  int32_t lo = 0, hi = -1, z = 0;
  uint32_t rm = 0;
  if (live) {
    const int2 ed = edits[e];
    const uint32_t p = (uint32_t)ed.x;
    const int64_t i2 = 2 * (int64_t)cell_i(p) + 1, j2 = 2 * (int64_t)cell_j(p) + 1;
    const int64_t yc = j2 * sl.c - i2 * sl.s;
    const int64_t hs = (int64_t)abs(sl.c) + (int64_t)abs(sl.s);
    lo = (int32_t)((yc - hs) >> 31);
    hi = (int32_t)((yc + hs - 1) >> 31);
    z = (int32_t)((i2 * sl.c + j2 * sl.s) >> 15);
    rm = ed.y < 0 ? 0x80000000u : 0u;
  }
  const uint32_t cnt = (uint32_t)(hi - lo + 1);
  const uint32_t incl = block_scan_incl(cnt, wt);
  // zero-point total change if every record applies (otherwise the structure is rebuilt)
  const uint32_t n_rm = block_scan_incl(rm ? cnt : 0u, wt);
  if (threadIdx.x == blockDim.x - 1 && incl > 0) {
    base = atomicAdd(&ctr->records, incl);
    atomicAdd(&ctr->delta, (int32_t)incl - 2 * (int32_t)n_rm);
  }
  __syncthreads();
  const uint32_t at = base + incl - cnt;
  for (int32_t r = lo; r <= hi; ++r) {
    Rec q;
    q.row = (uint32_t)(sl.row_off + r) | rm;
    q.z = z;
    rec[at + (uint32_t)(r - lo)] = q;
    rslice[at + (uint32_t)(r - lo)] = (uint16_t)blockIdx.y;
  }
}

// The first record of a band registers it: touched[s] = band, tzlo[s] = the
// lowest zero point of its slice (the origin of its bucket index).
__global__ void k_group_count(const Rec* __restrict__ rec, const uint16_t* __restrict__ rslice,
                              const SliceDev* __restrict__ slices, const UpdCounters* ctr_in,
                              uint32_t* __restrict__ rowcnt, uint32_t* __restrict__ row_slot,
                              uint32_t* __restrict__ touched, int32_t* __restrict__ tzlo,
                              uint32_t* __restrict__ local, UpdCounters* ctr) {
  const uint32_t n = ctr_in->records;
  for (uint32_t k = blockIdx.x * blockDim.x + threadIdx.x; k < n; k += gridDim.x * blockDim.x) {
    const uint32_t row = rec[k].row & 0x7fffffffu;
    const uint32_t l = atomicAdd(&rowcnt[row], 1u);
    local[k] = l;
    if (l == 0) {
      const uint32_t s = atomicAdd(&ctr->touched, 1u);
      row_slot[row] = s;
      touched[s] = row;
      tzlo[s] = slices[rslice[k]].zlo;
    }
  }
}

__global__ void k_touched_counts(const uint32_t* __restrict__ touched, const UpdCounters* ctr,
                                 const uint32_t* __restrict__ rowcnt, uint32_t* __restrict__ tcount) {
  const uint32_t n = ctr->touched;
  for (uint32_t k = blockIdx.x * blockDim.x + threadIdx.x; k < n; k += gridDim.x * blockDim.x)
    tcount[k] = rowcnt[touched[k]];
}

// --- exclusive scan of tcount[0, *n) in place (n read on the device) ---------
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
  const uint32_t n = ctr->records;
  for (uint32_t k = blockIdx.x * blockDim.x + threadIdx.x; k < n; k += gridDim.x * blockDim.x) {
    const Rec r = rec[k];
    grp[toff[row_slot[r.row & 0x7fffffffu]] + local[k]] = r;
  }
}

// Orders the keys the lanes of a wave move: in LDS a wave's operations are in
// order (a compiler fence suffices); in global memory the wave waits.
template <bool Lds>
__device__ __forceinline__ void keys_fence() {
  if constexpr (Lds)
    wave_fence();
  else
    __threadfence_block();
}

// Shift keys[a, b) one slot right (towards b), last chunk first.
template <bool Lds>
__device__ __forceinline__ void shift_right(int32_t* keys, int32_t a, int32_t b) {
  const int lane = threadIdx.x & 63;
  for (int32_t e = b; e > a; e -= 64) {
    const int32_t s = max(a, e - 64);
    const int32_t i = s + lane;
    int32_t v = 0;
    if (i < e) v = keys[i];
    keys_fence<Lds>();
    if (i < e) keys[i + 1] = v;
    keys_fence<Lds>();
  }
}

// Shift keys[a, b) one slot left (towards a), first chunk first.
template <bool Lds>
__device__ __forceinline__ void shift_left(int32_t* keys, int32_t a, int32_t b) {
  const int lane = threadIdx.x & 63;
  for (int32_t s = a; s < b; s += 64) {
    const int32_t i = s + lane;
    int32_t v = 0;
    if (i < b) v = keys[i];
    keys_fence<Lds>();
    if (i < b) keys[i - 1] = v;
    keys_fence<Lds>();
  }
}

// Position in keys[0, len) of the first key >= z (lower) or > z (upper), for
// keys in LDS and len <= 1024 = 64 x 16: lane l compares key 16 l, which
// finds the group of 16 that holds the position; lanes 0..15 then compare the
// group's keys.  Two LDS reads and two ballots; the same on every lane.
__device__ __forceinline__ int32_t bound_lds(const int32_t* keys, int32_t len, int32_t z, bool upper) {
  const int lane = threadIdx.x & 63;
  auto before = [&](int32_t k) {  // key k lies before the position
    const int32_t v = keys[k];
    return upper ? v <= z : v < z;
  };
  const int32_t g = __popcll(__ballot(16 * lane < len && before(16 * lane)));  // groups that start before it
  if (g == 0) return 0;
  const int32_t base = 16 * (g - 1);
  return base + __popcll(__ballot(lane < 16 && base + lane < len && before(base + lane)));
}

// Position in keys[0, len) of the first key >= z (lower) or > z (upper); every lane computes it.
__device__ __forceinline__ int32_t bound(const int32_t* keys, int32_t len, int32_t z, bool upper) {
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

// The bucket index of the map being edited (lines null: none).
struct EditBuckets {
  int32_t* lines;
  int32_t shift, nbk, zp16;
};

// Bands of up to kStageKeys keys, before and after the edit, with at most 64
// records are edited in an LDS copy.  Per wave: the copy, first[] after and
// (for bands edited in place) before the edit, one mark byte per bucket.
constexpr int kStageKeys = 1024;
__host__ __device__ constexpr int32_t edit_wave_words(int32_t nbk) {  // a multiple of 4 (16-byte groups)
  return (kStageKeys + (nbk > 0 ? 2 * (nbk + 1) + (nbk + 3) / 4 : 0) + 3) & ~3;
}
static_assert(kStageKeys == 4 * 4 * 64, "a staged band is four 16-byte groups per lane");

// One wave per touched band: its records are applied, removals first (each
// must find its key), then inserts after any equal keys.  A band whose new
// length exceeds its capacity moves to a new region taken from the spare area
// at the end of the zero-point array (1.5x its length plus inserts, plus the
// usual slack); only when the spare area is used up is the overflow flagged
// (the host then re-lays the whole structure).  Then the band's bucket lines
// that the edits can change are rewritten (bucket_lines.h); the old lines'
// overflow count follows from the records (LDS copy) or from first[] before
// the edit (in place).
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(6, 8))) void k_edit_bands(int32_t* __restrict__ hdr, int32_t* __restrict__ zeros,
                                                    const uint32_t* __restrict__ touched,
                                                    const int32_t* __restrict__ tzlo,
                                                    const uint32_t* __restrict__ toff, uint32_t* __restrict__ rowcnt,
                                                    const Rec* __restrict__ grp, UpdCounters* ctr,
                                                    unsigned long long* __restrict__ spare_cursor, uint64_t spare_end,
                                                    EditBuckets eb) {
  extern __shared__ int4 edit_lds[];
  const int lane = threadIdx.x & 63;
  const uint32_t wpb = blockDim.x >> 6;
  int32_t* stage = reinterpret_cast<int32_t*>(edit_lds) + (threadIdx.x >> 6) * edit_wave_words(eb.nbk);
  int32_t* first = stage + kStageKeys;
  int32_t* first_old = first + eb.nbk + 1;
  uint8_t* mark = reinterpret_cast<uint8_t*>(first_old + eb.nbk + 1);
  const uint32_t n_touched = ctr->touched, n_records = ctr->records;
  int over_n = 0;
  const uint32_t stride = gridDim.x * wpb;
  // Loads run ahead of the band being edited: a band's keys are loaded
  // together with the next band's header and records and the band after
  // that's number, record range and slice origin, so that one wait covers
  // all three.
  uint32_t t = blockIdx.x * wpb + (threadIdx.x >> 6);
  uint32_t row_a = 0, o0_a = 0, cnt_a = 0, row_b = 0, o0_b = 0, cnt_b = 0;
  int32_t zlo_a = 0, zlo_b = 0, hv_a = 0;
  Rec r_a{0u, 0};
  auto indices = [&](uint32_t u, uint32_t& row_, uint32_t& o0_, uint32_t& cnt_, int32_t& zlo_) {
    if (u < n_touched) {
      row_ = touched[u];
      o0_ = toff[u];
      cnt_ = (u + 1 < n_touched ? toff[u + 1] : n_records) - o0_;
      zlo_ = eb.lines ? tzlo[u] : 0;
    }
  };
  auto header = [&](uint32_t u) {  // band u's header words and records (lane k: record k < 64)
    if (u < n_touched) {
      hv_a = lane < kHeaderWords ? hdr[(int64_t)row_a * kNodeInts + lane] : 0;
      r_a = lane < (int)cnt_a ? grp[o0_a + lane] : Rec{0u, 0};
    }
  };
  indices(t, row_a, o0_a, cnt_a, zlo_a);
  header(t);
  indices(t + stride, row_b, o0_b, cnt_b, zlo_b);
  for (; t < n_touched; t += stride) {
    const uint32_t row = row_a, o0 = o0_a, cnt = cnt_a;
    const int32_t zlo = zlo_a, hv = hv_a;
    const Rec r = r_a;
    row_a = row_b, o0_a = o0_b, cnt_a = cnt_b, zlo_a = zlo_b;
    header(t + stride);
    indices(t + 2 * stride, row_b, o0_b, cnt_b, zlo_b);
    const Rec* g = grp + o0;
    int32_t* node = hdr + (int64_t)row * kNodeInts;
    const uint32_t old_start = (uint32_t)__builtin_amdgcn_readlane(hv, 0);
    const int32_t len = __builtin_amdgcn_readlane(hv, 1);
    uint32_t cap = (uint32_t)__builtin_amdgcn_readlane(hv, 2);
    const bool removal = (r.row & 0x80000000u) != 0;
    const uint64_t rm_mask = __ballot(lane < (int)cnt && removal);
    const uint64_t in_mask = __ballot(lane < (int)cnt && !removal);
    int32_t nrem = __popcll(rm_mask), nins = __popcll(in_mask);
    for (uint32_t k0 = 64; k0 < cnt; k0 += 64) {
      const bool live = k0 + lane < cnt;
      const bool rm = live && (g[k0 + lane].row & 0x80000000u);
      nrem += __popcll(__ballot(rm));
      nins += __popcll(__ballot(live && !rm));
    }
    const int32_t new_len = len - nrem + nins;
    uint32_t start = old_start;
    if (new_len > (int32_t)cap) {
      const uint32_t need = (uint32_t)(len + nins);
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
        continue;
      }
      start = (uint32_t)pos;
      cap = ncap;
    }
    int32_t* lines = eb.lines ? eb.lines + (int64_t)row * eb.nbk * kLineInts : nullptr;
    if (len <= kStageKeys && new_len <= kStageKeys && cnt <= 64) {
      {  // whole 16-byte groups up to the end of the band's last line (inside its region), loads first
        const int4* src = reinterpret_cast<const int4*>(zeros + old_start);
        int4* dst = reinterpret_cast<int4*>(stage);
        const int32_t groups = (int32_t)round_line((uint64_t)len) >> 2;
        int4 v0 = make_int4(0, 0, 0, 0), v1 = v0, v2 = v0, v3 = v0;
        if (lane < groups) v0 = src[lane];
        if (64 + lane < groups) v1 = src[64 + lane];
        if (128 + lane < groups) v2 = src[128 + lane];
        if (192 + lane < groups) v3 = src[192 + lane];
        if (lane < groups) dst[lane] = v0;
        if (64 + lane < groups) dst[64 + lane] = v1;
        if (128 + lane < groups) dst[128 + lane] = v2;
        if (192 + lane < groups) dst[192 + lane] = v3;
      }
      wave_fence();
      int32_t n = len;
      bool missing = false;
      for (uint64_t mm = rm_mask; mm; mm &= mm - 1) {
        const int32_t z = __builtin_amdgcn_readlane(r.z, (int)__builtin_ctzll(mm));
        const int32_t pos = bound_lds(stage, n, z, false);
        if (pos >= n || stage[pos] != z) {
          missing = true;
          break;
        }
        shift_left<true>(stage, pos + 1, n);
        --n;
      }
      if (missing) {  // never expected; the host rebuilds the structure
        if (lane == 0) {
          atomicOr(&ctr->missing, 1u);
          rowcnt[row] = 0;
        }
        wave_fence();
        continue;
      }
      for (uint64_t mm = in_mask; mm; mm &= mm - 1) {
        const int32_t z = __builtin_amdgcn_readlane(r.z, (int)__builtin_ctzll(mm));
        const int32_t pos = bound_lds(stage, n, z, true);
        shift_right<true>(stage, pos, n);
        if (lane == 0) stage[pos] = z;
        wave_fence();
        ++n;
      }
      {  // the keys and the INT_MAX padding of the last line, 16 bytes a lane
        const int4* src = reinterpret_cast<const int4*>(stage);
        int4* dst = reinterpret_cast<int4*>(zeros + start);
        const int32_t groups = (int32_t)round_line((uint64_t)n) >> 2;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int32_t gi = u * 64 + lane;
          if (gi < groups) {
            int4 v = src[gi];
            const int32_t k = 4 * gi;
            if (k >= n) v.x = INT_MAX;
            if (k + 1 >= n) v.y = INT_MAX;
            if (k + 2 >= n) v.z = INT_MAX;
            if (k + 3 >= n) v.w = INT_MAX;
            dst[gi] = v;
          }
        }
      }
      band_levels(node, zeros, start, n, cap, stage);
      if (lane == 0) {
        node[0] = (int32_t)start;
        node[1] = n;
        node[2] = (int32_t)cap;
        rowcnt[row] = 0;
      }
      if (lines) {
        bucket_firsts4(stage, n, zlo, eb.shift, eb.nbk, first);
        for (int32_t b = lane; b < eb.nbk; b += 64) mark[b] = 0;
        wave_fence();
        if (lane < (int)cnt) mark_around(r.z, zlo, eb.shift, eb.nbk, first, mark);
        wave_fence();
        // a bucket's key count before the edit: now, less its inserts, plus its removals
        auto old_n = [&](int32_t b) {
          int32_t c = first[b + 1] - first[b];
          for (uint32_t k = 0; k < cnt; ++k)
            if (bucket_of(__builtin_amdgcn_readlane(r.z, (int)k), zlo, eb.shift, eb.nbk) == b)
              c += ((rm_mask >> k) & 1) ? 1 : -1;
          return c;
        };
        for (int32_t b0 = 0; b0 < eb.nbk; b0 += 64) {
          const uint64_t mk = __ballot(b0 + lane < eb.nbk && mark[b0 + lane]);
          over_n += write_lines_halves(stage, n, zlo, eb.shift, b0, mk, first, lines, eb.zp16, old_n);
        }
      }
      wave_fence();  // the LDS tables are rewritten for the wave's next band
      continue;
    }
    // long bands, and bands with many records: edited in place
    if (lines) bucket_firsts(zeros + old_start, len, zlo, eb.shift, eb.nbk, first_old);
    if (start != old_start) {
      int32_t* nk = zeros + start;
      for (int32_t k = lane; k < len; k += 64) nk[k] = zeros[old_start + k];
      __threadfence_block();
      if (lane == 0) {
        node[0] = (int32_t)start;
        node[2] = (int32_t)cap;
      }
      __threadfence_block();
    }
    int32_t* keys = zeros + start;
    int32_t n = len;
    for (uint32_t k = 0; k < cnt; ++k) {  // removals first: every one must find its key
      if (!(g[k].row & 0x80000000u)) continue;
      const int32_t z = g[k].z;
      const int32_t pos = bound(keys, n, z, false);
      if (pos >= n || keys[pos] != z) {
        if (lane == 0) atomicOr(&ctr->missing, 1u);
        continue;
      }
      shift_left<false>(keys, pos + 1, n);
      --n;
    }
    for (uint32_t k = 0; k < cnt; ++k) {
      if (g[k].row & 0x80000000u) continue;
      if (n >= (int32_t)cap) {  // only reachable if a removal above found no key
        if (lane == 0) atomicOr(&ctr->overflow, 1u);
        break;
      }
      const int32_t z = g[k].z;
      const int32_t pos = bound(keys, n, z, true);
      shift_right<false>(keys, pos, n);
      if (lane == 0) keys[pos] = z;
      __threadfence_block();
      ++n;
    }
    if (lane == 0) {
      node[1] = n;
      rowcnt[row] = 0;
    }
    __threadfence_block();
    finalize_band(node, zeros);
    if (lines) {
      __threadfence_block();
      bucket_firsts(keys, n, zlo, eb.shift, eb.nbk, first);
      for (int32_t b = lane; b < eb.nbk; b += 64) mark[b] = 0;
      __threadfence_block();
      for (uint32_t k = lane; k < cnt; k += 64) mark_around(g[k].z, zlo, eb.shift, eb.nbk, first, mark);
      __threadfence_block();
      over_n += write_bucket_lines<false>(keys, n, zlo, eb.shift, eb.nbk, first, mark, first_old, lines, eb.zp16);
    }
    __threadfence_block();
  }
  if (over_n != 0) atomicAdd(&ctr->bk_over, over_n);
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
  // A chunk's ops and its zeroed counters go to the device in one copy from
  // pinned staging (the counters sit right after the ops on both sides); the
  // counters come back into pinned memory.
  CDDT_TRY(ensure(m->alloc, m->upd_ops, kStageBytes, "update ops"));
  if (!m->upd_host &&
      hipHostMalloc(&m->upd_host, kStageBytes + sizeof(UpdCounters), hipHostMallocDefault) != hipSuccess) {
    m->upd_host = nullptr;
    return fail(CDDT_ENOMEM, "cddt_update: pinned staging allocation failed");
  }
  CDDT_TRY(ensure(m->alloc, m->upd_changed, (size_t)kOpChunk * sizeof(int2), "changed cells"));
  CDDT_TRY(ensure(m->alloc, m->upd_cand, (size_t)kOpChunk * 9 * sizeof(int2), "candidate cells"));
  CDDT_TRY(ensure(m->alloc, m->upd_edits, (size_t)kOpChunk * 9 * sizeof(int2), "edge flips"));
  UpdCounters* ctr = (UpdCounters*)((uint8_t*)m->upd_ops.ptr + kCounterOffset);
  uint8_t* packed = (uint8_t*)m->upd_host;
  UpdCounters* host_ctr = (UpdCounters*)(packed + kStageBytes);
  // A pruned (PCDDT) structure depends on every free cell, not only on edge
  // flips: its grid takes the ops and the structure is rebuilt and pruned.
  const bool pruned = (m->flags & CDDT_FLAG_PRUNE) != 0;
  bool grid_changed = false;

  for (int64_t o0 = 0; o0 < n_ops; o0 += kOpChunk) {
    const int32_t n = (int32_t)std::min<int64_t>(kOpChunk, n_ops - o0);
    int32_t* d_xs = (int32_t*)m->upd_ops.ptr;
    int32_t* d_ys = d_xs + kOpChunk;
    uint8_t* d_vs = (uint8_t*)(d_ys + kOpChunk);
    // (the previous chunk ended with a wait, so its copy has read the staging)
    std::memcpy(packed, xs_h + o0, 4 * (size_t)n);
    std::memcpy(packed + 4 * (size_t)kOpChunk, ys_h + o0, 4 * (size_t)n);
    std::memcpy(packed + 8 * (size_t)kOpChunk, vals_h + o0, (size_t)n);
    std::memset(packed + kCounterOffset, 0, sizeof(UpdCounters));
    CDDT_HIP(hipMemcpyAsync(d_xs, packed, kCounterOffset + sizeof(UpdCounters), hipMemcpyHostToDevice, st));
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
    // Records: at most 9 edge flips per op (a changed cell's 3x3 block), and
    // each flipped cell covers at most 3 bands of every slice.  When arrays
    // for that bound are small enough the launches follow at once, sized by
    // the bound (the kernels read the counts on the device); otherwise the
    // host waits for the count of flips.
    UpdCounters hc{};
    const uint64_t bound_rec = (uint64_t)n * 9 * m->half * 3;
    const bool no_wait = !pruned && bound_rec * kRecordBytes <= kNoWaitBytes;
    uint64_t max_rec = bound_rec, max_edits = (uint64_t)n * 9;
    if (!no_wait) {
      CDDT_HIP(hipMemcpyAsync(host_ctr, ctr, sizeof(hc), hipMemcpyDeviceToHost, st));
      CDDT_HIP(hipStreamSynchronize(st));
      hc = *host_ctr;
      if (pruned) {
        grid_changed = grid_changed || hc.changed > 0;
        continue;
      }
      if (hc.edits == 0) continue;
      max_edits = hc.edits;
      max_rec = (uint64_t)hc.edits * m->half * 3;
    }

    // band records, grouped per band
    CDDT_TRY(ensure(m->alloc, m->upd_rec, max_rec * (sizeof(Rec) + 4 + 2), "update records"));
    CDDT_TRY(ensure(m->alloc, m->upd_grp, max_rec * sizeof(Rec), "grouped records"));
    CDDT_TRY(ensure(m->alloc, m->upd_touched, max_rec * 12, "touched bands"));
    const uint64_t ntiles = (max_rec + kScanTile - 1) / kScanTile;
    CDDT_TRY(ensure(m->alloc, m->upd_tiles, ntiles * 4, "update scan tiles"));
    Rec* rec = (Rec*)m->upd_rec.ptr;
    uint32_t* local = (uint32_t*)(rec + max_rec);
    uint32_t* touched = (uint32_t*)m->upd_touched.ptr;
    uint32_t* toff = touched + max_rec;
    int32_t* tzlo = (int32_t*)(toff + max_rec);
    uint16_t* rslice = (uint16_t*)(local + max_rec);
    uint32_t* rowcnt = (uint32_t*)m->upd_rowcnt.ptr;
    uint32_t* slot = (uint32_t*)m->upd_slot.ptr;
    const unsigned rblocks = std::min<unsigned>(blocks_for(max_rec, kThreads), kStrideBlocks);
    hipLaunchKernelGGL(k_records, dim3(blocks_for(max_edits, kThreads), m->half), dim3(kThreads), 0, st,
                       m->d_slices, edits, (const UpdCounters*)ctr, rec, rslice, ctr);
    hipLaunchKernelGGL(k_group_count, dim3(rblocks), dim3(kThreads), 0, st, rec,
                       (const uint16_t*)rslice, (const SliceDev*)m->d_slices, (const UpdCounters*)ctr, rowcnt, slot,
                       touched, tzlo, local, ctr);
    hipLaunchKernelGGL(k_touched_counts, dim3(rblocks), dim3(kThreads), 0, st, touched,
                       (const UpdCounters*)ctr, rowcnt, toff);
    hipLaunchKernelGGL(k_scan_sum, dim3((unsigned)ntiles), dim3(kScanThreads), 0, st, toff, (const UpdCounters*)ctr,
                       (uint32_t*)m->upd_tiles.ptr);
    hipLaunchKernelGGL(k_scan_tiles, dim3(1), dim3(kScanThreads), 0, st, (uint32_t*)m->upd_tiles.ptr,
                       (uint32_t)ntiles);
    hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)ntiles), dim3(kScanThreads), 0, st, toff,
                       (const UpdCounters*)ctr, (const uint32_t*)m->upd_tiles.ptr);
    hipLaunchKernelGGL(k_group_fill, dim3(rblocks), dim3(kThreads), 0, st, rec,
                       (const UpdCounters*)ctr, slot, toff, local, (Rec*)m->upd_grp.ptr);
    EditBuckets eb{};
    if (m->d_bk) {
      if (m->nbk > kFillMaxBuckets) return fail(CDDT_EINTERNAL, "cddt_update: more buckets per band than planned");
      eb = EditBuckets{m->d_bk, 16 + m->blog2, m->nbk, (m->flags & CDDT_FLAG_ZP16) ? 1 : 0};
    }
    const size_t wave_bytes = (size_t)edit_wave_words(eb.nbk) * 4;
    const unsigned wpb = (unsigned)std::max<size_t>(1, std::min<size_t>(4, 65536 / wave_bytes));
    const unsigned eblocks = std::min<unsigned>(blocks_for(max_rec, (int)wpb), kEditBlocks);
    hipLaunchKernelGGL(k_edit_bands, dim3(eblocks), dim3(64 * wpb), wpb * wave_bytes, st, m->d_hdr, m->d_zeros,
                       touched, (const int32_t*)tzlo, toff, rowcnt, (const Rec*)m->upd_grp.ptr, ctr, m->d_spare,
                       (uint64_t)m->spare_end, eb);
    CDDT_HIP(hipGetLastError());
    CDDT_HIP(hipMemcpyAsync(host_ctr, ctr, sizeof(hc), hipMemcpyDeviceToHost, st));
    CDDT_HIP(hipStreamSynchronize(st));
    hc = *host_ctr;
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
      if (m->d_bk) m->bucket_overflow += hc.bk_over;
    }
  }
  if (grid_changed) {
    CDDT_TRY(build_structure(m, st));
    ++m->rebuilds;
  }
  return CDDT_OK;
}

}  // namespace cddt
