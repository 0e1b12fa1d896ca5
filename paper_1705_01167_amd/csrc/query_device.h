// Device-side CDDT query: bin selection, projection into a slice, band search
// and the per-particle beam log-weight.  Shared by the plain cast kernel, the
// per-filter weight kernel and the persistent batched kernel, so every entry
// point produces identical bits.
//
// Method: Sec. IV-B (project the query, take its band, successor search,
// difference), Sec. IV-C (bins k >= n/2 search the same band backwards; the
// overlap check on the full grid; opposite rays share one search), Sec. VI
// (beam-model log-likelihood summed over the rays of a particle).
//
// Band layout (see band_layout.h): a 128-byte header node per band holds
// {start, len, cap} and up to 29 entries of the band's top search level; the
// keys sit in 128-byte lines of 32 starting at `start`, followed by stored
// sample levels (every 32nd key, every 1024th key, ...) when the band is long.
// A search reads the header line and then one 128-byte line per level below
// the top: two lines for bands of <= 928 keys, three up to 29696.
//
// Searches are cooperative: 8 lanes share one search, each lane loading 16 of
// a line's 128 bytes, so one load instruction fetches 8 lines for 8 searches.
#pragma once

#include <climits>

#include "band_layout.h"
#include "cddt_common.h"

namespace cddt {

// Loads and stores through the global address space.  Pointers read from a
// descriptor table in memory are generic, and generic (flat) loads count
// against the LDS wait counter too, which would serialise them with the
// lane shuffles; global loads keep several lines in flight.
template <typename T>
__device__ __forceinline__ T ldg(const T* p) {
  return *(const __attribute__((address_space(1))) T*)p;
}
template <typename T>
__device__ __forceinline__ void stg(T* p, T v) {
  *(__attribute__((address_space(1))) T*)p = v;
}
// 16-byte load as a native vector (int4's copy constructor would take a
// generic reference and turn the load back into a flat one).
typedef int32_t cddt_v4i __attribute__((ext_vector_type(4)));
__device__ __forceinline__ int4 ldg4(const int4* p) {
  const cddt_v4i v = *(const __attribute__((address_space(1))) cddt_v4i*)p;
  return make_int4(v.x, v.y, v.z, v.w);
}

// Loads and stores of a request's own inputs and outputs.  With Sys they are
// system-coherent (relaxed atomics at system scope): they bypass the L2, so
// data that the host rewrites while a kernel runs (a resident server's slots
// in pinned host memory) is read fresh, and results reach host memory when
// the store is acknowledged.
template <bool Sys, typename T>
__device__ __forceinline__ T ldx(const T* p) {
  if constexpr (Sys)
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
  else
    return ldg(p);
}
template <bool Sys, typename T>
__device__ __forceinline__ void stx(T* p, T v) {
  if constexpr (Sys)
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
  else
    stg(p, v);
}

// Quantised query position: floor(v * 2^16); v * 2^16 is exact in float32.
__device__ __forceinline__ int32_t quantize16(float v) {
  return (int32_t)floorf(__fmul_rn(v, 65536.0f));
}

__device__ __forceinline__ bool pose_inside(const MapDev& m, float x, float y) {
  return x >= 0.0f && x < (float)m.w && y >= 0.0f && y < (float)m.h;
}

// Bin over the full circle: floor(fl(fl(theta * K) + 0.5)) mod n, Euclidean.
// The multiply and the add round separately (no FMA contraction).
__device__ __forceinline__ int32_t theta_bin(float theta, float k_scale, int32_t n) {
  float t = __fmul_rn(theta, k_scale);
  float u = __fadd_rn(t, 0.5f);
  int32_t k = (int32_t)floorf(u);
  if (k >= -n && k < 2 * n) return k < 0 ? k + n : (k >= n ? k - n : k);  // angles within one turn of [0, 2pi)
  k %= n;
  return k < 0 ? k + n : k;
}

// First index in a[0, len) whose value is >= key (number of values < key).
__device__ __forceinline__ int32_t lower_bound_i32(const int32_t* __restrict__ a, int32_t len, int32_t key) {
  int32_t lo = 0, cnt = len;
  while (cnt > 0) {
    int32_t half = cnt >> 1;
    int32_t v = ldg(a + lo + half);
    if (v < key) {
      lo += half + 1;
      cnt -= half + 1;
    } else {
      cnt = half;
    }
  }
  return lo;
}

// Round the Q16 distance half up and clamp to the max range.
// Range from the distance d >= 0 (Q16) between a query and a zero point,
// rounded half up, capped at max_range.  Zero points and in-map queries lie
// within 2^31 - 2^28 of 0, so d < 2^32 - 2^29 and d + 2^15 fits 32 unsigned bits.
__device__ __forceinline__ int32_t range_of(uint32_t d, int32_t max_range) {
  const uint32_t v = (d + 32768u) >> 16;
  return v < (uint32_t)max_range ? (int32_t)v : max_range;
}

// Where a valid query lands: along-ray coordinate and global band index.
// With a bucket index the coordinate is taken relative to the slice's bucket
// origin (the keys of the bucket lines are stored the same way).
struct Landing {
  int32_t xq;
  int32_t row;
};

__device__ __forceinline__ Landing land(const MapDev& m, int32_t slice, int32_t xf, int32_t yf) {
  const int4 sv = ldg4(reinterpret_cast<const int4*>(m.slices + slice));
  int64_t along = (int64_t)xf * sv.x + (int64_t)yf * sv.y;
  int64_t lat = (int64_t)yf * sv.x - (int64_t)xf * sv.y;
  Landing l;
  l.xq = (int32_t)(along >> 30) - (m.bk ? sv.w : 0);
  l.row = sv.z + (int32_t)(lat >> 46);
  return l;
}

// Cross-lane moves inside a row of 16 lanes (DPP; VALU, no LDS traffic).
// quad_perm patterns swap lanes 1 / 2 apart inside each group of 4; the
// half-row mirror pairs lane i with 7 - i inside each group of 8; the row
// mirror pairs lane i with 15 - i.
constexpr int kDppQuadXor1 = 0xB1;    // quad_perm [1, 0, 3, 2]
constexpr int kDppQuadXor2 = 0x4E;    // quad_perm [2, 3, 0, 1]
constexpr int kDppQuadBcast0 = 0x00;  // quad_perm [0, 0, 0, 0]
constexpr int kDppRowMirror = 0x140;
constexpr int kDppHalfMirror = 0x141;

template <int Ctrl>
__device__ __forceinline__ int32_t dpp(int32_t v) {
  return __builtin_amdgcn_update_dpp(0, v, Ctrl, 0xF, 0xF, false);
}
template <int Ctrl>
__device__ __forceinline__ float dppf(float v) {
  return __builtin_bit_cast(float, dpp<Ctrl>(__builtin_bit_cast(int32_t, v)));
}

// Sum / min / max over the 8 lanes of a search group (lanes 8g .. 8g+7): two
// quad exchanges, then the other quad of the group through the half mirror.
__device__ __forceinline__ int32_t group_sum(int32_t v) {
  v += dpp<kDppQuadXor1>(v);
  v += dpp<kDppQuadXor2>(v);
  return v + dpp<kDppHalfMirror>(v);
}
__device__ __forceinline__ int32_t group_min(int32_t v) {
  v = min(v, dpp<kDppQuadXor1>(v));
  v = min(v, dpp<kDppQuadXor2>(v));
  return min(v, dpp<kDppHalfMirror>(v));
}
__device__ __forceinline__ int32_t group_max(int32_t v) {
  v = max(v, dpp<kDppQuadXor1>(v));
  v = max(v, dpp<kDppQuadXor2>(v));
  return max(v, dpp<kDppHalfMirror>(v));
}
// Value of the group's first lane in all 8 lanes.
__device__ __forceinline__ int32_t group_bcast0(int32_t v, int sub) {
  const int32_t q = dpp<kDppQuadBcast0>(v);  // first lane of each quad
  const int32_t o = dpp<kDppHalfMirror>(q);  // the other quad's first lane
  return sub < 4 ? q : o;
}

// Float sum over the whole wave in a fixed order: each row of 16 lanes is
// reduced with DPP (all lanes of a row end with the same bits), then the
// four row totals are added as (row0 + row1) + (row2 + row3).
__device__ __forceinline__ float wave_sum(float v) {
  v += dppf<kDppQuadXor1>(v);
  v += dppf<kDppQuadXor2>(v);
  v += dppf<kDppHalfMirror>(v);
  v += dppf<kDppRowMirror>(v);
  const float r0 = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int32_t, v), 0));
  const float r1 = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int32_t, v), 16));
  const float r2 = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int32_t, v), 32));
  const float r3 = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int32_t, v), 48));
  return (r0 + r1) + (r2 + r3);
}

// Scan this lane's four entries (indices 4*sub .. 4*sub+3 of a 32-entry line,
// shifted by `skip` header words) against x: entries with index in [0, valid).
__device__ __forceinline__ void scan4(int4 v, int sub, int skip, int32_t valid, int32_t x, int32_t& cnt,
                                      int32_t& nxt, int32_t& prv) {
  const int32_t e[4] = {v.x, v.y, v.z, v.w};
  cnt = 0;
  nxt = INT_MAX;
  prv = INT_MIN;
#pragma unroll
  for (int q = 3; q >= 0; --q) {
    const int32_t idx = 4 * sub + q - skip;
    if (idx >= 0 && idx < valid) {
      if (e[q] <= x) {
        ++cnt;
        prv = max(prv, e[q]);
      } else {
        nxt = e[q];  // ascending: the lowest index > x wins (scanned last)
      }
    }
  }
}

// Cooperative band search for one wave.  Each lane may own one query (want)
// with band `row` and along-ray coordinate `xq`.  On return that lane holds
// r_succ, the range to the smallest zero point > xq, and r_pred, the range to
// the largest zero point < xq (max_range when there is none).  Must be called
// by all 64 lanes together.
//
// The eight 8-lane groups each run K searches side by side: the K header
// lines are requested before any is used, then the searches descend their
// levels in lock-step, one line request per search per level.  K raises the
// number of independent lines a wave keeps in flight from 8 to 8K.
template <int K>
__device__ __forceinline__ void wave_search(const MapDev& m, bool want, int32_t row, int32_t xq, int32_t max_range,
                                            int32_t& r_succ, int32_t& r_pred) {
  const int lane = threadIdx.x & (kWave - 1);
  const uint64_t mask = __ballot(want);
  const int n = __popcll(mask);
  const int rank = __popcll(mask & ((1ull << lane) - 1ull));
  // rank -> lane table: want lanes go to their rank, the rest fill the tail
  const int dest = want ? rank : n + (lane - rank);
  const int list = __builtin_amdgcn_ds_permute(dest << 2, lane);
  const int g = lane >> 3, sub = lane & 7;
  r_succ = max_range;
  r_pred = max_range;
  for (int base = 0; base < n; base += 8 * K) {
    int32_t x[K], len[K], cap[K], c[K], nxt[K], prv[K], lvl[K];
    uint32_t start[K];
    int4 v[K];
#pragma unroll
    for (int j = 0; j < K; ++j) {  // request all K header lines first
      const int k = base + 8 * j + g;
      const bool act = k < n;
      const int src = __shfl(list, act ? k : 0);
      const int32_t qrow = __shfl(row, src);
      x[j] = __shfl(xq, src);
      v[j] = act ? ldg4(reinterpret_cast<const int4*>(m.hdr + (int64_t)qrow * kNodeInts) + sub) : make_int4(0, 0, 0, 0);
    }
#pragma unroll
    for (int j = 0; j < K; ++j) {  // top level, held in the header node
      start[j] = (uint32_t)group_bcast0(v[j].x, sub);
      len[j] = group_bcast0(v[j].y, sub);
      cap[j] = group_bcast0(v[j].z, sub);
      int32_t T = 0, nT = len[j];
      while (nT > kTopEntries) {
        nT = (nT + kLineInts - 1) >> kLineShift;
        ++T;
      }
      int32_t lc, ln, lp;
      scan4(v[j], sub, kHeaderWords, nT, x[j], lc, ln, lp);
      c[j] = group_sum(lc);
      nxt[j] = group_min(ln);
      prv[j] = group_max(lp);
      lvl[j] = c[j] > 0 ? T - 1 : -1;
    }
    for (;;) {  // one level of every unfinished search per round
      bool more = false;
#pragma unroll
      for (int j = 0; j < K; ++j) more |= lvl[j] >= 0;
      if (!more) break;
#pragma unroll
      for (int j = 0; j < K; ++j)
        if (lvl[j] >= 0) {
          const uint32_t off = level_base(start[j], (uint32_t)cap[j], lvl[j]) + (uint32_t)(c[j] - 1) * kLineInts;
          v[j] = ldg4(reinterpret_cast<const int4*>(m.zeros + off) + sub);
        }
#pragma unroll
      for (int j = 0; j < K; ++j)
        if (lvl[j] >= 0) {
          const int32_t blk = c[j] - 1;
          const int32_t valid = min(kLineInts, level_count(len[j], lvl[j]) - blk * kLineInts);
          int32_t lc, ln, lp;
          scan4(v[j], sub, 0, valid, x[j], lc, ln, lp);
          c[j] = blk * kLineInts + group_sum(lc);
          const int32_t gn = group_min(ln);
          nxt[j] = gn != INT_MAX ? gn : nxt[j];  // none in this block: the next block's first entry
          prv[j] = group_max(lp);
          --lvl[j];
        }
    }
    // c = number of keys <= x; nxt = smallest key > x; prv = largest key <= x
    int32_t gs[K], gp[K];
#pragma unroll
    for (int j = 0; j < K; ++j) {
      gs[j] = c[j] < len[j] ? range_of((uint32_t)nxt[j] - (uint32_t)x[j], max_range) : max_range;
      gp[j] = max_range;
      if (c[j] > 0) {
        int32_t pv = prv[j];
        if (pv == x[j]) {  // rare: x equals a key; find the last key strictly below it
          const int32_t lb = lower_bound_i32(m.zeros + start[j], c[j], x[j]);
          pv = lb > 0 ? ldg(m.zeros + start[j] + lb - 1) : INT_MIN;
        }
        if (pv != INT_MIN) gp[j] = range_of((uint32_t)x[j] - (uint32_t)pv, max_range);
      }
    }
    // hand results back: search k = base + 8j + g sits in slot j of group g;
    // both ranges (<= 65535) travel packed in one word
    const int rel = rank - base;
    const int leader = (rel & 7) << 3;
#pragma unroll
    for (int j = 0; j < K; ++j) {
      const int32_t pk = __shfl(gs[j] | (gp[j] << 16), leader);
      if (want && rel >= 0 && (rel >> 3) == j) {
        r_succ = pk & 0xffff;
        r_pred = (int32_t)((uint32_t)pk >> 16);
      }
    }
  }
}

// One 128-byte line of 32 entries, loaded by a single lane (8 x 16 bytes).
struct Line32 {
  int32_t e[32];
};

__device__ __forceinline__ Line32 load_line(const int32_t* p) {
  Line32 L;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const int4 q = ldg4(reinterpret_cast<const int4*>(p) + i);
    L.e[4 * i] = q.x;
    L.e[4 * i + 1] = q.y;
    L.e[4 * i + 2] = q.z;
    L.e[4 * i + 3] = q.w;
  }
  return L;
}

// Nearest entries by unsigned minima instead of compare-and-select chains
// (whose 64-bit lane masks would all be held in scalar registers at once).
// Modulo 2^32, d = e - x - 1 puts the entries above x first: e > x exactly
// when d < INT_MAX - x, and then e = x + 1 + d.  Likewise d = x - e puts the
// entries <= x first: e <= x exactly when d <= x + 2^31, and then e = x - d.
// Both hold for every pair of int32 values.
__device__ __forceinline__ uint32_t above_gap(int32_t e, int32_t x) { return (uint32_t)e - (uint32_t)x - 1u; }
__device__ __forceinline__ uint32_t below_gap(int32_t e, int32_t x) { return (uint32_t)x - (uint32_t)e; }
__device__ __forceinline__ bool has_above(uint32_t d, int32_t x) { return d < (uint32_t)INT_MAX - (uint32_t)x; }
__device__ __forceinline__ bool has_below(uint32_t d, int32_t x) { return d <= ((uint32_t)x ^ 0x80000000u); }

// Entries First..31 of a sorted line (unused slots hold INT_MAX): c = number
// of entries <= x, prv = the largest of them (INT_MIN if none), nxt = the
// smallest entry > x, or `carried` when every entry is <= x.
template <int First>
__device__ __forceinline__ void scan_line(const Line32& L, int32_t x, int32_t carried, int32_t& c, int32_t& nxt,
                                          int32_t& prv) {
  uint32_t dn = 0xffffffffu, dp = 0xffffffffu;
  c = 0;
#pragma unroll
  for (int i = First; i < 32; ++i) {
    dn = min(dn, above_gap(L.e[i], x));
    dp = min(dp, below_gap(L.e[i], x));
    c += L.e[i] <= x ? 1 : 0;
  }
  nxt = has_above(dn, x) ? (int32_t)((uint32_t)x + 1u + dn) : carried;
  prv = has_below(dp, x) ? (int32_t)((uint32_t)x - dp) : INT_MIN;
}

// Band search by one lane: the header line, then one line per level below the
// top.  Same results as wave_search; no cross-lane traffic, and a wave keeps up
// to 64 independent lines in flight.  Lanes without a query return max_range.
// The band's nearest keys around x: succ = smallest key > x, pred = largest
// key < x, or <= x when strict_pred is false (INT_MAX / INT_MIN when there is
// none).
__device__ __forceinline__ void tree_keys(const MapDev& m, int32_t row, int32_t x, bool strict_pred, int32_t& succ,
                                          int32_t& pred) {
  Line32 L = load_line(m.hdr + (int64_t)row * kNodeInts);
  const uint32_t start = (uint32_t)L.e[0];
  const int32_t len = L.e[1];
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
  succ = c < len ? nxt : INT_MAX;
  pred = INT_MIN;
  if (c > 0) {
    int32_t pv = prv;
    if (strict_pred && pv == x) {  // rare: x equals a key; find the last key strictly below it
      const int32_t lb = lower_bound_i32(m.zeros + start, c, x);
      pv = lb > 0 ? ldg(m.zeros + start + lb - 1) : INT_MIN;
    }
    pred = pv;
  }
}

__device__ __forceinline__ void tree_search(const MapDev& m, bool want, int32_t row, int32_t x, int32_t max_range,
                                            int32_t& r_succ, int32_t& r_pred) {
  r_succ = max_range;
  r_pred = max_range;
  if (!want) return;
  int32_t succ, pred;
  tree_keys(m, row, x, true, succ, pred);
  if (succ != INT_MAX) r_succ = range_of((uint32_t)succ - (uint32_t)x, max_range);
  if (pred != INT_MIN) r_pred = range_of((uint32_t)x - (uint32_t)pred, max_range);
}

// Bucket-index search by one lane: the bucket line of (band, x) gives the
// nearest key above x (within the bucket, else the carried next key) and the
// nearest key below x (within the bucket, else the carried previous key);
// keys equal to x count on neither side, as in tree_search.  x is relative to
// the slice's bucket origin.  An overflowing bucket defers to tree_search.
__device__ __forceinline__ int32_t bucket_of(const MapDev& m, int32_t x) {
  const int32_t b = x >> m.bshift;
  return b < 0 ? 0 : (b >= m.nbk ? m.nbk - 1 : b);
}

__device__ __forceinline__ void scan_bucket(const Line32& L, int32_t x, int32_t max_range, int32_t& r_succ,
                                            int32_t& r_pred) {
  // x > INT_MIN here (x >= 0 relative to the bucket origin), so the keys < x
  // are the keys <= x - 1
  const int32_t xm = x - 1;
  uint32_t dn = 0xffffffffu, dp = 0xffffffffu;
#pragma unroll
  for (int i = 2; i < 32; ++i) {
    dn = min(dn, above_gap(L.e[i], x));
    dp = min(dp, below_gap(L.e[i], xm));
  }
  int32_t nxt = has_above(dn, x) ? (int32_t)((uint32_t)x + 1u + dn) : INT_MAX;
  const int32_t prv = has_below(dp, xm) ? (int32_t)((uint32_t)xm - dp) : L.e[0];
  nxt = nxt < L.e[1] ? nxt : L.e[1];
  r_succ = nxt != INT_MAX ? range_of((uint32_t)nxt - (uint32_t)x, max_range) : max_range;
  r_pred = prv != INT_MIN ? range_of((uint32_t)x - (uint32_t)prv, max_range) : max_range;
}

// 16-bit zero points: a key of bin B stands for the bin centre B 8192 + 4096
// (relative to zlo).  The successor is the first key of bin >= bmin, the
// predecessor the last key of bin <= bmax, with bmin / bmax the bins whose
// centres lie strictly above / below x.
__device__ __forceinline__ int32_t bin_min_above(int32_t x) { return ((x - 4096) >> kBinShift) + 1; }
__device__ __forceinline__ int32_t bin_max_below(int32_t x) { return ((x - 4096 + 8191) >> kBinShift) - 1; }
__device__ __forceinline__ int32_t bin_centre(int32_t b) { return b * 8192 + 4096; }

__device__ __forceinline__ void scan_bucket16(const MapDev& m, const Line32& L, int32_t x, int32_t b,
                                              int32_t max_range, int32_t& r_succ, int32_t& r_pred) {
  const int32_t base = b << (m.bshift - kBinShift);  // first bin of the bucket
  const int32_t ts = bin_min_above(x) - base, tp = bin_max_below(x) - base;
  // One pass of unsigned minima, each word read once: the smallest key >= ts
  // and the largest key <= tp.  Keys, ts and tp are far below 2^31 in
  // magnitude, so v - ts (tp - v) is below 2^31 as an unsigned number exactly
  // when v >= ts (v <= tp).  Padding 0xffff lies above every bin of a bucket:
  // it never counts as <= tp, and as the only key >= ts it reads as none.
  uint32_t ds = 0xffffffffu, dp = 0xffffffffu;
#pragma unroll
  for (int i = 2; i < 32; ++i) {
    const uint32_t w = (uint32_t)L.e[i];
    const uint32_t lo = w & 0xffffu, hi = w >> 16;
    ds = min(ds, min(lo - (uint32_t)ts, hi - (uint32_t)ts));
    dp = min(dp, min((uint32_t)tp - lo, (uint32_t)tp - hi));
  }
  const int32_t s16 = ds < 0x80000000u ? ts + (int32_t)ds : 0xffff;
  const int32_t p16 = dp < 0x80000000u ? tp - (int32_t)dp : -1;
  const int32_t nxt = s16 != 0xffff ? bin_centre(base + s16) : L.e[1];
  const int32_t prv = p16 >= 0 ? bin_centre(base + p16) : L.e[0];
  r_succ = nxt != INT_MAX ? range_of((uint32_t)nxt - (uint32_t)x, max_range) : max_range;
  r_pred = prv != INT_MIN ? range_of((uint32_t)x - (uint32_t)prv, max_range) : max_range;
}

// Overflowing bucket: the band's exact keys by one tree descent, in a kernel
// that also serves maps with 16-bit zero points (z).  32-bit keys: the nearest
// keys around x, as tree_search.  16-bit: the first key >= t1 (the start of
// bin bmin) and the last key < t2 (the end of bin bmax), mapped to their bin
// centres; t2 = t1 unless x is itself a bin centre (t2 = t1 - 8192), the one
// case that takes a second descent.  A single call site of tree_keys keeps the
// kernel's register count down.
__device__ __forceinline__ void tree_search_any(const MapDev& m, bool z, int32_t row, int32_t x, int32_t zlo,
                                                int32_t max_range, int32_t& r_succ, int32_t& r_pred) {
  const int32_t t1 = zlo + bin_min_above(x) * 8192, t2 = zlo + (bin_max_below(x) + 1) * 8192;
  int32_t xt = z ? t1 - 1 : x + zlo, succ = INT_MAX, pred = INT_MIN;
  for (int pass = 0; pass < 2; ++pass) {
    int32_t s1, p1;
    tree_keys(m, row, xt, !z, s1, p1);
    if (pass == 0) succ = s1;
    pred = p1;
    if (!z || t2 == t1) break;
    xt = t2 - 1;
  }
  int32_t vs = succ, vp = pred, xr = x + zlo;
  if (z) {  // bin centres, relative to zlo like x
    vs = bin_centre((succ - zlo) >> kBinShift);
    vp = bin_centre((pred - zlo) >> kBinShift);
    xr = x;
  }
  r_succ = succ != INT_MAX ? range_of((uint32_t)vs - (uint32_t)xr, max_range) : max_range;
  r_pred = pred != INT_MIN ? range_of((uint32_t)xr - (uint32_t)vp, max_range) : max_range;
}

// Z: the caller's kernel handles maps with 16-bit zero points (Z = false
// compiles the 32-bit line scan alone; the host never hands such a kernel a
// map with 16-bit zero points).
template <bool Z>
__device__ __forceinline__ void scan_bucket_any(const MapDev& m, const Line32& L, int32_t row, int32_t x,
                                                int32_t max_range, int32_t& r_succ, int32_t& r_pred) {
  // The scan runs before the overflow test and its results pass through an
  // empty asm statement, which the compiler cannot move into a branch: this
  // keeps all eight loads of the line ahead of the test.  (Otherwise the
  // compiler moves the loads of words 4..31 into the branch that reads them,
  // and every search waits for two memory round trips in a row.)  An
  // overflowing line's scan result is discarded.
  if constexpr (Z) {
    if (m.zp16)
      scan_bucket16(m, L, x, bucket_of(m, x), max_range, r_succ, r_pred);
    else
      scan_bucket(L, x, max_range, r_succ, r_pred);
  } else {
    scan_bucket(L, x, max_range, r_succ, r_pred);
  }
  asm volatile("" : "+v"(r_succ), "+v"(r_pred));
  if (L.e[0] == kBucketOverflow) {
    if constexpr (Z)
      tree_search_any(m, m.zp16, row, x, L.e[1], max_range, r_succ, r_pred);
    else
      tree_search(m, true, row, x + L.e[1], max_range, r_succ, r_pred);
  }
}

template <bool Z>
__device__ __forceinline__ void bucket_search(const MapDev& m, bool want, int32_t row, int32_t x, int32_t max_range,
                                              int32_t& r_succ, int32_t& r_pred) {
  r_succ = max_range;
  r_pred = max_range;
  if (!want) return;
  const Line32 L = load_line(m.bk + ((int64_t)row * m.nbk + bucket_of(m, x)) * kLineInts);
  scan_bucket_any<Z>(m, L, row, x, max_range, r_succ, r_pred);
}

// Band search by one lane (bucket index when the map has one, else the
// band's search lines).
template <bool Z>
__device__ __forceinline__ void lane_search(const MapDev& m, bool want, int32_t row, int32_t x, int32_t max_range,
                                            int32_t& r_succ, int32_t& r_pred) {
  if (m.bk)
    bucket_search<Z>(m, want, row, x, max_range, r_succ, r_pred);
  else
    tree_search(m, want, row, x, max_range, r_succ, r_pred);
}

// Two bucket searches by one lane, both lines in flight together.
template <bool Z>
__device__ __forceinline__ void bucket_search2(const MapDev& m, bool wa, int32_t ra, int32_t xa, bool wb, int32_t rb,
                                               int32_t xb, int32_t max_range, int32_t& sa, int32_t& pa, int32_t& sb,
                                               int32_t& pb) {
  sa = pa = sb = pb = max_range;
  if (!wa && !wb) return;
  Line32 A, B;
  if (wa) A = load_line(m.bk + ((int64_t)ra * m.nbk + bucket_of(m, xa)) * kLineInts);
  if (wb) B = load_line(m.bk + ((int64_t)rb * m.nbk + bucket_of(m, xb)) * kLineInts);
  if (wa) scan_bucket_any<Z>(m, A, ra, xa, max_range, sa, pa);
  if (wb) scan_bucket_any<Z>(m, B, rb, xb, max_range, sb, pb);
}

// Two independent band searches by one lane, their line requests issued side
// by side (the second search's lines are in flight while the first's are
// scanned).  Same results as two lane_search calls.
template <bool Z>
__device__ __forceinline__ void lane_search2(const MapDev& m, bool wa, int32_t ra, int32_t xa, bool wb, int32_t rb,
                                             int32_t xb, int32_t max_range, int32_t& sa, int32_t& pa, int32_t& sb,
                                             int32_t& pb) {
  if (m.bk) {
    bucket_search2<Z>(m, wa, ra, xa, wb, rb, xb, max_range, sa, pa, sb, pb);
    return;
  }
  sa = pa = sb = pb = max_range;
  if (!wa && !wb) return;
  Line32 A, B;
  if (wa) A = load_line(m.hdr + (int64_t)ra * kNodeInts);
  if (wb) B = load_line(m.hdr + (int64_t)rb * kNodeInts);
  uint32_t st_a = 0, st_b = 0, cp_a = 0, cp_b = 0;
  int32_t ln_a = 0, ln_b = 0, ca = 0, cb = 0, na = INT_MAX, nb = INT_MAX, va = INT_MIN, vb = INT_MIN, ta = -1, tb = -1;
  if (wa) {
    st_a = (uint32_t)A.e[0];
    ln_a = A.e[1];
    cp_a = (uint32_t)A.e[2];
    scan_line<kHeaderWords>(A, xa, INT_MAX, ca, na, va);
    ta = ca > 0 ? top_level(ln_a) - 1 : -1;
  }
  if (wb) {
    st_b = (uint32_t)B.e[0];
    ln_b = B.e[1];
    cp_b = (uint32_t)B.e[2];
    scan_line<kHeaderWords>(B, xb, INT_MAX, cb, nb, vb);
    tb = cb > 0 ? top_level(ln_b) - 1 : -1;
  }
  while (ta >= 0 || tb >= 0) {
    const int32_t ka = ca - 1, kb = cb - 1;
    if (ta >= 0) A = load_line(m.zeros + level_base(st_a, cp_a, ta) + (uint32_t)ka * kLineInts);
    if (tb >= 0) B = load_line(m.zeros + level_base(st_b, cp_b, tb) + (uint32_t)kb * kLineInts);
    if (ta >= 0) {
      int32_t lc;
      scan_line<0>(A, xa, na, lc, na, va);
      ca = ka * kLineInts + lc;
      --ta;
    }
    if (tb >= 0) {
      int32_t lc;
      scan_line<0>(B, xb, nb, lc, nb, vb);
      cb = kb * kLineInts + lc;
      --tb;
    }
  }
  auto finish = [&](bool w, uint32_t st, int32_t ln, int32_t c, int32_t nx, int32_t pv, int32_t x, int32_t& rs,
                    int32_t& rp) {
    if (!w) return;
    if (c < ln) rs = range_of((uint32_t)nx - (uint32_t)x, max_range);
    if (c > 0) {
      if (pv == x) {  // rare: x equals a key; find the last key strictly below it
        const int32_t lb = lower_bound_i32(m.zeros + st, c, x);
        pv = lb > 0 ? ldg(m.zeros + st + lb - 1) : INT_MIN;
      }
      if (pv != INT_MIN) rp = range_of((uint32_t)x - (uint32_t)pv, max_range);
    }
  };
  finish(wa, st_a, ln_a, ca, na, va, xa, sa, pa);
  finish(wb, st_b, ln_b, cb, nb, vb, xb, sb, pb);
}

// One round of first passes over jobs [b, b + 64) by quads of lanes: in step
// k the 16 quads take jobs b + 16k .. b + 16k + 15, each lane of a quad
// reading one 16-byte quarter of the first half of the job's bucket line, so
// one load instruction covers 16 lines.  Each lane reduces its four words to
// the smallest above-gap and below-gap (unsigned minima as in scan_line; the
// carried neighbours in words 0 and 1 lie below and above x, so they take
// part like keys), then the quad combines them with two DPP exchanges.  Lane
// 4q + s keeps step s's result: job jo = b + 16s + q.  Returns whether jo
// exists; rs < 0 when the half line cannot settle it (x at or beyond the 14th
// key, or an overflowing bucket), else the ranges.  The first half of a line
// holds the carried neighbours and the bucket's lowest 14 keys (words 2..15);
// when x lies below the 14th key, the successor is among those keys (the 14th
// is above x) and every key below x is among them too (keys ascend), so the
// half gives the whole line's results.  Half a line halves the loads issued
// per search (the L2 still fills whole lines from memory).  All 64 lanes call.
__device__ __forceinline__ bool quad_half_round(const MapDev& m, const int2* jobs, int32_t b, int32_t njobs,
                                                int32_t max_range, int32_t& jo, int32_t& rs, int32_t& rp) {
  const int lane = threadIdx.x & (kWave - 1), sub = lane & 3, quad = lane >> 2;
  // Slots b .. b + 63 all lie inside the wave's queue (b < njobs <= the
  // queue's size, a multiple of 64), so the four job reads need no condition;
  // slots at or past njobs read stale entries, which load band 0's first line
  // instead (a valid address) and whose results are dropped.
  int2 jb[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) jb[k] = jobs[b + 16 * k + quad];
  const int4* lines = reinterpret_cast<const int4*>(m.bk) + sub;
  int4 v[4];
  int32_t xs[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const bool ok = b + 16 * k + quad < njobs;
    const int32_t row = ok ? jb[k].x : 0, x = ok ? jb[k].y : 0;
    xs[k] = x;
    const int32_t bkt = min(max(x >> m.bshift, 0), m.nbk - 1);
    v[k] = ldg4(lines + ((int64_t)row * m.nbk + bkt) * (kLineInts / 4));
  }
  const bool first = sub == 0, last = sub == 3;
  uint32_t dn[4], dp[4];
  int32_t bad[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int32_t x = xs[k], xm = x - 1;
    uint32_t a = min(min(above_gap(v[k].x, x), above_gap(v[k].y, x)), min(above_gap(v[k].z, x), above_gap(v[k].w, x)));
    uint32_t c = min(min(below_gap(v[k].x, xm), below_gap(v[k].y, xm)), min(below_gap(v[k].z, xm), below_gap(v[k].w, xm)));
    int32_t f = (int32_t)((first & (v[k].x == kBucketOverflow)) | (last & (x >= v[k].w)));
    a = min(a, (uint32_t)dpp<kDppQuadXor1>((int32_t)a));
    c = min(c, (uint32_t)dpp<kDppQuadXor1>((int32_t)c));
    f = max(f, dpp<kDppQuadXor1>(f));
    a = min(a, (uint32_t)dpp<kDppQuadXor2>((int32_t)a));
    c = min(c, (uint32_t)dpp<kDppQuadXor2>((int32_t)c));
    f = max(f, dpp<kDppQuadXor2>(f));
    dn[k] = a;
    dp[k] = c;
    bad[k] = f;
  }
  const bool s1 = sub == 1, s2 = sub == 2;
  const uint32_t d1 = first ? dn[0] : s1 ? dn[1] : s2 ? dn[2] : dn[3];
  const uint32_t d2 = first ? dp[0] : s1 ? dp[1] : s2 ? dp[2] : dp[3];
  const int32_t f = first ? bad[0] : s1 ? bad[1] : s2 ? bad[2] : bad[3];
  const int32_t x = first ? xs[0] : s1 ? xs[1] : s2 ? xs[2] : xs[3];
  jo = b + 16 * sub + quad;
  const int32_t xm = x - 1;
  const int32_t nxt = has_above(d1, x) ? (int32_t)((uint32_t)x + 1u + d1) : INT_MAX;
  const int32_t prv = has_below(d2, xm) ? (int32_t)((uint32_t)xm - d2) : INT_MIN;
  rs = nxt != INT_MAX ? range_of((uint32_t)nxt - (uint32_t)x, max_range) : max_range;
  rp = prv != INT_MIN ? range_of((uint32_t)x - (uint32_t)prv, max_range) : max_range;
  if (f) rs = -1;
  return jo < njobs;
}

// quad_half_round for 16-bit bucket lines.  The first half holds the carried
// neighbours as bin centres (words 0 and 1) and the lowest 28 bin indices of
// the bucket (words 2..15, two per word).  The successor is the first key of
// bin >= ts; when the 28th index is >= ts (or is padding), it lies in the half
// and so do all keys of bin <= tp < ts, and the half settles the search as
// scan_bucket16 would.  The quad reduces the indices' unsigned gaps and takes
// the carried centres from its first lane.  All 64 lanes call.
__device__ __forceinline__ bool quad_half_round16(const MapDev& m, const int2* jobs, int32_t b, int32_t njobs,
                                                  int32_t max_range, int32_t& jo, int32_t& rs, int32_t& rp) {
  const int lane = threadIdx.x & (kWave - 1), sub = lane & 3, quad = lane >> 2;
  int4 v[4];
  int32_t xs[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int32_t j = b + 16 * k + quad;
    const int2 jb = j < njobs ? jobs[j] : make_int2(0, 0);
    xs[k] = jb.y;
    v[k] = make_int4(-1, -1, -1, -1);
    if (j < njobs)
      v[k] = ldg4(reinterpret_cast<const int4*>(m.bk + ((int64_t)jb.x * m.nbk + bucket_of(m, jb.y)) * kLineInts) +
                  sub);
  }
  uint32_t dsk[4], dpk[4];
  int32_t e0k[4], e1k[4], bad[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int32_t x = xs[k], base = bucket_of(m, x) << (m.bshift - kBinShift);
    const uint32_t ts = (uint32_t)(bin_min_above(x) - base), tp = (uint32_t)(bin_max_below(x) - base);
    // words 0 and 1 of the first lane are the carried centres, not indices: read as padding here
    const uint32_t w0 = sub == 0 ? 0xffffffffu : (uint32_t)v[k].x, w1 = sub == 0 ? 0xffffffffu : (uint32_t)v[k].y;
    const uint32_t w[4] = {w0, w1, (uint32_t)v[k].z, (uint32_t)v[k].w};
    uint32_t ds = 0xffffffffu, dp = 0xffffffffu;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const uint32_t lo = w[q] & 0xffffu, hi = w[q] >> 16;
      ds = min(ds, min(lo - ts, hi - ts));
      dp = min(dp, min(tp - lo, tp - hi));
    }
    int32_t f = (sub == 0 && v[k].x == kBucketOverflow) ||
                        (sub == 3 && !((int32_t)((uint32_t)v[k].w >> 16) >= (int32_t)ts))
                    ? 1
                    : 0;
    ds = min(ds, (uint32_t)dpp<kDppQuadXor1>((int32_t)ds));
    dp = min(dp, (uint32_t)dpp<kDppQuadXor1>((int32_t)dp));
    f = max(f, dpp<kDppQuadXor1>(f));
    ds = min(ds, (uint32_t)dpp<kDppQuadXor2>((int32_t)ds));
    dp = min(dp, (uint32_t)dpp<kDppQuadXor2>((int32_t)dp));
    f = max(f, dpp<kDppQuadXor2>(f));
    dsk[k] = ds;
    dpk[k] = dp;
    bad[k] = f;
    e0k[k] = dpp<kDppQuadBcast0>(v[k].x);
    e1k[k] = dpp<kDppQuadBcast0>(v[k].y);
  }
  const uint32_t ds = sub == 0 ? dsk[0] : sub == 1 ? dsk[1] : sub == 2 ? dsk[2] : dsk[3];
  const uint32_t dp = sub == 0 ? dpk[0] : sub == 1 ? dpk[1] : sub == 2 ? dpk[2] : dpk[3];
  const int32_t f = sub == 0 ? bad[0] : sub == 1 ? bad[1] : sub == 2 ? bad[2] : bad[3];
  const int32_t e0 = sub == 0 ? e0k[0] : sub == 1 ? e0k[1] : sub == 2 ? e0k[2] : e0k[3];
  const int32_t e1 = sub == 0 ? e1k[0] : sub == 1 ? e1k[1] : sub == 2 ? e1k[2] : e1k[3];
  const int32_t x = sub == 0 ? xs[0] : sub == 1 ? xs[1] : sub == 2 ? xs[2] : xs[3];
  jo = b + 16 * sub + quad;
  const int32_t base = bucket_of(m, x) << (m.bshift - kBinShift);
  const int32_t ts = bin_min_above(x) - base, tp = bin_max_below(x) - base;
  const int32_t s16 = ds < 0x80000000u ? ts + (int32_t)ds : 0xffff;
  const int32_t p16 = dp < 0x80000000u ? tp - (int32_t)dp : -1;
  const int32_t nxt = s16 != 0xffff ? bin_centre(base + s16) : e1;
  const int32_t prv = p16 >= 0 ? bin_centre(base + p16) : e0;
  rs = nxt != INT_MAX ? range_of((uint32_t)nxt - (uint32_t)x, max_range) : max_range;
  rp = prv != INT_MIN ? range_of((uint32_t)x - (uint32_t)prv, max_range) : max_range;
  if (f) rs = -1;
  return jo < njobs;
}

// Search strategy: K = 0 one lane per search, K >= 1 eight lanes per search
// with K searches per group in flight (maps with a bucket index always search
// one lane per bucket line).
template <int K, bool Z>
__device__ __forceinline__ void band_search(const MapDev& m, bool want, int32_t row, int32_t xq, int32_t max_range,
                                            int32_t& r_succ, int32_t& r_pred) {
  if constexpr (K == 0) {
    lane_search<Z>(m, want, row, xq, max_range, r_succ, r_pred);
  } else {
    if (m.bk)
      bucket_search<Z>(m, want, row, xq, max_range, r_succ, r_pred);
    else
      wave_search<K>(m, want, row, xq, max_range, r_succ, r_pred);
  }
}

// Plain casts for up to 64 rays, one per lane (Sec. IV-B).  All lanes call.
template <int K, bool Z>
__device__ __forceinline__ int32_t wave_cast(const MapDev& m, bool active, float x, float y, float theta,
                                             int32_t max_range) {
  // the query's cell is read while the search runs (an occupied cell gives 0)
  const bool valid = active && (fabsf(theta) < 1e6f) && pose_inside(m, x, y);
  int32_t xf = 0, yf = 0;
  uint8_t cell = 1;
  bool fwd = true;
  Landing l{0, 0};
  if (valid) {
    xf = quantize16(x);
    yf = quantize16(y);
    cell = ldg(m.occ + (size_t)(yf >> 16) * (size_t)m.w + (size_t)(xf >> 16));
    int32_t k = theta_bin(theta, m.k_scale, m.n);
    fwd = k < m.half;
    l = land(m, fwd ? k : k - m.half, xf, yf);
  }
  int32_t rs, rp;
  band_search<K, Z>(m, valid, l.row, l.xq, max_range, rs, rp);
  return valid && cell == 0 ? (fwd ? rs : rp) : 0;
}

// Log-weight of one particle, computed by all 64 lanes of a wave (lane = ray
// within a chunk of 64 rays).  Every lane returns the same value.  The sum is
// float32: each lane accumulates its rays in chunk order, then wave_sum adds
// the lanes in a fixed order, so the bits depend only on n_rays.
//
// Radial pairing (Sec. IV-C): if pair_off > 0, lane l + pair_off reuses the
// search of lane l when both rays land in the same slice (their bins differ by
// n/2): every search returns both the successor and the predecessor.
// Sys: observations are read system-coherently (ldx).
template <int K, bool Z, bool Sys = false>
__device__ __forceinline__ float wave_particle_logw(const MapDev& m, float px, float py, float pth,
                                                    const float* __restrict__ offsets,
                                                    const int32_t* __restrict__ obs, int32_t n_rays,
                                                    int32_t pair_off, const float* __restrict__ table,
                                                    int32_t max_range, int32_t* __restrict__ ranges_row) {
  const int lane = threadIdx.x & (kWave - 1);
  const int32_t m1 = max_range + 1;
  // The pose's cell is read while the searches run: the searches assume a
  // free cell, and an occupied one zeroes the ranges afterwards (the same for
  // the whole wave, so the pairing below is unaffected).
  const bool inside = pose_inside(m, px, py);
  int32_t xf = 0, yf = 0;
  uint8_t cell = 1;
  if (inside) {
    xf = quantize16(px);
    yf = quantize16(py);
    cell = ldg(m.occ + (size_t)(yf >> 16) * (size_t)m.w + (size_t)(xf >> 16));
  }
  float acc = 0.0f;
  for (int32_t base = 0; base < n_rays; base += kWave) {
    const int32_t r = base + lane;
    const bool active = r < n_rays;
    float th = active ? __fadd_rn(pth, ldg(offsets + r)) : 0.0f;
    bool valid = active && inside && (fabsf(th) < 1e6f);
    int32_t slice = 0;
    bool fwd = true;
    if (valid) {
      int32_t k = theta_bin(th, m.k_scale, m.n);
      fwd = k < m.half;
      slice = fwd ? k : k - m.half;
    }
    // Pairing: does my partner below (lane - P) share my slice?
    bool paired = false;
    int src_c = lane;
    if (pair_off > 0) {
      const int src = lane - pair_off;
      src_c = src >= 0 ? src : lane;
      const int32_t ps = __shfl(valid ? slice : -1, src_c);  // partner's slice, -1 if it casts nothing
      const bool cand = src >= 0 && valid && ps == slice;
      // a partner that itself reuses a search does not search: no chains
      const int pc = __shfl(cand ? 1 : 0, src_c);
      paired = cand && !pc;
    }
    Landing l{0, 0};
    if (valid && !paired) l = land(m, slice, xf, yf);
    int32_t rs, rp;
    band_search<K, Z>(m, valid && !paired, l.row, l.xq, max_range, rs, rp);
    const int32_t opk = __shfl(rs | (rp << 16), src_c);  // partner's (successor, predecessor) ranges
    int32_t range = 0;
    if (valid && cell == 0)
      range = paired ? (fwd ? (opk & 0xffff) : (int32_t)((uint32_t)opk >> 16)) : (fwd ? rs : rp);
    if (active) {
      int32_t zo = ldx<Sys>(obs + r);
      zo = zo < 0 ? 0 : (zo > max_range ? max_range : zo);
      acc += ldg(table + (int64_t)zo * m1 + range);
      if (ranges_row) stg(ranges_row + r, range);
    }
  }
  return wave_sum(acc);
}

// Runs one wave's queued searches jobs[0, njobs) (band, Xq), one search per
// lane per round; each job's first word is replaced by its packed result
// (successor range | predecessor range << 16).  On maps with a bucket index
// a round reads only the first half of each line (quad_half_round, or
// quad_half_round16 for 16-bit lines); the searches it cannot settle are
// queued in `later` and run in full after the last round, so that a round
// never waits for a second line.  All 64 lanes call.
template <bool Z>
__device__ __forceinline__ void drain_jobs(const MapDev& m, int2* jobs, int32_t* later, int32_t njobs, int32_t M) {
  const int lane = threadIdx.x & (kWave - 1);
  const bool halves = m.bk != nullptr;  // the same for the whole wave
  int32_t nlater = 0;
  if (halves) {
    for (int32_t b = 0; b < njobs; b += kWave) {
      int32_t jo, rs, rp;
      bool wo;  // this lane's job jo and its result
      if (Z && m.zp16)
        wo = quad_half_round16(m, jobs, b, njobs, M, jo, rs, rp);
      else
        wo = quad_half_round(m, jobs, b, njobs, M, jo, rs, rp);
      const bool done = wo && rs >= 0;
      const bool defer = wo && rs < 0;
      const uint64_t dm = __ballot(defer);
      if (defer) later[nlater + __popcll(dm & ((1ull << lane) - 1ull))] = jo;
      nlater += __popcll(dm);
      if (done) jobs[jo].x = rs | (rp << 16);
    }
  } else {
    for (int32_t b = 0; b < njobs; b += kWave) {
      const int32_t j = b + lane;
      const bool w = j < njobs;
      const int2 jb = w ? jobs[j] : make_int2(0, 0);
      int32_t rs, rp;
      lane_search<Z>(m, w, jb.x, jb.y, M, rs, rp);
      if (w) jobs[j].x = rs | (rp << 16);
    }
  }
  __threadfence_block();
  for (int32_t b = 0; b < nlater; b += kWave) {  // the whole line, or the band's search lines
    const int32_t k = b + lane;
    const bool w = k < nlater;
    const int32_t j = w ? later[k] : 0;
    const int2 jb = w ? jobs[j] : make_int2(0, 0);
    int32_t rs, rp;
    lane_search<Z>(m, w, jb.x, jb.y, M, rs, rp);
    if (w) jobs[j].x = rs | (rp << 16);
  }
}

// Plain casts of rays [base, base + 64 Q) by one wave through the search queue
// (ray base + 64 q + lane in lane `lane`): the landings of all Q rays per lane
// are queued, drained by drain_jobs, and each result is picked as wave_cast
// picks it.  Same results as wave_cast.  jobs / codes / later: this wave's LDS
// slices of Q * 64 entries.  All 64 lanes call.
template <int Q, bool Z>
__device__ __forceinline__ void wave_cast_tile(const MapDev& m, const float* __restrict__ x,
                                               const float* __restrict__ y, const float* __restrict__ th,
                                               int64_t n, int64_t base, int32_t max_range, int32_t* __restrict__ out,
                                               int2* jobs, int32_t* codes, int32_t* later,
                                               int32_t* __restrict__ ticks = nullptr) {
  const int lane = threadIdx.x & (kWave - 1);
  const uint64_t t0 = ticks ? wall_clock64() : 0;
  int32_t njobs = 0;
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int64_t i = base + (int64_t)q * kWave + lane;
    const bool active = i < n;
    const float xi = active ? ldg(x + i) : 0.0f, yi = active ? ldg(y + i) : 0.0f, ti = active ? ldg(th + i) : 0.0f;
    bool valid = active && (fabsf(ti) < 1e6f) && pose_inside(m, xi, yi);
    int32_t xf = 0, yf = 0;
    if (valid) {
      xf = quantize16(xi);
      yf = quantize16(yi);
      valid = ldg(m.occ + (size_t)(yf >> 16) * (size_t)m.w + (size_t)(xf >> 16)) == 0;
    }
    bool fwd = true;
    Landing l{0, 0};
    if (valid) {
      const int32_t k = theta_bin(ti, m.k_scale, m.n);
      fwd = k < m.half;
      l = land(m, fwd ? k : k - m.half, xf, yf);
    }
    const uint64_t mask = __ballot(valid);
    const int32_t slot = njobs + __popcll(mask & ((1ull << lane) - 1ull));
    if (valid) jobs[slot] = make_int2(l.row, l.xq);
    codes[q * kWave + lane] = valid ? ((slot << 1) | (fwd ? 1 : 0)) : -1;
    njobs += __popcll(mask);
  }
  __threadfence_block();
  drain_jobs<Z>(m, jobs, later, njobs, max_range);
  __threadfence_block();
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int64_t i = base + (int64_t)q * kWave + lane;
    if (i < n) {
      const int32_t code = codes[q * kWave + lane];
      int32_t r = 0;
      if (code >= 0) {
        const int32_t pk = jobs[code >> 1].x;
        r = (code & 1) ? (pk & 0xffff) : (int32_t)((uint32_t)pk >> 16);
      }
      stg(out + i, r);
      if (ticks) stg(ticks + i, (int32_t)(wall_clock64() - t0));
    }
  }
}

// Log-weights of `cnt` (<= Q) consecutive particles by one wave, for ray
// layouts of at most 64 rays.  Same results as wave_particle_logw for each
// particle, computed in three phases so that one particle's chain of
// dependent reads (occupancy byte, header line, key line, table entry) does not
// serialise the wave:
//   A  lane q loads particle q's pose and occupancy byte (all Q at once);
//   B  each particle's rays (lane = ray) are binned and paired, and the rays
//      that search append (band, Xq) jobs to this wave's LDS queue; the queue
//      is then drained 64 jobs per round, one lane per search;
//   C  every ray reads its (or its partner's) result, the Q table gathers are
//      issued together, and each particle's sum is reduced in the fixed order.
// jobs / codes / later: this wave's LDS slices of Q * 64 entries (a job's
// first word is overwritten by its packed result).  With Lanes2 each lane
// runs two searches of a round side by side (128 searches per round).
// Otherwise the queue is drained by drain_jobs (half-line first pass on maps
// with a bucket index, deferred full searches).
// Sys: poses and observations are read, and log-weights written,
// system-coherently (ldx / stx).
template <int Q, int Lanes2, bool Z, bool Sys = false>
__device__ __forceinline__ void wave_tile_logw(const FilterDev& f, int64_t p0, int32_t cnt, int2* jobs,
                                               int32_t* codes, int32_t* later) {
  const int lane = threadIdx.x & (kWave - 1);
  const MapDev& m = f.map;
  const int32_t M = f.max_range, m1 = M + 1;
  // A: poses and the overlap check
  float qt = 0.0f;
  int32_t qxf = 0, qyf = 0, qok = 0;
  if (lane < cnt) {
    const float x = ldx<Sys>(f.px + p0 + lane), y = ldx<Sys>(f.py + p0 + lane);
    qt = ldx<Sys>(f.pth + p0 + lane);
    if (pose_inside(m, x, y)) {
      qxf = quantize16(x);
      qyf = quantize16(y);
      qok = ldg(m.occ + (size_t)(qyf >> 16) * (size_t)m.w + (size_t)(qxf >> 16)) == 0;
    }
  }
  const bool active = lane < f.n_rays;
  const float off = active ? ldg(f.offsets + lane) : 0.0f;
  int32_t zo = active ? ldx<Sys>(f.obs + lane) : 0;
  zo = zo < 0 ? 0 : (zo > M ? M : zo);
  const int P = f.pair_offset;
  // B: bins, pairing and the search queue
  // codes[q][lane]: -1 no cast (range 0); else (result slot << 1) | forward.
  // Kept in LDS rather than registers while the searches run.
  int32_t njobs = 0;
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    int32_t code = -1;
    if (q < cnt) {
      const float pth = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int32_t, qt), q));
      const int32_t xf = __builtin_amdgcn_readlane(qxf, q), yf = __builtin_amdgcn_readlane(qyf, q);
      const bool ok = __builtin_amdgcn_readlane(qok, q) != 0;
      const float th = active ? __fadd_rn(pth, off) : 0.0f;
      const bool valid = active && ok && (fabsf(th) < 1e6f);
      int32_t slice = 0;
      bool fwd = true;
      if (valid) {
        const int32_t k = theta_bin(th, m.k_scale, m.n);
        fwd = k < m.half;
        slice = fwd ? k : k - m.half;
      }
      bool paired = false;
      int src_c = lane;
      if (P > 0) {
        const int src = lane - P;
        src_c = src >= 0 ? src : lane;
        const int32_t ps = __shfl(valid ? slice : -1, src_c);
        const bool cand = src >= 0 && valid && ps == slice;
        const int pc = __shfl(cand ? 1 : 0, src_c);
        paired = cand && !pc;
      }
      const bool want = valid && !paired;
      const uint64_t mask = __ballot(want);
      const int32_t slot = njobs + __popcll(mask & ((1ull << lane) - 1ull));
      if (want) {
        const Landing l = land(m, slice, xf, yf);
        jobs[slot] = make_int2(l.row, l.xq);
      }
      const int32_t pslot = __shfl(slot, src_c);
      if (valid) code = ((paired ? pslot : slot) << 1) | (fwd ? 1 : 0);
      njobs += __popcll(mask);
    }
    codes[q * kWave + lane] = code;
  }
  __threadfence_block();
  if constexpr (Lanes2) {  // two searches per lane per round
    for (int32_t b = 0; b < njobs; b += 2 * kWave) {
      const int32_t ja = b + lane, jb = b + kWave + lane;
      const bool wa = ja < njobs, wb = jb < njobs;
      const int2 qa = wa ? jobs[ja] : make_int2(0, 0);
      const int2 qb = wb ? jobs[jb] : make_int2(0, 0);
      int32_t sa, pa, sb, pb;
      lane_search2<Z>(m, wa, qa.x, qa.y, wb, qb.x, qb.y, M, sa, pa, sb, pb);
      if (wa) jobs[ja].x = sa | (pa << 16);  // the result replaces its job
      if (wb) jobs[jb].x = sb | (pb << 16);
    }
  } else {
    drain_jobs<Z>(m, jobs, later, njobs, M);
  }
  __threadfence_block();
  // C: table gathers, then one fixed-order sum per particle
  float tv[Q];
  int32_t rg[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    tv[q] = 0.0f;
    rg[q] = 0;
    if (q < cnt && active) {
      const int32_t code = codes[q * kWave + lane];
      if (code >= 0) {
        const int32_t pk = jobs[code >> 1].x;
        rg[q] = (code & 1) ? (pk & 0xffff) : (int32_t)((uint32_t)pk >> 16);
      }
      tv[q] = ldg(f.table + (int64_t)zo * m1 + rg[q]);
    }
  }
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    if (q < cnt) {
      if (f.ranges && active) stg(f.ranges + (p0 + q) * f.n_rays + lane, rg[q]);
      const float lw = wave_sum(tv[q]);
      if (lane == 0) stx<Sys>(f.logw + p0 + q, lw);
    }
  }
}

}  // namespace cddt
