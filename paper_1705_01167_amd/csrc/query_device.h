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
  int32_t k = (int32_t)floorf(u) % n;
  return k < 0 ? k + n : k;
}

// First index in a[0, len) whose value is >= key (number of values < key).
__device__ __forceinline__ int32_t lower_bound_i32(const int32_t* __restrict__ a, int32_t len, int32_t key) {
  int32_t lo = 0, cnt = len;
  while (cnt > 0) {
    int32_t half = cnt >> 1;
    int32_t v = a[lo + half];
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
__device__ __forceinline__ int32_t range_of(int64_t d, int32_t max_range) {
  int64_t v = (d + 32768) >> 16;
  return v < (int64_t)max_range ? (int32_t)v : max_range;
}

// Where a valid query lands: along-ray coordinate and global band index.
struct Landing {
  int32_t xq;
  int32_t row;
};

__device__ __forceinline__ Landing land(const MapDev& m, int32_t slice, int32_t xf, int32_t yf) {
  SliceDev sl = m.slices[slice];
  int64_t along = (int64_t)xf * sl.c + (int64_t)yf * sl.s;
  int64_t lat = (int64_t)yf * sl.c - (int64_t)xf * sl.s;
  Landing l;
  l.xq = (int32_t)(along >> 30);
  l.row = sl.row_base + ((int32_t)(lat >> 46) - sl.row_min);
  return l;
}

// Sum / min / max over the 8 lanes of a search group (lanes 8g .. 8g+7).
__device__ __forceinline__ int32_t group_sum(int32_t v) {
  v += __shfl_xor(v, 1);
  v += __shfl_xor(v, 2);
  v += __shfl_xor(v, 4);
  return v;
}
__device__ __forceinline__ int32_t group_min(int32_t v) {
  v = min(v, __shfl_xor(v, 1));
  v = min(v, __shfl_xor(v, 2));
  v = min(v, __shfl_xor(v, 4));
  return v;
}
__device__ __forceinline__ int32_t group_max(int32_t v) {
  v = max(v, __shfl_xor(v, 1));
  v = max(v, __shfl_xor(v, 2));
  v = max(v, __shfl_xor(v, 4));
  return v;
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
  for (int base = 0; base < n; base += 8) {
    const int k = base + g;
    const bool act = k < n;
    const int src = __shfl(list, act ? k : 0);
    const int32_t qrow = __shfl(row, src);
    const int32_t x = __shfl(xq, src);
    int32_t gs = max_range, gp = max_range;
    if (act) {
      const int4* hn = reinterpret_cast<const int4*>(m.hdr + (int64_t)qrow * kNodeInts);
      const int4 h = hn[sub];
      const uint32_t start = (uint32_t)__shfl(h.x, lane & ~7);
      const int32_t len = __shfl(h.y, lane & ~7);
      const int32_t cap0 = __shfl(h.z, lane & ~7);
      // top level T: the smallest level with at most kTopEntries entries
      int32_t T = 0, nT = len;
      while (nT > kTopEntries) {
        nT = (nT + kLineInts - 1) >> kLineShift;
        ++T;
      }
      int32_t c, nxt, prv;
      {
        int32_t lc, ln, lp;
        scan4(h, sub, kHeaderWords, nT, x, lc, ln, lp);
        c = group_sum(lc);
        nxt = group_min(ln);
        prv = group_max(lp);
      }
      for (int32_t t = T - 1; t >= 0 && c > 0; --t) {
        const int32_t blk = c - 1;
        const int32_t nt = level_count(len, t);
        const int32_t valid = min(kLineInts, nt - blk * kLineInts);
        const int4* line = reinterpret_cast<const int4*>(m.zeros + level_base(start, cap0, t) + (uint32_t)blk * kLineInts);
        const int4 v = line[sub];
        int32_t lc, ln, lp;
        scan4(v, sub, 0, valid, x, lc, ln, lp);
        c = blk * kLineInts + group_sum(lc);
        const int32_t gn = group_min(ln);
        nxt = gn != INT_MAX ? gn : nxt;  // none in this block: the next block's first entry
        prv = group_max(lp);
      }
      // c = number of keys <= x; nxt = smallest key > x; prv = largest key <= x
      if (c < len) gs = range_of((int64_t)nxt - x, max_range);
      if (c > 0) {
        int32_t pv = prv;
        if (pv == x) {  // rare: x equals a key; find the last key strictly below it
          const int32_t lb = lower_bound_i32(m.zeros + start, c, x);
          pv = lb > 0 ? m.zeros[start + lb - 1] : INT_MIN;
        }
        if (pv != INT_MIN) gp = range_of((int64_t)x - pv, max_range);
      }
    }
    // hand results back: lanes whose rank falls in this pass pull from their group leader
    const int leader = (rank & 7) << 3;
    const int32_t ps = __shfl(gs, leader);
    const int32_t pp = __shfl(gp, leader);
    if (want && (rank >> 3) == (base >> 3)) {
      r_succ = ps;
      r_pred = pp;
    }
  }
}

// Plain casts for up to 64 rays, one per lane (Sec. IV-B).  All lanes call.
__device__ __forceinline__ int32_t wave_cast(const MapDev& m, bool active, float x, float y, float theta,
                                             int32_t max_range) {
  bool valid = active && (fabsf(theta) < 1e6f) && pose_inside(m, x, y);
  int32_t xf = 0, yf = 0;
  if (valid) {
    xf = quantize16(x);
    yf = quantize16(y);
    valid = m.occ[(size_t)(yf >> 16) * (size_t)m.w + (size_t)(xf >> 16)] == 0;
  }
  bool fwd = true;
  Landing l{0, 0};
  if (valid) {
    int32_t k = theta_bin(theta, m.k_scale, m.n);
    fwd = k < m.half;
    l = land(m, fwd ? k : k - m.half, xf, yf);
  }
  int32_t rs, rp;
  wave_search(m, valid, l.row, l.xq, max_range, rs, rp);
  return valid ? (fwd ? rs : rp) : 0;
}

// Log-weight of one particle, computed by all 64 lanes of a wave (lane = ray
// within a chunk of 64 rays).  Every lane returns the same value.  The sum is
// float32: each lane accumulates its rays in chunk order, then a fixed xor
// butterfly adds the lanes, so the bits depend only on n_rays.
//
// Radial pairing (Sec. IV-C): if pair_off > 0, lane l + pair_off reuses the
// search of lane l when both rays land in the same slice (their bins differ by
// n/2): every search returns both the successor and the predecessor.
__device__ __forceinline__ float wave_particle_logw(const MapDev& m, float px, float py, float pth,
                                                    const float* __restrict__ offsets,
                                                    const int32_t* __restrict__ obs, int32_t n_rays,
                                                    int32_t pair_off, const float* __restrict__ table,
                                                    int32_t max_range, int32_t* __restrict__ ranges_row) {
  const int lane = threadIdx.x & (kWave - 1);
  const int32_t m1 = max_range + 1;
  bool xy_ok = pose_inside(m, px, py);
  int32_t xf = 0, yf = 0;
  if (xy_ok) {
    xf = quantize16(px);
    yf = quantize16(py);
    xy_ok = m.occ[(size_t)(yf >> 16) * (size_t)m.w + (size_t)(xf >> 16)] == 0;
  }
  float acc = 0.0f;
  for (int32_t base = 0; base < n_rays; base += kWave) {
    const int32_t r = base + lane;
    const bool active = r < n_rays;
    float th = active ? __fadd_rn(pth, offsets[r]) : 0.0f;
    bool valid = active && xy_ok && (fabsf(th) < 1e6f);
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
      const int32_t ps = __shfl(slice, src_c);
      const int pv = __shfl(valid ? 1 : 0, src_c);
      const bool cand = src >= 0 && valid && pv && ps == slice;
      // a partner that itself reuses a search does not search: no chains
      const int pc = __shfl(cand ? 1 : 0, src_c);
      paired = cand && !pc;
    }
    Landing l{0, 0};
    if (valid && !paired) l = land(m, slice, xf, yf);
    int32_t rs, rp;
    wave_search(m, valid && !paired, l.row, l.xq, max_range, rs, rp);
    const int32_t os = __shfl(rs, src_c);
    const int32_t op = __shfl(rp, src_c);
    int32_t range = 0;
    if (valid) range = paired ? (fwd ? os : op) : (fwd ? rs : rp);
    if (active) {
      int32_t zo = obs[r];
      zo = zo < 0 ? 0 : (zo > max_range ? max_range : zo);
      acc += table[(int64_t)zo * m1 + range];
      if (ranges_row) ranges_row[r] = range;
    }
  }
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
  return acc;
}

}  // namespace cddt
