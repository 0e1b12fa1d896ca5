// Device-side CDDT query: bin selection, projection into a slice, band search
// and the per-particle beam log-weight.  Shared by the plain cast kernel, the
// per-filter weight kernel and the persistent batched kernel, so every entry
// point produces identical bits.
//
// Method: Sec. IV-B (project the query, take its band, successor search,
// difference), Sec. IV-C (bins k >= n/2 search the same band backwards; the
// overlap check on the full grid; opposite rays share one search), Sec. VI
// (beam-model log-likelihood summed over the rays of a particle).
#pragma once

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

// First index in a[0, len) whose value is > key (number of values <= key).
__device__ __forceinline__ int32_t upper_bound_i32(const int32_t* __restrict__ a, int32_t len,
                                                   int32_t key) {
  int32_t lo = 0, cnt = len;
  while (cnt > 0) {
    int32_t half = cnt >> 1;
    int32_t v = a[lo + half];
    if (v <= key) {
      lo += half + 1;
      cnt -= half + 1;
    } else {
      cnt = half;
    }
  }
  return lo;
}

// First index in a[0, len) whose value is >= key (number of values < key).
__device__ __forceinline__ int32_t lower_bound_i32(const int32_t* __restrict__ a, int32_t len,
                                                   int32_t key) {
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

// One ray, one lane (Sec. IV-B).
__device__ __forceinline__ int32_t cast_one(const MapDev& m, float x, float y, float theta,
                                            int32_t max_range) {
  if (!(fabsf(theta) < 1e6f)) return 0;
  if (!pose_inside(m, x, y)) return 0;
  int32_t xf = quantize16(x), yf = quantize16(y);
  if (m.occ[(size_t)(yf >> 16) * (size_t)m.w + (size_t)(xf >> 16)] != 0) return 0;
  int32_t k = theta_bin(theta, m.k_scale, m.n);
  bool fwd = k < m.half;
  Landing l = land(m, fwd ? k : k - m.half, xf, yf);
  int2 hd = m.hdr[l.row];
  const int32_t* z = m.zeros + (uint32_t)hd.x;
  if (fwd) {
    int32_t i = upper_bound_i32(z, hd.y, l.xq);
    return i < hd.y ? range_of((int64_t)z[i] - l.xq, max_range) : max_range;
  }
  int32_t i = lower_bound_i32(z, hd.y, l.xq);
  return i > 0 ? range_of((int64_t)l.xq - z[i - 1], max_range) : max_range;
}

// Log-weight of one particle, computed by all 64 lanes of a wave (lane = ray
// within a chunk of 64 rays).  Every lane returns the same value.  The sum is
// float32: each lane accumulates its rays in chunk order, then a fixed xor
// butterfly adds the lanes, so the bits depend only on n_rays.
//
// Radial pairing (Sec. IV-C): if pair_off > 0, lane l + pair_off reuses the
// search of lane l when both rays land in the same slice (their bins differ by
// n/2): one upper bound gives the successor for one direction and, at index
// i - 1 (after skipping values equal to Xq), the predecessor for the other.
__device__ __forceinline__ float wave_particle_logw(const MapDev& m, float px, float py, float pth,
                                                    const float* __restrict__ offsets,
                                                    const int32_t* __restrict__ obs, int32_t n_rays,
                                                    int32_t pair_off,
                                                    const float* __restrict__ table,
                                                    int32_t max_range,
                                                    int32_t* __restrict__ ranges_row) {
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
    // Pairing: does my partner below (lane - P) share my slice?  Does the
    // lane above (lane + P) reuse my search?
    bool paired = false, serve_up = false;
    if (pair_off > 0) {
      int src = lane - pair_off;
      int src_c = src >= 0 ? src : lane;
      int32_t ps = __shfl(slice, src_c);
      int pv = __shfl(valid ? 1 : 0, src_c);
      bool cand = src >= 0 && valid && pv && ps == slice;
      // a partner that itself reuses a search does not search: no chains
      int pc = __shfl(cand ? 1 : 0, src_c);
      paired = cand && !pc;
      int dst = lane + pair_off;
      int up = __shfl(paired ? 1 : 0, dst < kWave ? dst : lane);
      serve_up = dst < kWave && up;
    }
    int32_t r_succ = max_range, r_pred = max_range;
    if (valid && !paired) {
      Landing l = land(m, slice, xf, yf);
      int2 hd = m.hdr[l.row];
      const int32_t* z = m.zeros + (uint32_t)hd.x;
      const bool want_succ = fwd || serve_up;
      const bool want_pred = !fwd || serve_up;
      int32_t ub = 0, lb = 0;
      if (want_succ) {
        ub = upper_bound_i32(z, hd.y, l.xq);
        if (ub < hd.y) r_succ = range_of((int64_t)z[ub] - l.xq, max_range);
        if (want_pred) {
          lb = ub;
          if (ub > 0 && z[ub - 1] == l.xq) lb = lower_bound_i32(z, ub, l.xq);
        }
      } else {
        lb = lower_bound_i32(z, hd.y, l.xq);
      }
      if (want_pred && lb > 0) r_pred = range_of((int64_t)l.xq - z[lb - 1], max_range);
    }
    int32_t got_succ = r_succ, got_pred = r_pred;
    if (pair_off > 0) {
      int src = lane - pair_off;
      int src_c = src >= 0 ? src : lane;
      got_succ = __shfl(r_succ, src_c);
      got_pred = __shfl(r_pred, src_c);
    }
    int32_t range = 0;
    if (valid) {
      if (paired)
        range = fwd ? got_succ : got_pred;
      else
        range = fwd ? r_succ : r_pred;
    }
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
