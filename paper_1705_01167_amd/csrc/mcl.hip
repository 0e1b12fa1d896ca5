// The particle-filter steps on either side of the sensor model: the odometry
// motion model and systematic resampling (the paper's Monte Carlo
// localization update moves, weighs and resamples the particles, Sec. I and
// Sec. VI; it gives no formulas, so the library fixes them as documented in
// cddt.h).
//
//   k_motion     one thread per particle: robot-frame odometry rotated by the
//                particle's heading plus caller-drawn noise, in double
//                precision, rounded once to float32; heading wrapped to
//                [-pi, pi).  Many filters in one launch (particle prefix).
//   k_resample   one workgroup for one filter: the largest finite log-weight, the
//                integer weights q = floor(2^20 exp(l - max)) and their total,
//                then a chunked exclusive scan of q gives every particle its
//                first output slot; the slot array is max-scanned into the
//                source index of every output, and the poses are gathered.
//                After the weights everything is integer arithmetic, so the
//                result is independent of the order of the scan.
//   k_rs_*       the same for many filters in segments of kResampleSegment
//                particles, one workgroup per segment (five launches).
//
// exp, sin and cos come from range reduction and Taylor series by Horner's
// rule in a fixed order of IEEE double operations (below), so the results are
// the same bits on any implementation that performs the same operations.
#include <algorithm>
#include <climits>

#include "cddt_common.h"
#include "det_math.h"

namespace cddt {
namespace {

constexpr double kPi = 3.141592653589793;
constexpr double kTwoPi = 6.283185307179586;
constexpr int kResampleThreads = 1024;
constexpr int kMotionThreads = 256;

__device__ __forceinline__ void move_one(float* px, float* py, float* pth, int64_t i, float dx, float dy, float dth,
                                         const float* ex, const float* ey, const float* et) {
  double s, c;
  const float th = pth[i];
  sin_cos((double)th, s, c);
  const double x = (((double)px[i] + c * (double)dx) - s * (double)dy) + (double)ex[i];
  const double y = (((double)py[i] + s * (double)dx) + c * (double)dy) + (double)ey[i];
  double t = ((double)th + (double)dth) + (double)et[i];
  t = t - kTwoPi * floor((t + kPi) / kTwoPi);
  px[i] = (float)x;
  py[i] = (float)y;
  pth[i] = (float)t;
}

// One filter: noise = [ex(n), ey(n), eth(n)].
__global__ void k_motion(float* px, float* py, float* pth, int64_t n, float dx, float dy, float dth,
                         const float* __restrict__ noise) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    move_one(px, py, pth, i, dx, dy, dth, noise, noise + n, noise + 2 * n);
}

// Many filters: particle g belongs to the filter f with pre[f] <= g < pre[f+1];
// its noise block starts at 3 pre[f]; odom holds (dx, dy, dth) per filter.
__global__ void k_motion_many(const FilterDev* __restrict__ filters, const int64_t* __restrict__ pre, int32_t nf,
                              const float* __restrict__ odom, const float* __restrict__ noise) {
  const int64_t total = pre[nf];
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < total; g += stride) {
    int32_t lo = 0, cnt = nf;  // last pre[lo] <= g
    while (cnt > 1) {
      const int32_t h = cnt >> 1;
      if (pre[lo + h] <= g) {
        lo += h;
        cnt -= h;
      } else {
        cnt = h;
      }
    }
    const FilterDev& f = filters[lo];
    const int64_t n = f.n_particles, i = g - pre[lo];
    const float* nz = noise + 3 * pre[lo];
    move_one(const_cast<float*>(f.px), const_cast<float*>(f.py), const_cast<float*>(f.pth), i, odom[3 * lo],
             odom[3 * lo + 1], odom[3 * lo + 2], nz, nz + n, nz + 2 * n);
  }
}

// ---------------------------------------------------------------------------
// Workgroup reductions and scans (kResampleThreads threads = 16 waves): a
// shuffle scan inside each wave, then one wave scans the 16 wave totals.
// ---------------------------------------------------------------------------
constexpr int kWaves = kResampleThreads / 64;
constexpr int kItems = 4;  // consecutive elements per thread in every pass
constexpr int kChunk = kResampleThreads * kItems;
static_assert(kChunk == kResampleSegment, "a resampling segment is one chunk of one workgroup");

struct ResampleShared {
  unsigned long long w64[kWaves];
  int32_t w32[kWaves];
  float wf[kWaves];
};

__device__ __forceinline__ unsigned long long wave_incl_scan_u64(unsigned long long x, int lane) {
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const unsigned long long y = __shfl_up(x, d, 64);
    if (lane >= d) x += y;
  }
  return x;
}

__device__ __forceinline__ int32_t wave_incl_max_i32(int32_t x, int lane) {
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int32_t y = __shfl_up(x, d, 64);
    if (lane >= d) x = max(x, y);
  }
  return x;
}

// Exclusive prefix sum over the block; *total gets the block's sum.
__device__ unsigned long long block_exscan_u64(unsigned long long v, ResampleShared& sh, unsigned long long* total) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const unsigned long long x = wave_incl_scan_u64(v, lane);
  if (lane == 63) sh.w64[wid] = x;
  __syncthreads();
  if (wid == 0) {
    unsigned long long w = lane < kWaves ? sh.w64[lane] : 0ull;
    w = wave_incl_scan_u64(w, lane);
    if (lane < kWaves) sh.w64[lane] = w;
  }
  __syncthreads();
  const unsigned long long before = wid > 0 ? sh.w64[wid - 1] : 0ull;
  *total = sh.w64[kWaves - 1];
  __syncthreads();
  return before + x - v;
}

__device__ unsigned long long block_sum_u64(unsigned long long v, ResampleShared& sh) {
  unsigned long long total = 0;
  (void)block_exscan_u64(v, sh, &total);
  return total;
}

// Exclusive running maximum over the block (INT_MIN for thread 0); *last
// gets the block's maximum.
__device__ int32_t block_excl_max_i32(int32_t v, ResampleShared& sh, int32_t* last) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int32_t x = wave_incl_max_i32(v, lane);
  int32_t ex = __shfl_up(x, 1, 64);
  if (lane == 0) ex = INT_MIN;
  if (lane == 63) sh.w32[wid] = x;
  __syncthreads();
  if (wid == 0) {
    int32_t w = lane < kWaves ? sh.w32[lane] : INT_MIN;
    w = wave_incl_max_i32(w, lane);
    if (lane < kWaves) sh.w32[lane] = w;
  }
  __syncthreads();
  if (wid > 0) ex = max(ex, sh.w32[wid - 1]);
  *last = sh.w32[kWaves - 1];
  __syncthreads();
  return ex;
}

// (largest finite value, whether there is one) over the block.
__device__ float block_max_finite(float v, bool ok, ResampleShared& sh, bool* any) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  float m = ok ? v : -INFINITY;
  int32_t a = ok ? 1 : 0;
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) {
    m = fmaxf(m, __shfl_xor(m, d, 64));
    a |= __shfl_xor(a, d, 64);
  }
  if (lane == 0) {
    sh.wf[wid] = m;
    sh.w32[wid] = a;
  }
  __syncthreads();
  float r = sh.wf[0];
  int32_t ra = sh.w32[0];
  for (int w = 1; w < kWaves; ++w) {
    r = fmaxf(r, sh.wf[w]);
    ra |= sh.w32[w];
  }
  *any = ra != 0;
  __syncthreads();
  return r;
}

__device__ __forceinline__ unsigned long long weight_q(float l, bool any, float m) {
  if (!any) return 1ull;
  if (!isfinite(l)) return 0ull;
  return (unsigned long long)floor(exp_neg((double)l - (double)m) * 1048576.0);
}

// First output slot of cumulative weight c: ceil((n c - s) / T), 0 when n c <= s.
// A double-precision estimate (inv_t = 1 / T) is corrected by exact integer
// products, so the result is the exact ceiling without a 64-bit division
// (n c <= 2^60, the estimate is off by at most one or two).
__device__ __forceinline__ int64_t first_slot(unsigned long long n, unsigned long long c, unsigned long long s,
                                              unsigned long long T, double inv_t) {
  const unsigned long long num = n * c;
  if (num <= s) return 0;
  const unsigned long long d = num - s;
  unsigned long long j = (unsigned long long)((double)d * inv_t);
  while (j * T < d) ++j;
  while (j > 0 && (j - 1) * T >= d) --j;
  return (int64_t)j;
}

// Systematic resampling of one filter by one workgroup.  Reads logw and the
// poses in (ix, iy, it); writes idx (n) and the gathered poses to (ox, oy, ot).
// With stage != nullptr the poses are first copied there and gathered from it,
// so (ix, iy, it) may equal (ox, oy, ot).  Scans run over chunks of kChunk
// elements, kItems consecutive ones per thread, with a running carry.
__device__ void resample_block(const float* __restrict__ logw, int64_t n, uint32_t u, const float* ix,
                               const float* iy, const float* it, float* ox, float* oy, float* ot, int32_t* idx,
                               float* stage, ResampleShared& sh) {
  const int tid = threadIdx.x;
  if (n <= 0) return;
  // 1. largest finite log-weight; optional staging copy; clear the slot marks
  // (kItems strided elements per thread per iteration, loads issued together)
  float m = -INFINITY;
  bool mine = false;
  for (int64_t c0 = 0; c0 < n; c0 += kChunk) {
    float l[kItems];
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
      const int64_t i = c0 + tid + (int64_t)k * kResampleThreads;
      l[k] = i < n ? logw[i] : NAN;
    }
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
      const int64_t i = c0 + tid + (int64_t)k * kResampleThreads;
      if (isfinite(l[k]) && (!mine || l[k] > m)) {
        m = l[k];
        mine = true;
      }
      if (i < n) {
        idx[i] = -1;
        if (stage) {
          stage[i] = ix[i];
          stage[n + i] = iy[i];
          stage[2 * n + i] = it[i];
        }
      }
    }
  }
  bool any = false;
  m = block_max_finite(m, mine, sh, &any);
  // 2. total integer weight
  unsigned long long part = 0;
  for (int64_t c0 = 0; c0 < n; c0 += kChunk) {
    float l[kItems];
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
      const int64_t i = c0 + tid + (int64_t)k * kResampleThreads;
      l[k] = i < n ? logw[i] : NAN;
    }
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
      const int64_t i = c0 + tid + (int64_t)k * kResampleThreads;
      part += i < n ? weight_q(l[k], any, m) : 0ull;
    }
  }
  const unsigned long long T = block_sum_u64(part, sh);
  const unsigned long long s = ((unsigned long long)(u >> 12) * T) >> 20;
  const double inv_t = 1.0 / (double)T;
  // 3. first output slot of every particle with copies
  unsigned long long carry = 0;
  for (int64_t c0 = 0; c0 < n; c0 += kChunk) {
    const int64_t i0 = c0 + (int64_t)tid * kItems;
    float l[kItems];
#pragma unroll
    for (int k = 0; k < kItems; ++k) l[k] = i0 + k < n ? logw[i0 + k] : NAN;
    uint32_t q[kItems];  // q <= 2^20
    unsigned long long local = 0;
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
      q[k] = i0 + k < n ? (uint32_t)weight_q(l[k], any, m) : 0u;
      local += q[k];
    }
    unsigned long long chunk = 0;
    unsigned long long before = carry + block_exscan_u64(local, sh, &chunk);
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
      if (q[k] > 0) {
        const int64_t a0 = first_slot((unsigned long long)n, before, s, T, inv_t);
        int64_t a1 = first_slot((unsigned long long)n, before + q[k], s, T, inv_t);
        if (a1 > n) a1 = n;
        if (a0 < a1) idx[a0] = (int32_t)(i0 + k);
      }
      before += q[k];
    }
    carry += chunk;
  }
  __threadfence_block();
  __syncthreads();
  // 4. every output takes the last marked particle at or before it, then the gather
  const float* gx = stage ? stage : ix;
  const float* gy = stage ? stage + n : iy;
  const float* gt = stage ? stage + 2 * n : it;
  int32_t run = -1;
  for (int64_t c0 = 0; c0 < n; c0 += kChunk) {
    const int64_t j0 = c0 + (int64_t)tid * kItems;
    int32_t v[kItems], local = -1;
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
      v[k] = j0 + k < n ? idx[j0 + k] : -1;
      local = max(local, v[k]);
    }
    int32_t last = -1;
    int32_t k_run = max(run, block_excl_max_i32(local, sh, &last));  // everything before this thread's items
    run = max(run, last);
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
      k_run = max(k_run, v[k]);
      const int32_t src = k_run < 0 ? 0 : k_run;  // slot 0 is always marked (T > 0); kept in bounds regardless
      if (j0 + k < n) {
        idx[j0 + k] = src;
        ox[j0 + k] = gx[src];
        oy[j0 + k] = gy[src];
        ot[j0 + k] = gt[src];
      }
    }
  }
}

__global__ __launch_bounds__(kResampleThreads) void k_resample(const float* __restrict__ logw, int64_t n, uint32_t u,
                                                               const float* ix, const float* iy, const float* it,
                                                               float* ox, float* oy, float* ot, int32_t* idx) {
  __shared__ ResampleShared sh;
  resample_block(logw, n, u, ix, iy, it, ox, oy, ot, idx, nullptr, sh);
}

// ---------------------------------------------------------------------------
// Many filters: the same resampling split into segments of kResampleSegment
// particles, one workgroup per segment and five launches, so large filters
// use many compute units.  Every segment recomputes what it needs from the
// per-segment partial results of its filter (at most 256 segments for 2^20
// particles), so the integer results are those of resample_block.
// ---------------------------------------------------------------------------
struct SegView {
  int32_t f;
  int64_t lo, hi, n;  // segment particles [lo, hi) of a filter of n
  int32_t first, last;  // the filter's segments [first, last)
};

__device__ __forceinline__ SegView seg_view(const FilterDev* filters, const ResampleSegs& sg, int32_t g) {
  SegView v;
  v.f = sg.seg_f[g];
  v.n = filters[v.f].n_particles;
  v.lo = sg.seg_lo[g];
  v.hi = min(v.n, v.lo + (int64_t)kResampleSegment);
  v.first = sg.fseg[v.f];
  v.last = sg.fseg[v.f + 1];
  return v;
}

__device__ __forceinline__ float filter_max(const ResampleSegs& sg, const SegView& v, bool* any) {
  float m = -INFINITY;
  bool a = false;
  for (int32_t h = v.first; h < v.last; ++h) {
    if (sg.seg_any[h]) {
      const float x = sg.seg_max[h];
      if (!a || x > m) m = x;
      a = true;
    }
  }
  *any = a;
  return m;
}

// 1. segment maxima; slot marks cleared; poses staged
__global__ __launch_bounds__(kResampleThreads) void k_rs_max(const FilterDev* __restrict__ filters,
                                                             const int64_t* __restrict__ pre, ResampleSegs sg,
                                                             float* stage, int32_t* idx) {
  __shared__ ResampleShared sh;
  const SegView v = seg_view(filters, sg, blockIdx.x);
  const FilterDev& fd = filters[v.f];
  const int64_t base = pre[v.f];
  float m = -INFINITY;
  bool mine = false;
#pragma unroll
  for (int k = 0; k < kItems; ++k) {
    const int64_t i = v.lo + threadIdx.x + (int64_t)k * kResampleThreads;
    if (i < v.hi) {
      const float l = fd.logw[i];
      if (isfinite(l) && (!mine || l > m)) {
        m = l;
        mine = true;
      }
      idx[base + i] = -1;
      float* st = stage + 3 * base;
      st[i] = fd.px[i];
      st[v.n + i] = fd.py[i];
      st[2 * v.n + i] = fd.pth[i];
    }
  }
  bool any = false;
  m = block_max_finite(m, mine, sh, &any);
  if (threadIdx.x == 0) {
    sg.seg_max[blockIdx.x] = m;
    sg.seg_any[blockIdx.x] = any ? 1 : 0;
  }
}

// 2. segment sums of the integer weights
__global__ __launch_bounds__(kResampleThreads) void k_rs_sum(const FilterDev* __restrict__ filters, ResampleSegs sg) {
  __shared__ ResampleShared sh;
  const SegView v = seg_view(filters, sg, blockIdx.x);
  const FilterDev& fd = filters[v.f];
  bool any = false;
  const float m = filter_max(sg, v, &any);
  unsigned long long part = 0;
#pragma unroll
  for (int k = 0; k < kItems; ++k) {
    const int64_t i = v.lo + threadIdx.x + (int64_t)k * kResampleThreads;
    if (i < v.hi) part += weight_q(fd.logw[i], any, m);
  }
  const unsigned long long t = block_sum_u64(part, sh);
  if (threadIdx.x == 0) sg.seg_sum[blockIdx.x] = t;
}

// 3. first output slot of every particle with copies
__global__ __launch_bounds__(kResampleThreads) void k_rs_mark(const FilterDev* __restrict__ filters,
                                                              const int64_t* __restrict__ pre,
                                                              const uint32_t* __restrict__ u, ResampleSegs sg,
                                                              int32_t* idx) {
  __shared__ ResampleShared sh;
  const int32_t g = blockIdx.x;
  const SegView v = seg_view(filters, sg, g);
  const FilterDev& fd = filters[v.f];
  bool any = false;
  const float m = filter_max(sg, v, &any);
  unsigned long long T = 0, carry = 0;
  for (int32_t h = v.first; h < v.last; ++h) {
    T += sg.seg_sum[h];
    if (h < g) carry += sg.seg_sum[h];
  }
  const unsigned long long s = ((unsigned long long)(u[v.f] >> 12) * T) >> 20;
  const double inv_t = 1.0 / (double)T;
  const int64_t i0 = v.lo + (int64_t)threadIdx.x * kItems;
  float l[kItems];
#pragma unroll
  for (int k = 0; k < kItems; ++k) l[k] = i0 + k < v.hi ? fd.logw[i0 + k] : NAN;
  uint32_t q[kItems];
  unsigned long long local = 0;
#pragma unroll
  for (int k = 0; k < kItems; ++k) {
    q[k] = i0 + k < v.hi ? (uint32_t)weight_q(l[k], any, m) : 0u;
    local += q[k];
  }
  unsigned long long chunk = 0;
  unsigned long long before = carry + block_exscan_u64(local, sh, &chunk);
  int32_t* fidx = idx + pre[v.f];
#pragma unroll
  for (int k = 0; k < kItems; ++k) {
    if (q[k] > 0) {
      const int64_t a0 = first_slot((unsigned long long)v.n, before, s, T, inv_t);
      int64_t a1 = first_slot((unsigned long long)v.n, before + q[k], s, T, inv_t);
      if (a1 > v.n) a1 = v.n;
      if (a0 < a1) fidx[a0] = (int32_t)(i0 + k);
    }
    before += q[k];
  }
}

// 4. largest mark in every output segment
__global__ __launch_bounds__(kResampleThreads) void k_rs_segmax(const FilterDev* __restrict__ filters,
                                                                const int64_t* __restrict__ pre, ResampleSegs sg,
                                                                const int32_t* __restrict__ idx) {
  __shared__ ResampleShared sh;
  const SegView v = seg_view(filters, sg, blockIdx.x);
  const int32_t* fidx = idx + pre[v.f];
  int32_t mx = -1;
#pragma unroll
  for (int k = 0; k < kItems; ++k) {
    const int64_t j = v.lo + threadIdx.x + (int64_t)k * kResampleThreads;
    if (j < v.hi) mx = max(mx, fidx[j]);
  }
  int32_t last = -1;
  (void)block_excl_max_i32(mx, sh, &last);
  if (threadIdx.x == 0) sg.seg_mmax[blockIdx.x] = last;
}

// 5. every output takes the last mark at or before it; poses gathered in place
__global__ __launch_bounds__(kResampleThreads) void k_rs_fill(const FilterDev* __restrict__ filters,
                                                              const int64_t* __restrict__ pre, ResampleSegs sg,
                                                              const float* __restrict__ stage, int32_t* idx) {
  __shared__ ResampleShared sh;
  const int32_t g = blockIdx.x;
  const SegView v = seg_view(filters, sg, g);
  const FilterDev& fd = filters[v.f];
  int32_t run = -1;
  for (int32_t h = v.first; h < g; ++h) run = max(run, sg.seg_mmax[h]);
  int32_t* fidx = idx + pre[v.f];
  const float* st = stage + 3 * pre[v.f];
  const int64_t j0 = v.lo + (int64_t)threadIdx.x * kItems;
  int32_t w[kItems], local = -1;
#pragma unroll
  for (int k = 0; k < kItems; ++k) {
    w[k] = j0 + k < v.hi ? fidx[j0 + k] : -1;
    local = max(local, w[k]);
  }
  int32_t last = -1;
  int32_t k_run = max(run, block_excl_max_i32(local, sh, &last));
  float* px = const_cast<float*>(fd.px);
  float* py = const_cast<float*>(fd.py);
  float* pt = const_cast<float*>(fd.pth);
#pragma unroll
  for (int k = 0; k < kItems; ++k) {
    k_run = max(k_run, w[k]);
    const int32_t src = k_run < 0 ? 0 : k_run;  // slot 0 is always marked (T > 0); kept in bounds regardless
    if (j0 + k < v.hi) {
      fidx[j0 + k] = src;
      px[j0 + k] = st[src];
      py[j0 + k] = st[v.n + src];
      pt[j0 + k] = st[2 * v.n + src];
    }
  }
}

}  // namespace

cddt_status launch_motion_many(const FilterDev* d_filters, const int64_t* d_pre, int32_t nf, int64_t total,
                               const float* d_odom, const float* d_noise, hipStream_t st) {
  if (total <= 0) return CDDT_OK;
  const int64_t blocks = std::min<int64_t>((total + kMotionThreads - 1) / kMotionThreads, 65536);
  hipLaunchKernelGGL(k_motion_many, dim3((unsigned)blocks), dim3(kMotionThreads), 0, st, d_filters, d_pre, nf,
                     d_odom, d_noise);
  CDDT_HIP(hipGetLastError());
  return CDDT_OK;
}

cddt_status launch_resample_many(const FilterDev* d_filters, const int64_t* d_pre, const uint32_t* d_u,
                                 float* d_stage, int32_t* d_idx, const ResampleSegs& segs, hipStream_t st) {
  if (segs.nseg <= 0) return CDDT_OK;
  const dim3 grid((unsigned)segs.nseg), block(kResampleThreads);
  hipLaunchKernelGGL(k_rs_max, grid, block, 0, st, d_filters, d_pre, segs, d_stage, d_idx);
  hipLaunchKernelGGL(k_rs_sum, grid, block, 0, st, d_filters, segs);
  hipLaunchKernelGGL(k_rs_mark, grid, block, 0, st, d_filters, d_pre, d_u, segs, d_idx);
  hipLaunchKernelGGL(k_rs_segmax, grid, block, 0, st, d_filters, d_pre, segs, (const int32_t*)d_idx);
  hipLaunchKernelGGL(k_rs_fill, grid, block, 0, st, d_filters, d_pre, segs, (const float*)d_stage, d_idx);
  CDDT_HIP(hipGetLastError());
  return CDDT_OK;
}

}  // namespace cddt

using namespace cddt;

extern "C" {

cddt_status cddt_motion(float* px, float* py, float* ptheta, int64_t n, float dx, float dy, float dtheta,
                        const float* noise, void* stream) {
  if (n < 0) return fail(CDDT_EINVAL, "cddt_motion: n < 0");
  if (n == 0) return CDDT_OK;
  if (!px || !py || !ptheta || !noise) return fail(CDDT_EINVAL, "cddt_motion: NULL array");
  const int64_t blocks = std::min<int64_t>((n + kMotionThreads - 1) / kMotionThreads, 65536);
  hipLaunchKernelGGL(k_motion, dim3((unsigned)blocks), dim3(kMotionThreads), 0, (hipStream_t)stream, px, py, ptheta,
                     n, dx, dy, dtheta, noise);
  CDDT_HIP(hipGetLastError());
  return CDDT_OK;
}

cddt_status cddt_resample(const float* logw, int64_t n, uint32_t u, const float* px, const float* py,
                          const float* ptheta, float* px_out, float* py_out, float* ptheta_out, int32_t* idx_out,
                          void* stream) {
  if (n < 0 || n > kMaxResample) return fail(CDDT_EINVAL, "cddt_resample: n must be in 0..2^20");
  if (n == 0) return CDDT_OK;
  if (!logw || !px || !py || !ptheta || !px_out || !py_out || !ptheta_out || !idx_out)
    return fail(CDDT_EINVAL, "cddt_resample: NULL array");
  hipLaunchKernelGGL(k_resample, dim3(1), dim3(kResampleThreads), 0, (hipStream_t)stream, logw, n, u, px, py, ptheta,
                     px_out, py_out, ptheta_out, idx_out);
  CDDT_HIP(hipGetLastError());
  return CDDT_OK;
}

}  // extern "C"
