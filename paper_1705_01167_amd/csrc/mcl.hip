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
//   k_resample   one workgroup per filter: the largest finite log-weight, the
//                integer weights q = floor(2^20 exp(l - max)) and their total,
//                then a chunked exclusive scan of q gives every particle its
//                first output slot; the slot array is max-scanned into the
//                source index of every output, and the poses are gathered.
//                After the weights everything is integer arithmetic, so the
//                result is independent of the order of the scan.
//
// exp, sin and cos come from range reduction and Taylor series in a fixed
// order of IEEE double operations (below), so the results are the same bits
// on any implementation that performs the same operations.
#include <algorithm>
#include <climits>

#include "cddt_common.h"

namespace cddt {
namespace {

constexpr double kLog2e = 1.4426950408889634;
constexpr double kLn2 = 0.6931471805599453;
constexpr double kPio2Hi = 1.5707963267948966;
constexpr double kPio2Lo = 6.123233995736766e-17;
constexpr double kTwoOverPi = 0.6366197723675814;
constexpr double kPi = 3.141592653589793;
constexpr double kTwoPi = 6.283185307179586;
constexpr int kResampleThreads = 1024;
constexpr int kMotionThreads = 256;

// e^x for x <= 0 (0 below -64 and for NaN): x log2 e = k + f, e^(f ln 2) by
// the Taylor series to degree 15 (nested), scaled by 2^k.
__device__ double exp_neg(double x) {
  if (!(x >= -64.0)) return 0.0;
  const double y = x * kLog2e;
  const double k = floor(y);
  const double t = (y - k) * kLn2;
  double p = 1.0;
  for (int n = 15; n >= 1; --n) p = 1.0 + (t / (double)n) * p;
  return ldexp(p, (int)k);
}

// sin and cos by quadrant reduction with a two-part pi/2 and Taylor series in
// r^2 (to r^21 / r^20, nested).
__device__ void sin_cos(double a, double& s_out, double& c_out) {
  const double k = floor(a * kTwoOverPi + 0.5);
  const double r = (a - k * kPio2Hi) - k * kPio2Lo;
  const double r2 = r * r;
  double qs = 1.0, qc = 1.0;
  for (int n = 10; n >= 1; --n) {
    qs = 1.0 - (r2 / (double)((2 * n) * (2 * n + 1))) * qs;
    qc = 1.0 - (r2 / (double)((2 * n - 1) * (2 * n))) * qc;
  }
  const double sr = r * qs, cr = qc;
  const long long kq = (long long)k;
  const int quad = (int)(((kq % 4) + 4) % 4);
  if (quad == 0) {
    s_out = sr;
    c_out = cr;
  } else if (quad == 1) {
    s_out = cr;
    c_out = -sr;
  } else if (quad == 2) {
    s_out = -sr;
    c_out = -cr;
  } else {
    s_out = -cr;
    c_out = sr;
  }
}

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
// Workgroup reductions and scans (kResampleThreads threads)
// ---------------------------------------------------------------------------
struct ResampleShared {
  unsigned long long s64[kResampleThreads];
  int32_t s32[kResampleThreads];
  float f32[kResampleThreads];
};

__device__ unsigned long long block_sum_u64(unsigned long long v, ResampleShared& sh) {
  sh.s64[threadIdx.x] = v;
  __syncthreads();
  for (int w = kResampleThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh.s64[threadIdx.x] += sh.s64[threadIdx.x + w];
    __syncthreads();
  }
  const unsigned long long r = sh.s64[0];
  __syncthreads();
  return r;
}

// Exclusive prefix sum over the block; *total gets the block's sum.
__device__ unsigned long long block_exscan_u64(unsigned long long v, ResampleShared& sh, unsigned long long* total) {
  sh.s64[threadIdx.x] = v;
  __syncthreads();
  for (int d = 1; d < kResampleThreads; d <<= 1) {
    const unsigned long long add = (int)threadIdx.x >= d ? sh.s64[threadIdx.x - d] : 0ull;
    __syncthreads();
    sh.s64[threadIdx.x] += add;
    __syncthreads();
  }
  const unsigned long long incl = sh.s64[threadIdx.x];
  *total = sh.s64[kResampleThreads - 1];
  __syncthreads();
  return incl - v;
}

__device__ int32_t block_inclusive_max_i32(int32_t v, ResampleShared& sh, int32_t* last) {
  sh.s32[threadIdx.x] = v;
  __syncthreads();
  for (int d = 1; d < kResampleThreads; d <<= 1) {
    const int32_t o = (int)threadIdx.x >= d ? sh.s32[threadIdx.x - d] : INT_MIN;
    __syncthreads();
    sh.s32[threadIdx.x] = max(sh.s32[threadIdx.x], o);
    __syncthreads();
  }
  const int32_t r = sh.s32[threadIdx.x];
  *last = sh.s32[kResampleThreads - 1];
  __syncthreads();
  return r;
}

// (largest finite value, whether there is one) over the block.
__device__ float block_max_finite(float v, bool ok, ResampleShared& sh, bool* any) {
  sh.f32[threadIdx.x] = ok ? v : -INFINITY;
  sh.s32[threadIdx.x] = ok ? 1 : 0;
  __syncthreads();
  for (int w = kResampleThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      sh.f32[threadIdx.x] = fmaxf(sh.f32[threadIdx.x], sh.f32[threadIdx.x + w]);
      sh.s32[threadIdx.x] |= sh.s32[threadIdx.x + w];
    }
    __syncthreads();
  }
  const float r = sh.f32[0];
  *any = sh.s32[0] != 0;
  __syncthreads();
  return r;
}

__device__ __forceinline__ unsigned long long weight_q(float l, bool any, float m) {
  if (!any) return 1ull;
  if (!isfinite(l)) return 0ull;
  return (unsigned long long)floor(exp_neg((double)l - (double)m) * 1048576.0);
}

// First output slot of cumulative weight c: ceil((n c - s) / T), 0 when n c <= s.
__device__ __forceinline__ int64_t first_slot(unsigned long long n, unsigned long long c, unsigned long long s,
                                              unsigned long long T) {
  const unsigned long long num = n * c;
  return num <= s ? 0 : (int64_t)((num - s + T - 1) / T);
}

// Systematic resampling of one filter by one workgroup.  Reads logw and the
// poses in (ix, iy, it); writes idx (n) and the gathered poses to (ox, oy, ot).
// With stage != nullptr the poses are first copied there and gathered from it,
// so (ix, iy, it) may equal (ox, oy, ot).
__device__ void resample_block(const float* __restrict__ logw, int64_t n, uint32_t u, const float* ix,
                               const float* iy, const float* it, float* ox, float* oy, float* ot, int32_t* idx,
                               float* stage, ResampleShared& sh) {
  const int tid = threadIdx.x;
  if (n <= 0) return;
  // 1. largest finite log-weight; optional staging copy; clear the slot marks
  float m = -INFINITY;
  bool mine = false;
  for (int64_t i = tid; i < n; i += kResampleThreads) {
    const float l = logw[i];
    if (isfinite(l) && (!mine || l > m)) {
      m = l;
      mine = true;
    }
    idx[i] = -1;
    if (stage) {
      stage[i] = ix[i];
      stage[n + i] = iy[i];
      stage[2 * n + i] = it[i];
    }
  }
  bool any = false;
  m = block_max_finite(m, mine, sh, &any);
  // 2. total integer weight
  unsigned long long part = 0;
  for (int64_t i = tid; i < n; i += kResampleThreads) part += weight_q(logw[i], any, m);
  const unsigned long long T = block_sum_u64(part, sh);
  const unsigned long long s = ((unsigned long long)(u >> 12) * T) >> 20;
  // 3. first output slot of every particle with copies (chunks of the block size, running carry)
  unsigned long long carry = 0;
  for (int64_t c0 = 0; c0 < n; c0 += kResampleThreads) {
    const int64_t i = c0 + tid;
    const unsigned long long q = i < n ? weight_q(logw[i], any, m) : 0ull;
    unsigned long long chunk = 0;
    const unsigned long long before = carry + block_exscan_u64(q, sh, &chunk);
    if (i < n && q > 0) {
      const int64_t a0 = first_slot((unsigned long long)n, before, s, T);
      int64_t a1 = first_slot((unsigned long long)n, before + q, s, T);
      if (a1 > n) a1 = n;
      if (a0 < a1) idx[a0] = (int32_t)i;
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
  for (int64_t c0 = 0; c0 < n; c0 += kResampleThreads) {
    const int64_t j = c0 + tid;
    const int32_t v = j < n ? idx[j] : -1;
    int32_t last = -1;
    int32_t k = block_inclusive_max_i32(v, sh, &last);
    k = max(k, run);
    run = max(run, last);
    k = k < 0 ? 0 : k;  // slot 0 is always marked (T > 0); kept in bounds regardless
    if (j < n) {
      idx[j] = k;
      ox[j] = gx[k];
      oy[j] = gy[k];
      ot[j] = gt[k];
    }
  }
}

__global__ __launch_bounds__(kResampleThreads) void k_resample(const float* __restrict__ logw, int64_t n, uint32_t u,
                                                               const float* ix, const float* iy, const float* it,
                                                               float* ox, float* oy, float* ot, int32_t* idx) {
  __shared__ ResampleShared sh;
  resample_block(logw, n, u, ix, iy, it, ox, oy, ot, idx, nullptr, sh);
}

// Many filters, one workgroup each, in place: stage holds 3 pre[f] + ...
// floats of scratch per filter and idx pre[f] + ... ints.
__global__ __launch_bounds__(kResampleThreads) void k_resample_many(const FilterDev* __restrict__ filters,
                                                                    const int64_t* __restrict__ pre,
                                                                    const uint32_t* __restrict__ u, float* stage,
                                                                    int32_t* idx) {
  __shared__ ResampleShared sh;
  const int32_t f = blockIdx.x;
  const FilterDev& fd = filters[f];
  float* px = const_cast<float*>(fd.px);
  float* py = const_cast<float*>(fd.py);
  float* pt = const_cast<float*>(fd.pth);
  resample_block(fd.logw, fd.n_particles, u[f], px, py, pt, px, py, pt, idx + pre[f], stage + 3 * pre[f], sh);
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

cddt_status launch_resample_many(const FilterDev* d_filters, const int64_t* d_pre, int32_t nf,
                                 const uint32_t* d_u, float* d_stage, int32_t* d_idx, hipStream_t st) {
  if (nf <= 0) return CDDT_OK;
  hipLaunchKernelGGL(k_resample_many, dim3((unsigned)nf), dim3(kResampleThreads), 0, st, d_filters, d_pre, d_u,
                     d_stage, d_idx);
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
