/* Plain CPU reference for the particle-filter steps on either side of the
 * sensor model (test infrastructure only): the odometry motion model and
 * systematic resampling.  The paper names the steps of the Monte Carlo
 * localization update (move every particle by the odometry, weigh it with the
 * sensor model, resample by the belief; Sec. I and Sec. VI) without formulas;
 * the readings written out here are:
 *
 *   Motion.  Odometry (dx, dy, dth) is given in the robot frame; the caller
 *   draws the noise (ex, ey, eth) and passes it in.  In double precision,
 *     x' = ((x + cos(th) dx) - sin(th) dy) + ex
 *     y' = ((y + sin(th) dx) + cos(th) dy) + ey
 *     t' = (th + dth) + eth, wrapped to [-pi, pi) by t' - 2pi floor((t' + pi) / 2pi)
 *   each rounded once to float32.
 *
 *   Resampling (systematic, one uniform draw).  m = the largest finite
 *   log-weight; every particle gets the integer weight
 *     q_k = floor(2^20 exp(l_k - m))   (0 when l_k is not finite; all 1 when
 *                                      no l_k is finite),
 *   T = sum q_k, s = floor((u >> 12) T / 2^20) for the caller's 32-bit u, and
 *   particle k fills output slots [a_k, a_(k+1)) with
 *     a_k = ceil((n C_k - s) / T) clamped at 0,  C_k = q_0 + ... + q_(k-1).
 *   All of it is integer arithmetic once q is known, so the result does not
 *   depend on summation order.  (Equivalently: output j takes the first k
 *   whose cumulative weight n C_(k+1) exceeds s + j T.)
 *
 *   exp, sin and cos are evaluated by the functions below (range reduction
 *   and Taylor series by Horner's rule with the coefficients below, in a
 *   fixed order of IEEE double operations), so a
 *   second implementation that performs the same operations gets the same
 *   bits and takes the same integer decisions.
 *
 * Build: part of libcddt_ref.so (gcc -O2 -ffp-contract=off).
 */
#include <math.h>
#include <stdint.h>
#include <string.h>

#define MCL_LOG2E 1.4426950408889634
#define MCL_LN2 0.6931471805599453
#define MCL_PIO2_HI 1.5707963267948966
#define MCL_PIO2_LO 6.123233995736766e-17
#define MCL_TWO_OVER_PI 0.6366197723675814
#define MCL_PI 3.141592653589793
#define MCL_TWO_PI 6.283185307179586

/* Taylor coefficients: 1/k! (exp), (-1)^n/(2n+1)! (sin), (-1)^n/(2n)! (cos),
 * each the double nearest to the exact value. */
static const double kExpC[16] = {
    1.0, 1.0, 0.5, 0.16666666666666666,
    0.041666666666666664, 0.008333333333333333, 0.001388888888888889, 0.0001984126984126984,
    2.48015873015873e-05, 2.7557319223985893e-06, 2.755731922398589e-07, 2.505210838544172e-08,
    2.08767569878681e-09, 1.6059043836821613e-10, 1.1470745597729725e-11, 7.647163731819816e-13};
static const double kSinC[11] = {
    1.0, -0.16666666666666666, 0.008333333333333333, -0.0001984126984126984,
    2.7557319223985893e-06, -2.505210838544172e-08, 1.6059043836821613e-10, -7.647163731819816e-13,
    2.8114572543455206e-15, -8.22063524662433e-18, 1.9572941063391263e-20};
static const double kCosC[11] = {
    1.0, -0.5, 0.041666666666666664, -0.001388888888888889,
    2.48015873015873e-05, -2.755731922398589e-07, 2.08767569878681e-09, -1.1470745597729725e-11,
    4.779477332387385e-14, -1.5619206968586225e-16, 4.110317623312165e-19};

/* exp(x) for x <= 0: x log2(e) = k + f with k = floor, 2^f = e^(f ln 2) by
 * its Taylor series to degree 15 (Horner), times 2^k.  0 below -64. */
double ref_det_exp_neg(double x) {
  if (!(x >= -64.0)) return 0.0; /* also NaN and -inf */
  const double y = x * MCL_LOG2E;
  const double k = floor(y);
  const double t = (y - k) * MCL_LN2;
  double p = kExpC[15];
  for (int n = 14; n >= 0; --n) p = p * t + kExpC[n];
  return ldexp(p, (int)k);
}

/* sin and cos: a = k pi/2 + r with k = floor(a 2/pi + 1/2) and a two-part
 * pi/2, |r| <= about pi/4; Taylor series in r^2 by Horner (terms to r^21 and
 * r^20); the quadrant k mod 4 picks and signs the results. */
void ref_det_sincos(double a, double* s_out, double* c_out) {
  const double k = floor(a * MCL_TWO_OVER_PI + 0.5);
  const double r = (a - k * MCL_PIO2_HI) - k * MCL_PIO2_LO;
  const double r2 = r * r;
  double qs = kSinC[10], qc = kCosC[10];
  for (int n = 9; n >= 0; --n) {
    qs = qs * r2 + kSinC[n];
    qc = qc * r2 + kCosC[n];
  }
  const double sr = r * qs, cr = qc;
  const long long kq = (long long)k;
  const int quad = (int)(((kq % 4) + 4) % 4);
  switch (quad) {
    case 0: *s_out = sr; *c_out = cr; break;
    case 1: *s_out = cr; *c_out = -sr; break;
    case 2: *s_out = -sr; *c_out = -cr; break;
    default: *s_out = -cr; *c_out = sr; break;
  }
}

void ref_motion(const float* px, const float* py, const float* pth, int64_t n, float dx, float dy, float dth,
                const float* ex, const float* ey, const float* eth, float* ox, float* oy, float* oth) {
  for (int64_t i = 0; i < n; ++i) {
    double s, c;
    ref_det_sincos((double)pth[i], &s, &c);
    const double x = (((double)px[i] + c * (double)dx) - s * (double)dy) + (double)ex[i];
    const double y = (((double)py[i] + s * (double)dx) + c * (double)dy) + (double)ey[i];
    double t = ((double)pth[i] + (double)dth) + (double)eth[i];
    t = t - MCL_TWO_PI * floor((t + MCL_PI) / MCL_TWO_PI);
    ox[i] = (float)x;
    oy[i] = (float)y;
    oth[i] = (float)t;
  }
}

/* Integer weights q (n entries) from the log-weights; returns T. */
static uint64_t ref_quantize(const float* logw, int64_t n, uint64_t* q) {
  int any = 0;
  float m = 0.0f;
  for (int64_t i = 0; i < n; ++i) {
    if (isfinite(logw[i]) && (!any || logw[i] > m)) {
      m = logw[i];
      any = 1;
    }
  }
  uint64_t total = 0;
  for (int64_t i = 0; i < n; ++i) {
    if (!any) {
      q[i] = 1;
    } else if (!isfinite(logw[i])) {
      q[i] = 0;
    } else {
      q[i] = (uint64_t)floor(ref_det_exp_neg((double)logw[i] - (double)m) * 1048576.0);
    }
    total += q[i];
  }
  return total;
}

/* n <= 2^20.  idx[j] = source particle of output j; poses gathered into o*.
 * q is caller scratch of n entries.  Returns 0, or -1 for a bad n. */
int ref_resample(const float* logw, int64_t n, uint32_t u, const float* px, const float* py, const float* pth,
                 int32_t* idx, float* ox, float* oy, float* oth, uint64_t* q) {
  if (n < 0 || n > (1 << 20)) return -1;
  if (n == 0) return 0;
  const uint64_t T = ref_quantize(logw, n, q);
  const uint64_t s = ((uint64_t)(u >> 12) * T) >> 20;
  uint64_t C = 0;
  for (int64_t k = 0; k < n; ++k) {
    const uint64_t lo_num = (uint64_t)n * C, hi_num = (uint64_t)n * (C + q[k]);
    const uint64_t a0 = lo_num <= s ? 0 : (lo_num - s + T - 1) / T;
    uint64_t a1 = hi_num <= s ? 0 : (hi_num - s + T - 1) / T;
    if (a1 > (uint64_t)n) a1 = (uint64_t)n;
    for (uint64_t j = a0; j < a1; ++j) {
      idx[j] = (int32_t)k;
      ox[j] = px[k];
      oy[j] = py[k];
      oth[j] = pth[k];
    }
    C += q[k];
  }
  return 0;
}

/* The integer weights alone (for tests). */
uint64_t ref_resample_weights(const float* logw, int64_t n, uint64_t* q) { return ref_quantize(logw, n, q); }
