// exp and sin/cos in a fixed order of IEEE double operations: range
// reduction, then Taylor series by Horner's rule, so the results are the same
// bits on any implementation that performs the same operations (the particle
// motion model, and the cell-walk comparator's ray directions).
#pragma once

#include <hip/hip_runtime.h>

namespace cddt {
namespace {

constexpr double kLog2e = 1.4426950408889634;
constexpr double kLn2 = 0.6931471805599453;
constexpr double kPio2Hi = 1.5707963267948966;
constexpr double kPio2Lo = 6.123233995736766e-17;
constexpr double kTwoOverPi = 0.6366197723675814;

// Taylor coefficients, the nearest doubles to 1/k! (exp), (-1)^n/(2n+1)! (sin)
// and (-1)^n/(2n)! (cos).
__constant__ const double kExpC[16] = {
    1.0, 1.0, 0.5, 0.16666666666666666,
    0.041666666666666664, 0.008333333333333333, 0.001388888888888889, 0.0001984126984126984,
    2.48015873015873e-05, 2.7557319223985893e-06, 2.755731922398589e-07, 2.505210838544172e-08,
    2.08767569878681e-09, 1.6059043836821613e-10, 1.1470745597729725e-11, 7.647163731819816e-13};
__constant__ const double kSinC[11] = {
    1.0, -0.16666666666666666, 0.008333333333333333, -0.0001984126984126984,
    2.7557319223985893e-06, -2.505210838544172e-08, 1.6059043836821613e-10, -7.647163731819816e-13,
    2.8114572543455206e-15, -8.22063524662433e-18, 1.9572941063391263e-20};
__constant__ const double kCosC[11] = {
    1.0, -0.5, 0.041666666666666664, -0.001388888888888889,
    2.48015873015873e-05, -2.755731922398589e-07, 2.08767569878681e-09, -1.1470745597729725e-11,
    4.779477332387385e-14, -1.5619206968586225e-16, 4.110317623312165e-19};

// e^x for x <= 0 (0 below -64 and for NaN): x log2 e = k + f, e^(f ln 2) by
// the Taylor series to degree 15 (Horner), scaled by 2^k.
__device__ double exp_neg(double x) {
  if (!(x >= -64.0)) return 0.0;
  const double y = x * kLog2e;
  const double k = floor(y);
  const double t = (y - k) * kLn2;
  double p = kExpC[15];
#pragma unroll
  for (int n = 14; n >= 0; --n) p = p * t + kExpC[n];
  return ldexp(p, (int)k);
}

// sin and cos by quadrant reduction with a two-part pi/2 and Taylor series in
// r^2 by Horner (to r^21 / r^20).
__device__ void sin_cos(double a, double& s_out, double& c_out) {
  const double k = floor(a * kTwoOverPi + 0.5);
  const double r = (a - k * kPio2Hi) - k * kPio2Lo;
  const double r2 = r * r;
  double qs = kSinC[10], qc = kCosC[10];
#pragma unroll
  for (int n = 9; n >= 0; --n) {
    qs = qs * r2 + kSinC[n];
    qc = qc * r2 + kCosC[n];
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

}  // namespace
}  // namespace cddt
