// FP64 sine and cosine for the kernels' moderate arguments (|x| < 2^20).
//
// Cody-Waite reduction x = q (pi/2) + r, |r| <= pi/4, with pi/2 split into
// three doubles (the products q * P_i are exact inside fused multiply-adds),
// followed by the Taylor series of sin (through r^17) and cos (through r^16),
// whose truncation errors are below 5e-17 on |r| <= pi/4, and the quadrant
// selection by q mod 4.
#pragma once

#include <hip/hip_runtime.h>

namespace qax {

__device__ __forceinline__ void sincos_cw(double x, double* sp, double* cp) {
  const double q = rint(x * 0.6366197723675814);   // 2/pi
  double r = fma(-q, 1.5707963267948966, x);         // pi/2 = P1 + P2 + P3
  r = fma(-q, 6.123233995736766e-17, r);
  r = fma(-q, -1.4973849048591698e-33, r);
  const double r2 = r * r;
  // sin r = r + r^3 (-1/3! + r^2 (1/5! - ... + r^2 / 17!))
  double ps = 2.8114572543455206e-15;
  ps = fma(ps, r2, -7.647163731819816e-13);
  ps = fma(ps, r2, 1.6059043836821613e-10);
  ps = fma(ps, r2, -2.505210838544172e-08);
  ps = fma(ps, r2, 2.7557319223985893e-06);
  ps = fma(ps, r2, -0.0001984126984126984);
  ps = fma(ps, r2, 0.008333333333333333);
  ps = fma(ps, r2, -0.16666666666666666);
  const double S = fma(r * r2, ps, r);
  // cos r = 1 + r^2 (-1/2! + r^2 (1/4! - ... + r^2 / 16!))
  double pc = 4.779477332387385e-14;
  pc = fma(pc, r2, -1.1470745597729725e-11);
  pc = fma(pc, r2, 2.08767569878681e-09);
  pc = fma(pc, r2, -2.755731922398589e-07);
  pc = fma(pc, r2, 2.48015873015873e-05);
  pc = fma(pc, r2, -0.001388888888888889);
  pc = fma(pc, r2, 0.041666666666666664);
  pc = fma(pc, r2, -0.5);
  const double C = fma(r2, pc, 1.0);
  const int n = (int)q;
  double s = (n & 1) ? C : S;
  double c = (n & 1) ? S : C;
  if (n & 2) s = -s;
  if ((n + 1) & 2) c = -c;
  *sp = s;
  *cp = c;
}

}  // namespace qax
