// FP64 sine and cosine for the kernels' moderate arguments (|x| < 2^20).
// (sincos_2pi, sincos_tab512 and rsqrt_pos below: the pair-sum variants.)
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

// sin(2 pi t) and cos(2 pi t) for |t| < 2^50 (t in revolutions).  With
// n = rint(2 t) the remainder g = t - n / 2 is exact and |g| <= 1/4, so
// sin(2 pi t) = (-1)^n sin(2 pi g) and cos(2 pi t) = (-1)^n cos(2 pi g): one
// sign for both, no quadrant swap.  Taylor series in g: sin(2 pi g) through
// g^21 and cos(2 pi g) through g^22, truncation below 2e-18 on |g| <= 1/4
// (the coefficients (-1)^k (2 pi)^m / m! rounded to double).
__device__ __forceinline__ void sincos_2pi(double t, double* sp, double* cp) {
  const double n = rint(t + t);
  const double g = fma(n, -0.5, t);
  const double g2 = g * g;
  double ps = 0.0011309237482517963;
  ps = fma(ps, g2, -0.012031585942120627);
  ps = fma(ps, g2, 0.10422916220813984);
  ps = fma(ps, g2, -0.7181223017785006);
  ps = fma(ps, g2, 3.819952584848282);
  ps = fma(ps, g2, -15.09464257682299);
  ps = fma(ps, g2, 42.058693944897655);
  ps = fma(ps, g2, -76.70585975306139);
  ps = fma(ps, g2, 81.60524927607506);
  ps = fma(ps, g2, -41.34170224039976);
  ps = fma(ps, g2, 6.283185307179586);
  double pc = -0.0003229910672070978;
  pc = fma(pc, g2, 0.0037798342006800396);
  pc = fma(pc, g2, -0.03638284114254567);
  pc = fma(pc, g2, 0.28200596845579123);
  pc = fma(pc, g2, -1.714390711088672);
  pc = fma(pc, g2, 7.903536371318469);
  pc = fma(pc, g2, -26.4262567833744);
  pc = fma(pc, g2, 60.24464137187666);
  pc = fma(pc, g2, -85.45681720669373);
  pc = fma(pc, g2, 64.9393940226683);
  pc = fma(pc, g2, -19.739208802178716);
  pc = fma(pc, g2, 1.0);
  const int sgn = ((int)n & 1) << 31;
  const double S = g * ps;
  *sp = __hiloint2double(__double2hiint(S) ^ sgn, __double2loint(S));
  *cp = __hiloint2double(__double2hiint(pc) ^ sgn, __double2loint(pc));
}

// sin and cos of 2 pi u / 512 (u in 512ths of a revolution, |u| < 2^31) from
// a table of (sin, cos)(2 pi i / 512), i = 0..511: with m = rint(u) the
// remainder g = u - m is exact and |g| <= 1/2, so the Taylor series of
// sin(2 pi g / 512) through g^5 (the next term is below 7e-20) and of
// cos(2 pi g / 512) - 1 through g^4 (the next term is below 7.5e-17, under
// half a unit in the last place of 1) and the angle-addition formulas with
// the table entry of m mod 512 give both.  The coefficients are
// (-1)^k (2 pi / 512)^m / m! rounded to double; the error is a few units in
// the last place.
__device__ __forceinline__ void sincos_tab512(double u, const double2* tab, double* sp, double* cp) {
  const double m = rint(u);
  const double g = u - m;
  const double2 T = tab[(int)m & 511];
  const double g2 = g * g;
  const double S = g * fma(fma(g2, 2.3193606829202922e-12, -3.080196845561248e-07), g2, 0.01227184630308513);
  const double Cm1 = g2 * fma(g2, 9.44992556799382e-10, -7.529910584327208e-05);
  *sp = fma(T.x, Cm1, fma(T.y, S, T.x));
  *cp = fma(T.y, Cm1, fma(-T.x, S, T.y));
}

// The table for sincos_tab512: (sin, cos)(2 pi i / 512) in tab[i], filled by
// the `nthreads` threads of a workgroup (a barrier must follow before use).
__device__ __forceinline__ void fill_tab512(double2* tab, int tid, int nthreads) {
  for (int i = tid; i < 512; i += nthreads) {
    double s, c;
    sincos_2pi(i * (1.0 / 512.0), &s, &c);
    tab[i] = make_double2(s, c);
  }
}

// 1 / sqrt(x) for finite x > 0: the hardware estimate (relative error about
// 2^-23) and one third-order correction y (1 + e/2 + 3 e^2 / 8),
// e = 1 - x y^2, leaving an error of order e^3 (no special-case handling).
__device__ __forceinline__ double rsqrt_pos(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  const double e = fma(-(x * y), y, 1.0);
  return fma(y * e, fma(e, 0.375, 0.5), y);
}

}  // namespace qax
