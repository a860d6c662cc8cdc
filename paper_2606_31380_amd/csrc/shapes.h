// Generating curves of the supported bodies and their cancellation-free
// differences (device code).
//
// Surface (Section 2, equation para_quasi): (r cos th + p, r sin th + q, z).
// sphere / spheroid: r = a cos t, z = c sin t; peanut: polar radius
// rho(t) = a (1 - c cos 2t) (= a (1 + c cos 2 psi), psi the polar angle),
// r = rho cos t, z = rho sin t.  Bent centreline: circle of curvature kappa
// tangent to the z-axis, p = kappa z^2 / (1 + sqrt(1 - kappa^2 z^2)), q = 0.
#pragma once

#include <hip/hip_runtime.h>

#include "fastmath.h"

namespace qax {

struct Curve {
  double r, dr, z, dz, p, dp, q, dq;
};

// Curve at parameter t from st = sin t, ct = cos t.
__device__ __forceinline__ Curve curve_from_sincos(int shape, double a, double c, double kappa,
                                                   double st, double ct) {
  Curve o;
  if (shape == QAX_PEANUT) {
    const double s2 = 2.0 * st * ct, c2 = 1.0 - 2.0 * st * st;
    const double rho = a * (1.0 - c * c2);
    const double drho = 2.0 * a * c * s2;
    o.r = rho * ct;
    o.dr = drho * ct - rho * st;
    o.z = rho * st;
    o.dz = drho * st + rho * ct;
  } else {
    o.r = a * ct;
    o.dr = -a * st;
    o.z = c * st;
    o.dz = c * ct;
  }
  if (kappa != 0.0) {
    const double root = sqrt(1.0 - kappa * kappa * o.z * o.z);
    o.p = kappa * o.z * o.z / (1.0 + root);
    o.dp = kappa * o.z / root * o.dz;
  } else {
    o.p = 0.0;
    o.dp = 0.0;
  }
  o.q = 0.0;
  o.dq = 0.0;
  return o;
}

__device__ __forceinline__ Curve curve_eval(int shape, double a, double c, double kappa, double t) {
  double st, ct;
  sincos_cw(t, &st, &ct);
  return curve_from_sincos(shape, a, c, kappa, st, ct);
}

// Differences between the slice at s = t + dl and the slice at t, written with
// product-to-sum identities so they keep full relative accuracy as dl -> 0:
// d_r = r(s) - r(t), d_z = z(t) - z(s), d_p = p(t) - p(s), d_q = q(t) - q(s).
struct CurveDiff {
  double d_r, d_z, d_p, d_q;
};

// From sin/cos of t, s = t + dl, dl/2 and sig = t + dl/2.
__device__ __forceinline__ CurveDiff curve_diff_sc(int shape, double a, double c, double kappa,
                                                   double st, double ct, double ss, double cs,
                                                   double sh, double chh, double ssig, double csig) {
  CurveDiff o;
  double z_t, z_s;
  if (shape == QAX_PEANUT) {
    const double rho_t = a * (1.0 - c * (1.0 - 2.0 * st * st));
    const double rho_s = a * (1.0 - c * (1.0 - 2.0 * ss * ss));
    // rho(s) - rho(t) = 2 a c sin(2 sig) sin(dl), sin(dl) = 2 sin(dl/2) cos(dl/2)
    const double d_rho = 2.0 * a * c * (2.0 * ssig * csig) * (2.0 * sh * chh);
    const double dcos = -2.0 * ssig * sh;   // cos s - cos t
    const double dsin = -2.0 * csig * sh;   // sin t - sin s
    o.d_r = d_rho * cs + rho_t * dcos;
    o.d_z = rho_t * dsin - d_rho * ss;
    z_t = rho_t * st;
    z_s = rho_s * ss;
  } else {
    o.d_r = -2.0 * a * ssig * sh;
    o.d_z = -2.0 * c * csig * sh;
    z_t = c * st;
    z_s = c * ss;
  }
  if (kappa != 0.0) {
    const double Rt = sqrt(1.0 - kappa * kappa * z_t * z_t);
    const double Rs = sqrt(1.0 - kappa * kappa * z_s * z_s);
    o.d_p = kappa * o.d_z * (z_t + z_s) / (Rt + Rs);
  } else {
    o.d_p = 0.0;
  }
  o.d_q = 0.0;
  return o;
}

__device__ __forceinline__ CurveDiff curve_diff(int shape, double a, double c, double kappa,
                                                double t, double dl) {
  double sh, chh, ssig, csig, st, ct, ss, cs;
  sincos_cw(0.5 * dl, &sh, &chh);
  sincos_cw(t + 0.5 * dl, &ssig, &csig);
  sincos_cw(t, &st, &ct);
  sincos_cw(t + dl, &ss, &cs);
  return curve_diff_sc(shape, a, c, kappa, st, ct, ss, cs, sh, chh, ssig, csig);
}

}  // namespace qax
