// Generating curves of the supported bodies and their cancellation-free
// differences (device code).
//
// Surface (Section 2, equation para_quasi): (r cos th + p, r sin th + q, z).
// sphere / spheroid: r = a cos t, z = c sin t; peanut: polar radius
// rho(t) = a (1 - c cos 2t) (= a (1 + c cos 2 psi), psi the polar angle),
// r = rho cos t, z = rho sin t.  Bent centreline: circle of curvature kappa
// tangent to the z-axis, p = kappa z^2 / (1 + sqrt(1 - kappa^2 z^2)), q = 0.
// The geometries of Section 6.1, Example 2 (equations quasiellipsoid, spiral,
// conch), scaled by a: quasi-ellipsoid r = 2a cos t, z = 3a sin t,
// p = a cos t; spiral r = 1.5a cos t, z = 2a sin t, p = 0.05a cos 4 pi t,
// q = 0.1a sin 4 pi t; conch r = a cos t, z = 1.5a sin t, p = a f cos t,
// q = a f sin t, f = 0.2 + 0.1 sin 8t.
//
// Panels: n_uni uniform panels over [-pi/2, pi/2], the panel at each pole
// halved n_ref times toward the pole (dyadic refinement, Section 6).
#pragma once

#include <hip/hip_runtime.h>

#include "fastmath.h"
#include "internal.h"

namespace qax {

struct Curve {
  double r, dr, z, dz, p, dp, q, dq;
};

// Breakpoint m (0..n_uni + 2 n_ref) of the panels.
__host__ __device__ __forceinline__ double panel_edge(int n_uni, int n_ref, int m) {
  const double h = PI / n_uni;
  const int total = n_uni + 2 * n_ref;
  if (m <= 0) return -0.5 * PI;
  if (m >= total) return 0.5 * PI;
  if (m <= n_ref) return -0.5 * PI + h * ldexp(1.0, m - 1 - n_ref);
  if (m >= total - n_ref) return 0.5 * PI - h * ldexp(1.0, total - m - 1 - n_ref);
  return -0.5 * PI + h * (m - n_ref);
}

constexpr double FOUR_PI_SHAPE = 12.566370614359172954;

// Bodies mapped onto themselves by the reflections y -> -y (theta -> -theta)
// and z -> -z (t -> -t): r and p even in t, z odd, q = 0 (the sphere,
// spheroid and peanut, bent or not, and the quasi-ellipsoid; the panels and
// their Gauss-Legendre nodes are symmetric about t = 0).  Node (s, j), s the
// Gauss-Legendre node along the curve (panel * 16 + index, n_s in all) and j
// the azimuth, has the images (s, (2N - j) mod 2N) and (n_s - 1 - s, j), and
// every self-block entry is the same for a pair of nodes and for its images.
__host__ __device__ __forceinline__ bool mirror_symmetric(int shape) {
  return shape == QAX_SPHERE || shape == QAX_SPHEROID || shape == QAX_PEANUT ||
         shape == QAX_QUASI_ELLIPSOID;
}

// Curve at parameter t, given st = sin t, ct = cos t.
__device__ __forceinline__ Curve curve_from_sincos(int shape, double a, double c, double kappa,
                                                   double t, double st, double ct) {
  Curve o;
  if (shape >= QAX_QUASI_ELLIPSOID) {
    if (shape == QAX_QUASI_ELLIPSOID) {
      o.r = 2.0 * a * ct; o.dr = -2.0 * a * st;
      o.z = 3.0 * a * st; o.dz = 3.0 * a * ct;
      o.p = a * ct; o.dp = -a * st;
      o.q = 0.0; o.dq = 0.0;
    } else if (shape == QAX_SPIRAL) {
      double sw, cw;
      sincos_cw(FOUR_PI_SHAPE * t, &sw, &cw);
      o.r = 1.5 * a * ct; o.dr = -1.5 * a * st;
      o.z = 2.0 * a * st; o.dz = 2.0 * a * ct;
      o.p = 0.05 * a * cw; o.dp = -0.05 * a * FOUR_PI_SHAPE * sw;
      o.q = 0.1 * a * sw; o.dq = 0.1 * a * FOUR_PI_SHAPE * cw;
    } else {
      double s8, c8;
      sincos_cw(8.0 * t, &s8, &c8);
      const double f = 0.2 + 0.1 * s8, df = 0.8 * c8;
      o.r = a * ct; o.dr = -a * st;
      o.z = 1.5 * a * st; o.dz = 1.5 * a * ct;
      o.p = a * f * ct; o.dp = a * (df * ct - f * st);
      o.q = a * f * st; o.dq = a * (df * st + f * ct);
    }
    return o;
  }
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
  return curve_from_sincos(shape, a, c, kappa, t, st, ct);
}

// Differences between the slice at s = t + dl and the slice at t, written with
// product-to-sum identities so they keep full relative accuracy as dl -> 0:
// d_r = r(s) - r(t), d_z = z(t) - z(s), d_p = p(t) - p(s), d_q = q(t) - q(s).
struct CurveDiff {
  double d_r, d_z, d_p, d_q;
};

// From t, dl and the sines / cosines of t, s = t + dl, dl/2 and
// sig = t + dl/2.
__device__ __forceinline__ CurveDiff curve_diff_sc(int shape, double a, double c, double kappa,
                                                   double t, double dl, double st, double ct,
                                                   double ss, double cs, double sh, double chh,
                                                   double ssig, double csig) {
  CurveDiff o;
  double z_t, z_s;
  if (shape >= QAX_QUASI_ELLIPSOID) {
    const double dcos = -2.0 * ssig * sh;   // cos s - cos t
    const double dsin = -2.0 * csig * sh;   // sin t - sin s
    if (shape == QAX_QUASI_ELLIPSOID) {
      o.d_r = 2.0 * a * dcos; o.d_z = 3.0 * a * dsin;
      o.d_p = -a * dcos; o.d_q = 0.0;
    } else if (shape == QAX_SPIRAL) {
      // cos wt - cos ws = 2 sin(w sig) sin(w dl / 2), sin wt - sin ws = -2 cos(w sig) sin(w dl / 2)
      double sws, cws, swh, cwh;
      sincos_cw(FOUR_PI_SHAPE * (t + 0.5 * dl), &sws, &cws);
      sincos_cw(0.5 * FOUR_PI_SHAPE * dl, &swh, &cwh);
      o.d_r = 1.5 * a * dcos; o.d_z = 2.0 * a * dsin;
      o.d_p = 0.1 * a * sws * swh;
      o.d_q = -0.2 * a * cws * swh;
    } else {
      // f(t) - f(s) = -0.2 cos(8 sig) sin(4 dl)
      double s8s, c8s, s4, c4, s8, c8;
      sincos_cw(8.0 * (t + 0.5 * dl), &s8s, &c8s);
      sincos_cw(4.0 * dl, &s4, &c4);
      sincos_cw(8.0 * (t + dl), &s8, &c8);
      const double f_s = 0.2 + 0.1 * s8;
      const double df = -0.2 * c8s * s4;
      o.d_r = a * dcos; o.d_z = 1.5 * a * dsin;
      o.d_p = a * (df * ct - f_s * dcos);
      o.d_q = a * (df * st + f_s * dsin);
    }
    return o;
  }
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
  return curve_diff_sc(shape, a, c, kappa, t, dl, st, ct, ss, cs, sh, chh, ssig, csig);
}

}  // namespace qax
