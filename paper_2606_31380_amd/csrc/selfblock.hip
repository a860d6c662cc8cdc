// FP64 assembly of the self blocks B = 1/2 I + D_bb (Sections 3.1-3.4).
//
// Row T (target x at (t_T, theta_T), panel p), columns (i, l, j):
//   near panel i (|i - p| <= 1):  int_{panel i} P_l(s) G_j(x, s) ds,
//     G_j(x, s) = int_0^{2pi} K(x, y(s,theta)) L_j(theta) dtheta,
//     K = grad_y G^k . (d_theta x d_s)   (the density is interpolated by
//     P_l(s) L_j(theta); the area normal is kept exact, so its theta
//     dependence through p', q' becomes the mode shifts m -/+ 1)
//   far panel i:  K(x, y_ilj) (pi/N) omega_il   (Section 3.1, equation sx).
//
// Inner integral G_j, two routes, both producing the theta-frame modes K_m,
// |m| <= N, of the kernel on the source slice:
//  * modal route (Section 3.3) when chi - 1 < CHI_SPLIT: toroidal Legendre
//    functions Q_{m-1/2}(chi) by the recurrence leg_recur (forward where it is
//    stable, Miller's backward recurrence normalised by Q_{-1/2} = mu K(mu)
//    otherwise; K and E by the arithmetic-geometric mean), Q' by dleg_recur,
//    static derivative modes, the smooth factors F = cos k rho + k rho sin k rho
//    and Hs = (k rho cos k rho - sin k rho)/(4 pi rho^3) sampled on 128 azimuths
//    and transformed by FFT in LDS, the convolution of F^ with the static modes
//    and the shift to the theta frame;
//  * direct route otherwise: trapezoidal rule on L = 128 or 256 azimuths
//    (chosen from the decay rate acosh(chi) of the modes so that aliasing stays
//    below rounding) applied to the kernel itself, its modes by FFT in LDS.
// The map from modes to the Lagrange basis (inverse DFT, G_j = (1/2N) sum'_m
// K_m e^{i m theta_j}, +-N halved) is linear, so the outer sum
// sum_q w_q P_l(s_q) K_m(s_q) is accumulated in registers (lane = mode) and the
// inverse DFT is applied once per work item.  FFTs are radix-4 Stockham
// (self-sorting) passes with a final radix-2 pass where L = 128.
// Outer integral: the paper's generalized Gaussian tables are not available;
// this uses the substitution s - e = (s_end - e) u^5 with 64-point
// Gauss-Legendre in u on each side of the target (self panel) and toward the
// shared end (adjacent panels), which integrates the logarithmic singularity to
// about 1e-13.  Geometry near the target uses cancellation-free differences of
// the generating curve (chi - 1 keeps full relative accuracy).
//
// One wavefront (64 lanes) per (target row, panel) work item.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "fastmath.h"
#include "internal.h"
#include "shapes.h"

namespace qax {

constexpr int LM = 128;                       // modal FFT length
constexpr int NF_CAP = 48;                    // largest convolution half-width
constexpr int NTH_MAX = 64;                   // largest n_theta
constexpr int MQ_CAP = NTH_MAX / 2 + 2 + NF_CAP;   // highest Q index kept (82)
constexpr int QB = 32;                        // nodes per recurrence batch
constexpr int LD = 256;                       // direct-route azimuthal samples (FFT length)
// outer Gauss-Legendre order per side of the target: 48 on two or more
// uniform panels (self-block entries converged to ~1e-14 there), 64 on a
// single panel (the self panel is the whole curve) and on dyadically
// refined curves (small end panels next to panels twice their length)
constexpr int NGO = 64;
constexpr int NGO_UNIFORM = 48;
constexpr double CHI_SPLIT = 0.02;
constexpr double NEAR_EXP = 40.0;   // smooth rule where 2N acosh(chi) >= 40 on the whole panel
constexpr double INV_4PI = 0.0795774715459476678844;

struct NodeLoc {
  double r, dr, dz, dp, dq, rt, alpha, c, chim1, rmrt, z, p, q, w, s;
};

// CF: the single-layer arrays are only sized for the combined-field kernel.
template <bool CF>
struct ModalScratch {
  double2 fa[LM];
  double2 fb[LM];
  double Fh[LM / 2];
  double Hrh[NTH_MAX / 2 + 2];
  double Hh[NTH_MAX / 2 + 2];
  double2 AB0[MQ_CAP + 1];      // static modes (dr, dz) of the kernel, n = 0..nmax+nf
  double2 Am[NTH_MAX / 2 + 2];
  double2 Bm[NTH_MAX / 2 + 2];
  // single layer (combined field only)
  double2 fc[CF ? LM : 1];               // sin(k rho) / (4 pi rho) samples, then transform
  double Ch[CF ? LM / 2 : 1];            // modes of cos(k rho)
  double Sh[CF ? NTH_MAX / 2 + 2 : 1];   // modes of sin(k rho) / (4 pi rho)
  double G0[CF ? MQ_CAP + 1 : 1];        // static modes of G
  double2 Gm[CF ? NTH_MAX / 2 + 2 : 1];  // phi-frame modes of G
};

template <bool CF>
struct SelfShared {
  union {
    double Q[QB][MQ_CAP + 1];     // toroidal functions of one recurrence batch, node-major
                                  // (odd row stride: conflict-free rows and columns)
    double2 acc[GL_ORDER][64];    // accumulated modes (final inverse DFT)
  };
  double2 tw[LD + LD / 16];     // e^{-2 pi i q / LD} at twi(q) (FFT twiddles, azimuth table)
  double2 tw2n[NTH_MAX];        // e^{i pi m / N}
  int modal_idx[64];
  union {
    ModalScratch<CF> m;
    double2 K[CF ? 2 : 1][LD];   // direct-route samples: double layer (, single layer)
  } u;
};

// ---------------------------------------------------------------- elliptic / Q
// K(k), E(k) (modulus k, complementary modulus kp) by the AGM
// (Abramowitz & Stegun 17.6.3-17.6.4), c_n = c_{n-1}^2 / (4 a_n).
__device__ void agm_ke(double kmod, double kp, double& K, double& E) {
  double a = 1.0, b = kp, c = kmod;
  double s = 0.5 * c * c, p2 = 0.5;
  for (int it = 0; it < 40; ++it) {
    const double an = 0.5 * (a + b);
    const double bn = sqrt(a * b);
    const double cn = c * c / (4.0 * an);
    a = an;
    b = bn;
    c = cn;
    p2 *= 2.0;
    s += p2 * c * c;
    if (c <= 1e-17 * a) break;
  }
  K = PI / (2.0 * a);
  E = K * (1.0 - s);
}

// 1/x for exact small integers x: hardware reciprocal + two Newton steps.
__device__ __forceinline__ double recip(double x) {
  double y = __builtin_amdgcn_rcp(x);
  y = fma(y, fma(-x, y, 1.0), y);
  y = fma(y, fma(-x, y, 1.0), y);
  return y;
}

// Wavefront maxima by DPP row shifts and row broadcasts (lane 15 of each row
// of 16 ends with its row's maximum, lane 63 with the wavefront's), read
// back from lane 63: of a non-negative int, and of a non-negative double
// (whose bits order like its values).  Lanes without a DPP source read 0.
template <int CTRL, int ROWM>
__device__ __forceinline__ int dpp_i32(int v) {
  return __builtin_amdgcn_update_dpp(0, v, CTRL, ROWM, 0xf, false);
}
__device__ __forceinline__ int wave_max_int(int v) {
  v = max(v, dpp_i32<0x111, 0xf>(v));   // row_shr:1
  v = max(v, dpp_i32<0x112, 0xf>(v));   // row_shr:2
  v = max(v, dpp_i32<0x114, 0xf>(v));   // row_shr:4
  v = max(v, dpp_i32<0x118, 0xf>(v));   // row_shr:8
  v = max(v, dpp_i32<0x142, 0xa>(v));   // row_bcast:15 into rows 1, 3
  v = max(v, dpp_i32<0x143, 0xc>(v));   // row_bcast:31 into rows 2, 3
  return __builtin_amdgcn_readlane(v, 63);
}
template <int CTRL, int ROWM>
__device__ __forceinline__ unsigned long long dpp_u64(unsigned long long v) {
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)v, CTRL, ROWM, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(v >> 32), CTRL, ROWM, 0xf, false);
  return ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo;
}
__device__ __forceinline__ double wave_max_nonneg(double x) {
  unsigned long long v = (unsigned long long)__double_as_longlong(x);
  auto mx = [](unsigned long long a, unsigned long long b) { return a > b ? a : b; };
  v = mx(v, dpp_u64<0x111, 0xf>(v));
  v = mx(v, dpp_u64<0x112, 0xf>(v));
  v = mx(v, dpp_u64<0x114, 0xf>(v));
  v = mx(v, dpp_u64<0x118, 0xf>(v));
  v = mx(v, dpp_u64<0x142, 0xa>(v));
  v = mx(v, dpp_u64<0x143, 0xc>(v));
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)v, 63);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(v >> 32), 63);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Uniform copy of lane l's value (v_readlane on both halves); l uniform.
__device__ __forceinline__ double readlane_f64(double v, int l) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b & 0xffffffffull), l);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), l);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Coefficients of the recurrence leg_recur with the division folded in,
// exact ratios rounded once at compile time; the index n is the same in every
// lane, so the kernels read them with scalar loads:
//   forward   Q_{n+1/2} = chi fa[n] Q_{n-1/2} - fb[n] Q_{n-3/2},
//             fa[n] = 4n / (2n + 1), fb[n] = (2n - 1) / (2n + 1)   (f[n]);
//   backward  Q_{n-3/2} = chi ba[n] Q_{n-1/2} - bb[n] Q_{n+1/2},
//             ba[n] = 4n / (2n - 1), bb[n] = (2n + 1) / (2n - 1)   (b[n]).
constexpr int QREC_MAX = 1024;
struct QRecTables {
  double2 f[QREC_MAX + 1];   // (fa, fb)
  double2 b[QREC_MAX + 1];   // (ba, bb)
};
constexpr QRecTables make_qrec() {
  QRecTables t{};
  for (int n = 1; n <= QREC_MAX; ++n) {
    const double d = n;
    t.f[n].x = 4.0 * d / (2.0 * d + 1.0);
    t.f[n].y = (2.0 * d - 1.0) / (2.0 * d + 1.0);
    t.b[n].x = 4.0 * d / (2.0 * d - 1.0);
    t.b[n].y = (2.0 * d + 1.0) / (2.0 * d - 1.0);
  }
  return t;
}
__constant__ QRecTables qrec = make_qrec();

// Q[col][n] = Q_{n-1/2}(chi), n = 0..mq, for the node of each lane with `act`
// (one batch of nodes, one node per lane).  Starting values Q_{-1/2} = mu K,
// Q_{1/2} = chi mu K - sqrt(2 (chi + 1)) E (K, E of modulus mu by the AGM).
// Where m acosh(chi) stays small the recurrence leg_recur runs forward; else
// Miller's backward recurrence from one common start index for the batch
// (20 / acosh(chi) + 10 beyond mq for the slowest-decaying lane, which only
// adds accuracy for the others; at most 9 mq + 19 since backward lanes have
// acosh(chi) > 2.5 / (mq + 1); values above 1e150 are rescaled while no entry
// is stored yet), normalised by Q_{-1/2}.  One dependent fma per step: the
// coefficients come from qrec and the older term's product is formed a step
// ahead.
__device__ __forceinline__ void toroidal_q_batch(bool act, double chi, double chim1, int mq,
                                                 double (*Q)[MQ_CAP + 1], int col) {
  if (!act) {
    chi = 2.0;
    chim1 = 1.0;
  }
  const double mu = sqrt(2.0 / (chi + 1.0));
  const double mup = sqrt(chim1 / (chi + 1.0));
  double K, E;
  agm_ke(mu, mup, K, E);
  const double q0 = mu * K;
  const double q1 = chi * mu * K - sqrt(2.0 * (chi + 1.0)) * E;
  const double a = log(chi + sqrt(chim1 * (chi + 1.0)));   // acosh(chi)
  const bool fwd = act && a * (mq + 1) <= 2.5;
  const bool bwd = act && !fwd;
  if (__ballot(fwd)) {
    if (fwd) {
      Q[col][0] = q0;
      Q[col][1] = q1;
    }
    double qm = q0, qn = q1;
    const double2* tf = qrec.f;
#pragma unroll 4
    for (int n = 1; n < mq; ++n) {
      const double2 c = tf[n];
      const double qp = fma(chi * c.x, qn, -c.y * qm);
      if (fwd) Q[col][n + 1] = qp;
      qm = qn;
      qn = qp;
    }
  }
  int start = bwd ? mq + (int)ceil(20.0 / a) + 10 : 0;
  start = __builtin_amdgcn_readfirstlane(min(wave_max_int(start), QREC_MAX));
  if (start > 0) {
    double hi = 0.0, lo = 1e-200;
    const double2* tb = qrec.b;
    auto step = [&](double2 c) {
      const double nw = fma(chi * c.x, lo, -c.y * hi);
      hi = lo;
      lo = nw;
    };
    int n = start;
    // no entry stored yet: 16 steps between checks for rescaling, their
    // coefficients loaded first
    for (; n > mq + 16; n -= 16) {
      double2 c[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) c[u] = tb[n - u];
#pragma unroll
      for (int u = 0; u < 16; ++u) step(c[u]);
      if (fabs(lo) > 1e150) {
        lo *= 1e-150;
        hi *= 1e-150;
      }
    }
    for (; n > mq; --n) step(tb[n]);
    for (; n >= 1; --n) {
      if (bwd) Q[col][n] = lo;
      step(tb[n]);
    }
    if (bwd) {
      const double scale = q0 / lo;
      Q[col][0] = q0;
      for (int m = 1; m <= mq; ++m) Q[col][m] *= scale;
    }
  }
}

// position of twiddle q in the padded table (see below)
__device__ __forceinline__ int twi(int q) { return q + (q >> 4); }

// ---------------------------------------------------------------- FFT in LDS
// Forward DFT X_q = sum_l x_l e^{-2 pi i q l / L}, in place, natural order in
// and out: Stockham self-sorting passes.  A pass over sub-transforms of length
// Ns takes butterfly j (inputs x[j + i L/r], i < r), multiplies input i by
// e^{-2 pi i i (j mod Ns) / (r Ns)}, applies the r-point DFT and stores output i
// at (j - j mod Ns) r + (j mod Ns) + i Ns.  Every lane reads its inputs before a
// barrier and writes after it, so one buffer serves as source and target.
// tw[twi(q)] = e^{-2 pi i q / LD}, q < LD: one padding entry after every 16,
// so the strided twiddle reads of a pass (q = 16 k or 4 k across lanes) fall
// on different LDS banks.
__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// 4-point forward DFT in place: y_q = sum_n a_n (-i)^{n q}
__device__ __forceinline__ void dft4(double2& a0, double2& a1, double2& a2, double2& a3) {
  const double2 t0 = make_double2(a0.x + a2.x, a0.y + a2.y);
  const double2 t1 = make_double2(a0.x - a2.x, a0.y - a2.y);
  const double2 t2 = make_double2(a1.x + a3.x, a1.y + a3.y);
  const double2 t3 = make_double2(a1.x - a3.x, a1.y - a3.y);
  a0 = make_double2(t0.x + t2.x, t0.y + t2.y);
  a2 = make_double2(t0.x - t2.x, t0.y - t2.y);
  a1 = make_double2(t1.x + t3.y, t1.y - t3.x);   // t1 - i t3
  a3 = make_double2(t1.x - t3.y, t1.y + t3.x);   // t1 + i t3
}

// One radix-4 pass of an L-point transform; butterfly j in lanes with `active`.
// The twiddles (a read-only table) are read together with the data, before
// the barrier; the first pass (Ns = 1) has none.
template <int L, int Ns>
__device__ __forceinline__ void r4_pass(double2* x, int j, bool active, const double2* tw) {
  double2 a0, a1, a2, a3, w1, w2, w3;
  const int k = j & (Ns - 1);
  if (active) {
    a0 = x[j];
    a1 = x[j + L / 4];
    a2 = x[j + L / 2];
    a3 = x[j + 3 * L / 4];
    if (Ns > 1) {
      constexpr int step = LD / (4 * Ns);
      w1 = tw[twi(k * step)];
      w2 = tw[twi(2 * k * step)];
      w3 = tw[twi(3 * k * step)];
    }
  }
  __syncthreads();
  if (active) {
    if (Ns > 1) {
      a1 = cmul(a1, w1);
      a2 = cmul(a2, w2);
      a3 = cmul(a3, w3);
    }
    dft4(a0, a1, a2, a3);
    const int o = 4 * (j - k) + k;
    x[o] = a0;
    x[o + Ns] = a1;
    x[o + 2 * Ns] = a2;
    x[o + 3 * Ns] = a3;
  }
  __syncthreads();
}

// Last pass of a 128-point transform (radix 2, Ns = 64): butterfly j = lane
// reads and writes x[j], x[j + 64] only.
__device__ __forceinline__ void r2_last128(double2* x, int j, const double2* tw) {
  const double2 a0 = x[j];
  const double2 a1 = cmul(x[j + 64], tw[twi(2 * j)]);
  x[j] = make_double2(a0.x + a1.x, a0.y + a1.y);
  x[j + 64] = make_double2(a0.x - a1.x, a0.y - a1.y);
}

// Two 128-point transforms at once: lanes 0-31 take xa, lanes 32-63 take xb in
// the radix-4 passes; every lane finishes one butterfly of each.
__device__ void fft128x2(double2* xa, double2* xb, const double2* tw) {
  const int lane = threadIdx.x;
  double2* x = lane < 32 ? xa : xb;
  const int j = lane & 31;
  r4_pass<128, 1>(x, j, true, tw);
  r4_pass<128, 4>(x, j, true, tw);
  r4_pass<128, 16>(x, j, true, tw);
  r2_last128(xa, lane, tw);
  r2_last128(xb, lane, tw);
  __syncthreads();
}

__device__ void fft128(double2* x, const double2* tw) {
  const int lane = threadIdx.x;
  r4_pass<128, 1>(x, lane, lane < 32, tw);
  r4_pass<128, 4>(x, lane, lane < 32, tw);
  r4_pass<128, 16>(x, lane, lane < 32, tw);
  r2_last128(x, lane, tw);
  __syncthreads();
}

__device__ void fft256(double2* x, const double2* tw) {
  const int lane = threadIdx.x;
  r4_pass<256, 1>(x, lane, true, tw);
  r4_pass<256, 4>(x, lane, true, tw);
  r4_pass<256, 16>(x, lane, true, tw);
  r4_pass<256, 64>(x, lane, true, tw);
}

__device__ __forceinline__ double wave_min(double v) {
  for (int off = 32; off > 0; off >>= 1) v = fmin(v, __shfl_xor(v, off));
  return v;
}

__device__ __forceinline__ double wave_max(double v) {
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off));
  return v;
}

// Hs = (x cos x - sin x)/(4 pi rho^3), x = k rho, given irho = 1 / rho,
// sx = sin x, cx = cos x;
// for x < 0.5 the Taylor series sum_{j>=1} (-1)^j 2j/(2j+1)! x^{2j-2} (times
// k^3 / 4 pi), which avoids the cancellation.
__device__ __forceinline__ double smooth_h(double k, double rho, double irho, double sx, double cx) {
  const double x = k * rho;
  if (x < 0.5) {
    const double x2 = x * x;
    double p = 1.5472680682522736e-24;
    p = fma(p, x2, -8.509974375387505e-22);
    p = fma(p, x2, 3.9145882126782523e-19);
    p = fma(p, x2, -1.4797143443923793e-16);
    p = fma(p, x2, 4.498331606952833e-14);
    p = fma(p, x2, -1.0706029224547743e-11);
    p = fma(p, x2, 1.9270852604185937e-09);
    p = fma(p, x2, -2.505210838544172e-07);
    p = fma(p, x2, 2.2045855379188714e-05);
    p = fma(p, x2, -0.0011904761904761906);
    p = fma(p, x2, 0.03333333333333333);
    p = fma(p, x2, -0.3333333333333333);
    return k * k * k * INV_4PI * p;
  }
  return (x * cx - sx) * INV_4PI * irho * irho * irho;
}

// phi-frame modes m = 0..nmax of A = dr G, B = dz G for one node (all lanes),
// given its Q column.  Results in M.Am, M.Bm.
// CF: also the modes of G itself (the single layer, Section 3.3 equations
// conv and I1): cos(k rho) convolved with the static modes of G plus
// i times the modes of sin(k rho) / (4 pi rho).
template <bool CF>
__device__ void modal_modes(double k, double r, double rt, double c, double chim1, double rmrt,
                            int nmax, const double (*Q)[MQ_CAP + 1], int col, ModalScratch<CF>& M,
                            const double2* tw) {
  const int lane = threadIdx.x;
  const double chi = 1.0 + chim1;
  int nf = 0;
  if (k != 0.0) {
    const double k2pi = k / TWO_PI;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int l = lane + 64 * h;
      // sin(phi/2) with phi = 2 pi l / LM from the table e^{-2 pi i q / LD}
      const double sh = -tw[twi(l * (LD / (2 * LM)))].y;
      const double rho2 = 2.0 * r * rt * (chim1 + 2.0 * sh * sh);
      const double irho = rsqrt_pos(rho2);
      const double rho = rho2 * irho;
      double sk, ck;
      sincos_2pi(rho * k2pi, &sk, &ck);
      const double F = ck + k * rho * sk;
      const double Hs = smooth_h(k, rho, irho, sk, ck);
      const double cphi = 1.0 - 2.0 * sh * sh;
      M.fa[l] = make_double2(F, Hs);
      M.fb[l] = make_double2(Hs * (r - rt * cphi), CF ? ck : 0.0);
      if constexpr (CF) {
        const double x = k * rho;
        // sin(x) / (4 pi rho) = (k / 4 pi) sin(x) / x
        const double sx = x < 1e-3 ? 1.0 - x * x * (1.0 / 6.0 - x * x * (1.0 / 120.0)) : sk / x;
        M.fc[l] = make_double2(k * INV_4PI * sx, 0.0);
      }
    }
    __syncthreads();
    fft128x2(M.fa, M.fb, tw);
    if constexpr (CF) fft128(M.fc, tw);
    const double sc = TWO_PI / LM;
    M.Fh[lane] = M.fa[lane].x * sc;
    if constexpr (CF) M.Ch[lane] = M.fb[lane].y * sc;
    if (lane < nmax + 1) {
      M.Hh[lane] = M.fa[lane].y * sc;
      M.Hrh[lane] = M.fb[lane].x * sc;
      if constexpr (CF) M.Sh[lane] = M.fc[lane].x * sc;
    }
    const double mag = fabs(M.fa[lane].x * sc);
    const double mx = wave_max_nonneg(mag);
    const bool above = mag > 1e-15 * mx;
    const unsigned long long bal = __ballot(above);
    nf = bal ? 63 - __clzll(bal) : 0;
    nf = min(nf + 1, NF_CAP);
    nf = min(nf, MQ_CAP - nmax - 1);
    __syncthreads();
  }
  // static modes n = 0..nmax+nf
  const int mtot = nmax + nf;
  const double pref = 1.0 / (TWO_PI * sqrt(rt * r));
  const double ir = 1.0 / r, irt = 1.0 / rt;
  const double half_inv_chi2m1 = 0.5 / (chim1 * (chi + 1.0));
  const double drchi = (rmrt * (r + rt) - c * c) * 0.5 * irt * ir * ir;
  const double dzchi = -c * ir * irt;
  for (int n = lane; n <= mtot; n += 64) {
    const double qn = Q[col][n];
    const double qm = n == 0 ? Q[col][1] : Q[col][n - 1];
    const double qp = (2.0 * n - 1.0) * half_inv_chi2m1 * (chi * qn - qm);
    M.AB0[n] = make_double2(pref * (drchi * qp - 0.5 * ir * qn), pref * dzchi * qp);
    if constexpr (CF) M.G0[n] = pref * qn;
  }
  __syncthreads();
  if (k != 0.0 && nmax < 32) {
    // the convolution's sum over n split between the wavefront's halves
    // (lanes m and m + 32 take n <= nf / 2 and n > nf / 2 for mode m), the
    // halves' sums added across: half the dependent chain
    const int m = lane & 31, hf = lane >> 5, nh = nf / 2;
    const int n0 = hf ? nh + 1 : 1, n1 = hf ? nf : nh;
    double ar = 0.0, br = 0.0, gr = 0.0;
    if (m <= nmax) {
      if (!hf) {
        const double2 ab = M.AB0[m];
        ar = M.Fh[0] * ab.x;
        br = M.Fh[0] * ab.y;
        if constexpr (CF) gr = M.Ch[0] * M.G0[m];
      }
#pragma unroll 4
      for (int n = n0; n <= n1; ++n) {
        const double f = M.Fh[n];
        const double2 u = M.AB0[abs(m - n)], v = M.AB0[m + n];
        ar = fma(f, u.x + v.x, ar);
        br = fma(f, u.y + v.y, br);
      }
      if constexpr (CF) {
#pragma unroll 4
        for (int n = n0; n <= n1; ++n) gr = fma(M.Ch[n], M.G0[abs(m - n)] + M.G0[m + n], gr);
      }
    }
    ar += __shfl_xor(ar, 32);
    br += __shfl_xor(br, 32);
    if constexpr (CF) gr += __shfl_xor(gr, 32);
    if (!hf && m <= nmax) {
      M.Am[m] = make_double2(ar * (1.0 / TWO_PI), M.Hrh[m]);
      M.Bm[m] = make_double2(br * (1.0 / TWO_PI), -c * M.Hh[m]);
      if constexpr (CF) M.Gm[m] = make_double2(gr * (1.0 / TWO_PI), M.Sh[m]);
    }
  } else if (lane <= nmax) {
    const double2 ab = M.AB0[lane];
    if (k == 0.0) {
      M.Am[lane] = make_double2(ab.x, 0.0);
      M.Bm[lane] = make_double2(ab.y, 0.0);
      if constexpr (CF) M.Gm[lane] = make_double2(M.G0[lane], 0.0);
    } else {
      // F^ is even in n: (F^ * g)_m = F^_0 g_m + sum_{n>=1} F^_n (g_{|m-n|} + g_{m+n})
      double ar = M.Fh[0] * ab.x, br = M.Fh[0] * ab.y;
#pragma unroll 4
      for (int n = 1; n <= nf; ++n) {
        const double f = M.Fh[n];
        const double2 u = M.AB0[abs(lane - n)], v = M.AB0[lane + n];
        ar = fma(f, u.x + v.x, ar);
        br = fma(f, u.y + v.y, br);
      }
      M.Am[lane] = make_double2(ar * (1.0 / TWO_PI), M.Hrh[lane]);
      M.Bm[lane] = make_double2(br * (1.0 / TWO_PI), -c * M.Hh[lane]);
      if constexpr (CF) {
        double gr = M.Ch[0] * M.G0[lane];
#pragma unroll 4
        for (int n = 1; n <= nf; ++n) gr = fma(M.Ch[n], M.G0[abs(lane - n)] + M.G0[lane + n], gr);
        M.Gm[lane] = make_double2(gr * (1.0 / TWO_PI), M.Sh[lane]);
      }
    }
  }
  __syncthreads();
}

// theta-frame mode m of the kernel from the phi-frame modes A = dr G, B = dz G
// (even in m), with e^{-i m alpha} = (c0, s0) and e^{i alpha} = (ca, sa):
//   e^{-i m alpha} (r z' A_m - r r' B_m)
//   - r/2 (p' - i q') e^{-i(m-1) alpha} B_{m-1} - r/2 (p' + i q') e^{-i(m+1) alpha} B_{m+1}
template <bool CF>
__device__ __forceinline__ double2 theta_mode(int m, double c0, double s0, double ca, double sa,
                                              const NodeLoc& L, const ModalScratch<CF>& M) {
  const double r = L.r;
  const double c1 = c0 * ca - s0 * sa, s1 = s0 * ca + c0 * sa;   // e^{-i(m-1) alpha}
  const double c2 = c0 * ca + s0 * sa, s2 = s0 * ca - c0 * sa;   // e^{-i(m+1) alpha}
  const double2 A = M.Am[abs(m)], B = M.Bm[abs(m)];
  const double2 Bm1 = M.Bm[abs(m - 1)], Bp1 = M.Bm[abs(m + 1)];
  const double tr = r * L.dz * A.x - r * L.dr * B.x;
  const double ti = r * L.dz * A.y - r * L.dr * B.y;
  double kr = c0 * tr - s0 * ti;
  double ki = c0 * ti + s0 * tr;
  const double fr = 0.5 * r * L.dp, fq = 0.5 * r * L.dq;
  {
    const double er = c1 * Bm1.x - s1 * Bm1.y, ei = c1 * Bm1.y + s1 * Bm1.x;
    kr -= fr * er + fq * ei;
    ki -= fr * ei - fq * er;
  }
  {
    const double er = c2 * Bp1.x - s2 * Bp1.y, ei = c2 * Bp1.y + s2 * Bp1.x;
    kr -= fr * er - fq * ei;
    ki -= fr * ei + fq * er;
  }
  return make_double2(kr, ki);
}

// Mode slot of lane s < 2N: m = s - N, with slot 0 holding K_{-N} + K_{N}
// (the inverse DFT weighs both by 1/2 and e^{+-i N theta_j} agree).
// CF: ks receives the single-layer slot, e^{-i m alpha} G_|m| (the same
// pairing of -N and N in slot 0).
template <bool CF>
__device__ __forceinline__ double2 modal_slot(int N, const NodeLoc& L, const ModalScratch<CF>& M,
                                              double2& ks) {
  const int lane = threadIdx.x;
  double2 out = make_double2(0.0, 0.0);
  ks = make_double2(0.0, 0.0);
  const double arev = L.alpha * (1.0 / TWO_PI);   // alpha in revolutions
  double sa, ca;
  sincos_2pi(arev, &sa, &ca);
  if (lane < 2 * N) {
    const int m = lane - N;
    double s0, c0;
    sincos_2pi(-m * arev, &s0, &c0);
    out = theta_mode(m, c0, s0, ca, sa, L, M);
    if constexpr (CF) ks = cmul(make_double2(c0, s0), M.Gm[abs(m)]);
    if (lane == 0) {
      const double2 o2 = theta_mode(N, c0, -s0, ca, sa, L, M);
      out.x += o2.x;
      out.y += o2.y;
      if constexpr (CF) {
        const double2 k2 = cmul(make_double2(c0, -s0), M.Gm[N]);
        ks.x += k2.x;
        ks.y += k2.y;
      }
    }
  }
  return out;
}

// acc[l] += w_q P_l(s_q) K with w_q P_l(s_q) held by lane q (uniform) in P[l]
__device__ __forceinline__ void accumulate_node(double2 (&acc)[GL_ORDER], const double (&P)[GL_ORDER],
                                                int q, double2 K) {
#pragma unroll
  for (int l = 0; l < GL_ORDER; ++l) {
    const double p = readlane_f64(P[l], q);
    acc[l].x = fma(p, K.x, acc[l].x);
    acc[l].y = fma(p, K.y, acc[l].y);
  }
}

// ---------------------------------------------------------------- per-node geometry
// Target-side quantities shared by every outer node of a work item.
struct TargetGeom {
  double t, st, ct;      // parameter of the target slice and its sine / cosine
  double r;              // r(t)
  double sth, cth;       // sin / cos of the target azimuth
};

// Source slice at s = t + dl relative to the target (t, theta_t).
__device__ NodeLoc node_local(int shape, double a, double c, double kappa, const TargetGeom& T,
                              double dl) {
  NodeLoc L;
  double sh, chh, ssig, csig, ss, cs;
  sincos_cw(0.5 * dl, &sh, &chh);
  sincos_cw(T.t + 0.5 * dl, &ssig, &csig);
  sincos_cw(T.t + dl, &ss, &cs);
  const Curve cv = curve_from_sincos(shape, a, c, kappa, T.t + dl, ss, cs);
  const CurveDiff d = curve_diff_sc(shape, a, c, kappa, T.t, dl, T.st, T.ct, ss, cs, sh, chh, ssig,
                                    csig);
  const double ax = T.r * T.cth + d.d_p;
  const double by = T.r * T.sth + d.d_q;
  L.rt = sqrt(ax * ax + by * by);
  L.alpha = atan2(by, ax);
  const double drt = (2.0 * T.r * (T.cth * d.d_p + T.sth * d.d_q) + d.d_p * d.d_p + d.d_q * d.d_q) /
                     (L.rt + T.r);
  L.rmrt = d.d_r - drt;
  L.c = d.d_z;
  L.r = cv.r;
  L.dr = cv.dr;
  L.dz = cv.dz;
  L.dp = cv.dp;
  L.dq = cv.dq;
  L.z = cv.z;
  L.p = cv.p;
  L.q = cv.q;
  L.chim1 = (L.rmrt * L.rmrt + L.c * L.c) / (2.0 * L.r * L.rt);
  L.s = T.t + dl;
  return L;
}

// The node held by lane `src` (uniform), broadcast to the wavefront.
__device__ __forceinline__ NodeLoc read_node(const NodeLoc& v, int src) {
  NodeLoc o;
  o.r = readlane_f64(v.r, src); o.dr = readlane_f64(v.dr, src); o.dz = readlane_f64(v.dz, src);
  o.dp = readlane_f64(v.dp, src); o.dq = readlane_f64(v.dq, src); o.rt = readlane_f64(v.rt, src);
  o.alpha = readlane_f64(v.alpha, src); o.c = readlane_f64(v.c, src);
  o.chim1 = readlane_f64(v.chim1, src); o.rmrt = readlane_f64(v.rmrt, src);
  o.z = readlane_f64(v.z, src); o.p = readlane_f64(v.p, src); o.q = readlane_f64(v.q, src);
  o.w = 0.0;
  o.s = readlane_f64(v.s, src);
  return o;
}

__device__ __forceinline__ NodeLoc shfl_node(const NodeLoc& v, int src) {
  NodeLoc o;
  o.r = __shfl(v.r, src); o.dr = __shfl(v.dr, src); o.dz = __shfl(v.dz, src);
  o.dp = __shfl(v.dp, src); o.dq = __shfl(v.dq, src); o.rt = __shfl(v.rt, src);
  o.alpha = __shfl(v.alpha, src); o.c = __shfl(v.c, src); o.chim1 = __shfl(v.chim1, src);
  o.rmrt = __shfl(v.rmrt, src); o.z = __shfl(v.z, src); o.p = __shfl(v.p, src);
  o.q = __shfl(v.q, src); o.w = __shfl(v.w, src); o.s = __shfl(v.s, src);
  return o;
}

// ---------------------------------------------------------------- assembly kernel
struct OuterRule {
  double x[2][NGO];   // [0]: NGO_UNIFORM nodes (rest unused), [1]: NGO nodes
  double w[2][NGO];
};

// Inverse DFT of the accumulated mode slots (S.acc) onto the Lagrange basis
// for lane j < 2N: g_l = (1/2N) sum_s acc_l[s] e^{i (s - N) theta_j}, slot 0
// weighted 1/2 (applied when the slots were stored);
// e^{i (s - N) j pi / N} = (-1)^j e^{i pi s j / N}.
template <bool CF>
__device__ __forceinline__ void slots_to_nodes(const SelfShared<CF>& S, int N,
                                               double2 (&g)[GL_ORDER]) {
  const int lane = threadIdx.x;
#pragma unroll
  for (int l = 0; l < GL_ORDER; ++l) g[l] = make_double2(0.0, 0.0);
  int e = 0;
  for (int sl = 0; sl < 2 * N; ++sl) {
    const double2 t = S.tw2n[e];
    e += lane;
    if (e >= 2 * N) e -= 2 * N;
#pragma unroll
    for (int l = 0; l < GL_ORDER; ++l) {
      const double2 v = S.acc[l][sl];
      g[l].x = fma(v.x, t.x, fma(-v.y, t.y, g[l].x));
      g[l].y = fma(v.x, t.y, fma(v.y, t.x, g[l].y));
    }
  }
  const double scale = ((lane & 1) ? -1.0 : 1.0) / (2 * N);
#pragma unroll
  for (int l = 0; l < GL_ORDER; ++l) g[l] = make_double2(g[l].x * scale, g[l].y * scale);
}

template <bool CF>
__device__ __forceinline__ void store_slots(SelfShared<CF>& S, const double2 (&acc)[GL_ORDER], bool conj) {
  const int lane = threadIdx.x;
  const double f = lane == 0 ? 0.5 : 1.0;
  const double fy = conj ? -f : f;
#pragma unroll
  for (int l = 0; l < GL_ORDER; ++l) S.acc[l][lane] = make_double2(acc[l].x * f, acc[l].y * fy);
}

// One radix-4 Stockham pass (as r4_pass) over the NR rows X[l][0..L) at once:
// NR L / 4 butterflies, NR L / 256 per lane, read before the barrier, written
// after it.
template <int L, int Ns, int NR>
__device__ __forceinline__ void r4_pass_rows(double2 (*X)[64], const double2* tw) {
  constexpr int NB = L / 4, NBT = NR * NB, PER = NBT >= 64 ? NBT / 64 : 1;
  const int lane = threadIdx.x;
  const bool act = NBT >= 64 || lane < NBT;
  double2 a[PER][4], w[PER][3];
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int e = lane + 64 * u, row = e / NB, j = e % NB;
    if (!act) continue;
#pragma unroll
    for (int i = 0; i < 4; ++i) a[u][i] = X[row][j + i * NB];
    if (Ns > 1) {
      constexpr int step = LD / (4 * Ns);
      const int k = j & (Ns - 1);
#pragma unroll
      for (int i = 1; i < 4; ++i) w[u][i - 1] = tw[twi(i * k * step)];
    }
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int e = lane + 64 * u, row = e / NB, j = e % NB;
    if (!act) continue;
    const int k = j & (Ns - 1);
    if (Ns > 1) {
#pragma unroll
      for (int i = 1; i < 4; ++i) a[u][i] = cmul(a[u][i], w[u][i - 1]);
    }
    dft4(a[u][0], a[u][1], a[u][2], a[u][3]);
    const int o = 4 * (j - k) + k;
#pragma unroll
    for (int i = 0; i < 4; ++i) X[row][o + i * Ns] = a[u][i];
  }
  __syncthreads();
}

// slots_to_nodes for 2N = 16 or 64 (powers of 4): the inverse DFT of every
// row as conj(FFT(conj(row))) (the rows were stored conjugated), then the
// same scale and sign.
template <int L>
__device__ __forceinline__ void fft_rows(double2 (*X)[64], const double2* tw) {
  r4_pass_rows<L, 1, GL_ORDER>(X, tw);
  r4_pass_rows<L, 4, GL_ORDER>(X, tw);
  if constexpr (L == 64) r4_pass_rows<L, 16, GL_ORDER>(X, tw);
}

template <bool CF>
__device__ __forceinline__ void slots_to_nodes_fft(SelfShared<CF>& S, int N, double2 (&g)[GL_ORDER]) {
  const int lane = threadIdx.x;
  if (2 * N == 64) fft_rows<64>(S.acc, S.tw);
  else fft_rows<16>(S.acc, S.tw);
  const double scale = ((lane & 1) ? -1.0 : 1.0) / (2 * N);
#pragma unroll
  for (int l = 0; l < GL_ORDER; ++l) {
    const double2 v = lane < 2 * N ? S.acc[l][lane] : make_double2(0.0, 0.0);
    g[l] = make_double2(v.x * scale, -v.y * scale);
  }
}

// One work item = one target row T and one source panel ip of a block.
// CF = false: row of 1/2 I + D (Section 3.1, equations muJ and coef_ele, with
// the double-layer modes of Section 3.3).  CF = true: row of the combined
// field 1/2 I + D - i eta S (the combined-field remark of Section 2), where
// the single layer interpolates the density times |J|, so its column
// (ip, l, j) carries |J| at that node.
template <int FORM>
__global__ __launch_bounds__(64) void assemble_self_kernel(
    const SelfTask* __restrict__ tasks, const BlockDev* __restrict__ blocks,
    const BodyDev* __restrict__ bodies, const double* __restrict__ gl16,
    const OuterRule* __restrict__ orule, double2* __restrict__ pool) {
  constexpr bool CF = FORM != 0;   // single-layer modes needed
  __shared__ SelfShared<CF> S;
  const SelfTask task = tasks[blockIdx.x];
  const BlockDev K = blocks[task.block];
  const BodyDev& B = bodies[K.rep_body];
  const int lane = threadIdx.x;
  const int shape = B.shape;
  const double a = B.a, cc = B.c, kappa = B.kappa, k = B.k;
  const double eta = CF ? B.eta : 0.0;
  const int nth = B.n_theta, N = nth / 2;
  const int n = K.n;
  const int T = task.row, ip = task.panel;
  const int pT = T / (GL_ORDER * nth), lT = (T / nth) % GL_ORDER, jT = T % nth;
  const double eT0 = panel_edge(B.n_uni, B.n_ref, pT);
  const double hT = panel_edge(B.n_uni, B.n_ref, pT + 1) - eT0;
  const double tT = eT0 + 0.5 * hT * (gl16[lT] + 1.0);
  // source panel ip: [e0, e1], length h
  const double e0 = panel_edge(B.n_uni, B.n_ref, ip), e1 = panel_edge(B.n_uni, B.n_ref, ip + 1);
  const double h = e1 - e0;
  const double thT = jT * PI / N;
  double2* row = pool + K.elem_off + (int64_t)T * n;
  // Mirror-symmetric bodies: only the rows with s < n_s / 2 and j <= N are
  // work items, and each entry (T, (s, j)) is also stored at the images of
  // the pair: ((n_s - 1 - s_T, j_T), (n_s - 1 - s, j)) always, and, where
  // the row's azimuth is neither 0 nor N (other rows are their own theta
  // image), ((s_T, 2N - j_T), (s, -j)) and ((n_s - 1 - s_T, 2N - j_T), (n_s - 1 - s, -j)).
  const int ns = GL_ORDER * B.n_panels, sT = T / nth;
  const bool mir = mirror_symmetric(shape);
  const bool mth = mir && jT != 0 && jT != N;
  double2* row_t = pool + K.elem_off + (int64_t)((ns - 1 - sT) * nth + jT) * n;
  double2* row_h = pool + K.elem_off + (int64_t)(sT * nth + (nth - jT) % nth) * n;
  double2* row_ht = pool + K.elem_off + (int64_t)((ns - 1 - sT) * nth + (nth - jT) % nth) * n;
  auto put = [&](int l, int j, double2 v) {
    const int sc = ip * GL_ORDER + l;
    row[(int64_t)sc * nth + j] = v;
    if (mir) {
      const int jm = j ? nth - j : 0;
      const int64_t cm = (int64_t)(ns - 1 - sc) * nth;
      row_t[cm + j] = v;
      if (mth) {
        row_h[(int64_t)sc * nth + jm] = v;
        row_ht[cm + jm] = v;
      }
    }
  };

  // target point (body frame)
  TargetGeom TG;
  TG.t = tT;
  sincos_cw(tT, &TG.st, &TG.ct);
  const Curve cT = curve_from_sincos(shape, a, cc, kappa, tT, TG.st, TG.ct);
  TG.r = cT.r;
  sincos_cw(thT, &TG.sth, &TG.cth);
  const double xT = cT.r * TG.cth + cT.p, yT = cT.r * TG.sth + cT.q, zT = cT.z;

  // near panel: adjacent, or one whose rings are close enough for the smooth
  // rule's trapezoid in theta to alias (modes decay like e^{-|m| acosh chi};
  // 2N points resolve them to e^{-2N acosh chi}); happens near the poles of
  // dyadically refined curves, where the rings shrink with the panels
  bool near = abs(ip - pT) <= 1;
  if (!near) {
    double v = 1e300;
    if (lane < GL_ORDER) {
      const double s = e0 + 0.5 * h * (gl16[lane] + 1.0);
      const NodeLoc L = node_local(shape, a, cc, kappa, TG, s - tT);
      v = nth * log1p(L.chim1 + sqrt(L.chim1 * (L.chim1 + 2.0)));
    }
    near = wave_min(v) < NEAR_EXP;
  }
  if (!near) {
    // far panel: smooth rule (Section 3.1, equation sx)
    for (int e = lane; e < GL_ORDER * nth; e += 64) {
      const int l = e / nth, j = e % nth;
      const double t = e0 + 0.5 * h * (gl16[l] + 1.0);
      const double om = 0.5 * h * gl16[GL_ORDER + l];
      const Curve cv = curve_eval(shape, a, cc, kappa, t);
      double sj, cj;
      sincos_cw(j * PI / N, &sj, &cj);
      const double dx = cv.r * cj + cv.p - xT, dy = cv.r * sj + cv.q - yT, dz = cv.z - zT;
      const double nx = cv.r * cv.dz * cj, ny = cv.r * cv.dz * sj;
      const double nz = -cv.r * (cv.dr + cv.dp * cj + cv.dq * sj);
      const double r2 = dx * dx + dy * dy + dz * dz;
      const double ir = rsqrt(r2);
      const double rr = r2 * ir;
      double s, c;
      sincos_cw(k * rr, &s, &c);
      const double wq = om * PI / N;
      const double sc = (dx * nx + dy * ny + dz * nz) * ir * ir * ir * INV_4PI * wq;
      double2 v = make_double2(-(c + k * rr * s) * sc, (k * rr * c - s) * sc);
      if constexpr (FORM == 1) {
        // - i eta e^{i k rho} / (4 pi rho) |J| w
        const double g = eta * sqrt(nx * nx + ny * ny + nz * nz) * ir * INV_4PI * wq;
        v.x += s * g;
        v.y -= c * g;
      } else if constexpr (FORM == 2) {
        // e^{i k rho} / (4 pi rho) |J| w alone
        const double g = sqrt(nx * nx + ny * ny + nz * nz) * ir * INV_4PI * wq;
        v = make_double2(c * g, s * g);
      }
      put(l, j, v);
    }
    return;
  }

  // tables: FFT twiddles (also the azimuth samples) and e^{i pi m / N}
  for (int q = lane; q < LD; q += 64) {
    double s, c;
    sincos_cw(-TWO_PI * q / LD, &s, &c);
    S.tw[twi(q)] = make_double2(c, s);
  }
  for (int q = lane; q < 2 * N; q += 64) {
    double s, c;
    sincos_cw(PI * q / N, &s, &c);
    S.tw2n[q] = make_double2(c, s);
  }
  __syncthreads();

  // lane s < 2N accumulates sum_q w_q P_l(s_q) K_{s-N}(s_q), l < 16
  // (CF: the single-layer modes in acs)
  double2 acc[GL_ORDER];
  double2 acs[CF ? GL_ORDER : 1];
#pragma unroll
  for (int l = 0; l < GL_ORDER; ++l) acc[l] = make_double2(0.0, 0.0);
  if constexpr (CF) {
#pragma unroll
    for (int l = 0; l < GL_ORDER; ++l) acs[l] = make_double2(0.0, 0.0);
  }
  const int nsides = (ip == pT) ? 2 : 1;
  for (int side = 0; side < nsides; ++side) {
    // outer node `lane` (lanes >= the rule's order idle): offset dl from tT
    // and weight (u^5 substitution)
    const int rk = (B.n_ref > 0 || B.n_uni < 2) ? 1 : 0;
    const bool onode = lane < (rk ? NGO : NGO_UNIFORM);
    double dl, w;
    {
      const double u = onode ? orule->x[rk][lane] : 0.5, wu = onode ? orule->w[rk][lane] : 0.0;
      const double u4 = u * u * u * u;
      if (ip == pT) {
        const double ell = (side == 0 ? e0 : e1) - tT;
        dl = ell * u4 * u;
        w = fabs(ell) * 5.0 * u4 * wu;
      } else {
        const double end = (ip < pT) ? e1 : e0;
        const double far = (ip < pT) ? e0 : e1;
        dl = (end - tT) + (far - end) * u4 * u;
        w = fabs(far - end) * 5.0 * u4 * wu;
      }
    }
    // the lane's own node, computed once and broadcast to the wavefront when
    // the node is processed
    const NodeLoc Lme = node_local(shape, a, cc, kappa, TG, dl);
    // and its Lagrange weights P_l(s) on the 16 GL nodes of the panel:
    // b_l prod_{m != l} (x - x_m) by prefix and suffix products
    double P[GL_ORDER];
    {
      const double x = 2.0 * (Lme.s - e0) / h - 1.0;
      double pre = 1.0;
#pragma unroll
      for (int l = 0; l < GL_ORDER; ++l) {
        P[l] = pre;
        pre *= x - gl16[l];
      }
      double suf = 1.0;
#pragma unroll
      for (int l = GL_ORDER - 1; l >= 0; --l) {
        P[l] *= suf * gl16[32 + l] * w;   // with the node's weight
        suf *= x - gl16[l];
      }
    }
    bool modal, wide;
    {
      const NodeLoc& L = Lme;
      modal = onode && L.chim1 < CHI_SPLIT;
      // direct route: modes decay like e^{-acosh(chi) |m|} beyond the width of
      // the oscillatory factor (about k rho_max); 128 samples when the aliased
      // modes |m| >= 128 - N are below 1e-17 of the leading ones
      const double acosh_chi = log1p(L.chim1 + sqrt(L.chim1 * (L.chim1 + 2.0)));
      const double rho_max = sqrt((L.r + L.rt) * (L.r + L.rt) + L.c * L.c);
      wide = acosh_chi * ((LD / 2) - N - (k * rho_max + 10.0)) < 40.0;
    }
    const unsigned long long mmask = __ballot(modal);
    const int nmodal = __popcll(mmask);
    {
      const unsigned long long below = lane ? (mmask & ((1ull << lane) - 1ull)) : 0ull;
      if (modal) S.modal_idx[__popcll(below)] = lane;
    }
    __syncthreads();
    // ---- modal route, in batches of QB nodes (recurrences one node per lane)
    for (int b0 = 0; b0 < nmodal; b0 += QB) {
      const bool qlane = lane < QB && b0 + lane < nmodal;
      const int src = qlane ? S.modal_idx[b0 + lane] : 0;
      const double cm1 = __shfl(Lme.chim1, src);
      const double qchim1 = qlane ? cm1 : 1.0;
      toroidal_q_batch(qlane, 1.0 + qchim1, qchim1, MQ_CAP, S.Q, lane & (QB - 1));
      __syncthreads();
      const int cnt = min(QB, nmodal - b0);
      for (int q = 0; q < cnt; ++q) {
        const int sl = __builtin_amdgcn_readfirstlane(S.modal_idx[b0 + q]);
        const NodeLoc Ln = read_node(Lme, sl);
        modal_modes<CF>(k, Ln.r, Ln.rt, Ln.c, Ln.chim1, Ln.rmrt, N + 1, S.Q, q, S.u.m, S.tw);
        double2 ks;
        const double2 Kq = modal_slot<CF>(N, Ln, S.u.m, ks);
        accumulate_node(acc, P, sl, Kq);
        if constexpr (CF) accumulate_node(acs, P, sl, ks);
        __syncthreads();
      }
    }
    // ---- direct route: trapezoidal rule on L azimuths of the kernel itself,
    // its modes by FFT
    const unsigned long long dmask = ~mmask & __ballot(onode);
    const double k2pi = k / TWO_PI;
    const unsigned long long wmask = __ballot(wide);
    // samples of node q at L azimuths into S.u.K[part][base + l]
    auto sample = [&](int q, int L, int base) {
      const int tstep = LD / L;
      const NodeLoc Lq = read_node(Lme, q);
      Curve cv;
      cv.r = Lq.r; cv.dr = Lq.dr; cv.z = Lq.z; cv.dz = Lq.dz;
      cv.p = Lq.p; cv.dp = Lq.dp; cv.q = Lq.q; cv.dq = Lq.dq;
#pragma unroll
      for (int hh = 0; hh < LD / 64; ++hh) {
        const int l = lane + 64 * hh;
        if (l < L) {
          // (cos, sin)(2 pi l / L) from the twiddle table
          const double2 t = S.tw[twi(l * tstep)];
          const double cth = t.x, sth = -t.y;
          const double dx = cv.r * cth + cv.p - xT, dy = cv.r * sth + cv.q - yT, dz = cv.z - zT;
          const double nx = cv.r * cv.dz * cth, ny = cv.r * cv.dz * sth;
          const double nz = -cv.r * (cv.dr + cv.dp * cth + cv.dq * sth);
          const double r2 = fma(dx, dx, fma(dy, dy, dz * dz));
          const double ir = rsqrt_pos(r2);
          const double rr = r2 * ir;
          double s, c;
          sincos_2pi(rr * k2pi, &s, &c);
          const double sc = (dx * nx + dy * ny + dz * nz) * ir * ir * ir * INV_4PI;
          S.u.K[0][base + l] = make_double2(-fma(k * rr, s, c) * sc, fma(k * rr, c, -s) * sc);
          if constexpr (CF)
            S.u.K[CF ? 1 : 0][base + l] = make_double2(c * ir * INV_4PI, s * ir * INV_4PI);
        }
      }
    };
    // mode slot s = lane of node q: m = s - N (slot 0 also takes m = +N),
    // K_m = (2 pi / L) X[m mod L], accumulated with the node's weights
    auto gather = [&](int q, int L, int base) {
#pragma unroll
      for (int part = 0; part < (CF ? 2 : 1); ++part) {
        double2 Kq = make_double2(0.0, 0.0);
        if (lane < 2 * N) {
          Kq = S.u.K[part][base + ((lane - N + L) & (L - 1))];
          if (lane == 0) {
            const double2 v = S.u.K[part][base + N];
            Kq.x += v.x;
            Kq.y += v.y;
          }
          const double f = TWO_PI / L;
          Kq.x *= f;
          Kq.y *= f;
        }
        if (part == 0) accumulate_node(acc, P, q, Kq);
        else if constexpr (CF) accumulate_node(acs, P, q, Kq);
      }
    };
    // nodes with 256 samples one at a time
    for (unsigned long long dm = dmask & wmask; dm; dm &= dm - 1) {
      const int q = __ffsll(dm) - 1;
      sample(q, LD, 0);
      __syncthreads();
      fft256(S.u.K[0], S.tw);
      if constexpr (CF) fft256(S.u.K[CF ? 1 : 0], S.tw);
      gather(q, LD, 0);
      __syncthreads();
    }
    // nodes with 128 samples two at a time, in the two halves of the buffer
    // through one pair of interleaved transforms (an odd last node leaves the
    // second half's result unused)
    for (unsigned long long dm = dmask & ~wmask; dm;) {
      const int q1 = __ffsll(dm) - 1;
      dm &= dm - 1;
      const int q2 = dm ? __ffsll(dm) - 1 : -1;
      if (dm) dm &= dm - 1;
      sample(q1, LD / 2, 0);
      if (q2 >= 0) sample(q2, LD / 2, LD / 2);
      __syncthreads();
      fft128x2(S.u.K[0], S.u.K[0] + LD / 2, S.tw);
      if constexpr (CF) fft128x2(S.u.K[CF ? 1 : 0], S.u.K[CF ? 1 : 0] + LD / 2, S.tw);
      gather(q1, LD / 2, 0);
      if (q2 >= 0) gather(q2, LD / 2, LD / 2);
      __syncthreads();
    }
  }
  __syncthreads();   // the recurrence batches are done with S.Q (shares S.acc)
  // inverse DFT over the 2N slots: radix-4 FFT passes when 2N is 16 or 64
  const bool fft_inv = 2 * N == 64 || 2 * N == 16;
  store_slots(S, acc, fft_inv);
  __syncthreads();
  double2 g[GL_ORDER];
  if (fft_inv) slots_to_nodes_fft(S, N, g);
  else if (lane < 2 * N) slots_to_nodes(S, N, g);
  if constexpr (CF) {
    // single layer: second inverse DFT, then - i eta |J| (combined field) or
    // |J| (single layer) at the column node
    __syncthreads();
    store_slots(S, acs, fft_inv);
    __syncthreads();
    double2 gs[GL_ORDER];
    if (fft_inv) slots_to_nodes_fft(S, N, gs);
    else if (lane < 2 * N) slots_to_nodes(S, N, gs);
    if (lane < 2 * N) {
      double sj, cj;
      sincos_cw(lane * PI / N, &sj, &cj);
#pragma unroll
      for (int l = 0; l < GL_ORDER; ++l) {
        const double t = e0 + 0.5 * h * (gl16[l] + 1.0);
        const Curve cv = curve_eval(shape, a, cc, kappa, t);
        const double dn = cv.dr + cv.dp * cj + cv.dq * sj;
        const double jac = cv.r * sqrt(cv.dz * cv.dz + dn * dn);
        if constexpr (FORM == 2) {
          g[l] = make_double2(jac * gs[l].x, jac * gs[l].y);
        } else {
          const double f = eta * jac;
          g[l].x = fma(f, gs[l].y, g[l].x);
          g[l].y = fma(-f, gs[l].x, g[l].y);
        }
      }
    }
  }
  if (lane < 2 * N) {
    const bool diag = FORM != 2 && ip == pT && lane == jT;
#pragma unroll
    for (int l = 0; l < GL_ORDER; ++l) {
      double2 v = g[l];
      if (diag && l == lT) v.x += 0.5;     // 1/2 I (second-kind formulations)
      put(l, lane, v);
    }
  }
}

// ---------------------------------------------------------------- launch
static void outer_rule_host(OuterRule& R) {
  const int orders[2] = {NGO_UNIFORM, NGO};
  for (int q = 0; q < 2; ++q) {
    double x[NGO], w[NGO];
    gauss_legendre_host(orders[q], x, w);
    for (int i = 0; i < NGO; ++i) {
      R.x[q][i] = i < orders[q] ? 0.5 * (x[i] + 1.0) : 0.5;
      R.w[q][i] = i < orders[q] ? 0.5 * w[i] : 0.0;
    }
  }
}

hipError_t launch_assemble_self(qax_problem* p) {
  std::vector<SelfTask> tasks;
  for (int bk = 0; bk < (int)p->hblocks.size(); ++bk) {
    const BodyDev& B = p->hbodies[p->hblocks[bk].rep_body];
    const int n = p->hblocks[bk].n, nth = B.n_theta, ns = n / nth;
    // mirror-symmetric bodies: the rows s < n_s / 2, j <= N (the kernel
    // stores the others as their images)
    const bool mir = mirror_symmetric(B.shape);
    for (int row = 0; row < n; ++row) {
      if (mir && (row / nth >= ns / 2 || row % nth > nth / 2)) continue;
      for (int pan = 0; pan < B.n_panels; ++pan) tasks.push_back(SelfTask{bk, row, pan});
    }
  }
  // self-panel work items first (outer nodes on both sides of the target,
  // most of them on the modal route), then adjacent panels, then the far
  // panels' smooth rule: the hardware issues workgroups in index order, so
  // the long items start early and the short ones fill the end of the launch
  // (1000-body workload: 82.6 -> 60.3 ms per assembly; 27-body lattice
  // 8.7 -> 5.6 ms)
  {
    auto rank = [&](const SelfTask& t) {
      const int nth = p->hbodies[p->hblocks[t.block].rep_body].n_theta;
      const int d = abs(t.panel - t.row / (GL_ORDER * nth));
      return d == 0 ? 0 : d == 1 ? 1 : 2;
    };
    std::stable_sort(tasks.begin(), tasks.end(),
                     [&](const SelfTask& a, const SelfTask& b) { return rank(a) < rank(b); });
  }
  OuterRule R;
  outer_rule_host(R);
  SelfTask* d_tasks = nullptr;
  OuterRule* d_rule = nullptr;
  hipError_t e = hipMalloc(&d_tasks, tasks.size() * sizeof(SelfTask));
  if (e != hipSuccess) return e;
  e = hipMalloc(&d_rule, sizeof(OuterRule));
  if (e != hipSuccess) { (void)hipFree(d_tasks); return e; }
  e = hipMemcpyAsync(d_tasks, tasks.data(), tasks.size() * sizeof(SelfTask), hipMemcpyHostToDevice, p->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(d_rule, &R, sizeof(R), hipMemcpyHostToDevice, p->stream);
  if (e == hipSuccess) {
    timing_begin(p, QAX_K_SELF_ASSEMBLY);
    const int form = p->form();
    auto kern = form == 1 ? assemble_self_kernel<1> : form == 2 ? assemble_self_kernel<2>
                                                                  : assemble_self_kernel<0>;
    hipLaunchKernelGGL(kern, dim3((unsigned)tasks.size()), dim3(64), 0, p->stream, d_tasks,
                       p->d_blocks, p->d_bodies, p->d_gl, d_rule, (double2*)p->d_B);
    timing_end(p, QAX_K_SELF_ASSEMBLY);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
  (void)hipFree(d_tasks);
  (void)hipFree(d_rule);
  return e;
}

// ---------------------------------------------------------------- test hook
__global__ __launch_bounds__(64) void modal_modes_kernel(const double* __restrict__ r,
                                                         const double* __restrict__ rt,
                                                         const double* __restrict__ c,
                                                         const double* __restrict__ chim1,
                                                         const double* __restrict__ rmrt, double k,
                                                         int nmax, double2* __restrict__ A,
                                                         double2* __restrict__ B) {
  __shared__ SelfShared<false> S;
  const int pt = blockIdx.x;
  const int lane = threadIdx.x;
  for (int q = lane; q < LD; q += 64) {
    double s, cc;
    sincos_cw(-TWO_PI * q / LD, &s, &cc);
    S.tw[twi(q)] = make_double2(cc, s);
  }
  toroidal_q_batch(lane == 0, 1.0 + chim1[pt], chim1[pt], MQ_CAP, S.Q, lane & (QB - 1));
  __syncthreads();
  modal_modes<false>(k, r[pt], rt[pt], c[pt], chim1[pt], rmrt[pt], nmax, S.Q, 0, S.u.m, S.tw);
  if (lane <= nmax) {
    A[(int64_t)pt * (nmax + 1) + lane] = S.u.m.Am[lane];
    B[(int64_t)pt * (nmax + 1) + lane] = S.u.m.Bm[lane];
  }
}

hipError_t launch_modal_modes(hipStream_t s, int n, const double* r, const double* rt,
                              const double* c, const double* chim1, const double* rmrt, double k,
                              int nmax, double* A, double* B) {
  if (nmax > NTH_MAX / 2 + 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(modal_modes_kernel, dim3(n), dim3(64), 0, s, r, rt, c, chim1, rmrt, k, nmax,
                     (double2*)A, (double2*)B);
  return hipGetLastError();
}

}  // namespace qax
