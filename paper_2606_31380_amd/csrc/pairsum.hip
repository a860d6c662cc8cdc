// Inter-body double-layer pair sum (Section 4, the display after the equation
// for the second part of the multi-body potential); with the combined field
// the single-layer term - i eta G(x_i, y_j) |aw_j| mu_j is added per pair:
//
//   w_i = 1/(4 pi) sum_{j in other bodies} (ik r - 1) e^{ikr} / r^3
//                                          (aw_j . (y_j - x_i)) mu_j,
//   r = |y_j - x_i|,  aw_j = n_j |J_j| (pi/N) omega_j.
//
// A tiled N-body kernel on the vector ALUs: source tiles are staged in LDS,
// every thread owns one target.  Work is cut into tasks (target block x range
// of source bodies) listed in a table sorted by cost, so that uneven bodies and
// independent problems share one launch; the partial sums of the tasks of one
// target row are reduced by a second kernel in a fixed order (deterministic).
//
// FP64 path: plain FP64 arithmetic.
// FP32 path: the phase k r is never formed in FP32.  For target x_i and source
// body b with centre c_b, D = c_b - x_i, |D| and frac(k|D|/2pi) are formed in
// FP64 once per (target, body).  Per pair, with y' = y_j - c_b stored in FP32,
// num = 2 D.y' + |y'|^2 = r^2 - |D|^2 is formed without cancellation, r^2 =
// |D|^2 + num, and delta = r - |D| = num / (r + |D|); the phase
// frac(k|D|/2pi) + k delta/2pi then carries only the FP32 rounding of delta
// (relative), not that of r (absolute, ulp(|D|)).  Sums are accumulated in FP32 per
// tile and the tile sums are added with an error-free TwoSum (compensated
// accumulation).
#include <algorithm>
#include <cmath>
#include <vector>

#include "fastmath.h"
#include "internal.h"

namespace qax {

constexpr double INV_FOUR_PI = 0.0795774715459476678844;

// Lockstep solves pass seg_active[problem * nrhs + r] (0 once that GMRES
// segment has converged in the current cycle; its basis vectors are then
// zero).  A task none of whose right-hand sides is active writes zeros to its
// partial sums and does no pair work.  The test is uniform over the block.
template <int NRC>
__device__ __forceinline__ bool skip_task(const PairTask& T, const BodyDev* __restrict__ bodies,
                                          const int32_t* __restrict__ seg_active, int nrhs, int rc0,
                                          bool active, int64_t i, int64_t N,
                                          double2* __restrict__ partial) {
  if (!seg_active) return false;
  const int pr = bodies[T.tbody_lo].problem;
  bool any = false;
  for (int r = rc0; r < rc0 + NRC && r < nrhs; ++r) any = any || seg_active[pr * nrhs + r] != 0;
  if (any) return false;
  if (active) {
    double2* dst = partial + (int64_t)T.slot * N * nrhs;
    for (int r = rc0; r < rc0 + NRC && r < nrhs; ++r) dst[i * nrhs + r] = make_double2(0.0, 0.0);
  }
  return true;
}

template <int TPB, int NRC, int FORM>
__global__ __launch_bounds__(TPB) void pair_sum_f64_kernel(
    const PairTask* __restrict__ tasks, const BodyDev* __restrict__ bodies,
    const int32_t* __restrict__ node_body, const double* __restrict__ pos,
    const double* __restrict__ aw, const double* __restrict__ ew, int64_t N,
    const double2* __restrict__ mu, int nrhs,
    const int32_t* __restrict__ seg_active, double2* __restrict__ partial) {
  const PairTask T = tasks[blockIdx.x];
  const int rc0 = blockIdx.y * NRC;  // first right-hand side of this chunk
  const int tid = threadIdx.x;
  const bool active = tid < T.nt;
  const int64_t i = T.t0 + (active ? tid : 0);
  if (skip_task<NRC>(T, bodies, seg_active, nrhs, rc0, active, i, N, partial)) return;
  const double xi = pos[i], yi = pos[N + i], zi = pos[2 * N + i];
  const int mybody = node_body[i];
  const double k = T.k;

  __shared__ double sx[TPB], sy[TPB], sz[TPB], sax[TPB], say[TPB], saz[TPB];
  __shared__ double sew[FORM ? TPB : 1];
  __shared__ double2 smu[TPB * NRC];

  double accr[NRC], acci[NRC];
#pragma unroll
  for (int r = 0; r < NRC; ++r) { accr[r] = 0.0; acci[r] = 0.0; }
  // one right-hand side: S1 = sum sc z, S2 = sum u z (S3 = sum t z), see below
  double ar = 0.0, ai = 0.0, br = 0.0, bi = 0.0, er = 0.0, ei = 0.0;
  const double k2pi = k / TWO_PI;

  for (int b = T.b0; b < T.b1; ++b) {
    if (T.tbody_lo == b && T.tbody_hi == b) continue;  // every target is in body b
    const int64_t s0 = bodies[b].off;
    const int nb = bodies[b].n;
    const bool own = (mybody == b);
    for (int base = 0; base < nb; base += TPB) {
      const int cnt = min(TPB, nb - base);
      __syncthreads();
      if (tid < cnt) {
        const int64_t j = s0 + base + tid;
        sx[tid] = pos[j]; sy[tid] = pos[N + j]; sz[tid] = pos[2 * N + j];
        sax[tid] = aw[j]; say[tid] = aw[N + j]; saz[tid] = aw[2 * N + j];
        if (FORM) sew[tid] = ew[j];
#pragma unroll
        for (int r = 0; r < NRC; ++r)
          smu[tid * NRC + r] = (rc0 + r < nrhs) ? mu[j * nrhs + rc0 + r] : make_double2(0.0, 0.0);
      }
      __syncthreads();
      if (!own && NRC == 1 && FORM != 2) {
        // with e = e^{ikr}, z = e mu and r ir = 1 the double-layer term is
        // (ikr - 1) e (aw . (y - x)) / r^3 mu = -sc z + i k u z, sc = dot ir^3,
        // u = dot ir^2; the phase kr / 2 pi = r^2 ir k / 2 pi in revolutions
        // (combined field: - i eta G |aw| mu = - i t z, t = eta |aw| ir)
        for (int jj = 0; jj < cnt; ++jj) {
          const double dx = sx[jj] - xi, dy = sy[jj] - yi, dz = sz[jj] - zi;
          const double r2 = fma(dx, dx, fma(dy, dy, dz * dz));
          const double ir = rsqrt_pos(r2);
          double s, c;
          sincos_2pi(r2 * ir * k2pi, &s, &c);
          const double2 m = smu[jj];
          const double zr = fma(c, m.x, -s * m.y);
          const double zi = fma(c, m.y, s * m.x);
          const double dot = fma(sax[jj], dx, fma(say[jj], dy, saz[jj] * dz));
          const double u = dot * ir * ir;
          const double sc = u * ir;
          ar = fma(sc, zr, ar);
          ai = fma(sc, zi, ai);
          br = fma(u, zr, br);
          bi = fma(u, zi, bi);
          if constexpr (FORM == 1) {
            const double t = sew[jj] * ir;
            er = fma(t, zr, er);
            ei = fma(t, zi, ei);
          }
        }
      } else if (!own) {
        for (int jj = 0; jj < cnt; ++jj) {
          const double dx = sx[jj] - xi, dy = sy[jj] - yi, dz = sz[jj] - zi;
          const double r2 = fma(dx, dx, fma(dy, dy, dz * dz));
          const double ir = rsqrt_pos(r2);
          const double r = r2 * ir;
          const double kr = k * r;
          double s, c;
          sincos_cw(kr, &s, &c);
          double re, im;
          if constexpr (FORM == 2) {   // G |aw|: (|aw| / r)(cos kr + i sin kr)
            const double t = sew[jj] * ir;
            re = c * t;
            im = s * t;
          } else {
            const double dot = sax[jj] * dx + say[jj] * dy + saz[jj] * dz;
            const double sc = dot * ir * ir * ir;
            re = -(c + kr * s) * sc;
            im = (kr * c - s) * sc;
            if constexpr (FORM == 1) {   // - i eta G |aw|: (eta |aw| / r)(sin kr - i cos kr)
              const double t = sew[jj] * ir;
              re = fma(t, s, re);
              im = fma(-t, c, im);
            }
          }
#pragma unroll
          for (int r_ = 0; r_ < NRC; ++r_) {
            const double2 m = smu[jj * NRC + r_];
            accr[r_] = fma(re, m.x, fma(-im, m.y, accr[r_]));
            acci[r_] = fma(re, m.y, fma(im, m.x, acci[r_]));
          }
        }
      }
    }
  }
  if (NRC == 1 && FORM != 2) {   // -S1 + i k S2 (- i S3)
    accr[0] += fma(-k, bi, ei - ar);
    acci[0] += fma(k, br, -ai - er);
  }
  if (active) {
    double2* dst = partial + (int64_t)T.slot * N * nrhs;
#pragma unroll
    for (int r = 0; r < NRC; ++r)
      if (rc0 + r < nrhs)
        dst[i * nrhs + rc0 + r] = make_double2(accr[r] * INV_FOUR_PI, acci[r] * INV_FOUR_PI);
  }
}

__device__ __forceinline__ void two_sum(float& s, float& c, float a) {
  const float t = s + a;
  const float bp = t - s;
  const float e = (s - (t - bp)) + (a - bp);
  s = t;
  c += e;
}

template <int TPB, int NRC, int FORM>
__global__ __launch_bounds__(TPB) void pair_sum_f32_kernel(
    const PairTask* __restrict__ tasks, const BodyDev* __restrict__ bodies,
    const int32_t* __restrict__ node_body, const double* __restrict__ pos,
    const float4* __restrict__ loc32, const float4* __restrict__ aw32,
    const float* __restrict__ ew32, int64_t N,
    const double2* __restrict__ mu, int nrhs, const int32_t* __restrict__ seg_active,
    double2* __restrict__ partial) {
  const PairTask T = tasks[blockIdx.x];
  const int rc0 = blockIdx.y * NRC;
  const int tid = threadIdx.x;
  const bool active = tid < T.nt;
  const int64_t i = T.t0 + (active ? tid : 0);
  if (skip_task<NRC>(T, bodies, seg_active, nrhs, rc0, active, i, N, partial)) return;
  const double xi = pos[i], yi = pos[N + i], zi = pos[2 * N + i];
  const int mybody = node_body[i];
  const double k = T.k;
  const float kf = (float)k;
  const float k2pi = (float)(k / TWO_PI);

  __shared__ float4 sloc[TPB];
  __shared__ float4 saw[TPB];
  __shared__ float sew[FORM ? TPB : 1];
  __shared__ float2 smu[TPB * NRC];

  float sr[NRC], si[NRC], cr[NRC], ci[NRC];
#pragma unroll
  for (int r = 0; r < NRC; ++r) { sr[r] = si[r] = cr[r] = ci[r] = 0.0f; }

  for (int b = T.b0; b < T.b1; ++b) {
    if (T.tbody_lo == b && T.tbody_hi == b) continue;
    const BodyDev& B = bodies[b];
    const int64_t s0 = B.off;
    const int nb = B.n;
    const bool own = (mybody == b);
    // per (target, source body) set-up in FP64: D = c_b - x_i, |D|, |D|^2 and
    // the phase frac(k |D| / 2 pi)
    const double Dx = B.cen[0] - xi, Dy = B.cen[1] - yi, Dz = B.cen[2] - zi;
    const double D2 = Dx * Dx + Dy * Dy + Dz * Dz;
    const double Dn = sqrt(D2);
    double ph0d = k * Dn / TWO_PI;
    ph0d -= floor(ph0d);
    const float dxf = (float)Dx, dyf = (float)Dy, dzf = (float)Dz;
    const float dx2 = 2.0f * dxf, dy2 = 2.0f * dyf, dz2 = 2.0f * dzf;
    const float d2f = (float)D2;
    const float dnf = (float)Dn;
    // scaled set-up of the one-right-hand-side loop (k > 0): kappa = 2 pi / k
    const double kap = k > 0.0 ? TWO_PI / k : 1.0;
    const float kap2 = (float)(kap * kap), d2s = (float)(kap * kap * D2), dns = (float)(kap * Dn);
    const float ck1 = (float)kap, ck2 = (float)(k * kap * kap), ck3 = (float)(kap * kap * kap);
    const float ph0 = (float)ph0d;
    for (int base = 0; base < nb; base += TPB) {
      const int cnt = min(TPB, nb - base);
      __syncthreads();
      if (tid < cnt) {
        const int64_t j = s0 + base + tid;
        sloc[tid] = loc32[j];
        saw[tid] = aw32[j];
        if (FORM) sew[tid] = ew32[j];
#pragma unroll
        for (int r = 0; r < NRC; ++r) {
          const double2 m = (rc0 + r < nrhs) ? mu[j * nrhs + rc0 + r] : make_double2(0.0, 0.0);
          smu[tid * NRC + r] = make_float2((float)m.x, (float)m.y);
        }
      }
      __syncthreads();
      if (!own && NRC == 1 && FORM != 2 && k == 0.0) {
        // Laplace (e = 1): -S1 (- i S3) with S1 = sum dot ir^3 mu
        float ar = 0.0f, ai = 0.0f, er = 0.0f, ei = 0.0f;
#pragma unroll 4
        for (int jj = 0; jj < cnt; ++jj) {
          const float4 yl = sloc[jj];
          const float4 a4 = saw[jj];
          const float num = fmaf(dx2, yl.x, fmaf(dy2, yl.y, fmaf(dz2, yl.z, yl.w)));
          const float ir = __builtin_amdgcn_rsqf(d2f + num);
          const float2 m = smu[jj];
          const float dot = fmaf(a4.x, dxf, fmaf(a4.y, dyf, fmaf(a4.z, dzf, a4.w)));
          const float sc = dot * ir * ir * ir;
          ar = fmaf(sc, m.x, ar);
          ai = fmaf(sc, m.y, ai);
          if constexpr (FORM == 1) {
            const float t = sew[jj] * ir;
            er = fmaf(t, m.x, er);
            ei = fmaf(t, m.y, ei);
          }
        }
        two_sum(sr[0], cr[0], ei - ar);
        two_sum(si[0], ci[0], -ai - er);
      } else if (!own && NRC == 1 && FORM != 2) {
        // one right-hand side: with e = e^{ikr}, z = e mu and r ir = 1 the
        // double-layer term is (ikr - 1) e (aw . (y - x)) / r^3 mu
        // = -sc z + i k u z, sc = dot ir^3, u = dot ir^2, so the tile sums
        // S1 = sum sc z and S2 = sum u z need neither r nor kr
        // (combined-field: - i eta G |aw| mu = - i t z, t = eta |aw| ir).
        // Distances scaled by kappa = 2 pi / k: r'^2 = kappa^2 (|D|^2 + num),
        // ir' = ir / kappa, r'^2 ir' + kappa |D| = kappa (r + |D|), so the
        // phase increment k delta / 2 pi = num / (kappa (r + |D|)) is one fma;
        // the sums carry kappa^-3 (S1), kappa^-2 (S2), kappa^-1 (S3), undone
        // per tile
        float ar = 0.0f, ai = 0.0f, br = 0.0f, bi = 0.0f, er = 0.0f, ei = 0.0f;
#pragma unroll 4
        for (int jj = 0; jj < cnt; ++jj) {
          const float4 yl = sloc[jj];
          const float4 a4 = saw[jj];
          const float num = fmaf(dx2, yl.x, fmaf(dy2, yl.y, fmaf(dz2, yl.z, yl.w)));
          const float r2s = fmaf(kap2, num, d2s);
          const float irs = __builtin_amdgcn_rsqf(r2s);
          const float ph = fmaf(num, __builtin_amdgcn_rcpf(fmaf(r2s, irs, dns)), ph0);
          const float s = __builtin_amdgcn_sinf(ph);
          const float c = __builtin_amdgcn_cosf(ph);
          const float2 m = smu[jj];
          const float zr = fmaf(c, m.x, -s * m.y);
          const float zi = fmaf(c, m.y, s * m.x);
          const float dot = fmaf(a4.x, dxf, fmaf(a4.y, dyf, fmaf(a4.z, dzf, a4.w)));
          const float u = dot * irs * irs;
          const float sc = u * irs;
          ar = fmaf(sc, zr, ar);
          ai = fmaf(sc, zi, ai);
          br = fmaf(u, zr, br);
          bi = fmaf(u, zi, bi);
          if constexpr (FORM == 1) {
            const float t = sew[jj] * irs;
            er = fmaf(t, zr, er);
            ei = fmaf(t, zi, ei);
          }
        }
        // -S1 + i k S2 (- i S3)
        two_sum(sr[0], cr[0], fmaf(-ck2, bi, fmaf(ck1, ei, -ck3 * ar)));
        two_sum(si[0], ci[0], fmaf(ck2, br, fmaf(-ck1, er, -ck3 * ai)));
      } else if (!own) {
        float tr[NRC], ti[NRC];
#pragma unroll
        for (int r = 0; r < NRC; ++r) { tr[r] = 0.0f; ti[r] = 0.0f; }
#pragma unroll 4
        for (int jj = 0; jj < cnt; ++jj) {
          const float4 yl = sloc[jj];      // y' = y_j - c_b, |y'|^2
          const float4 a4 = saw[jj];       // aw_j, aw_j . y'
          // num = 2 D.y' + |y'|^2 = r^2 - |D|^2 without cancellation
          const float num = fmaf(dx2, yl.x, fmaf(dy2, yl.y, fmaf(dz2, yl.z, yl.w)));
          const float r2 = d2f + num;
          const float ir = __builtin_amdgcn_rsqf(r2);
          const float r = r2 * ir;
          // delta = r - |D| = num / (r + |D|): the phase is never formed from r
          const float delta = num * __builtin_amdgcn_rcpf(r + dnf);
          const float ph = fmaf(delta, k2pi, ph0);            // revolutions
          const float s = __builtin_amdgcn_sinf(ph);
          const float c = __builtin_amdgcn_cosf(ph);
          float re, im;
          if constexpr (FORM == 2) {   // G |aw|: (|aw| / r)(cos kr + i sin kr)
            const float t = sew[jj] * ir;
            re = c * t;
            im = s * t;
          } else {
            const float kr = kf * r;
            // aw . (y - x) = aw . D + aw . y'
            const float dot = fmaf(a4.x, dxf, fmaf(a4.y, dyf, fmaf(a4.z, dzf, a4.w)));
            const float sc = dot * (ir * ir * ir);
            re = -fmaf(kr, s, c) * sc;                         // Re (ikr - 1) e^{ikr} / r^3 (.)
            im = fmaf(kr, c, -s) * sc;
            if constexpr (FORM == 1) {   // - i eta G |aw|: (eta |aw| / r)(sin kr - i cos kr)
              const float t = sew[jj] * ir;
              re = fmaf(t, s, re);
              im = fmaf(-t, c, im);
            }
          }
#pragma unroll
          for (int r_ = 0; r_ < NRC; ++r_) {
            const float2 m = smu[jj * NRC + r_];
            tr[r_] = fmaf(re, m.x, tr[r_]);
            tr[r_] = fmaf(-im, m.y, tr[r_]);
            ti[r_] = fmaf(re, m.y, ti[r_]);
            ti[r_] = fmaf(im, m.x, ti[r_]);
          }
        }
#pragma unroll
        for (int r = 0; r < NRC; ++r) {
          two_sum(sr[r], cr[r], tr[r]);
          two_sum(si[r], ci[r], ti[r]);
        }
      }
    }
  }
  if (active) {
    double2* dst = partial + (int64_t)T.slot * N * nrhs;
#pragma unroll
    for (int r = 0; r < NRC; ++r)
      if (rc0 + r < nrhs)
        dst[i * nrhs + rc0 + r] =
            make_double2(((double)sr[r] + (double)cr[r]) * INV_FOUR_PI,
                         ((double)si[r] + (double)ci[r]) * INV_FOUR_PI);
  }
}

// out[e] = (accumulate ? out[e] : 0) + sum_s partial[s][e], fixed order.
__global__ void reduce_slots_kernel(const double2* __restrict__ partial, int slots, int64_t count,
                                    double2* __restrict__ out, int accumulate) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= count) return;
  double2 acc = accumulate ? out[e] : make_double2(0.0, 0.0);
  for (int s = 0; s < slots; ++s) {
    const double2 v = partial[(int64_t)s * count + e];
    acc.x += v.x;
    acc.y += v.y;
  }
  out[e] = acc;
}

// ---------------------------------------------------------------------------
// Reciprocal FP32 pair sum (one right-hand side, double layer or combined
// field, k > 0).  For x_i on body a and y_j on body b != a, the distance r,
// the phase and e^{ikr} are the same for the pair (target i, source j) and
// the pair (target j, source i); only the double-layer dot products and the
// densities differ.  Each unordered pair of bodies a < b is visited once, as
// tasks of a block of SYM_T nodes of a against a block of SYM_T nodes of b,
// so the shared part of a pair is computed once for both directions.  The
// blocks keep tasks small enough that the workgroups fill the chip evenly.
//
// Coordinates are local to each body: x_i = c_a + x', y_j = c_b + y',
// C = c_b - c_a.  With P_j = 2 C.y' + |y'|^2 and Q_i = |x'|^2 - 2 C.x',
//   num = r^2 - |C|^2 = P_j + Q_i - 2 x'.y'
// (no cancellation against |C|^2), delta = r - |C| = num / (r + |C|), and the
// phase is frac(k |C| / 2 pi) + k delta / 2 pi, in the kappa-scaled form of
// the per-target kernel.  The dot products are
//   aw_j . (y_j - x_i) = A_j - aw_j . x',  A_j = aw_j . (C + y'),
//   aw_i . (x_i - y_j) = B_i - aw_i . y',  B_i = aw_i . (x' - C).
//
// A workgroup is two wavefronts; lane l owns targets l and l + 64 of its
// wavefront's 128.  Sources pass in chunks of 64; at step s lane l meets
// source (l + s) mod 64 of the chunk, so the 64 lanes of a wavefront see 64
// distinct sources at every step.  The chunk is staged twice over (indices
// 0..127), which turns (l + s) mod 64 into l + s.  The target-side sums stay
// in registers (FP32 per chunk, compensated across chunks).  The source-side
// sums travel with their source: lane l holds the running sums of source
// (l + s) mod 64 at step s, and the next step receives them from lane l + 1
// (a wavefront rotation fused into the add), so after the chunk lane l holds
// those of source (l + 63) mod 64.  The two wavefronts' sums of a source are
// added through LDS (FP32 sums over the task's targets).  Both sides' task
// sums are stored as complex64 and added in FP64 by the reduction.
__device__ __forceinline__ float from_next_lane(float x) {
  // DPP wavefront rotation: lane l reads lane (l + 1) mod 64
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x134, 0xf, 0xf, false));
}

template <int FORM>
__global__ __launch_bounds__(128) void pair_sum_f32_sym_kernel(
    const SymTask* __restrict__ tasks, const BodyDev* __restrict__ bodies,
    const float4* __restrict__ loc32, const float4* __restrict__ aw32,
    const float* __restrict__ ew32, const double2* __restrict__ mu,
    const int32_t* __restrict__ seg_active, float2* __restrict__ part) {
  constexpr int NA = FORM ? 6 : 4;   // source-side sums: S1, S2 (, S3), re/im
  const SymTask T = tasks[blockIdx.x];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const BodyDev& BA = bodies[T.a];
  const BodyDev& BB = bodies[T.b];
  if (seg_active && seg_active[BA.problem] == 0) {
    for (int t = tid; t < T.nt; t += 128) part[T.ioff + t] = make_float2(0.0f, 0.0f);
    for (int j = tid; j < T.nb; j += 128) part[T.joff + j] = make_float2(0.0f, 0.0f);
    return;
  }
  const double k = BA.k;
  const double Cx = BB.cen[0] - BA.cen[0], Cy = BB.cen[1] - BA.cen[1], Cz = BB.cen[2] - BA.cen[2];
  const double C2 = Cx * Cx + Cy * Cy + Cz * Cz;
  const double Cn = sqrt(C2);
  double ph0d = k * Cn / TWO_PI;
  ph0d -= floor(ph0d);
  const double kap = TWO_PI / k;
  const float kap2 = (float)(kap * kap), d2s = (float)(kap * kap * C2), dns = (float)(kap * Cn);
  const float ck1 = (float)kap, ck2 = (float)(k * kap * kap), ck3 = (float)(kap * kap * kap);
  const float ph0 = (float)ph0d;
  const float cx = (float)Cx, cy = (float)Cy, cz = (float)Cz;

  // the lane's two targets: -x', Q_i, -aw_i / 2, B_i, mu_i (0 past the block)
  float mx[2], my[2], mz[2], q[2], hx[2], hy[2], hz[2], bv[2], mr[2], mi[2], ew[2];
  float sr[2], si[2], cr[2], ci[2];
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    const int loc = wv * 128 + t * 64 + lane;
    const bool act = loc < T.nt;
    const int64_t i = T.t0 + (act ? loc : 0);
    const float4 x4 = loc32[i];
    const float4 a4 = aw32[i];
    mx[t] = -x4.x;
    my[t] = -x4.y;
    mz[t] = -x4.z;
    q[t] = fmaf(-2.0f * cx, x4.x, fmaf(-2.0f * cy, x4.y, fmaf(-2.0f * cz, x4.z, x4.w)));
    hx[t] = -0.5f * a4.x;
    hy[t] = -0.5f * a4.y;
    hz[t] = -0.5f * a4.z;
    bv[t] = a4.w - fmaf(a4.x, cx, fmaf(a4.y, cy, a4.z * cz));
    const double2 m = act ? mu[i] : make_double2(0.0, 0.0);
    mr[t] = (float)m.x;
    mi[t] = (float)m.y;
    ew[t] = FORM ? ew32[i] : 0.0f;
    sr[t] = si[t] = cr[t] = ci[t] = 0.0f;
  }

  __shared__ float4 sY[128];           // 2 y', P_j
  __shared__ float4 sW[128];           // aw_j, A_j
  __shared__ float4 sM[128];           // mu_j, eta |aw_j|
  __shared__ float sX[NA][64];         // second wavefront's source-side sums

  const int src = (lane + 63) & 63;    // source of the lane's sums after a chunk
  const int nch = (T.nb + 63) / 64;
  for (int c = 0; c < nch; ++c) {
    if (tid < 64) {
      const int jl = c * 64 + tid;
      const bool act = jl < T.nb;
      const int64_t j = T.s0 + (act ? jl : 0);
      const float4 y4 = loc32[j];
      const float4 b4 = aw32[j];
      const double2 m = act ? mu[j] : make_double2(0.0, 0.0);
      const float4 Y = make_float4(2.0f * y4.x, 2.0f * y4.y, 2.0f * y4.z,
                                   fmaf(2.0f * cx, y4.x, fmaf(2.0f * cy, y4.y, fmaf(2.0f * cz, y4.z, y4.w))));
      const float4 W = make_float4(b4.x, b4.y, b4.z, b4.w + fmaf(b4.x, cx, fmaf(b4.y, cy, b4.z * cz)));
      const float4 M = make_float4((float)m.x, (float)m.y, FORM ? ew32[j] : 0.0f, 0.0f);
      sY[tid] = Y;
      sY[tid + 64] = Y;
      sW[tid] = W;
      sW[tid + 64] = W;
      sM[tid] = M;
      sM[tid + 64] = M;
    }
    __syncthreads();
    float ar[2], ai[2], br[2], bi[2], er[2], ei[2];
#pragma unroll
    for (int t = 0; t < 2; ++t) ar[t] = ai[t] = br[t] = bi[t] = er[t] = ei[t] = 0.0f;
    float acc[NA];
#pragma unroll
    for (int a = 0; a < NA; ++a) acc[a] = 0.0f;
    const float4* pY = &sY[lane];
    const float4* pW = &sW[lane];
    const float4* pM = &sM[lane];
#pragma unroll 4
    for (int st = 0; st < 64; ++st) {
      const float4 Y = pY[st];
      const float4 W = pW[st];
      const float4 M = pM[st];
      float cn[NA];
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        // shared: r, e^{ikr} (scaled as in the per-target kernel)
        const float num = fmaf(mx[t], Y.x, fmaf(my[t], Y.y, fmaf(mz[t], Y.z, Y.w + q[t])));
        const float r2s = fmaf(kap2, num, d2s);
        const float irs = __builtin_amdgcn_rsqf(r2s);
        const float ph = fmaf(num, __builtin_amdgcn_rcpf(fmaf(r2s, irs, dns)), ph0);
        const float sn = __builtin_amdgcn_sinf(ph);
        const float cs = __builtin_amdgcn_cosf(ph);
        const float ir2 = irs * irs;
        // target i, source j
        {
          const float zr = fmaf(cs, M.x, -sn * M.y);
          const float zi = fmaf(cs, M.y, sn * M.x);
          const float dot = fmaf(W.x, mx[t], fmaf(W.y, my[t], fmaf(W.z, mz[t], W.w)));
          const float u = dot * ir2;
          const float sc = u * irs;
          ar[t] = fmaf(sc, zr, ar[t]);
          ai[t] = fmaf(sc, zi, ai[t]);
          br[t] = fmaf(u, zr, br[t]);
          bi[t] = fmaf(u, zi, bi[t]);
          if constexpr (FORM == 1) {
            const float tt = M.z * irs;
            er[t] = fmaf(tt, zr, er[t]);
            ei[t] = fmaf(tt, zi, ei[t]);
          }
        }
        // target j, source i
        {
          const float zr = fmaf(cs, mr[t], -sn * mi[t]);
          const float zi = fmaf(cs, mi[t], sn * mr[t]);
          const float dot = fmaf(hx[t], Y.x, fmaf(hy[t], Y.y, fmaf(hz[t], Y.z, bv[t])));
          const float u = dot * ir2;
          const float sc = u * irs;
          const float tt = FORM ? ew[t] * irs : 0.0f;
          if (t == 0) {
            cn[0] = sc * zr;
            cn[1] = sc * zi;
            cn[2] = u * zr;
            cn[3] = u * zi;
            if constexpr (FORM == 1) {
              cn[4] = tt * zr;
              cn[5] = tt * zi;
            }
          } else {
            cn[0] = fmaf(sc, zr, cn[0]);
            cn[1] = fmaf(sc, zi, cn[1]);
            cn[2] = fmaf(u, zr, cn[2]);
            cn[3] = fmaf(u, zi, cn[3]);
            if constexpr (FORM == 1) {
              cn[4] = fmaf(tt, zr, cn[4]);
              cn[5] = fmaf(tt, zi, cn[5]);
            }
          }
        }
      }
#pragma unroll
      for (int a = 0; a < NA; ++a) acc[a] = from_next_lane(acc[a]) + cn[a];
    }
    // -S1 + i k S2 (- i S3), undoing the kappa scaling
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      two_sum(sr[t], cr[t], fmaf(-ck2, bi[t], fmaf(ck1, ei[t], -ck3 * ar[t])));
      two_sum(si[t], ci[t], fmaf(ck2, br[t], fmaf(-ck1, er[t], -ck3 * ai[t])));
    }
    if (wv == 1) {
#pragma unroll
      for (int a = 0; a < NA; ++a) sX[a][lane] = acc[a];
    }
    __syncthreads();
    if (wv == 0 && c * 64 + src < T.nb) {
      float v[NA];
#pragma unroll
      for (int a = 0; a < NA; ++a) v[a] = acc[a] + sX[a][lane];
      const float e3r = FORM ? v[4] : 0.0f, e3i = FORM ? v[5] : 0.0f;
      const float vr = fmaf(-ck2, v[3], fmaf(ck1, e3i, -ck3 * v[0]));
      const float vi = fmaf(ck2, v[2], fmaf(-ck1, e3r, -ck3 * v[1]));
      part[T.joff + c * 64 + src] =
          make_float2(vr * (float)INV_FOUR_PI, vi * (float)INV_FOUR_PI);
    }
  }
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    const int loc = wv * 128 + t * 64 + lane;
    if (loc < T.nt)
      part[T.ioff + loc] = make_float2((float)(((double)sr[t] + (double)cr[t]) * INV_FOUR_PI),
                                       (float)(((double)si[t] + (double)ci[t]) * INV_FOUR_PI));
  }
}

// FP64 reciprocal pair sum: the same tasks, lane mapping and rotation of the
// source-side sums as the FP32 kernel, in plain FP64 on absolute positions
// (d = y_j - x_i, r^2 = |d|^2, phase r k / 2 pi in revolutions for
// sincos_2pi); aw_j . (y_j - x_i) = aw_j . d and aw_i . (x_i - y_j) =
// -aw_i . d.  Task sums are stored as complex128.
__device__ __forceinline__ double from_next_lane(double x) {
  const long long v = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(v & 0xffffffffLL), 0x134, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(v >> 32), 0x134, 0xf, 0xf, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

template <int FORM>
__global__ __launch_bounds__(128) void pair_sum_f64_sym_kernel(
    const SymTask* __restrict__ tasks, const BodyDev* __restrict__ bodies,
    const double* __restrict__ pos, const double* __restrict__ aw,
    const double* __restrict__ ew, int64_t N, const double2* __restrict__ mu,
    const int32_t* __restrict__ seg_active, double2* __restrict__ part) {
  constexpr int NA = FORM ? 6 : 4;   // source-side sums: S1, S2 (, S3), re/im
  const SymTask T = tasks[blockIdx.x];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const BodyDev& BA = bodies[T.a];
  if (seg_active && seg_active[BA.problem] == 0) {
    for (int t = tid; t < T.nt; t += 128) part[T.ioff + t] = make_double2(0.0, 0.0);
    for (int j = tid; j < T.nb; j += 128) part[T.joff + j] = make_double2(0.0, 0.0);
    return;
  }
  const double k = BA.k;
  const double k2pi = k / TWO_PI;

  // the lane's two targets: x_i, -aw_i, mu_i (0 past the block)
  double xx[2], xy[2], xz[2], nx[2], ny[2], nz[2], mr[2], mi[2], ewi[2];
  double ar[2], ai[2], br[2], bi[2], er[2], ei[2];
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    const int loc = wv * 128 + t * 64 + lane;
    const bool act = loc < T.nt;
    const int64_t i = T.t0 + (act ? loc : 0);
    xx[t] = pos[i];
    xy[t] = pos[N + i];
    xz[t] = pos[2 * N + i];
    nx[t] = -aw[i];
    ny[t] = -aw[N + i];
    nz[t] = -aw[2 * N + i];
    const double2 m = act ? mu[i] : make_double2(0.0, 0.0);
    mr[t] = m.x;
    mi[t] = m.y;
    ewi[t] = FORM ? ew[i] : 0.0;
    ar[t] = ai[t] = br[t] = bi[t] = er[t] = ei[t] = 0.0;
  }

  __shared__ double2 sQ0[128];         // y.x, y.y
  __shared__ double2 sQ1[128];         // y.z, aw.z
  __shared__ double2 sQ2[128];         // aw.x, aw.y
  __shared__ double2 sM[128];          // mu_j
  __shared__ double sE[FORM ? 128 : 1];
  __shared__ double sX[NA][64];        // second wavefront's source-side sums

  const int src = (lane + 63) & 63;    // source of the lane's sums after a chunk
  const int nch = (T.nb + 63) / 64;
  for (int c = 0; c < nch; ++c) {
    if (tid < 64) {
      const int jl = c * 64 + tid;
      const bool act = jl < T.nb;
      const int64_t j = T.s0 + (act ? jl : 0);
      const double2 q0 = make_double2(pos[j], pos[N + j]);
      const double2 q1 = make_double2(pos[2 * N + j], aw[2 * N + j]);
      const double2 q2 = make_double2(aw[j], aw[N + j]);
      const double2 m = act ? mu[j] : make_double2(0.0, 0.0);
      sQ0[tid] = q0;
      sQ0[tid + 64] = q0;
      sQ1[tid] = q1;
      sQ1[tid + 64] = q1;
      sQ2[tid] = q2;
      sQ2[tid + 64] = q2;
      sM[tid] = m;
      sM[tid + 64] = m;
      if (FORM) {
        sE[tid] = ew[j];
        sE[tid + 64] = ew[j];
      }
    }
    __syncthreads();
    double acc[NA];
#pragma unroll
    for (int a = 0; a < NA; ++a) acc[a] = 0.0;
#pragma unroll 2
    for (int st = 0; st < 64; ++st) {
      const double2 q0 = sQ0[lane + st];
      const double2 q1 = sQ1[lane + st];
      const double2 q2 = sQ2[lane + st];
      const double2 m = sM[lane + st];
      const double e = FORM ? sE[lane + st] : 0.0;
      double cn[NA];
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        const double dx = q0.x - xx[t], dy = q0.y - xy[t], dz = q1.x - xz[t];
        const double r2 = fma(dx, dx, fma(dy, dy, dz * dz));
        const double ir = rsqrt_pos(r2);
        double sn, cs;
        sincos_2pi(r2 * ir * k2pi, &sn, &cs);
        const double ir2 = ir * ir;
        // target i, source j
        {
          const double zr = fma(cs, m.x, -sn * m.y);
          const double zi = fma(cs, m.y, sn * m.x);
          const double dot = fma(q2.x, dx, fma(q2.y, dy, q1.y * dz));
          const double u = dot * ir2;
          const double sc = u * ir;
          ar[t] = fma(sc, zr, ar[t]);
          ai[t] = fma(sc, zi, ai[t]);
          br[t] = fma(u, zr, br[t]);
          bi[t] = fma(u, zi, bi[t]);
          if constexpr (FORM == 1) {
            const double tt = e * ir;
            er[t] = fma(tt, zr, er[t]);
            ei[t] = fma(tt, zi, ei[t]);
          }
        }
        // target j, source i
        {
          const double zr = fma(cs, mr[t], -sn * mi[t]);
          const double zi = fma(cs, mi[t], sn * mr[t]);
          const double dot = fma(nx[t], dx, fma(ny[t], dy, nz[t] * dz));
          const double u = dot * ir2;
          const double sc = u * ir;
          const double tt = FORM ? ewi[t] * ir : 0.0;
          if (t == 0) {
            cn[0] = sc * zr;
            cn[1] = sc * zi;
            cn[2] = u * zr;
            cn[3] = u * zi;
            if constexpr (FORM == 1) {
              cn[4] = tt * zr;
              cn[5] = tt * zi;
            }
          } else {
            cn[0] = fma(sc, zr, cn[0]);
            cn[1] = fma(sc, zi, cn[1]);
            cn[2] = fma(u, zr, cn[2]);
            cn[3] = fma(u, zi, cn[3]);
            if constexpr (FORM == 1) {
              cn[4] = fma(tt, zr, cn[4]);
              cn[5] = fma(tt, zi, cn[5]);
            }
          }
        }
      }
#pragma unroll
      for (int a = 0; a < NA; ++a) acc[a] = from_next_lane(acc[a]) + cn[a];
    }
    if (wv == 1) {
#pragma unroll
      for (int a = 0; a < NA; ++a) sX[a][lane] = acc[a];
    }
    __syncthreads();
    if (wv == 0 && c * 64 + src < T.nb) {
      double v[NA];
#pragma unroll
      for (int a = 0; a < NA; ++a) v[a] = acc[a] + sX[a][lane];
      const double e3r = FORM ? v[4] : 0.0, e3i = FORM ? v[5] : 0.0;
      // -S1 + i k S2 (- i S3)
      part[T.joff + c * 64 + src] = make_double2(fma(-k, v[3], e3i - v[0]) * INV_FOUR_PI,
                                                 fma(k, v[2], -v[1] - e3r) * INV_FOUR_PI);
    }
  }
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    const int loc = wv * 128 + t * 64 + lane;
    if (loc < T.nt)
      part[T.ioff + loc] = make_double2(fma(-k, bi[t], ei[t] - ar[t]) * INV_FOUR_PI,
                                        fma(k, br[t], -ai[t] - er[t]) * INV_FOUR_PI);
  }
}

// out[n] = (accumulate ? out[n] : 0) + the task sums of n's block.  A
// workgroup takes 64 consecutive nodes; wavefront w adds the list entries
// w, w + 4, ... of each node, and the four sums are added in wavefront order
// (a fixed order).
template <typename P>
__global__ __launch_bounds__(256) void reduce_sym_kernel(
    const P* __restrict__ part, const int32_t* __restrict__ node_body,
    const BodyDev* __restrict__ bodies, const int32_t* __restrict__ blk_base,
    const int32_t* __restrict__ ptr, const int64_t* __restrict__ list, int64_t N,
    double2* __restrict__ out, int accumulate) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t n = (int64_t)blockIdx.x * 64 + lane;
  __shared__ double2 red[4][64];
  double2 acc = make_double2(0.0, 0.0);
  if (n < N) {
    const int b = node_body[n];
    const int blk = blk_base[b] + (int)((n - bodies[b].off) / SYM_T);
    const int e1 = ptr[blk + 1];
#pragma unroll 4
    for (int e = ptr[blk] + w; e < e1; e += 4) {
      const P v = part[list[e] + n];
      acc.x += (double)v.x;
      acc.y += (double)v.y;
    }
  }
  red[w][lane] = acc;
  __syncthreads();
  if (w == 0 && n < N) {
    double2 o = accumulate ? out[n] : make_double2(0.0, 0.0);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      o.x += red[q][lane].x;
      o.y += red[q][lane].y;
    }
    out[n] = o;
  }
}

// Tasks of the reciprocal kernel: for every problem, every pair of bodies
// a < b and every pair of blocks (one of a, one of b).  Partial-sum offsets
// follow the order of construction; each block lists, in that order, the
// tasks whose target or source block it is.  The table is then sorted by
// decreasing cost.
static void plan_sym(qax_problem* p) {
  auto& S = p->sym;
  S.tasks.clear();
  S.ok = p->n_problems > 0;
  for (int pr = 0; pr < p->n_problems; ++pr) S.ok = S.ok && p->k[pr] > 0.0;
  const int nbody = (int)p->hbodies.size();
  std::vector<int32_t> blk_base(nbody + 1, 0);
  for (int b = 0; b < nbody; ++b)
    blk_base[b + 1] = blk_base[b] + (p->hbodies[b].n + SYM_T - 1) / SYM_T;
  std::vector<std::vector<int64_t>> lists(blk_base[nbody]);
  int64_t off = 0;
  for (int pr = 0; pr < p->n_problems; ++pr) {
    const int b0 = (int)p->prob_body0[pr], b1 = (int)p->prob_body0[pr + 1];
    for (int a = b0; a < b1; ++a)
      for (int b = a + 1; b < b1; ++b)
        for (int qa = 0; qa * SYM_T < p->hbodies[a].n; ++qa)
          for (int qb = 0; qb * SYM_T < p->hbodies[b].n; ++qb) {
            SymTask T;
            T.t0 = p->hbodies[a].off + (int64_t)qa * SYM_T;
            T.nt = std::min(SYM_T, p->hbodies[a].n - qa * SYM_T);
            T.s0 = p->hbodies[b].off + (int64_t)qb * SYM_T;
            T.nb = std::min(SYM_T, p->hbodies[b].n - qb * SYM_T);
            T.a = a;
            T.b = b;
            T.ioff = off;
            T.joff = off + T.nt;
            lists[blk_base[a] + qa].push_back(T.ioff - T.t0);
            lists[blk_base[b] + qb].push_back(T.joff - T.s0);
            off += T.nt + T.nb;
            S.tasks.push_back(T);
          }
  }
  S.nparts = off;
  auto cost = [](const SymTask& x) { return (int64_t)x.nt * x.nb; };
  bool uniform = true;
  for (const SymTask& T : S.tasks) uniform = uniform && cost(T) == cost(S.tasks[0]);
  if (!uniform)
    std::stable_sort(S.tasks.begin(), S.tasks.end(),
                     [&](const SymTask& x, const SymTask& y) { return cost(x) > cost(y); });
  S.h_blk_base = blk_base;
  S.h_ptr.assign(1, 0);
  S.h_list.clear();
  for (auto& v : lists) {
    S.h_list.insert(S.h_list.end(), v.begin(), v.end());
    S.h_ptr.push_back((int32_t)S.h_list.size());
  }
}

static hipError_t upload_sym(qax_problem* p) {
  auto& S = p->sym;
  if (S.d_mem) {
    hipError_t e = hipStreamSynchronize(p->stream);
    if (e != hipSuccess) return e;
    dev_release(p, S.d_mem);
    S.d_mem = nullptr;
  }
  auto al = [](size_t x) { return (x + 255) / 256 * 256; };
  const size_t bt = al(sizeof(SymTask) * std::max<size_t>(1, S.tasks.size()));
  const size_t bb = al(sizeof(int32_t) * S.h_blk_base.size());
  const size_t bp = al(sizeof(int32_t) * S.h_ptr.size());
  const size_t bl = al(sizeof(int64_t) * std::max<size_t>(1, S.h_list.size()));
  hipError_t e = dev_alloc(p, &S.d_mem, bt + bb + bp + bl);
  if (e != hipSuccess) return e;
  char* m = (char*)S.d_mem;
  S.d_tasks = (SymTask*)m;
  S.d_blk_base = (int32_t*)(m + bt);
  S.d_ptr = (int32_t*)(m + bt + bb);
  S.d_list = (int64_t*)(m + bt + bb + bp);
  auto cp = [&](void* d, const void* h, size_t n) {
    if (e == hipSuccess && n) e = hipMemcpyAsync(d, h, n, hipMemcpyHostToDevice, p->stream);
  };
  cp(S.d_tasks, S.tasks.data(), sizeof(SymTask) * S.tasks.size());
  cp(S.d_blk_base, S.h_blk_base.data(), sizeof(int32_t) * S.h_blk_base.size());
  cp(S.d_ptr, S.h_ptr.data(), sizeof(int32_t) * S.h_ptr.size());
  cp(S.d_list, S.h_list.data(), sizeof(int64_t) * S.h_list.size());
  if (e != hipSuccess) return e;
  return hipStreamSynchronize(p->stream);
}

// Build the task table: target blocks of `tpb` rows inside one problem, each
// paired with `slots` contiguous chunks of that problem's source bodies
// (balanced by node count).  Sorted by decreasing cost so that the hardware
// dispatcher, which issues workgroups in index order, balances uneven work.
void plan_pair_sum(qax_problem* p, int prec, int cu_count) {
  const int pi = prec == QAX_FP64 ? 0 : 1;
  const int tpb = p->tune.pair_tpb[pi];
  const int64_t mult = p->tune.pair_mult[pi];
  std::vector<PairTask> tasks;
  int64_t tblocks = 0;
  for (int pr = 0; pr < p->n_problems; ++pr)
    tblocks += (p->off[p->prob_body0[pr + 1]] - p->off[p->prob_body0[pr]] + tpb - 1) / tpb;
  int slots = (int)std::max<int64_t>(1, (mult * cu_count + tblocks - 1) / std::max<int64_t>(tblocks, 1));
  slots = std::min(slots, 32);
  for (int pr = 0; pr < p->n_problems; ++pr) {
    const int b0 = (int)p->prob_body0[pr], b1 = (int)p->prob_body0[pr + 1];
    const int64_t n0 = p->off[b0], n1 = p->off[b1];
    // split bodies into `slots` chunks of similar node counts
    std::vector<int> cut(slots + 1, b1);
    cut[0] = b0;
    {
      int b = b0;
      for (int s = 1; s < slots; ++s) {
        const int64_t target = n0 + (n1 - n0) * s / slots;
        while (b < b1 && p->off[b + 1] <= target) ++b;
        cut[s] = std::max(cut[s - 1], b);
      }
      cut[slots] = b1;
    }
    for (int64_t t0 = n0; t0 < n1; t0 += tpb) {
      const int nt = (int)std::min<int64_t>(tpb, n1 - t0);
      // bodies spanned by the targets
      int lo = b0, hi = b0;
      while (lo + 1 < b1 && p->off[lo + 1] <= t0) ++lo;
      hi = lo;
      while (hi + 1 < b1 && p->off[hi + 1] <= t0 + nt - 1) ++hi;
      for (int s = 0; s < slots; ++s) {
        PairTask T;
        T.t0 = t0;
        T.nt = nt;
        T.b0 = cut[s];
        T.b1 = cut[s + 1];
        T.slot = s;
        T.tbody_lo = lo;
        T.tbody_hi = hi;
        T.k = p->k[pr];
        T.eta = p->eta_of(p->k[pr]);
        tasks.push_back(T);
      }
    }
  }
  auto cost = [&](const PairTask& T) {
    return (double)T.nt * (double)(p->off[T.b1] - p->off[T.b0]);
  };
  std::stable_sort(tasks.begin(), tasks.end(),
                   [&](const PairTask& a, const PairTask& b) { return cost(a) > cost(b); });
  if (prec == QAX_FP64) {
    p->tasks64 = tasks;
    p->slots64 = slots;
  } else {
    p->tasks32 = tasks;
    p->slots32 = slots;
  }
  p->plan_tpb[pi] = tpb;
}

hipError_t upload_pair_plan(qax_problem* p, int prec, int cu_count) {
  plan_pair_sum(p, prec, cu_count);
  if (!p->sym.d_mem) {
    // the reciprocal task table depends on the geometry only
    plan_sym(p);
    hipError_t e = upload_sym(p);
    if (e != hipSuccess) return e;
  }
  ++p->generation;   // captured solver steps hold the old launch sizes
  std::vector<PairTask>& t = prec == QAX_FP64 ? p->tasks64 : p->tasks32;
  PairTask*& d = prec == QAX_FP64 ? p->d_tasks64 : p->d_tasks32;
  if (d) {
    hipError_t e = hipStreamSynchronize(p->stream);
    if (e != hipSuccess) return e;
    dev_release(p, d);
    d = nullptr;
  }
  hipError_t e = dev_alloc(p, (void**)&d, sizeof(PairTask) * t.size());
  if (e != hipSuccess) return e;
  e = hipMemcpyAsync(d, t.data(), sizeof(PairTask) * t.size(), hipMemcpyHostToDevice, p->stream);
  if (e != hipSuccess) return e;
  return hipStreamSynchronize(p->stream);
}

// LDS per workgroup (with the combined-field weights): FP64 7 TPB doubles +
// TPB NRC complex128; FP32 2 TPB float4 + TPB floats + TPB NRC complex64
constexpr size_t lds_f64(int tpb, int nrc) { return (size_t)tpb * (56 + 16 * nrc); }
constexpr size_t lds_f32(int tpb, int nrc) { return (size_t)tpb * (36 + 8 * nrc); }

bool pair_config_ok(int prec, int tpb, int nrc) {
  if (tpb != 128 && tpb != 256 && tpb != 512) return false;
  if (prec == QAX_FP64) {
    if (nrc != 1 && nrc != 2 && nrc != 4 && nrc != 8) return false;
    return lds_f64(tpb, nrc) <= 65536;
  }
  if (nrc != 1 && nrc != 2 && nrc != 4 && nrc != 8 && nrc != 16 && nrc != 32) return false;
  return lds_f32(tpb, nrc) <= 65536;
}

template <int TPB, int NRC, int FORM>
static void launch_f64(qax_problem* p, const double* mu, int nrhs, double* partial) {
  if constexpr (lds_f64(TPB, NRC) <= 65536) {
    dim3 grid((unsigned)p->tasks64.size(), (unsigned)((nrhs + NRC - 1) / NRC));
    hipLaunchKernelGGL((pair_sum_f64_kernel<TPB, NRC, FORM>), grid, dim3(TPB), 0, p->stream,
                       p->d_tasks64, p->d_bodies, p->d_node_body, p->d_pos, p->d_aw, p->d_ew, p->N,
                       (const double2*)mu, nrhs, p->seg_active, (double2*)partial);
  }
}

template <int TPB, int NRC, int FORM>
static void launch_f32(qax_problem* p, const double* mu, int nrhs, double* partial) {
  if constexpr (lds_f32(TPB, NRC) <= 65536) {
    dim3 grid((unsigned)p->tasks32.size(), (unsigned)((nrhs + NRC - 1) / NRC));
    hipLaunchKernelGGL((pair_sum_f32_kernel<TPB, NRC, FORM>), grid, dim3(TPB), 0, p->stream,
                       p->d_tasks32, p->d_bodies, p->d_node_body, p->d_pos,
                       (const float4*)p->d_loc32, (const float4*)p->d_aw32, p->d_ew32, p->N,
                       (const double2*)mu, nrhs, p->seg_active, (double2*)partial);
  }
}

template <int TPB, int FORM>
static void launch_f64_nrc(qax_problem* p, int nrc, const double* mu, int nrhs, double* partial) {
  switch (nrc) {
    case 1: launch_f64<TPB, 1, FORM>(p, mu, nrhs, partial); break;
    case 2: launch_f64<TPB, 2, FORM>(p, mu, nrhs, partial); break;
    case 4: launch_f64<TPB, 4, FORM>(p, mu, nrhs, partial); break;
    default: launch_f64<TPB, 8, FORM>(p, mu, nrhs, partial); break;
  }
}

template <int TPB, int FORM>
static void launch_f32_nrc(qax_problem* p, int nrc, const double* mu, int nrhs, double* partial) {
  switch (nrc) {
    case 1: launch_f32<TPB, 1, FORM>(p, mu, nrhs, partial); break;
    case 2: launch_f32<TPB, 2, FORM>(p, mu, nrhs, partial); break;
    case 4: launch_f32<TPB, 4, FORM>(p, mu, nrhs, partial); break;
    case 8: launch_f32<TPB, 8, FORM>(p, mu, nrhs, partial); break;
    case 16: launch_f32<TPB, 16, FORM>(p, mu, nrhs, partial); break;
    default: launch_f32<TPB, 32, FORM>(p, mu, nrhs, partial); break;
  }
}

template <int FORM>
static void launch_any(qax_problem* p, bool f64, int tpb, int nrc, const double* mu, int nrhs,
                       double* partial) {
  if (f64) {
    if (tpb == 128) launch_f64_nrc<128, FORM>(p, nrc, mu, nrhs, partial);
    else if (tpb == 256) launch_f64_nrc<256, FORM>(p, nrc, mu, nrhs, partial);
    else launch_f64_nrc<512, FORM>(p, nrc, mu, nrhs, partial);
  } else {
    if (tpb == 128) launch_f32_nrc<128, FORM>(p, nrc, mu, nrhs, partial);
    else if (tpb == 256) launch_f32_nrc<256, FORM>(p, nrc, mu, nrhs, partial);
    else launch_f32_nrc<512, FORM>(p, nrc, mu, nrhs, partial);
  }
}

// partial: slots x N x nrhs complex128 workspace; out = pair sum, or
// out += pair sum when accumulate is set.  The workgroup size is the one the
// task table was planned with; right-hand sides per pass from the tuning
// (clamped to a supported configuration).
size_t pair_work_bytes(const qax_problem* p, int prec, int nrhs) {
  const int slots = prec == QAX_FP64 ? p->slots64 : p->slots32;
  size_t b = std::max((size_t)slots * p->N * nrhs * 16, lattice_work_bytes(p, nrhs));
  if (nrhs == 1 && p->sym.ok)
    b = std::max(b, (size_t)p->sym.nparts * (prec == QAX_FP64 ? 16 : 8));
  return b;
}

static bool use_sym(const qax_problem* p, int prec, int nrhs) {
  return nrhs == 1 && p->sym.ok && p->sym.enabled && p->sym.d_mem && p->form() != 2;
}

hipError_t launch_pair_sum(qax_problem* p, int prec, const double* mu, double* out, int nrhs,
                           double* partial, bool accumulate) {
  if (p->lat.active) {
    // regular array of identical bodies: block-Toeplitz apply
    const int kind = prec == QAX_FP64 ? QAX_K_PAIRSUM_FP64 : QAX_K_PAIRSUM_FP32;
    timing_begin(p, kind);
    hipError_t e = launch_lattice_apply(p, prec, mu, out, nrhs, partial, accumulate);
    timing_end(p, kind);
    return e;
  }
  const bool f64 = prec == QAX_FP64;
  const int pi = f64 ? 0 : 1;
  const int kind = f64 ? QAX_K_PAIRSUM_FP64 : QAX_K_PAIRSUM_FP32;
  if (use_sym(p, prec, nrhs)) {
    auto& S = p->sym;
    const int form = p->form();
    timing_begin(p, kind);
    if (!S.tasks.empty()) {
      const dim3 grid((unsigned)S.tasks.size());
      if (f64) {
        double2* part = (double2*)partial;
        if (form == 1)
          hipLaunchKernelGGL(pair_sum_f64_sym_kernel<1>, grid, dim3(128), 0, p->stream, S.d_tasks,
                             p->d_bodies, p->d_pos, p->d_aw, p->d_ew, p->N, (const double2*)mu,
                             p->seg_active, part);
        else
          hipLaunchKernelGGL(pair_sum_f64_sym_kernel<0>, grid, dim3(128), 0, p->stream, S.d_tasks,
                             p->d_bodies, p->d_pos, p->d_aw, p->d_ew, p->N, (const double2*)mu,
                             p->seg_active, part);
      } else {
        float2* part = (float2*)partial;
        if (form == 1)
          hipLaunchKernelGGL(pair_sum_f32_sym_kernel<1>, grid, dim3(128), 0, p->stream, S.d_tasks,
                             p->d_bodies, (const float4*)p->d_loc32, (const float4*)p->d_aw32,
                             p->d_ew32, (const double2*)mu, p->seg_active, part);
        else
          hipLaunchKernelGGL(pair_sum_f32_sym_kernel<0>, grid, dim3(128), 0, p->stream, S.d_tasks,
                             p->d_bodies, (const float4*)p->d_loc32, (const float4*)p->d_aw32,
                             p->d_ew32, (const double2*)mu, p->seg_active, part);
      }
    }
    timing_end(p, kind);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const dim3 rgrid((unsigned)((p->N + 63) / 64));
    if (f64)
      hipLaunchKernelGGL(reduce_sym_kernel<double2>, rgrid, dim3(256), 0, p->stream,
                         (const double2*)partial, p->d_node_body, p->d_bodies, S.d_blk_base,
                         S.d_ptr, S.d_list, p->N, (double2*)out, accumulate ? 1 : 0);
    else
      hipLaunchKernelGGL(reduce_sym_kernel<float2>, rgrid, dim3(256), 0, p->stream,
                         (const float2*)partial, p->d_node_body, p->d_bodies, S.d_blk_base,
                         S.d_ptr, S.d_list, p->N, (double2*)out, accumulate ? 1 : 0);
    return hipGetLastError();
  }
  const int tpb = p->tune.pair_tpb[pi];
  int nrc = nrhs == 1 ? 1 : p->tune.pair_nrc[pi][nrhs_class(nrhs)];
  while (nrc > 1 && !pair_config_ok(prec, tpb, nrc)) nrc /= 2;
  if (!pair_config_ok(prec, tpb, nrc) || p->plan_tpb[pi] != tpb) return hipErrorInvalidConfiguration;
  timing_begin(p, kind);
  switch (p->form()) {
    case 1: launch_any<1>(p, f64, tpb, nrc, mu, nrhs, partial); break;
    case 2: launch_any<2>(p, f64, tpb, nrc, mu, nrhs, partial); break;
    default: launch_any<0>(p, f64, tpb, nrc, mu, nrhs, partial); break;
  }
  timing_end(p, kind);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int slots = prec == QAX_FP64 ? p->slots64 : p->slots32;
  const int64_t count = p->N * nrhs;
  hipLaunchKernelGGL(reduce_slots_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0,
                     p->stream, (const double2*)partial, slots, count, (double2*)out,
                     accumulate ? 1 : 0);
  return hipGetLastError();
}

}  // namespace qax
