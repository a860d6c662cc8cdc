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
#include <functional>
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
// Reciprocal pair sums (one right-hand side, double layer or combined field,
// k > 0).  For x_i on body a and y_j on body b != a, the distance r, the phase
// and e^{ikr} are the same for the pair (target i, source j) and the pair
// (target j, source i); only the double-layer dot products and the densities
// differ, so each unordered pair of nodes is evaluated once for both
// directions.
//
// Work layout.  Each problem's node range is cut into blocks of SYM_T
// consecutive nodes (a block may hold the end of one body and the start of
// the next).  A task is a pair of blocks (I, J), I <= J, of one problem: for
// I < J every pair (i in I, j in J) on different bodies is taken in both
// directions; for I == J every ordered pair on different bodies is taken in
// the target direction only.  Tasks are grouped into super-tasks of up to
// S x S block pairs (block rows [i0, i0 + ni) x columns [j0, j0 + nj); on the
// diagonal only J >= I), one workgroup each.  A super-task keeps the target
// sums of its current row in registers across its columns and writes one
// target slot per row; it accumulates the source sums of each column over
// its rows in one source slot per column (read-modify-write by the thread
// that owns the entry).  Slots hold SYM_T complex values (complex128 for the
// FP64 kernel, complex64 for the FP32 kernel), so the workspace is
// (ni + nj) SYM_T values per super-task, N nblk / S in all; the super-tasks
// are split into launches whose slots fit a fixed cap, each followed by a
// reduction that adds, per node, the slots of its block in FP64 in a fixed
// order (deterministic results).
//
// Lanes.  A workgroup is two wavefronts; lane l of wavefront w owns targets
// w 128 + l and w 128 + 64 + l of block I.  The sources of block J pass in
// chunks of at most 64 nodes of one body (a chunk ends at a body's last
// node), staged twice over in LDS; at step s lane l meets source
// (l + s) mod 64 (index l + s), so the 64 lanes of a wavefront see 64
// distinct sources at every step.  A chunk of at most 32 sources (the end of
// a body part; node counts are multiples of 32) takes 32 steps with each
// source in two slots l and l + 32, whose sums are added at the end.  The target-side sums stay in registers.
// The source-side sums travel with their source: each step adds lane l + 1's
// running sums to lane l's contribution with a DPP wavefront rotation fused
// into the add, so after the chunk lane l holds those of source
// (l + 63) mod 64 (no LDS read-modify-write per step).  Since a chunk lies in
// one body b, the exclusion of pairs on the same body is a per-lane choice
// for the whole chunk: a lane whose target is on b (or past the end of the
// block) gets a far-away stand-in target and a zero density, so its pairs are
// finite and add nothing to the source sums, and its target sum of the chunk
// is dropped.
__device__ __forceinline__ float from_next_lane(float x) {
  // DPP wavefront rotation: lane l reads lane (l + 1) mod 64
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x134, 0xf, 0xf, false));
}

__device__ __forceinline__ double from_next_lane(double x) {
  // the rotation writes every lane, so the "old" operand is never used; with
  // the source itself as old the move needs no zeroed destination first
  const long long v = __double_as_longlong(x);
  const int vl = (int)(v & 0xffffffffLL), vh = (int)(v >> 32);
  const int lo = __builtin_amdgcn_update_dpp(vl, vl, 0x134, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(vh, vh, 0x134, 0xf, 0xf, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Rows of super-task T whose block pair (row ii, column jj) is evaluated.
__device__ __forceinline__ uint32_t sym_row_mask(const SymSuper& T, int ii) {
  uint32_t m = 0;
  for (int jj = T.diag ? ii : 0; jj < T.nj; ++jj)
    if (!((T.skip >> (ii * SYM_SMAX + jj)) & 1ull)) m |= 1u << jj;
  return m;
}

// Inactive problem of a lockstep solve: the super-task's slots hold zeros.
template <typename S2>
__device__ __forceinline__ bool sym_inactive(const SymSuper& T, const int32_t* __restrict__ seg_active,
                                             S2* __restrict__ part) {
  if (!seg_active || seg_active[T.problem] != 0) return false;
  for (int e = threadIdx.x; e < (T.ni + T.nj) * SYM_T; e += blockDim.x) {
    part[T.toff + e].x = 0;
    part[T.toff + e].y = 0;
  }
  return true;
}

// FP32 reciprocal pair sum.  Source coordinates are local to their body,
// y_j = c_b + y'; per target and source body, D = c_b - x_i, |D| and
// frac(k |D| / 2 pi) are formed in FP64 (from the centres and the target's
// local coordinates) and, with c = k^2 / 2 pi, m = 2 c D in FP32, so that
//   num = c (r^2 - |D|^2) = m.y' + c |y'|^2
// is three fmas with no cancellation against |D|^2 (c |y'|^2 is staged with
// the source), delta = r - |D| = (r^2 - |D|^2) / (r + |D|), and the phase in
// revolutions is frac(k |D| / 2 pi) + k delta / 2 pi, so FP32 rounding enters
// relative to delta, not to r.  Distances are scaled by k:
// r_s^2 = k^2 r^2 = 2 pi num + k^2 |D|^2, irs = 1 / (k r) and
// num rcp(r_s^2 irs + k |D|) = k delta / 2 pi.  The double-layer factor of a
// pair, (ik/r - 1/r^2) e^{ikr} / (4 pi r), is k^3 / (4 pi) w with
// w = e^{ikr} irs^2 (i - irs), shared by both directions; the direction
// (i <- j) adds w aw_j.(y_j - x_i) mu_j and the direction (j <- i) adds
// w aw_i.(x_i - y_j) mu_i, with
//   aw_j.(y_j - x_i) = aw_j.y' + (aw_j / 2 c).m,
//   aw_i.(x_i - y_j) = -aw_i.D - aw_i.y'
// (aw_j / 2 c staged with the source).  The combined field adds
// - i eta e^{ikr} |aw| mu / (4 pi r) per direction, i.e.
// - i (ew / k^2) irs e^{ikr} mu in the same scaling (ew = eta |aw|).
// Real parts are accumulated negated (one sign flip per slot).  Target sums
// are FP32 per chunk of at most 64 sources and FP64 across chunks and
// columns; source sums are FP32 over the chunk's 128 targets of a
// wavefront, then FP64.
// A square's sums are stored rounded to complex64 slots (half the bytes of
// complex128, so a launch holds twice the squares in the same workspace) and
// the reduction adds the slots in FP64.
// Five wavefronts per SIMD (at most 102 registers; the few spills are outside
// the pair loop): 1.4 % faster than the four the unconstrained allocation
// allows, on the 1000-body workload.
template <int FORM>
__global__ __launch_bounds__(128) __attribute__((amdgpu_waves_per_eu(5))) void pair_sum_f32_sym_kernel(
    const SymSuper* __restrict__ supers, const SymBlock* __restrict__ blocks,
    const BodyDev* __restrict__ bodies, const int32_t* __restrict__ node_body,
    const float4* __restrict__ loc32, const float4* __restrict__ aw32,
    const float* __restrict__ ew32, const double2* __restrict__ mu,
    const int32_t* __restrict__ seg_active, float2* __restrict__ part) {
  const SymSuper T = supers[blockIdx.x];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  if (sym_inactive(T, seg_active, part)) return;
  const double k = T.k;
  const double cnum = k * k / TWO_PI;  // scale of num
  const double sc3 = k * k * k / FOUR_PI;
  const float c32 = (float)cnum, hw = (float)(0.5 / cnum), ik2 = (float)(1.0 / (k * k));
  const float twopi = (float)TWO_PI;

  __shared__ float4 sY[128];           // y', c |y'|^2
  __shared__ float4 sW[128];           // aw_j / 2 c, aw_j . y'
  __shared__ float4 sM[128];           // mu_j, ew_j / kappa^2
  __shared__ float sX[2][64];          // second wavefront's source-side sums
  const int src = (lane + 63) & 63;    // source of the lane's sums after a chunk

  uint32_t touched = 0;                // columns whose source slot holds a value
  for (int ii = 0; ii < T.ni; ++ii) {
    const uint32_t rowmask = sym_row_mask(T, ii);
    if (!rowmask) continue;
    const int I = T.i0 + ii;
    const SymBlock BI = blocks[I];
    // the lane's two targets
    float xx[2], xy[2], xz[2], nx[2], ny[2], nz[2], mr[2], mi[2], ew[2];
    int ab[2];
    bool act[2];
    double nsr[2], tsi[2];   // target sums of the row, FP64 across chunks and columns
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      const int loc = wv * 128 + t * 64 + lane;
      act[t] = loc < BI.n;
      const int64_t i = BI.n0 + (act[t] ? loc : 0);
      const float4 x4 = loc32[i];
      const float4 a4 = aw32[i];
      xx[t] = x4.x; xy[t] = x4.y; xz[t] = x4.z;
      nx[t] = -a4.x; ny[t] = -a4.y; nz[t] = -a4.z;
      const double2 m = act[t] ? mu[i] : make_double2(0.0, 0.0);
      mr[t] = (float)m.x;
      mi[t] = (float)m.y;
      ew[t] = FORM ? ew32[i] * ik2 : 0.0f;
      ab[t] = node_body[i];
      nsr[t] = tsi[t] = 0.0;
    }
    for (int jj = 0; jj < T.nj; ++jj) {
      if (!((rowmask >> jj) & 1u)) continue;
      const SymBlock BJ = blocks[T.j0 + jj];
      const bool dtask = (T.j0 + jj) == I;    // diagonal block: target direction only
      const bool first_src = !dtask && !((touched >> jj) & 1u);
      if (!dtask) touched |= 1u << jj;
      // per target and source body: m, Q, B, scaled |C|^2 and |C|, phase base
      float mx[2], my[2], mz[2], bq[2], d2s[2], dns[2], ph0[2], mre[2], mie[2];
      bool msk[2];
      int cur_b = -1;
      for (int cs = 0; cs < BJ.n;) {
        const int64_t node = BJ.n0 + cs;
        const int b = node_body[node];
        const BodyDev& BB = bodies[b];
        const int cl = (int)min((int64_t)min(64, BJ.n - cs), BB.off + BB.n - node);
        if (b != cur_b) {
          cur_b = b;
#pragma unroll
          for (int t = 0; t < 2; ++t) {
            const BodyDev& BA = bodies[ab[t]];
            msk[t] = !act[t] || ab[t] == b;
            // D = c_b - x_i in FP64 from the centres and the local coordinates
            const double Dx = (BB.cen[0] - BA.cen[0]) - (double)xx[t];
            const double Dy = (BB.cen[1] - BA.cen[1]) - (double)xy[t];
            const double Dz = (BB.cen[2] - BA.cen[2]) - (double)xz[t];
            const double D2 = fma(Dx, Dx, fma(Dy, Dy, Dz * Dz));
            const double Dn = sqrt(D2);
            double ph = k * Dn / TWO_PI;
            ph -= floor(ph);
            if (msk[t]) {
              // stand-in target 1e6 away: finite, negligible pairs
              mx[t] = (float)(2.0 * cnum * 1e6);
              my[t] = mz[t] = bq[t] = 0.0f;
              d2s[t] = (float)(k * k * 1e12);
              dns[t] = (float)(k * 1e6);
              ph0[t] = 0.0f;
            } else {
              mx[t] = (float)(2.0 * cnum * Dx);
              my[t] = (float)(2.0 * cnum * Dy);
              mz[t] = (float)(2.0 * cnum * Dz);
              bq[t] = (float)((double)nx[t] * Dx + (double)ny[t] * Dy + (double)nz[t] * Dz);
              d2s[t] = (float)(k * k * D2);
              dns[t] = (float)(k * Dn);
              ph0[t] = (float)ph;
            }
            mre[t] = msk[t] ? 0.0f : mr[t];
            mie[t] = msk[t] ? 0.0f : mi[t];
          }
        }
        // a chunk of at most 32 sources takes 32 steps, each source staged in
        // two slots of the rotation (lanes l and l + 32 then hold its sums)
        const bool half = cl <= 32;
        const int nst = half ? 32 : 64;
        __syncthreads();   // the previous chunk's LDS reads are done
        if (tid < 64) {
          const int sl = half ? (tid & 31) : tid;
          const bool sact = sl < cl;
          const int64_t j = node + (sact ? sl : 0);
          float4 y4 = loc32[j];
          y4.w *= c32;
          const float4 b4 = aw32[j];
          const double2 m = sact ? mu[j] : make_double2(0.0, 0.0);
          const float4 W = make_float4(hw * b4.x, hw * b4.y, hw * b4.z, b4.w);
          const float4 M = make_float4((float)m.x, (float)m.y, FORM && sact ? ew32[j] * ik2 : 0.0f, 0.0f);
          sY[tid] = y4;
          sY[tid + 64] = y4;
          sW[tid] = W;
          sW[tid + 64] = W;
          sM[tid] = M;
          sM[tid + 64] = M;
        }
        __syncthreads();
        float nar[2] = {0.0f, 0.0f}, tai[2] = {0.0f, 0.0f};
        float acc0 = 0.0f, acc1 = 0.0f;
        const float4* pY = &sY[lane];
        const float4* pW = &sW[lane];
        const float4* pM = &sM[lane];
        for (int st0 = 0; st0 < nst; st0 += 8)
#pragma unroll
        for (int st = st0; st < st0 + 8; ++st) {
          const float4 Y = pY[st];
          const float4 W = pW[st];
          const float4 M = pM[st];
          float cr = 0.0f, ci = 0.0f;
#pragma unroll
          for (int t = 0; t < 2; ++t) {
            // shared by both directions: r, e^{ikr}, w
            const float num = fmaf(mx[t], Y.x, fmaf(my[t], Y.y, fmaf(mz[t], Y.z, Y.w)));
            const float r2s = fmaf(twopi, num, d2s[t]);
            const float irs = __builtin_amdgcn_rsqf(r2s);
            const float ph = fmaf(num, __builtin_amdgcn_rcpf(fmaf(r2s, irs, dns[t])), ph0[t]);
            const float sn = __builtin_amdgcn_sinf(ph);
            const float cs_ = __builtin_amdgcn_cosf(ph);
            // w = irs^2 e^{i ph} (i - irs)
            const float ir2 = irs * irs;
            const float nwr = fmaf(cs_, irs, sn) * ir2;    // -Re w
            const float wi = fmaf(-sn, irs, cs_) * ir2;    //  Im w
            // target i, source j
            {
              const float d = fmaf(W.x, mx[t], fmaf(W.y, my[t], fmaf(W.z, mz[t], W.w)));
              const float vr = d * M.x, vi = d * M.y;
              nar[t] = fmaf(nwr, vr, fmaf(wi, vi, nar[t]));
              tai[t] = fmaf(wi, vr, fmaf(-nwr, vi, tai[t]));
              if constexpr (FORM == 1) {
                const float g = M.z * irs;
                const float p1 = fmaf(cs_, M.y, sn * M.x), p2 = fmaf(cs_, M.x, -(sn * M.y));
                nar[t] = fmaf(-g, p1, nar[t]);
                tai[t] = fmaf(-g, p2, tai[t]);
              }
            }
            // target j, source i
            {
              const float d = fmaf(nx[t], Y.x, fmaf(ny[t], Y.y, fmaf(nz[t], Y.z, bq[t])));
              const float ur = d * mre[t], ui = d * mie[t];
              if (t == 0) {
                cr = fmaf(nwr, ur, wi * ui);
                ci = fmaf(wi, ur, -(nwr * ui));
              } else {
                cr = fmaf(nwr, ur, fmaf(wi, ui, cr));
                ci = fmaf(wi, ur, fmaf(-nwr, ui, ci));
              }
              if constexpr (FORM == 1) {
                const float g = ew[t] * irs;
                const float p1 = fmaf(cs_, mie[t], sn * mre[t]), p2 = fmaf(cs_, mre[t], -(sn * mie[t]));
                cr = fmaf(-g, p1, cr);
                ci = fmaf(-g, p2, ci);
              }
            }
          }
          acc0 = from_next_lane(acc0) + cr;
          acc1 = from_next_lane(acc1) + ci;
        }
#pragma unroll
        for (int t = 0; t < 2; ++t) {
          if (!msk[t]) {
            nsr[t] += (double)nar[t];
            tsi[t] += (double)tai[t];
          }
        }
        if (!dtask) {
          if (half) {   // the two slots of a source: lanes l and l + 32
            acc0 += __shfl_xor(acc0, 32);
            acc1 += __shfl_xor(acc1, 32);
          }
          if (wv == 1) {
            sX[0][lane] = acc0;
            sX[1][lane] = acc1;
          }
          __syncthreads();
          const int sj = half ? ((lane + 31) & 31) : src;
          if (wv == 0 && (!half || lane < 32) && sj < cl) {
            const double vr = -((double)acc0 + (double)sX[0][lane]) * sc3;
            const double vi = ((double)acc1 + (double)sX[1][lane]) * sc3;
            float2* d = part + T.soff + (int64_t)jj * SYM_T + cs + sj;
            if (first_src) {
              *d = make_float2((float)vr, (float)vi);
            } else {
              const float2 o = *d;
              *d = make_float2((float)(o.x + vr), (float)(o.y + vi));
            }
          }
        }
        cs += cl;
      }
    }
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      const int loc = wv * 128 + t * 64 + lane;
      if (loc < BI.n)
        part[T.toff + (int64_t)ii * SYM_T + loc] =
            make_float2((float)(-nsr[t] * sc3), (float)(tsi[t] * sc3));
    }
  }
}

// FP64 reciprocal pair sum: the same super-tasks, chunks, lane mapping and
// rotation as the FP32 kernel, in plain FP64 on positions scaled by k: the
// sources local to their body, y' = k (y_j - c_b), D = k (c_b - x_i) per
// target and source body, so (k r)^2 = |D|^2 + 2 D.y' + |y'|^2 is four fmas
// with |y'|^2 / 2 staged (phase k r in 512ths of a revolution for
// sincos_tab512, whose table each workgroup fills in LDS);
// w = e^{ikr} ir^2 (i - ir) with ir = 1/(k r)
// is shared by both directions, aw_j.d and -aw_i.d are k aw_j.(y_j - x_i)
// and k aw_i.(x_i - y_j), and the sums carry the factor k^2 / 4 pi (the
// combined field's eta |aw| staged divided by k).
// Four wavefronts per SIMD (at most 128 registers, spills outside the pair
// loop; 19.5 KB of LDS per workgroup, eight workgroups in 160 KB): 1 % faster
// than three.
template <int FORM>
__global__ __launch_bounds__(128) __attribute__((amdgpu_waves_per_eu(4))) void pair_sum_f64_sym_kernel(
    const SymSuper* __restrict__ supers, const SymBlock* __restrict__ blocks,
    const BodyDev* __restrict__ bodies, const int32_t* __restrict__ node_body,
    const double* __restrict__ pos, const double* __restrict__ aw, const double* __restrict__ ewp,
    int64_t N, const double2* __restrict__ mu, const int32_t* __restrict__ seg_active,
    double2* __restrict__ part) {
  const SymSuper T = supers[blockIdx.x];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  if (sym_inactive(T, seg_active, part)) return;
  const double k = T.k;
  const double u512 = 512.0 / TWO_PI;      // k r in 512ths of a revolution
  const double sc2 = k * k * INV_FOUR_PI;   // positions scaled by k: k^2 w dot mu / 4 pi

  __shared__ double2 sQ0[128];         // y'.x, y'.y   (y' = k (y - c_b))
  __shared__ double2 sQ1[128];         // y'.z, |y'|^2 / 2
  __shared__ double2 sQ2[128];         // aw.x, aw.y
  __shared__ double2 sQ3[128];         // aw.z, aw.y'
  __shared__ double2 sM[128];          // mu_j
  __shared__ double sE[FORM ? 128 : 1];
  __shared__ double sX[2][64];         // second wavefront's source-side sums
  __shared__ double2 sTab[512];        // (sin, cos)(2 pi i / 512)
  const int src = (lane + 63) & 63;
  fill_tab512(sTab, tid, 128);         // ordered by the first chunk's barrier

  uint32_t touched = 0;
  for (int ii = 0; ii < T.ni; ++ii) {
    const uint32_t rowmask = sym_row_mask(T, ii);
    if (!rowmask) continue;
    const int I = T.i0 + ii;
    const SymBlock BI = blocks[I];
    double xx[2], xy[2], xz[2], nx[2], ny[2], nz[2], mr[2], mi[2], ewi[2];
    double sr[2], si[2];
    int ab[2];
    bool act[2];
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      const int loc = wv * 128 + t * 64 + lane;
      act[t] = loc < BI.n;
      const int64_t i = BI.n0 + (act[t] ? loc : 0);
      xx[t] = k * pos[i];
      xy[t] = k * pos[N + i];
      xz[t] = k * pos[2 * N + i];
      nx[t] = -aw[i];
      ny[t] = -aw[N + i];
      nz[t] = -aw[2 * N + i];
      const double2 m = act[t] ? mu[i] : make_double2(0.0, 0.0);
      mr[t] = m.x;
      mi[t] = m.y;
      ewi[t] = FORM ? ewp[i] / k : 0.0;
      ab[t] = node_body[i];
      sr[t] = si[t] = 0.0;
    }
    for (int jj = 0; jj < T.nj; ++jj) {
      if (!((rowmask >> jj) & 1u)) continue;
      const SymBlock BJ = blocks[T.j0 + jj];
      const bool dtask = (T.j0 + jj) == I;
      const bool first_src = !dtask && !((touched >> jj) & 1u);
      if (!dtask) touched |= 1u << jj;
      double Dx[2], Dy[2], Dz[2], d2[2], bq[2], mre[2], mie[2];
      bool msk[2];
      int cur_b = -1;
      for (int cs = 0; cs < BJ.n;) {
        const int64_t node = BJ.n0 + cs;
        const int b = node_body[node];
        const BodyDev& BB = bodies[b];
        const int cl = (int)min((int64_t)min(64, BJ.n - cs), BB.off + BB.n - node);
        if (b != cur_b) {
          cur_b = b;
#pragma unroll
          for (int t = 0; t < 2; ++t) {
            msk[t] = !act[t] || ab[t] == b;
            // D = k (c_b - x_i); a masked lane's stand-in target is far away:
            // finite, negligible pairs
            Dx[t] = msk[t] ? 1e10 : k * BB.cen[0] - xx[t];
            Dy[t] = msk[t] ? 0.0 : k * BB.cen[1] - xy[t];
            Dz[t] = msk[t] ? 0.0 : k * BB.cen[2] - xz[t];
            d2[t] = fma(Dx[t], Dx[t], fma(Dy[t], Dy[t], Dz[t] * Dz[t]));
            bq[t] = fma(nx[t], Dx[t], fma(ny[t], Dy[t], nz[t] * Dz[t]));
            mre[t] = msk[t] ? 0.0 : mr[t];
            mie[t] = msk[t] ? 0.0 : mi[t];
          }
        }
        const bool half = cl <= 32;   // 32 steps, each source in two slots
        const int nst = half ? 32 : 64;
        __syncthreads();
        if (tid < 64) {
          const int sl = half ? (tid & 31) : tid;
          const bool sact = sl < cl;
          const int64_t j = node + (sact ? sl : 0);
          const double yx = k * (pos[j] - BB.cen[0]), yy = k * (pos[N + j] - BB.cen[1]),
                       yz = k * (pos[2 * N + j] - BB.cen[2]);
          const double ax = aw[j], ay = aw[N + j], az = aw[2 * N + j];
          const double2 q0 = make_double2(yx, yy);
          const double2 q1 = make_double2(yz, 0.5 * fma(yx, yx, fma(yy, yy, yz * yz)));
          const double2 q2 = make_double2(ax, ay);
          const double2 q3 = make_double2(az, fma(ax, yx, fma(ay, yy, az * yz)));
          const double2 m = sact ? mu[j] : make_double2(0.0, 0.0);
          sQ0[tid] = q0;
          sQ0[tid + 64] = q0;
          sQ1[tid] = q1;
          sQ1[tid + 64] = q1;
          sQ2[tid] = q2;
          sQ2[tid + 64] = q2;
          sQ3[tid] = q3;
          sQ3[tid + 64] = q3;
          sM[tid] = m;
          sM[tid + 64] = m;
          if (FORM) {
            const double e = sact ? ewp[j] / k : 0.0;
            sE[tid] = e;
            sE[tid + 64] = e;
          }
        }
        __syncthreads();
        double ar[2] = {0.0, 0.0}, ai[2] = {0.0, 0.0};
        double acc0 = 0.0, acc1 = 0.0;
        for (int st0 = 0; st0 < nst; st0 += 2)
#pragma unroll
        for (int st = st0; st < st0 + 2; ++st) {
          const double2 q0 = sQ0[lane + st];
          const double2 q1 = sQ1[lane + st];
          const double2 q2 = sQ2[lane + st];
          const double2 q3 = sQ3[lane + st];
          const double2 m = sM[lane + st];
          const double e = FORM ? sE[lane + st] : 0.0;
          double cr = 0.0, ci = 0.0;
#pragma unroll
          for (int t = 0; t < 2; ++t) {
            // k^2 r^2 = |D|^2 + 2 D.y' + |y'|^2
            const double nh = fma(Dx[t], q0.x, fma(Dy[t], q0.y, fma(Dz[t], q1.x, q1.y)));
            const double r2 = fma(2.0, nh, d2[t]);
            const double ir = rsqrt_pos(r2);
            double sn, cs_;
            sincos_tab512(r2 * ir * u512, sTab, &sn, &cs_);
            const double ir2 = ir * ir;
            const double wr = -(fma(cs_, ir, sn) * ir2);
            const double wi = fma(-sn, ir, cs_) * ir2;
            // target i, source j
            {
              // k aw_j.(y_j - x_i) = aw_j.y' + aw_j.D
              const double d = fma(q2.x, Dx[t], fma(q2.y, Dy[t], fma(q3.x, Dz[t], q3.y)));
              const double vr = d * m.x, vi = d * m.y;
              ar[t] = fma(wr, vr, fma(-wi, vi, ar[t]));
              ai[t] = fma(wi, vr, fma(wr, vi, ai[t]));
              if constexpr (FORM == 1) {
                const double g = e * ir;
                ar[t] = fma(g, fma(cs_, m.y, sn * m.x), ar[t]);
                ai[t] = fma(-g, fma(cs_, m.x, -(sn * m.y)), ai[t]);
              }
            }
            // target j, source i
            {
              // k aw_i.(x_i - y_j) = -aw_i.D - aw_i.y'
              const double d = fma(nx[t], q0.x, fma(ny[t], q0.y, fma(nz[t], q1.x, bq[t])));
              const double ur = d * mre[t], ui = d * mie[t];
              if (t == 0) {
                cr = fma(wr, ur, -(wi * ui));
                ci = fma(wi, ur, wr * ui);
              } else {
                cr = fma(wr, ur, fma(-wi, ui, cr));
                ci = fma(wi, ur, fma(wr, ui, ci));
              }
              if constexpr (FORM == 1) {
                const double g = ewi[t] * ir;
                cr = fma(g, fma(cs_, mie[t], sn * mre[t]), cr);
                ci = fma(-g, fma(cs_, mre[t], -(sn * mie[t])), ci);
              }
            }
          }
          acc0 = from_next_lane(acc0) + cr;
          acc1 = from_next_lane(acc1) + ci;
        }
#pragma unroll
        for (int t = 0; t < 2; ++t) {
          if (!msk[t]) {
            sr[t] += ar[t];
            si[t] += ai[t];
          }
        }
        if (!dtask) {
          if (half) {   // the two slots of a source: lanes l and l + 32
            acc0 += __shfl_xor(acc0, 32);
            acc1 += __shfl_xor(acc1, 32);
          }
          if (wv == 1) {
            sX[0][lane] = acc0;
            sX[1][lane] = acc1;
          }
          __syncthreads();
          const int sj = half ? ((lane + 31) & 31) : src;
          if (wv == 0 && (!half || lane < 32) && sj < cl) {
            const double vr = (acc0 + sX[0][lane]) * sc2;
            const double vi = (acc1 + sX[1][lane]) * sc2;
            double2* d = part + T.soff + (int64_t)jj * SYM_T + cs + sj;
            if (first_src) {
              *d = make_double2(vr, vi);
            } else {
              const double2 o = *d;
              *d = make_double2(o.x + vr, o.y + vi);
            }
          }
        }
        cs += cl;
      }
    }
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      const int loc = wv * 128 + t * 64 + lane;
      if (loc < BI.n)
        part[T.toff + (int64_t)ii * SYM_T + loc] = make_double2(sr[t] * sc2, si[t] * sc2);
    }
  }
}

// out[n] (+)= the slots of n's block in this launch.  A workgroup takes 64
// consecutive nodes; wavefront w adds the list entries w, w + 4, ... of each
// node, and the four sums are added in wavefront order (a fixed order).
// mode 0: out = sum, 1: out += sum.
__global__ __launch_bounds__(256) void reduce_sym_kernel(
    const double2* __restrict__ part, const int32_t* __restrict__ node_block,
    const SymBlock* __restrict__ blocks, const int64_t* __restrict__ lptr,
    const int64_t* __restrict__ list, int64_t N, double2* __restrict__ out, int mode) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t n = (int64_t)blockIdx.x * 64 + lane;
  __shared__ double2 red[4][64];
  double2 acc = make_double2(0.0, 0.0);
  int64_t e0 = 0, e1 = 0;
  if (n < N) {
    const int blk = node_block[n];
    e0 = lptr[blk];
    e1 = lptr[blk + 1];
    const int64_t rel = n - blocks[blk].n0;
#pragma unroll 4
    for (int64_t e = e0 + w; e < e1; e += 4) {
      const double2 v = part[list[e] + rel];
      acc.x += v.x;
      acc.y += v.y;
    }
  }
  red[w][lane] = acc;
  __syncthreads();
  if (w == 0 && n < N && (mode == 0 || e1 > e0)) {
    double2 o = mode ? out[n] : make_double2(0.0, 0.0);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      o.x += red[q][lane].x;
      o.y += red[q][lane].y;
    }
    out[n] = o;
  }
}

// The same for complex64 slots, two nodes per lane (16-byte loads): a
// workgroup takes 128 consecutive nodes.  Block starts and lengths are even
// (node counts are multiples of 32), so both nodes of a lane share a block.
__global__ __launch_bounds__(256) void reduce_sym32_kernel(
    const float4* __restrict__ part, const int32_t* __restrict__ node_block,
    const SymBlock* __restrict__ blocks, const int64_t* __restrict__ lptr,
    const int64_t* __restrict__ list, int64_t N, double2* __restrict__ out, int mode) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t n = (int64_t)blockIdx.x * 128 + 2 * lane;
  __shared__ double4 red[4][64];
  double4 acc = make_double4(0.0, 0.0, 0.0, 0.0);
  int64_t e0 = 0, e1 = 0;
  if (n < N) {
    const int blk = node_block[n];
    e0 = lptr[blk];
    e1 = lptr[blk + 1];
    const int64_t rel2 = (n - blocks[blk].n0) >> 1;   // pair index within a slot
#pragma unroll 4
    for (int64_t e = e0 + w; e < e1; e += 4) {
      const float4 v = part[(list[e] >> 1) + rel2];
      acc.x += (double)v.x;
      acc.y += (double)v.y;
      acc.z += (double)v.z;
      acc.w += (double)v.w;
    }
  }
  red[w][lane] = acc;
  __syncthreads();
  if (w == 0 && n < N && (mode == 0 || e1 > e0)) {
    double2 o0 = mode ? out[n] : make_double2(0.0, 0.0);
    double2 o1 = mode ? out[n + 1] : make_double2(0.0, 0.0);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      o0.x += red[q][lane].x;
      o0.y += red[q][lane].y;
      o1.x += red[q][lane].z;
      o1.y += red[q][lane].w;
    }
    out[n] = o0;
    out[n + 1] = o1;
  }
}

// Blocks of SYM_T consecutive nodes per problem, and the block of each node.
static void plan_sym_blocks(qax_problem* p) {
  auto& S = p->sym;
  S.ok = p->n_problems > 0;
  for (int pr = 0; pr < p->n_problems; ++pr) S.ok = S.ok && p->k[pr] > 0.0;
  S.blocks.clear();
  S.prob_blk0.assign(p->n_problems + 1, 0);
  S.blk_body_lo.clear();
  S.blk_body_hi.clear();
  for (int pr = 0; pr < p->n_problems; ++pr) {
    S.prob_blk0[pr] = (int32_t)S.blocks.size();
    const int b0 = (int)p->prob_body0[pr], b1 = (int)p->prob_body0[pr + 1];
    const int64_t n0 = p->off[b0], n1 = p->off[b1];
    int lo = b0;
    for (int64_t a = n0; a < n1; a += SYM_T) {
      SymBlock B;
      B.n0 = a;
      B.n = (int32_t)std::min<int64_t>(SYM_T, n1 - a);
      B.problem = pr;
      while (lo + 1 < b1 && p->off[lo + 1] <= a) ++lo;
      int hi = lo;
      while (hi + 1 < b1 && p->off[hi + 1] <= a + B.n - 1) ++hi;
      S.blocks.push_back(B);
      S.blk_body_lo.push_back(lo);
      S.blk_body_hi.push_back(hi);
    }
  }
  S.prob_blk0[p->n_problems] = (int32_t)S.blocks.size();
}

// Super-tasks of s x s block pairs, sorted by decreasing cost, cut into
// launches whose slots fit `cap` complex values; per launch and block, the
// slots that hold sums of the block's nodes (in super-task order).
static void plan_sym_supers(qax_problem* p, int pi, int s, int64_t cap) {
  auto& S = p->sym;
  auto& P = S.plan[pi];
  P.supers.clear();
  const int nblk = (int)S.blocks.size();
  auto same_body = [&](int I, int J) {
    return S.blk_body_lo[I] == S.blk_body_hi[I] && S.blk_body_lo[J] == S.blk_body_hi[J] &&
           S.blk_body_lo[I] == S.blk_body_lo[J];
  };
  std::vector<double> cost;
  for (int pr = 0; pr < p->n_problems; ++pr) {
    const int g0 = S.prob_blk0[pr], g1 = S.prob_blk0[pr + 1];
    for (int r0 = g0; r0 < g1; r0 += s)
      for (int c0 = r0; c0 < g1; c0 += s) {
        SymSuper T;
        T.i0 = r0;
        T.ni = std::min(s, g1 - r0);
        T.j0 = c0;
        T.nj = std::min(s, g1 - c0);
        T.diag = r0 == c0 ? 1 : 0;
        T.problem = pr;
        T.k = p->k[pr];
        T.skip = 0;
        double c = 0.0;
        int visits = 0;
        for (int ii = 0; ii < T.ni; ++ii)
          for (int jj = T.diag ? ii : 0; jj < T.nj; ++jj) {
            const int I = r0 + ii, J = c0 + jj;
            if (same_body(I, J)) {
              T.skip |= 1ull << (ii * SYM_SMAX + jj);
              continue;
            }
            ++visits;
            c += (double)S.blocks[I].n * S.blocks[J].n;
          }
        if (!visits) continue;
        T.toff = T.soff = 0;
        P.supers.push_back(T);
        cost.push_back(c);
      }
  }
  // decreasing cost (stable: ties keep the construction order); the costs
  // take few distinct values (products of block sizes), so the order is
  // built by buckets of equal cost, which is the stable sort's order
  std::vector<int64_t> ord;
  {
    std::vector<double> uniq(cost);
    std::sort(uniq.begin(), uniq.end(), std::greater<double>());
    uniq.erase(std::unique(uniq.begin(), uniq.end()), uniq.end());
    ord.reserve(cost.size());
    if (uniq.size() <= 256) {
      std::vector<int64_t> cnt(uniq.size() + 1, 0);
      std::vector<int32_t> bucket(cost.size());
      for (size_t i = 0; i < cost.size(); ++i) {
        bucket[i] = (int32_t)(std::lower_bound(uniq.begin(), uniq.end(), cost[i], std::greater<double>()) -
                              uniq.begin());
        ++cnt[bucket[i] + 1];
      }
      for (size_t b = 1; b < cnt.size(); ++b) cnt[b] += cnt[b - 1];
      ord.resize(cost.size());
      for (size_t i = 0; i < cost.size(); ++i) ord[cnt[bucket[i]]++] = (int64_t)i;
    } else {
      for (size_t i = 0; i < cost.size(); ++i) ord.push_back((int64_t)i);
      std::stable_sort(ord.begin(), ord.end(), [&](int64_t a, int64_t b) { return cost[a] > cost[b]; });
    }
  }
  std::vector<SymSuper> sorted;
  sorted.reserve(ord.size());
  for (int64_t i : ord) sorted.push_back(P.supers[i]);
  P.supers.swap(sorted);
  // launches and slot offsets
  P.launch_super.assign(1, 0);
  P.max_slots = 0;
  int64_t used = 0;
  for (size_t i = 0; i < P.supers.size(); ++i) {
    SymSuper& T = P.supers[i];
    const int64_t need = (int64_t)(T.ni + T.nj) * SYM_T;
    if (used > 0 && used + need > cap) {
      P.launch_super.push_back((int64_t)i);
      used = 0;
    }
    T.toff = used;
    T.soff = used + (int64_t)T.ni * SYM_T;
    used += need;
    P.max_slots = std::max(P.max_slots, used);
  }
  P.launch_super.push_back((int64_t)P.supers.size());
  const int nl = (int)P.launch_super.size() - 1;
  // lists: per launch, per block, the slots in super-task order (counted,
  // then filled)
  P.lptr.assign((size_t)nl * (nblk + 1), 0);
  P.list.clear();
  std::vector<int64_t> fill(nblk + 1);
  for (int pass = 0; pass < 2; ++pass) {
    int64_t base = 0;
    for (int l = 0; l < nl; ++l) {
      int64_t* lp = P.lptr.data() + (size_t)l * (nblk + 1);
      if (pass == 0) std::fill(fill.begin(), fill.end(), 0);
      else std::copy(lp, lp + nblk + 1, fill.begin());
      for (int64_t i = P.launch_super[l]; i < P.launch_super[l + 1]; ++i) {
        const SymSuper& T = P.supers[i];
        uint32_t colseen = 0;
        for (int ii = 0; ii < T.ni; ++ii) {
          bool row = false;
          for (int jj = T.diag ? ii : 0; jj < T.nj; ++jj) {
            if ((T.skip >> (ii * SYM_SMAX + jj)) & 1ull) continue;
            row = true;
            if (T.i0 + ii != T.j0 + jj) colseen |= 1u << jj;
          }
          if (row) {
            if (pass == 0) ++fill[T.i0 + ii];
            else P.list[fill[T.i0 + ii]++] = T.toff + (int64_t)ii * SYM_T;
          }
        }
        for (int jj = 0; jj < T.nj; ++jj)
          if ((colseen >> jj) & 1u) {
            if (pass == 0) ++fill[T.j0 + jj];
            else P.list[fill[T.j0 + jj]++] = T.soff + (int64_t)jj * SYM_T;
          }
      }
      if (pass == 0) {
        for (int b = 0; b < nblk; ++b) {
          lp[b] = base;
          base += fill[b];
        }
        lp[nblk] = base;
      }
    }
    if (pass == 0) P.list.assign((size_t)base, 0);
  }
  P.s = s;
}

static hipError_t upload_sym_blocks(qax_problem* p) {
  auto& S = p->sym;
  if (S.d_bmem) {
    hipError_t e = hipStreamSynchronize(p->stream);
    if (e != hipSuccess) return e;
    dev_release(p, S.d_bmem);
    S.d_bmem = nullptr;
  }
  auto al = [](size_t x) { return (x + 255) / 256 * 256; };
  const size_t bb = al(sizeof(SymBlock) * std::max<size_t>(1, S.blocks.size()));
  const size_t bn = al(sizeof(int32_t) * std::max<int64_t>(1, p->N));
  hipError_t e = dev_alloc(p, &S.d_bmem, bb + bn);
  if (e != hipSuccess) return e;
  S.d_blocks = (SymBlock*)S.d_bmem;
  S.d_node_block = (int32_t*)((char*)S.d_bmem + bb);
  std::vector<int32_t> nb(p->N);
  for (size_t b = 0; b < S.blocks.size(); ++b)
    for (int t = 0; t < S.blocks[b].n; ++t) nb[S.blocks[b].n0 + t] = (int32_t)b;
  if (!S.blocks.empty())
    e = hipMemcpyAsync(S.d_blocks, S.blocks.data(), sizeof(SymBlock) * S.blocks.size(),
                       hipMemcpyHostToDevice, p->stream);
  if (e == hipSuccess && p->N)
    e = hipMemcpyAsync(S.d_node_block, nb.data(), sizeof(int32_t) * p->N, hipMemcpyHostToDevice, p->stream);
  if (e != hipSuccess) return e;
  return hipStreamSynchronize(p->stream);
}

// Drop plan pi's device arrays (after the stream has drained).
hipError_t release_sym_plan(qax_problem* p, int pi) {
  auto& P = p->sym.plan[pi];
  if (P.d_mem) {
    hipError_t e = hipStreamSynchronize(p->stream);
    if (e != hipSuccess) return e;
    dev_release(p, P.d_mem);
  }
  P.d_mem = nullptr;
  P.d_supers = nullptr;
  P.d_lptr = nullptr;
  P.d_list = nullptr;
  P.s = 0;
  P.supers.clear();
  P.launch_super.clear();
  P.lptr.clear();
  P.list.clear();
  P.max_slots = 0;
  return hipSuccess;
}

static hipError_t upload_sym_plan(qax_problem* p, int pi) {
  auto& P = p->sym.plan[pi];
  auto al = [](size_t x) { return (x + 255) / 256 * 256; };
  const size_t bs = al(sizeof(SymSuper) * std::max<size_t>(1, P.supers.size()));
  const size_t bp = al(sizeof(int64_t) * std::max<size_t>(1, P.lptr.size()));
  const size_t bl = al(sizeof(int64_t) * std::max<size_t>(1, P.list.size()));
  hipError_t e = dev_alloc(p, &P.d_mem, bs + bp + bl);
  if (e != hipSuccess) return e;
  char* m = (char*)P.d_mem;
  P.d_supers = (SymSuper*)m;
  P.d_lptr = (int64_t*)(m + bs);
  P.d_list = (int64_t*)(m + bs + bp);
  auto cp = [&](void* d, const void* h, size_t n) {
    if (e == hipSuccess && n) e = hipMemcpyAsync(d, h, n, hipMemcpyHostToDevice, p->stream);
  };
  cp(P.d_supers, P.supers.data(), sizeof(SymSuper) * P.supers.size());
  cp(P.d_lptr, P.lptr.data(), sizeof(int64_t) * P.lptr.size());
  cp(P.d_list, P.list.data(), sizeof(int64_t) * P.list.size());
  if (e != hipSuccess) return e;
  e = hipStreamSynchronize(p->stream);
  // the launches need only the launch ranges on the host
  std::vector<SymSuper>().swap(P.supers);
  std::vector<int64_t>().swap(P.lptr);
  std::vector<int64_t>().swap(P.list);
  return e;
}

// Default super-task size: the largest of 8, 4, 2, 1 that still gives every
// compute unit 16 super-tasks.
int sym_default_s(const qax_problem* p, int cu_count) {
  const auto& S = p->sym;
  for (int s : {8, 4, 2}) {
    int64_t n = 0;
    for (int pr = 0; pr < p->n_problems; ++pr) {
      const int64_t r = (S.prob_blk0[pr + 1] - S.prob_blk0[pr] + s - 1) / s;
      n += r * (r + 1) / 2;
    }
    if (n >= 16LL * cu_count) return s;
  }
  return 1;
}

// (Re)plan the reciprocal kernels for super-tasks of s x s block pairs
// (s <= 0: the default), precision index pi (0 FP64, 1 FP32).
hipError_t plan_sym(qax_problem* p, int pi, int s, int cu_count) {
  auto& S = p->sym;
  if (!S.d_bmem) {
    plan_sym_blocks(p);
    hipError_t e = upload_sym_blocks(p);
    if (e != hipSuccess) return e;
  }
  if (s <= 0) s = sym_default_s(p, cu_count);
  s = std::max(1, std::min(SYM_SMAX, s));
  if (S.plan[pi].d_mem && S.plan[pi].s == s) return hipSuccess;
  hipError_t e = release_sym_plan(p, pi);
  if (e != hipSuccess) return e;
  ++p->generation;   // captured solver steps hold the old launch sizes
  // the FP32 slots are complex64: twice as many fit the same workspace
  plan_sym_supers(p, pi, s, SYM_SLOT_CAP * (pi == 1 ? 2 : 1));
  return upload_sym_plan(p, pi);
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
  {
    // the reciprocal kernels' super-tasks (kept while the geometry and the
    // super-task size are unchanged)
    hipError_t e = plan_sym(p, prec == QAX_FP64 ? 0 : 1, p->tune.sym_s[prec == QAX_FP64 ? 0 : 1], cu_count);
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
    b = std::max(b, (size_t)p->sym.plan[prec == QAX_FP64 ? 0 : 1].max_slots * (prec == QAX_FP64 ? 16 : 8));
  return b;
}

static bool use_sym(const qax_problem* p, int prec, int nrhs) {
  return nrhs == 1 && p->sym.ok && p->sym.enabled && p->sym.plan[prec == QAX_FP64 ? 0 : 1].d_mem &&
         p->form() != 2;
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
    auto& P = S.plan[pi];
    const int form = p->form();
    double2* part = (double2*)partial;
    const int nblk = (int)S.blocks.size();
    const int nl = (int)P.launch_super.size() - 1;
    const dim3 rgrid((unsigned)((p->N + 63) / 64));
    for (int l = 0; l < nl; ++l) {
      const int64_t s0 = P.launch_super[l], s1 = P.launch_super[l + 1];
      if (s1 > s0) {
        const dim3 grid((unsigned)(s1 - s0));
        timing_begin(p, kind);
        if (f64) {
          if (form == 1)
            hipLaunchKernelGGL(pair_sum_f64_sym_kernel<1>, grid, dim3(128), 0, p->stream, P.d_supers + s0,
                               S.d_blocks, p->d_bodies, p->d_node_body, p->d_pos, p->d_aw, p->d_ew, p->N,
                               (const double2*)mu, p->seg_active, part);
          else
            hipLaunchKernelGGL(pair_sum_f64_sym_kernel<0>, grid, dim3(128), 0, p->stream, P.d_supers + s0,
                               S.d_blocks, p->d_bodies, p->d_node_body, p->d_pos, p->d_aw, p->d_ew, p->N,
                               (const double2*)mu, p->seg_active, part);
        } else {
          if (form == 1)
            hipLaunchKernelGGL(pair_sum_f32_sym_kernel<1>, grid, dim3(128), 0, p->stream, P.d_supers + s0,
                               S.d_blocks, p->d_bodies, p->d_node_body, (const float4*)p->d_loc32,
                               (const float4*)p->d_aw32, p->d_ew32, (const double2*)mu, p->seg_active,
                               (float2*)partial);
          else
            hipLaunchKernelGGL(pair_sum_f32_sym_kernel<0>, grid, dim3(128), 0, p->stream, P.d_supers + s0,
                               S.d_blocks, p->d_bodies, p->d_node_body, (const float4*)p->d_loc32,
                               (const float4*)p->d_aw32, p->d_ew32, (const double2*)mu, p->seg_active,
                               (float2*)partial);
        }
        timing_end(p, kind);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
      }
      const int mode = l == 0 ? (accumulate ? 1 : 0) : 1;
      if (f64)
        hipLaunchKernelGGL(reduce_sym_kernel, rgrid, dim3(256), 0, p->stream, (const double2*)part,
                           S.d_node_block, S.d_blocks, P.d_lptr + (size_t)l * (nblk + 1), P.d_list, p->N,
                           (double2*)out, mode);
      else
        hipLaunchKernelGGL(reduce_sym32_kernel, dim3((unsigned)((p->N + 127) / 128)), dim3(256), 0, p->stream,
                           (const float4*)partial, S.d_node_block, S.d_blocks, P.d_lptr + (size_t)l * (nblk + 1),
                           P.d_list, p->N, (double2*)out, mode);
      hipError_t e = hipGetLastError();
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
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
