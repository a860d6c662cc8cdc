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
  ++p->generation;   // captured solver steps hold the old launch sizes
  std::vector<PairTask>& t = prec == QAX_FP64 ? p->tasks64 : p->tasks32;
  PairTask*& d = prec == QAX_FP64 ? p->d_tasks64 : p->d_tasks32;
  if (d) {
    hipError_t e = hipStreamSynchronize(p->stream);
    if (e != hipSuccess) return e;
    (void)hipFree(d);
    d = nullptr;
  }
  hipError_t e = hipMalloc(&d, sizeof(PairTask) * t.size());
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
  return std::max((size_t)slots * p->N * nrhs * 16, lattice_work_bytes(p, nrhs));
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
