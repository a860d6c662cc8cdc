// Scattered field at points off the surfaces: the double-layer potential of
// the density (Section 4, equation multi-double; minus i eta times the
// single-layer potential for the combined field) by the smooth product rule of
// Section 3.1 (equation sx), the same kernel as the inter-body pair sum, for
// evaluation points that are not nodes (the near-field part of the error
// study of Section 6).  FP64.
#include <algorithm>

#include "fastmath.h"
#include "internal.h"

namespace qax {

constexpr double INV_FOUR_PI_NF = 0.0795774715459476678844;

// out[e] = sum_s partial[s][e] (fixed order), from the pair-sum translation unit
__global__ void reduce_slots_kernel(const double2* __restrict__ partial, int slots, int64_t count,
                                    double2* __restrict__ out, int accumulate);

// ---------------------------------------------------------------- near field
// u(x) = 1/(4 pi) sum_{j in problem} (ik r - 1) e^{ikr} / r^3 (aw_j . (y_j - x)) mu_j
// at points x away from the surfaces (the smooth rule, as the pair sum):
// one point per thread, source tiles in LDS, the source range of the problem
// cut into `slots` chunks (blockIdx.y) whose partial sums are reduced in a
// fixed order afterwards; right-hand side blockIdx.z.
template <int TPB>
__global__ __launch_bounds__(TPB) void nearfield_kernel(
    const double* __restrict__ pts, int64_t M, const double* __restrict__ pos,
    const double* __restrict__ aw, const double* __restrict__ ew, int form, int64_t N, int64_t s0,
    int64_t s1, int slots, double k,
    const double2* __restrict__ mu, int nrhs, double2* __restrict__ partial) {
  const int tid = threadIdx.x;
  const int64_t i = (int64_t)blockIdx.x * TPB + tid;
  const bool active = i < M;
  const int r = blockIdx.z;
  const double xi = active ? pts[i] : 0.0, yi = active ? pts[M + i] : 0.0,
               zi = active ? pts[2 * M + i] : 0.0;
  const int64_t len = s1 - s0;
  const int64_t c0 = s0 + len * blockIdx.y / slots, c1 = s0 + len * (blockIdx.y + 1) / slots;
  __shared__ double sx[TPB], sy[TPB], sz[TPB], sax[TPB], say[TPB], saz[TPB], sew[TPB];
  __shared__ double2 smu[TPB];
  double ar = 0.0, ai = 0.0;
  for (int64_t base = c0; base < c1; base += TPB) {
    const int cnt = (int)min((int64_t)TPB, c1 - base);
    __syncthreads();
    if (tid < cnt) {
      const int64_t j = base + tid;
      sx[tid] = pos[j]; sy[tid] = pos[N + j]; sz[tid] = pos[2 * N + j];
      sax[tid] = aw[j]; say[tid] = aw[N + j]; saz[tid] = aw[2 * N + j];
      sew[tid] = form ? ew[j] : 0.0;
      smu[tid] = mu[j * nrhs + r];
    }
    __syncthreads();
    for (int jj = 0; jj < cnt; ++jj) {
      const double dx = sx[jj] - xi, dy = sy[jj] - yi, dz = sz[jj] - zi;
      const double r2 = dx * dx + dy * dy + dz * dz;
      const double ir = rsqrt(r2);
      const double rr = r2 * ir;
      const double kr = k * rr;
      double sn, cs;
      sincos_cw(kr, &sn, &cs);
      const double t = sew[jj] * ir;
      double re, im;
      if (form == 2) {                    // single layer: (|aw| / r)(cos kr + i sin kr)
        re = cs * t;
        im = sn * t;
      } else {
        const double sc = (sax[jj] * dx + say[jj] * dy + saz[jj] * dz) * ir * ir * ir;
        re = -(cs + kr * sn) * sc;
        im = (kr * cs - sn) * sc;
        re = fma(t, sn, re);              // combined field: (eta |aw| / r)(sin kr - i cos kr)
        im = fma(-t, cs, im);
      }
      const double2 m = smu[jj];
      ar += re * m.x - im * m.y;
      ai += re * m.y + im * m.x;
    }
  }
  if (active)
    partial[((int64_t)blockIdx.y * M + i) * nrhs + r] = make_double2(ar * INV_FOUR_PI_NF, ai * INV_FOUR_PI_NF);
}

// partial: slots x M x nrhs complex128 (nearfield_slots); u = sum over slots.
int nearfield_slots(int64_t M, int cu_count) {
  const int64_t blocks = (M + 255) / 256;
  return (int)std::max<int64_t>(1, std::min<int64_t>(64, (8LL * cu_count + blocks - 1) / blocks));
}

hipError_t launch_nearfield(qax_problem* p, const double* mu, int nrhs, const double* pts, int64_t M,
                            int problem, int slots, double* partial, double* u) {
  const int64_t s0 = p->off[p->prob_body0[problem]], s1 = p->off[p->prob_body0[problem + 1]];
  dim3 grid((unsigned)((M + 255) / 256), (unsigned)slots, (unsigned)nrhs);
  hipLaunchKernelGGL((nearfield_kernel<256>), grid, dim3(256), 0, p->stream, pts, M, p->d_pos,
                     p->d_aw, p->d_ew, p->form(), p->N, s0, s1,
                     slots, p->k[problem], (const double2*)mu, nrhs, (double2*)partial);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t count = M * nrhs;
  hipLaunchKernelGGL(reduce_slots_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0,
                     p->stream, (const double2*)partial, slots, count, (double2*)u, 0);
  return hipGetLastError();
}

}  // namespace qax
