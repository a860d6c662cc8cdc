// Surface nodes of quasi-axisymmetric bodies (Section 2, equation para_quasi;
// Section 3.1: tangents d_s, d_theta, Jacobian |J| = |d_s x d_theta|, panels of
// 16 Gauss-Legendre nodes x 2N trapezoidal azimuths; Section 6.2, Example 5:
// rigid motion x = R x0 + c, n = R n0).
#include <cmath>

#include "internal.h"
#include "shapes.h"

namespace qax {

// Gauss-Legendre nodes and weights on [-1, 1] by Newton's method on P_n
// (three-term recurrence for P_n and its derivative).
void gauss_legendre_host(int n, double* x, double* w) {
  for (int i = 0; i < n; ++i) {
    double z = std::cos(PI * (i + 0.75) / (n + 0.5));
    double dp = 0.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= n; ++k) {
        double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      dp = n * (z * p1 - p0) / (z * z - 1.0);
      double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= n; ++k) {
        double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      dp = n * (z * p1 - p0) / (z * z - 1.0);
    }
    // ascending order
    x[n - 1 - i] = z;
    w[n - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
}

__device__ __forceinline__ int find_body(const BodyDev* __restrict__ b, int nb, int64_t i) {
  int lo = 0, hi = nb - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (b[mid].off <= i) lo = mid; else hi = mid - 1;
  }
  return lo;
}

__global__ void build_nodes_kernel(const BodyDev* __restrict__ bodies, int nb, int64_t N,
                                   const double* __restrict__ gl, int32_t* __restrict__ node_body,
                                   double* __restrict__ pos, double* __restrict__ aw,
                                   float4* __restrict__ loc32, float4* __restrict__ aw32) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const int bi = find_body(bodies, nb, i);
  const BodyDev& B = bodies[bi];
  const int li = (int)(i - B.off);
  const int nth = B.n_theta;
  const int panel = li / (GL_ORDER * nth);
  const int l = (li / nth) % GL_ORDER;
  const int j = li % nth;
  const double e0 = panel_edge(B.n_uni, B.n_ref, panel);
  const double h = panel_edge(B.n_uni, B.n_ref, panel + 1) - e0;
  const double t = e0 + 0.5 * h * (gl[l] + 1.0);
  const double omega = 0.5 * h * gl[GL_ORDER + l];
  const int Nh = nth / 2;
  const double th = j * PI / Nh;
  Curve cv = curve_eval(B.shape, B.a, B.c, B.kappa, t);
  double sth, cth;
  sincos(th, &sth, &cth);
  // body-frame point and area normal d_theta x d_s
  const double y0[3] = {cv.r * cth + cv.p, cv.r * sth + cv.q, cv.z};
  const double n0[3] = {cv.r * cv.dz * cth, cv.r * cv.dz * sth,
                        -cv.r * (cv.dr + cv.dp * cth + cv.dq * sth)};
  const double wgt = omega * PI / Nh;
  double yl[3], nl[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    yl[a] = B.R[3 * a] * y0[0] + B.R[3 * a + 1] * y0[1] + B.R[3 * a + 2] * y0[2];
    nl[a] = (B.R[3 * a] * n0[0] + B.R[3 * a + 1] * n0[1] + B.R[3 * a + 2] * n0[2]) * wgt;
  }
  node_body[i] = bi;
  pos[i] = yl[0] + B.cen[0];
  pos[N + i] = yl[1] + B.cen[1];
  pos[2 * N + i] = yl[2] + B.cen[2];
  aw[i] = nl[0];
  aw[N + i] = nl[1];
  aw[2 * N + i] = nl[2];
  loc32[i] = make_float4((float)yl[0], (float)yl[1], (float)yl[2],
                         (float)(yl[0] * yl[0] + yl[1] * yl[1] + yl[2] * yl[2]));
  aw32[i] = make_float4((float)nl[0], (float)nl[1], (float)nl[2],
                        (float)(nl[0] * yl[0] + nl[1] * yl[1] + nl[2] * yl[2]));
}

// Combined-field weights eta |aw| per node (|aw| = |J| (pi/N) omega, the
// single-layer smooth-rule weight); zero for the double layer.
__global__ void node_weights_kernel(const BodyDev* __restrict__ bodies,
                                    const int32_t* __restrict__ node_body, int64_t N,
                                    const double* __restrict__ aw, double* __restrict__ ew,
                                    float* __restrict__ ew32) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const double eta = bodies[node_body[i]].eta;
  const double w = sqrt(aw[i] * aw[i] + aw[N + i] * aw[N + i] + aw[2 * N + i] * aw[2 * N + i]);
  ew[i] = eta * w;
  ew32[i] = (float)(eta * w);
}

hipError_t launch_node_weights(qax_problem* p) {
  const int64_t blocks = (p->N + 255) / 256;
  hipLaunchKernelGGL(node_weights_kernel, dim3((unsigned)blocks), dim3(256), 0, p->stream,
                     p->d_bodies, p->d_node_body, p->N, p->d_aw, p->d_ew, p->d_ew32);
  return hipGetLastError();
}

hipError_t launch_build_nodes(qax_problem* p) {
  const int tpb = 256;
  const int64_t blocks = (p->N + tpb - 1) / tpb;
  hipLaunchKernelGGL(build_nodes_kernel, dim3((unsigned)blocks), dim3(tpb), 0, p->stream,
                     p->d_bodies, p->n_bodies, p->N, p->d_gl, p->d_node_body, p->d_pos, p->d_aw,
                     (float4*)p->d_loc32, (float4*)p->d_aw32);
  return hipGetLastError();
}

}  // namespace qax
