// Vector kernels of the solver: plane-wave right-hand side (Section 2 and
// Section 6, equation plane wave parameters), far field of the double-layer
// density (Section 6: the far-field pattern, with the normal derivative of the
// kernel for a double-layer density; plus the single-layer term for the
// combined field), and the GMRES building blocks.
//
// GMRES vectors are N x nrhs complex128 (right-hand sides fastest).  Every
// (problem, right-hand side) pair is an independent "segment": dot products
// and norms are segmented by problem node range and right-hand side, and are
// reduced in a fixed order so results do not depend on scheduling.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>

#include "fastmath.h"
#include "internal.h"
#include "krylov.h"

namespace qax {

constexpr double INV_FOUR_PI_K = 0.0795774715459476678844;

__global__ void rhs_kernel(const BodyDev* __restrict__ bodies, const int32_t* __restrict__ node_body,
                           const double* __restrict__ pos, int64_t N, const double* __restrict__ dirs,
                           int nrhs, double2* __restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= N * nrhs) return;
  const int64_t n = e / nrhs;
  const int r = (int)(e % nrhs);
  const BodyDev& B = bodies[node_body[n]];
  const double* d = dirs + ((int64_t)B.problem * nrhs + r) * 3;
  const double ph = B.k * (d[0] * pos[n] + d[1] * pos[N + n] + d[2] * pos[2 * N + n]);
  double s, c;
  sincos_cw(ph, &s, &c);
  out[e] = make_double2(-c, -s);
}

hipError_t launch_rhs(qax_problem* p, const double* dirs_dev, int nrhs, double* out) {
  const int64_t cnt = p->N * nrhs;
  hipLaunchKernelGGL(rhs_kernel, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, p->stream,
                     p->d_bodies, p->d_node_body, p->d_pos, p->N, dirs_dev, nrhs, (double2*)out);
  return hipGetLastError();
}

// out[e] = sum_s partial[s][e] (fixed order), from the pair-sum translation unit
__global__ void reduce_slots_kernel(const double2* __restrict__ partial, int slots, int64_t count,
                                    double2* __restrict__ out, int accumulate);

// u_inf[p][dir][r] = (1/4pi) sum_{n in problem p} (-i k_p xhat.aw_n)
// e^{-i k_p xhat.y_n} mu[n][r] (combined field: plus -i eta |aw_n| e^{...};
// single layer: |aw_n| e^{...} alone).  One item per thread: a direction, or a
// direction and its exact negation (the phase negated: one sin/cos for
// both); node tiles staged in LDS and read by broadcast, the problem's node
// range cut into `slots` chunks (blockIdx.y) whose partial sums are added in a
// fixed order afterwards; blockIdx.z = problem * nrhs + right-hand side.
// pinfo: the problems' first nodes (n_problems + 1 int64) then their k.
// The phase is taken in 512ths of a revolution for sincos_tab512 (table in
// LDS per workgroup); PAIRS: the list holds negated pairs (else the second
// direction's sums are not formed).
template <int TPB, bool PAIRS>
__global__ __launch_bounds__(TPB) void farfield_kernel(
    const double* __restrict__ xhat, const int2* __restrict__ items, int64_t M, int64_t Mi,
    const double* __restrict__ pos, const double* __restrict__ aw, const double* __restrict__ ew,
    int form, int64_t N, const int64_t* __restrict__ pinfo, int nprob, int slots,
    const double2* __restrict__ mu, int nrhs, double2* __restrict__ partial) {
  const int tid = threadIdx.x;
  const int64_t t = (int64_t)blockIdx.x * TPB + tid;
  const bool active = t < Mi;
  // direction i and, when the list holds its exact negation, that one (i2):
  // its phase is the negated phase, so sin flips sign and cos is unchanged
  // items == nullptr: one item per direction, no pairs
  const int2 it = active ? (items ? items[t] : make_int2((int)t, -1)) : make_int2(0, -1);
  const int64_t i = it.x, i2 = it.y;
  const double pair = i2 >= 0 ? 1.0 : 0.0;
  const int r = blockIdx.z % nrhs, pr = blockIdx.z / nrhs;
  const int64_t pn0 = pinfo[pr], pn = pinfo[pr + 1] - pn0;
  const double k = __longlong_as_double(pinfo[nprob + 1 + pr]);
  const double hx = active ? xhat[3 * i] : 0.0, hy = active ? xhat[3 * i + 1] : 0.0,
               hz = active ? xhat[3 * i + 2] : 0.0;
  // phase -k x.y / 2 pi in 512ths of a revolution and k x, per direction
  const double kr = -k * (512.0 / TWO_PI);
  const double px = kr * hx, py = kr * hy, pz = kr * hz;
  const double qx = k * hx, qy = k * hy, qz = k * hz;
  const int64_t c0 = pn0 + pn * blockIdx.y / slots, c1 = pn0 + pn * (blockIdx.y + 1) / slots;
  __shared__ double sx[TPB], sy[TPB], sz[TPB], sax[TPB], say[TPB], saz[TPB], sew[TPB];
  __shared__ double2 smu[TPB];
  __shared__ double2 sTab[512];
  fill_tab512(sTab, tid, TPB);   // ordered by the first tile's barrier
  double ar = 0.0, ai = 0.0, br = 0.0, bi = 0.0;
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
    if (form == 2) {
      for (int jj = 0; jj < cnt; ++jj) {
        double s, c;
        sincos_tab512(fma(px, sx[jj], fma(py, sy[jj], pz * sz[jj])), sTab, &s, &c);
        const double fr = sew[jj] * c, fi = sew[jj] * s;
        const double2 m = smu[jj];
        ar = fma(fr, m.x, fma(-fi, m.y, ar));
        ai = fma(fr, m.y, fma(fi, m.x, ai));
        if constexpr (PAIRS) {
          // -x: fr, -fi
          br = fma(fr, m.x, fma(fi, m.y, br));
          bi = fma(fr, m.y, fma(-fi, m.x, bi));
        }
      }
    } else {
      for (int jj = 0; jj < cnt; ++jj) {
        double s, c;
        sincos_tab512(fma(px, sx[jj], fma(py, sy[jj], pz * sz[jj])), sTab, &s, &c);
        // (-i k nd)(c + i s) = k nd s - i k nd c; combined field adds
        // (-i eta |aw|)(c + i s) = eta |aw| s - i eta |aw| c (ew = 0 otherwise)
        const double d = fma(qx, sax[jj], fma(qy, say[jj], qz * saz[jj]));
        const double a = d + sew[jj];
        const double fr = a * s, fi = -a * c;
        const double2 m = smu[jj];
        ar = fma(fr, m.x, fma(-fi, m.y, ar));
        ai = fma(fr, m.y, fma(fi, m.x, ai));
        if constexpr (PAIRS) {
          // -x: k nd -> -k nd, s -> -s: (eta |aw| - d)(-s) - i (eta |aw| - d) c
          const double a2 = sew[jj] - d;
          const double gr = -a2 * s, gi = -a2 * c;
          br = fma(gr, m.x, fma(-gi, m.y, br));
          bi = fma(gr, m.y, fma(gi, m.x, bi));
        }
      }
    }
  }
  if (active) {
    const int64_t base = ((int64_t)blockIdx.y * nprob + pr) * M;
    partial[(base + i) * nrhs + r] = make_double2(ar * INV_FOUR_PI_K, ai * INV_FOUR_PI_K);
    if (pair > 0.0)
      partial[(base + i2) * nrhs + r] = make_double2(br * INV_FOUR_PI_K, bi * INV_FOUR_PI_K);
  }
}

int farfield_slots(int64_t M, int cu_count) {
  const int64_t blocks = (M + 255) / 256;
  return (int)std::max<int64_t>(1, std::min<int64_t>(64, (8LL * cu_count + blocks - 1) / blocks));
}

// out[problem][dir][r] (directions xhat_dev, 3 doubles each; pinfo_dev as
// the kernel's pinfo; items_dev may be null: no pairs); partial:
// farfield_slots x n_problems x ndir x nrhs complex128.
hipError_t launch_farfield(qax_problem* p, const double* mu, int nrhs, const double* xhat_dev,
                           int ndir, const int2* items_dev, int nitems, const int64_t* pinfo_dev,
                           int slots, double* partial, double* out) {
  dim3 grid((unsigned)((nitems + 255) / 256), (unsigned)slots, (unsigned)(nrhs * p->n_problems));
  // items pair a direction with its negation only when there are fewer
  // items than directions
  auto kern = nitems < ndir ? farfield_kernel<256, true> : farfield_kernel<256, false>;
  hipLaunchKernelGGL(kern, grid, dim3(256), 0, p->stream, xhat_dev, items_dev,
                     (int64_t)ndir, (int64_t)nitems, p->d_pos, p->d_aw, p->d_ew, p->form(), p->N,
                     pinfo_dev, p->n_problems, slots, (const double2*)mu, nrhs, (double2*)partial);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t count = (int64_t)p->n_problems * ndir * nrhs;
  hipLaunchKernelGGL(reduce_slots_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0,
                     p->stream, (const double2*)partial, slots, count, (double2*)out, 0);
  return hipGetLastError();
}

// ---------------------------------------------------------------- segmented dots
// partial[i][chunk][r] = sum_{n in chunk} conj(V_i[n][r]) w[n][r]
// The block has U*nrhs threads (U = 256/nrhs rounded down); thread t handles
// right-hand side t % nrhs.
__global__ __launch_bounds__(256) void mdot_kernel(const double2* __restrict__ V, int64_t vstride,
                                                   const double2* __restrict__ w, int nrhs,
                                                   const Chunk* __restrict__ chunks,
                                                   double2* __restrict__ partial, int nchunks) {
  const Chunk C = chunks[blockIdx.x];
  const int i = blockIdx.y;
  const double2* v = V + (int64_t)i * vstride;
  const int nthr = blockDim.x;
  const int U = nthr / nrhs;
  const int t = threadIdx.x;
  const int r = t % nrhs;
  const int u = t / nrhs;
  double ar = 0.0, ai = 0.0;
  for (int64_t n = C.n0 + u; n < C.n1; n += U) {
    const double2 a = v[n * nrhs + r];
    const double2 b = w[n * nrhs + r];
    ar += a.x * b.x + a.y * b.y;
    ai += a.x * b.y - a.y * b.x;
  }
  __shared__ double sr[256], si[256];
  sr[t] = ar;
  si[t] = ai;
  __syncthreads();
  if (t < nrhs) {
    double xr = 0.0, xi = 0.0;
    for (int q = 0; q < U; ++q) {
      xr += sr[t + q * nrhs];
      xi += si[t + q * nrhs];
    }
    partial[((int64_t)i * nchunks + blockIdx.x) * nrhs + t] = make_double2(xr, xi);
  }
}

// h[i][problem][r] = sum over the chunks of the problem (in order).
__global__ void mdot_reduce_kernel(const double2* __restrict__ partial, int nchunks, int nrhs,
                                   const int32_t* __restrict__ prob_chunk0, int nprob,
                                   double2* __restrict__ h) {
  const int i = blockIdx.y;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nprob * nrhs) return;
  const int pr = e / nrhs, r = e % nrhs;
  double xr = 0.0, xi = 0.0;
  for (int c = prob_chunk0[pr]; c < prob_chunk0[pr + 1]; ++c) {
    const double2 v = partial[((int64_t)i * nchunks + c) * nrhs + r];
    xr += v.x;
    xi += v.y;
  }
  h[(int64_t)i * nprob * nrhs + e] = make_double2(xr, xi);
}

// w[n][r] -= sum_{i<m} V_i[n][r] h[i][problem(n)][r]
__global__ void orth_update_kernel(const double2* __restrict__ V, int64_t vstride, int m,
                                   const double2* __restrict__ h, const int32_t* __restrict__ node_prob,
                                   int nprob, int64_t N, int nrhs, double2* __restrict__ w) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= N * nrhs) return;
  const int64_t n = e / nrhs;
  const int r = (int)(e % nrhs);
  const int pr = node_prob[n];
  double2 acc = w[e];
  for (int i = 0; i < m; ++i) {
    const double2 v = V[(int64_t)i * vstride + e];
    const double2 c = h[((int64_t)i * nprob + pr) * nrhs + r];
    acc.x -= v.x * c.x - v.y * c.y;
    acc.y -= v.x * c.y + v.y * c.x;
  }
  w[e] = acc;
}

// out[n][r] = (accumulate ? out : 0) + sum_{i<m} V_i[n][r] y[i][problem(n)][r]
__global__ void combine_kernel(const double2* __restrict__ V, int64_t vstride, int m,
                               const double2* __restrict__ y, const int32_t* __restrict__ node_prob,
                               int nprob, int64_t N, int nrhs, double2* __restrict__ out,
                               int accumulate) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= N * nrhs) return;
  const int64_t n = e / nrhs;
  const int r = (int)(e % nrhs);
  const int pr = node_prob[n];
  double2 acc = accumulate ? out[e] : make_double2(0.0, 0.0);
  for (int i = 0; i < m; ++i) {
    const double2 v = V[(int64_t)i * vstride + e];
    const double2 c = y[((int64_t)i * nprob + pr) * nrhs + r];
    acc.x += v.x * c.x - v.y * c.y;
    acc.y += v.x * c.y + v.y * c.x;
  }
  out[e] = acc;
}

// out[n][r] = a[n][r] * s[problem(n)][r]  (complex scale per segment)
__global__ void seg_scale_kernel(const double2* __restrict__ a, const double2* __restrict__ s,
                                 const int32_t* __restrict__ node_prob, int64_t N, int nrhs,
                                 double2* __restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= N * nrhs) return;
  const int64_t n = e / nrhs;
  const int r = (int)(e % nrhs);
  const double2 c = s[(int64_t)node_prob[n] * nrhs + r];
  const double2 v = a[e];
  out[e] = make_double2(v.x * c.x - v.y * c.y, v.x * c.y + v.y * c.x);
}

// out = alpha*a + beta*b (real scalars)
__global__ void axpby_kernel(double alpha, const double2* __restrict__ a, double beta,
                             const double2* __restrict__ b, int64_t cnt, double2* __restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= cnt) return;
  const double2 x = a[e];
  const double2 y = b[e];
  out[e] = make_double2(alpha * x.x + beta * y.x, alpha * x.y + beta * y.y);
}

// ---------------------------------------------------------------- least squares
__device__ __forceinline__ double2 cmul_k(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 conj_k(double2 a) { return make_double2(a.x, -a.y); }

// One thread per segment: column j of the Hessenberg matrix (h1 + h2 for rows
// <= j, |w| below), the earlier rotations applied to it, the rotation that
// annihilates the subdiagonal (cs real, sn complex), g updated, the scale
// 1/h_{j+1,j} of the next basis vector, and the convergence count.  A
// segment that reaches its tolerance (or a breakdown, |w| ~ 0) stops: its
// step count is kept for the back substitution, its next basis vectors are
// zero and its `active` flag lets the operator skip it.
__global__ void givens_kernel(int nseg, int j, int m, const double2* __restrict__ h1,
                              const double2* __restrict__ h2, const double2* __restrict__ hn2,
                              GivensState G) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nseg) return;
  const bool stopped = G.frozen[s] != 0 || G.kconv[s] != 0;
  if (stopped) {
    G.scl[s] = make_double2(0.0, 0.0);
    return;
  }
  double2* col = G.H + ((int64_t)s * m + j) * (m + 1);
  for (int i = 0; i <= j; ++i) {
    const double2 a = h1[(int64_t)i * nseg + s], b = h2[(int64_t)i * nseg + s];
    col[i] = make_double2(a.x + b.x, a.y + b.y);
  }
  const double hn = sqrt(fmax(hn2[s].x, 0.0));
  col[j + 1] = make_double2(hn, 0.0);
  double* cs = G.cs + (int64_t)s * m;
  double2* sn = G.sn + (int64_t)s * m;
  double2* g = G.g + (int64_t)s * (m + 1);
  for (int i = 0; i < j; ++i) {
    const double2 a = col[i], b = col[i + 1];
    const double2 sb = cmul_k(sn[i], b);
    const double2 t = make_double2(cs[i] * a.x + sb.x, cs[i] * a.y + sb.y);
    const double2 na = cmul_k(conj_k(sn[i]), a);
    col[i + 1] = make_double2(cs[i] * b.x - na.x, cs[i] * b.y - na.y);
    col[i] = t;
  }
  const double2 a = col[j], b = col[j + 1];
  const double aa = hypot(a.x, a.y), bb = hypot(b.x, b.y);
  const double den = hypot(aa, bb);
  double c;
  double2 sv;
  if (den == 0.0) {
    c = 1.0;
    sv = make_double2(0.0, 0.0);
  } else if (aa == 0.0) {
    c = 0.0;
    sv = make_double2(1.0, 0.0);
  } else {
    c = aa / den;
    const double2 u = make_double2(a.x / aa, a.y / aa);
    const double2 q = cmul_k(u, conj_k(b));
    sv = make_double2(q.x / den, q.y / den);
  }
  cs[j] = c;
  sn[j] = sv;
  const double2 sb = cmul_k(sv, b);
  col[j] = make_double2(c * a.x + sb.x, c * a.y + sb.y);
  col[j + 1] = make_double2(0.0, 0.0);
  const double2 gj = g[j];
  const double2 ng = cmul_k(conj_k(sv), gj);
  g[j + 1] = make_double2(-ng.x, -ng.y);
  g[j] = make_double2(c * gj.x, c * gj.y);
  const double beta = G.beta[s];
  const bool tiny = !(hn > 1e-14 * beta);
  const double est = beta > 0.0 ? hypot(g[j + 1].x, g[j + 1].y) / beta : 0.0;
  if (est > G.tin[s] && !tiny) {
    G.scl[s] = make_double2(1.0 / hn, 0.0);
    atomicAdd(G.notdone + j, 1);
  } else {
    G.scl[s] = make_double2(0.0, 0.0);
    G.kconv[s] = j + 1;
    G.active[s] = 0;
  }
}

// One thread per segment: back substitution R y = g over the first k columns.
__global__ void back_solve_kernel(int nseg, int k, int m, GivensState G, double2* __restrict__ y) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nseg) return;
  const double2* H = G.H + (int64_t)s * m * (m + 1);
  const double2* g = G.g + (int64_t)s * (m + 1);
  const bool frozen = G.frozen[s] != 0;
  const int ks = G.kconv[s] > 0 ? min(G.kconv[s], k) : k;
  for (int i = k - 1; i >= ks; --i) y[(int64_t)i * nseg + s] = make_double2(0.0, 0.0);
  for (int i = ks - 1; i >= 0; --i) {
    double2 acc = g[i];
    for (int l = i + 1; l < ks; ++l) {
      const double2 t = cmul_k(H[(int64_t)l * (m + 1) + i], y[(int64_t)l * nseg + s]);
      acc.x -= t.x;
      acc.y -= t.y;
    }
    const double2 d = H[(int64_t)i * (m + 1) + i];
    const double dd = d.x * d.x + d.y * d.y;
    double2 v = make_double2(0.0, 0.0);
    if (!frozen && dd > 0.0) v = make_double2((acc.x * d.x + acc.y * d.y) / dd, (acc.y * d.x - acc.x * d.y) / dd);
    y[(int64_t)i * nseg + s] = v;
  }
}

static inline unsigned blocks_for(int64_t n) { return (unsigned)((n + 255) / 256); }

// vstride: distance between consecutive vectors of V in doubles (the kernels
// index complex elements, hence vstride / 2).
void Krylov::dots(const double* V, int64_t vstride, int m, const double* w, double* h) {
  const int nthr = (256 / nrhs) * nrhs;
  hipLaunchKernelGGL(mdot_kernel, dim3(nchunks, m), dim3(nthr), 0, stream, (const double2*)V,
                     vstride / 2, (const double2*)w, nrhs, d_chunks, (double2*)d_partial, nchunks);
  hipLaunchKernelGGL(mdot_reduce_kernel, dim3(blocks_for((int64_t)nprob * nrhs), m), dim3(256), 0,
                     stream, (const double2*)d_partial, nchunks, nrhs, d_prob_chunk0, nprob,
                     (double2*)h);
}

void Krylov::orth(const double* V, int64_t vstride, int m, const double* h, double* w) {
  hipLaunchKernelGGL(orth_update_kernel, dim3(blocks_for(N * nrhs)), dim3(256), 0, stream,
                     (const double2*)V, vstride / 2, m, (const double2*)h, d_node_prob, nprob, N, nrhs,
                     (double2*)w);
}

void Krylov::combine(const double* V, int64_t vstride, int m, const double* y, double* out,
                     bool accumulate) {
  hipLaunchKernelGGL(combine_kernel, dim3(blocks_for(N * nrhs)), dim3(256), 0, stream,
                     (const double2*)V, vstride / 2, m, (const double2*)y, d_node_prob, nprob, N, nrhs,
                     (double2*)out, accumulate ? 1 : 0);
}

void Krylov::scale(const double* a, const double* s, double* out) {
  hipLaunchKernelGGL(seg_scale_kernel, dim3(blocks_for(N * nrhs)), dim3(256), 0, stream,
                     (const double2*)a, (const double2*)s, d_node_prob, N, nrhs, (double2*)out);
}

void Krylov::givens(int nseg, int j, int m, const double* h1, const double* h2, const double* hn2,
                    const GivensState& G) {
  hipLaunchKernelGGL(givens_kernel, dim3(blocks_for(nseg)), dim3(256), 0, stream, nseg, j, m,
                     (const double2*)h1, (const double2*)h2, (const double2*)hn2, G);
}

void Krylov::back_solve(int nseg, int k, int m, const GivensState& G, double* y) {
  hipLaunchKernelGGL(back_solve_kernel, dim3(blocks_for(nseg)), dim3(256), 0, stream, nseg, k, m, G,
                     (double2*)y);
}

void Krylov::axpby(double alpha, const double* a, double beta, const double* b, double* out) {
  hipLaunchKernelGGL(axpby_kernel, dim3(blocks_for(N * nrhs)), dim3(256), 0, stream, alpha,
                     (const double2*)a, beta, (const double2*)b, N * nrhs, (double2*)out);
}

// ---------------------------------------------------------------- block Krylov products
// Blocks of the block GMRES basis: N x p complex matrices stored node-major
// with the p columns (right-hand sides) fastest, p <= 64.
//
// partial[chunk][i][b][a] = sum_{n in chunk} conj(V_i[n][b]) W[n][a] for the
// nb blocks V_i = V + i vstride.  A workgroup takes one block i and one chunk
// of rows; each thread owns a 4 x 4 tile of (b, a); rows pass through LDS 16
// at a time.
constexpr int BK_P = 64;
constexpr int BK_KT = 16;

__global__ __launch_bounds__(256) void block_dots_kernel(const double2* __restrict__ V, int64_t vstride,
                                                         const double2* __restrict__ W, int64_t N, int p,
                                                         int64_t rows_per_chunk, double2* __restrict__ partial) {
  const int tid = threadIdx.x, tb = tid >> 4, ta = tid & 15;
  const int i = blockIdx.y, chunk = blockIdx.x, nb = gridDim.y;
  const double2* Vi = V + (int64_t)i * vstride / 2;
  const int64_t k0 = (int64_t)chunk * rows_per_chunk, k1 = min(N, k0 + rows_per_chunk);
  __shared__ double2 sV[BK_KT][BK_P];
  __shared__ double2 sW[BK_KT][BK_P];
  double ar[4][4], ai[4][4];
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int y = 0; y < 4; ++y) ar[x][y] = ai[x][y] = 0.0;
  for (int64_t base = k0; base < k1; base += BK_KT) {
    __syncthreads();
    for (int e = tid; e < BK_KT * BK_P; e += 256) {
      const int kk = e / BK_P, c = e % BK_P;
      const int64_t n = base + kk;
      const bool ok = n < k1 && c < p;
      sV[kk][c] = ok ? Vi[n * p + c] : make_double2(0.0, 0.0);
      sW[kk][c] = ok ? W[n * p + c] : make_double2(0.0, 0.0);
    }
    __syncthreads();
#pragma unroll 4
    for (int kk = 0; kk < BK_KT; ++kk) {
      double2 v[4], w[4];
#pragma unroll
      for (int x = 0; x < 4; ++x) v[x] = sV[kk][tb * 4 + x];
#pragma unroll
      for (int y = 0; y < 4; ++y) w[y] = sW[kk][ta * 4 + y];
#pragma unroll
      for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y) {
          // conj(v) w
          ar[x][y] = fma(v[x].x, w[y].x, fma(v[x].y, w[y].y, ar[x][y]));
          ai[x][y] = fma(v[x].x, w[y].y, fma(-v[x].y, w[y].x, ai[x][y]));
        }
    }
  }
  double2* out = partial + ((int64_t)chunk * nb + i) * BK_P * BK_P;
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int y = 0; y < 4; ++y) out[(tb * 4 + x) * BK_P + ta * 4 + y] = make_double2(ar[x][y], ai[x][y]);
}

// out[i][b][a] = sum over chunks of partial (a fixed order), b, a < p.
__global__ void block_dots_reduce_kernel(const double2* __restrict__ partial, int nchunks, int nb, int p,
                                         double2* __restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t total = (int64_t)nb * p * p;
  if (e >= total) return;
  const int i = (int)(e / (p * p)), b = (int)(e / p % p), a = (int)(e % p);
  double2 acc = make_double2(0.0, 0.0);
  for (int c = 0; c < nchunks; ++c) {
    const double2 v = partial[((int64_t)c * nb + i) * BK_P * BK_P + b * BK_P + a];
    acc.x += v.x;
    acc.y += v.y;
  }
  out[e] = acc;
}

// out[n][a] = beta base[n][a] + alpha sum_{i < nb} sum_b V_i[n][b] C[i][b][a]
// (C: nb x p x p, row b, column a; base may be out or null when beta = 0).
// A workgroup takes 64 rows and all p columns; each thread a 4 x 4 tile of
// (row, column); the products' inner index passes through LDS 16 at a time.
__global__ __launch_bounds__(256) void block_update_kernel(const double2* __restrict__ V, int64_t vstride,
                                                           int nb, const double2* __restrict__ C, int p,
                                                           int64_t N, double alpha, double beta,
                                                           const double2* base, double2* out) {
  const int tid = threadIdx.x, tr = tid >> 4, tc = tid & 15;
  const int64_t r0 = (int64_t)blockIdx.x * 64;
  __shared__ double2 sV[64][BK_KT + 1];
  __shared__ double2 sC[BK_KT][BK_P];
  double sr[4][4], si[4][4];
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int y = 0; y < 4; ++y) sr[x][y] = si[x][y] = 0.0;
  const int K = nb * p;
  for (int k0 = 0; k0 < K; k0 += BK_KT) {
    __syncthreads();
    for (int e = tid; e < 64 * BK_KT; e += 256) {
      const int r = e / BK_KT, kk = e % BK_KT;
      const int k = k0 + kk;
      const int64_t n = r0 + r;
      double2 v = make_double2(0.0, 0.0);
      if (k < K && n < N) {
        const int i = k / p, b = k % p;
        v = V[(int64_t)i * vstride / 2 + n * p + b];
      }
      sV[r][kk] = v;
    }
    for (int e = tid; e < BK_KT * BK_P; e += 256) {
      const int kk = e / BK_P, a = e % BK_P;
      const int k = k0 + kk;
      sC[kk][a] = (k < K && a < p) ? C[(int64_t)k * p + a] : make_double2(0.0, 0.0);
    }
    __syncthreads();
#pragma unroll 4
    for (int kk = 0; kk < BK_KT; ++kk) {
      double2 v[4], c[4];
#pragma unroll
      for (int x = 0; x < 4; ++x) v[x] = sV[tr * 4 + x][kk];
#pragma unroll
      for (int y = 0; y < 4; ++y) c[y] = sC[kk][tc * 4 + y];
#pragma unroll
      for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y) {
          sr[x][y] = fma(v[x].x, c[y].x, fma(-v[x].y, c[y].y, sr[x][y]));
          si[x][y] = fma(v[x].x, c[y].y, fma(v[x].y, c[y].x, si[x][y]));
        }
    }
  }
#pragma unroll
  for (int x = 0; x < 4; ++x) {
    const int64_t n = r0 + tr * 4 + x;
    if (n >= N) continue;
#pragma unroll
    for (int y = 0; y < 4; ++y) {
      const int a = tc * 4 + y;
      if (a >= p) continue;
      double2 o = make_double2(alpha * sr[x][y], alpha * si[x][y]);
      if (beta != 0.0) {
        const double2 b0 = base[n * p + a];
        o.x = fma(beta, b0.x, o.x);
        o.y = fma(beta, b0.y, o.y);
      }
      out[n * p + a] = o;
    }
  }
}

// chunks x blocks <= ceil(1024 / nb) nb <= 1024 + nb_max for every nb <= nb_max
size_t block_dots_work_bytes(int64_t N, int nb_max) {
  const int64_t cells = std::min<int64_t>((N + 1023) / 1024 * nb_max, 1024 + (int64_t)nb_max);
  return (size_t)std::max<int64_t>(cells, nb_max) * BK_P * BK_P * 16;
}

hipError_t launch_block_dots(hipStream_t s, const double* V, int64_t vstride, int nb, const double* W,
                             int64_t N, int p, double* partial, double* out) {
  // enough chunks for about 1024 workgroups, at least 1024 rows each
  const int64_t nch = std::max<int64_t>(1, std::min<int64_t>((N + 1023) / 1024, (1024 + nb - 1) / nb));
  const int64_t rows = (N + nch - 1) / nch;
  hipLaunchKernelGGL(block_dots_kernel, dim3((unsigned)nch, (unsigned)nb), dim3(256), 0, s,
                     (const double2*)V, vstride, (const double2*)W, N, p, rows, (double2*)partial);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t total = (int64_t)nb * p * p;
  hipLaunchKernelGGL(block_dots_reduce_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s,
                     (const double2*)partial, (int)nch, nb, p, (double2*)out);
  return hipGetLastError();
}

hipError_t launch_block_update(hipStream_t s, const double* V, int64_t vstride, int nb, const double* C,
                               int p, int64_t N, double alpha, double beta, const double* base,
                               double* out) {
  hipLaunchKernelGGL(block_update_kernel, dim3((unsigned)((N + 63) / 64)), dim3(256), 0, s,
                     (const double2*)V, vstride, nb, (const double2*)C, p, N, alpha, beta,
                     (const double2*)base, (double2*)out);
  return hipGetLastError();
}

// ---------------------------------------------------------------- far field without allocation
// Workspace of qax_farfield_noalloc: the far field's partial sums, one array
// per GPU that holds it until the process ends, shared by every call on that
// GPU (calls that overlap on one GPU race on it).  Its device address on each
// GPU is taken once, by qax_create, with that GPU current; host code uses
// that address, never the array's name.
constexpr size_t FF_NOALLOC_BYTES = (size_t)64 << 20;
constexpr int NOALLOC_MAX_DEVICES = 64;
static __device__ __align__(256) char noalloc_scratch[FF_NOALLOC_BYTES];
static void* g_noalloc_ptr[NOALLOC_MAX_DEVICES] = {};
static int g_noalloc_cus[NOALLOC_MAX_DEVICES] = {};
static std::mutex g_noalloc_mu;

hipError_t noalloc_init(int device) {
  std::lock_guard<std::mutex> lock(g_noalloc_mu);
  if (device < 0 || device >= NOALLOC_MAX_DEVICES) return hipErrorInvalidDevice;
  if (g_noalloc_ptr[device]) return hipSuccess;
  void* ptr = nullptr;
  hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(noalloc_scratch));
  if (e != hipSuccess) return e;
  int cus = 0;
  e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device);
  if (e != hipSuccess) return e;
  g_noalloc_cus[device] = cus;
  g_noalloc_ptr[device] = ptr;
  return hipSuccess;
}

}  // namespace qax

extern "C" qax_status qax_farfield_noalloc(qax_problem* p, const void* d_mu, int32_t nrhs,
                                           const double* d_xhat, int32_t n_dirs, void* d_u_inf) {
  using namespace qax;
  if (!p) return QAX_ERR_ARG;
  if (!d_mu || !d_xhat || !d_u_inf || nrhs < 1 || nrhs > 256 || n_dirs < 1)
    return fail(p, QAX_ERR_ARG, "qax_farfield_noalloc: null pointer, nrhs out of [1, 256] or no directions");
  if (p->state < 1) return fail(p, QAX_ERR_STATE, "qax_farfield_noalloc: call qax_build first");
  if (p->device < 0 || p->device >= NOALLOC_MAX_DEVICES || !g_noalloc_ptr[p->device])
    return fail(p, QAX_ERR_DEVICE, "qax_farfield_noalloc: workspace address not set for this device");
  const size_t per_slot = (size_t)p->n_problems * n_dirs * nrhs * 16;
  if (per_slot > FF_NOALLOC_BYTES)
    return fail(p, QAX_ERR_ARG,
                "qax_farfield_noalloc: n_problems x n_dirs x nrhs exceeds the 64 MiB workspace "
                "(at most 4194304 complex values)");
  hipError_t e = hipSetDevice(p->device);
  if (e != hipSuccess) return hip_check(p, e, "hipSetDevice");
  int slots = farfield_slots((int64_t)n_dirs * p->n_problems, g_noalloc_cus[p->device]);
  slots = (int)std::min<size_t>((size_t)slots, FF_NOALLOC_BYTES / per_slot);
  e = launch_farfield(p, (const double*)d_mu, nrhs, d_xhat, n_dirs, nullptr, n_dirs, p->d_pinfo, slots,
                      (double*)g_noalloc_ptr[p->device], (double*)d_u_inf);
  return e == hipSuccess ? QAX_OK : hip_check(p, e, "qax_farfield_noalloc");
}
