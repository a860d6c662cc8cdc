// Block-Toeplitz inter-body apply on a regular array of identical bodies.
//
// Section 4 (the paragraph on identical scatterers on a P x Q x R array with
// uniform spacing): the interaction block between bodies t' and t depends
// only on the displacement d = c_t' - c_t, so the inter-body sum
//   w_t' = sum_{t != t'} D_{t' - t} mu_t
// is a three-level block-Toeplitz product with (2P-1)(2Q-1)(2R-1) - 1
// distinct blocks (Table 7 counts them).  The paper computes each distinct
// block once and copies it into a dense matrix.  Here the blocks are not
// copied at all: the Toeplitz product is embedded in a circulant one of
// period L = (2P-1, 2Q-1, 2R-1) (exactly large enough: every displacement
// has its own residue), transformed over the array indices, and the apply
// becomes one n_b x n_b product per frequency:
//   T_xi = sum_a D_a e^{-2 pi i xi.a / L}            (once, on the device)
//   mu^_xi = sum_t mu_t e^{-2 pi i xi.t / L}          (per apply)
//   w_t' = (1/F) sum_xi e^{+2 pi i xi.t' / L} T_xi mu^_xi,  F = L0 L1 L2.
// The transforms are direct DFTs along one axis at a time (the periods are
// small); the products reuse the block-diagonal GEMV / MFMA GEMM kernels
// with one "block" per frequency.  Memory per apply: F n_b^2 table entries
// read once (16 B FP64, 8 B FP32) against N^2 kernel evaluations for the
// direct pair sum.
#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "fastmath.h"
#include "internal.h"

namespace qax {

constexpr double INV_FOUR_PI_LAT = 0.0795774715459476678844;

#define LCHECK(expr, what)                                   \
  do {                                                       \
    qax_status _s = hip_check(p, (expr), what);              \
    if (_s != QAX_OK) return _s;                             \
  } while (0)
constexpr int LAT_LMAX = 127;         // longest period (P <= 64)
constexpr int64_t LAT_FMAX = 65535;   // frequencies (one grid dimension)

// D[a][i][j] = kernel from source node j of the reference body to target
// node i of the body displaced by d(a) (the pair-sum kernel of Section 4 with
// the smooth-rule weights in aw; minus i eta G |aw| for the combined field;
// G |aw| alone for the single layer),
// a = (a0, a1, a2) in the L0 x L1 x L2 grid, d = a or a - L per axis; zero
// block for d = 0 (the self block is applied separately).
__global__ __launch_bounds__(256) void lattice_blocks_kernel(
    const double* __restrict__ pos, const double* __restrict__ aw, const double* __restrict__ ew,
    int form, int64_t N, int64_t off, int nb, int L0, int L1, int L2, int P0, int P1, int P2,
    double h0, double h1, double h2, double k, double2* __restrict__ D) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t nn = (int64_t)nb * nb;
  if (e >= nn) return;
  const int a = blockIdx.y;
  const int a0 = a / (L1 * L2), a1 = (a / L2) % L1, a2 = a % L2;
  const int d0 = a0 < P0 ? a0 : a0 - L0;
  const int d1 = a1 < P1 ? a1 : a1 - L1;
  const int d2 = a2 < P2 ? a2 : a2 - L2;
  double2 v = make_double2(0.0, 0.0);
  if (d0 != 0 || d1 != 0 || d2 != 0) {
    const int i = (int)(e / nb), j = (int)(e % nb);
    const int64_t ti = off + i, sj = off + j;
    // y - x with x = pos_i + d h (target in the displaced body)
    const double dx = pos[sj] - pos[ti] - d0 * h0;
    const double dy = pos[N + sj] - pos[N + ti] - d1 * h1;
    const double dz = pos[2 * N + sj] - pos[2 * N + ti] - d2 * h2;
    const double r2 = dx * dx + dy * dy + dz * dz;
    const double ir = rsqrt(r2);
    const double r = r2 * ir;
    const double kr = k * r;
    double s, c;
    sincos_cw(kr, &s, &c);
    double re, im;
    if (form == 2) {   // single layer: (|aw| / r) e^{ikr}
      const double t = ew[sj] * ir;
      re = c * t;
      im = s * t;
    } else {
      const double dot = aw[sj] * dx + aw[N + sj] * dy + aw[2 * N + sj] * dz;
      const double sc = dot * ir * ir * ir;
      re = -(c + kr * s) * sc;
      im = (kr * c - s) * sc;
      if (form == 1) {
        const double t = ew[sj] * ir;
        re = fma(t, s, re);
        im = fma(-t, c, im);
      }
    }
    v = make_double2(re * INV_FOUR_PI_LAT, im * INV_FOUR_PI_LAT);
  }
  D[(int64_t)a * nn + e] = v;
}

// One axis of a DFT over the array indices:
//   out[o][e] = scale sum_{t < nin} in[o with o_ax -> t][e] e^{sign 2 pi i o_ax t / L}
// for every output site o of the n0 x n1 x n2 grid (the input has nin sites
// along axis `ax`, the output's extents elsewhere) and every element e < E of
// a site's contiguous run.  in_node / out_node: first node of each site's
// body (a run starts at node * mult), for the density and the result in the
// handle's node order; null for dense site-major arrays.  One thread per
// output element; loads and stores coalesced along e.
__global__ __launch_bounds__(256) void lattice_dft_kernel(
    const double2* __restrict__ in, const int64_t* __restrict__ in_node, double2* __restrict__ out,
    const int64_t* __restrict__ out_node, int64_t mult, int accumulate, int n0, int n1, int n2,
    int ax, int nin, int L, int sign, double scale, int64_t E) {
  __shared__ double2 tw[LAT_LMAX];
  for (int q = threadIdx.x; q < L; q += 256) {
    double s, c;
    sincospi(2.0 * q / L, &s, &c);
    tw[q] = make_double2(c, sign * s);
  }
  __syncthreads();
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t total = (int64_t)n0 * n1 * n2 * E;
  if (idx >= total) return;
  const int64_t e = idx % E;
  const int64_t so = idx / E;
  int o[3];
  o[2] = (int)(so % n2);
  o[1] = (int)((so / n2) % n1);
  o[0] = (int)(so / ((int64_t)n1 * n2));
  int din[3] = {n0, n1, n2};
  din[ax] = nin;
  const int oa = o[ax];
  double ar = 0.0, ai = 0.0;
  int q = 0;
  for (int t = 0; t < nin; ++t) {
    int c[3] = {o[0], o[1], o[2]};
    c[ax] = t;
    const int64_t si = ((int64_t)c[0] * din[1] + c[1]) * din[2] + c[2];
    const int64_t base = in_node ? in_node[si] * mult : si * E;
    const double2 v = in[base + e];
    const double2 w = tw[q];
    ar = fma(v.x, w.x, fma(-v.y, w.y, ar));
    ai = fma(v.x, w.y, fma(v.y, w.x, ai));
    q += oa;
    if (q >= L) q -= L;
  }
  const int64_t ob = (out_node ? out_node[so] * mult : so * E) + e;
  double2 r = make_double2(ar * scale, ai * scale);
  if (accumulate) {
    const double2 prev = out[ob];
    r.x += prev.x;
    r.y += prev.y;
  }
  out[ob] = r;
}

static hipError_t dft_axis(hipStream_t s, const double2* in, const int64_t* in_node, double2* out,
                           const int64_t* out_node, int64_t mult, bool accumulate, const int n[3],
                           int ax, int nin, int L, int sign, double scale, int64_t E) {
  const int64_t total = (int64_t)n[0] * n[1] * n[2] * E;
  hipLaunchKernelGGL(lattice_dft_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, in,
                     in_node, out, out_node, mult, accumulate ? 1 : 0, n[0], n[1], n[2], ax, nin, L,
                     sign, scale, E);
  return hipGetLastError();
}

void lattice_free(qax_problem* p) {
  auto& t = p->lat;
  void* ptrs[] = {t.T64, t.T32, t.d_fbodies, t.d_fblocks, t.d_frow, t.d_ftasks, t.d_site_node};
  for (void* q : ptrs)
    if (q) (void)hipFree(q);
  t = qax_problem::Lattice();
}

size_t lattice_work_bytes(const qax_problem* p, int nrhs) {
  if (!p->lat.active) return 0;
  return (size_t)2 * p->lat.F * p->lat.nb * nrhs * 16;
}

// Sites of a full regular array aligned with the axes, from the centres:
// per axis the distinct coordinates (merged within tol), uniform spacing.
static bool array_axis(const std::vector<double>& x, double tol, int& n, double& h,
                       std::vector<int>& idx) {
  std::vector<double> u(x);
  std::sort(u.begin(), u.end());
  std::vector<double> m{u[0]};
  for (double v : u)
    if (v - m.back() > tol) m.push_back(v);
  n = (int)m.size();
  h = n > 1 ? (m.back() - m.front()) / (n - 1) : 0.0;
  for (int i = 0; i < n; ++i)
    if (std::fabs(m[i] - (m[0] + h * i)) > tol) return false;
  idx.resize(x.size());
  for (size_t b = 0; b < x.size(); ++b) {
    const double f = n > 1 ? (x[b] - m[0]) / h : 0.0;
    const long r = std::lround(f);
    if (std::fabs(f - r) * (n > 1 ? h : 1.0) > tol || r < 0 || r >= n) return false;
    idx[b] = (int)r;
  }
  return true;
}

qax_status lattice_enable(qax_problem* p, int32_t* dims_out) {
  lattice_free(p);
  if (p->n_problems != 1) return fail(p, QAX_ERR_ARG, "qax_lattice: needs a single problem");
  const qax_body& b0 = p->bodies[0];
  double scale = 1.0;
  for (const auto& b : p->bodies) {
    if (b.shape != b0.shape || b.n_panels != b0.n_panels || b.n_ref != b0.n_ref ||
        b.n_theta != b0.n_theta ||
        b.a != b0.a || b.c != b0.c || b.kappa != b0.kappa || b.theta1 != b0.theta1 ||
        b.theta2 != b0.theta2)
      return fail(p, QAX_ERR_ARG, "qax_lattice: bodies differ in shape, discretisation or orientation");
    scale = std::max({scale, std::fabs(b.centre[0]), std::fabs(b.centre[1]), std::fabs(b.centre[2])});
  }
  const double tol = 1e-9 * scale;
  std::vector<double> cx, cy, cz;
  for (const auto& b : p->bodies) {
    cx.push_back(b.centre[0]);
    cy.push_back(b.centre[1]);
    cz.push_back(b.centre[2]);
  }
  int n[3];
  double h[3];
  std::vector<int> ix, iy, iz;
  if (!array_axis(cx, tol, n[0], h[0], ix) || !array_axis(cy, tol, n[1], h[1], iy) ||
      !array_axis(cz, tol, n[2], h[2], iz))
    return fail(p, QAX_ERR_ARG, "qax_lattice: centres are not uniformly spaced along the axes");
  const int64_t nsite = (int64_t)n[0] * n[1] * n[2];
  if (nsite != p->n_bodies) return fail(p, QAX_ERR_ARG, "qax_lattice: centres do not fill a regular array");
  std::vector<int64_t> site_node(nsite, -1);
  for (int b = 0; b < p->n_bodies; ++b) {
    const int64_t s = ((int64_t)ix[b] * n[1] + iy[b]) * n[2] + iz[b];
    if (site_node[s] >= 0) return fail(p, QAX_ERR_ARG, "qax_lattice: two bodies on one site");
    site_node[s] = p->off[b];
  }
  int L[3];
  int64_t F = 1;
  for (int a = 0; a < 3; ++a) {
    L[a] = 2 * n[a] - 1;
    if (L[a] > LAT_LMAX) return fail(p, QAX_ERR_ARG, "qax_lattice: array longer than 64 along an axis");
    F *= L[a];
  }
  if (F > LAT_FMAX) return fail(p, QAX_ERR_ARG, "qax_lattice: (2P-1)(2Q-1)(2R-1) exceeds 65535");
  const int nb = p->hbodies[0].n;
  const int64_t nn = (int64_t)nb * nb;
  size_t free_b = 0, total_b = 0;
  LCHECK(hipMemGetInfo(&free_b, &total_b), "memory info");
  const size_t need = (size_t)F * nn * (16 + 16 + 8);
  if (need > free_b) return fail(p, QAX_ERR_NOMEM, "qax_lattice: frequency tables do not fit in device memory");

  auto& t = p->lat;
  hipStream_t s = p->stream;
  double2* tmp = nullptr;
  LCHECK(hipMalloc(&t.T64, (size_t)F * nn * 16), "lattice tables");
  LCHECK(hipMalloc(&t.T32, (size_t)F * nn * 8), "lattice tables");
  LCHECK(hipMalloc(&tmp, (size_t)F * nn * 16), "lattice scratch");
  // representative: the body at site 0
  const int64_t off0 = site_node[0];
  const BodyDev& B0 = p->hbodies[0];
  hipLaunchKernelGGL(lattice_blocks_kernel, dim3((unsigned)((nn + 255) / 256), (unsigned)F), dim3(256),
                     0, s, p->d_pos, p->d_aw, p->d_ew, p->form(),
                     p->N, off0, nb, L[0], L[1], L[2], n[0], n[1], n[2], h[0], h[1], h[2], B0.k, tmp);
  hipError_t e = hipGetLastError();
  // T = DFT over the three displacement axes (tmp -> T64 -> tmp -> T64)
  const int full[3] = {L[0], L[1], L[2]};
  double2* T = (double2*)t.T64;
  if (e == hipSuccess) e = dft_axis(s, tmp, nullptr, T, nullptr, 0, false, full, 2, L[2], L[2], -1, 1.0, nn);
  if (e == hipSuccess) e = dft_axis(s, T, nullptr, tmp, nullptr, 0, false, full, 1, L[1], L[1], -1, 1.0, nn);
  if (e == hipSuccess) e = dft_axis(s, tmp, nullptr, T, nullptr, 0, false, full, 0, L[0], L[0], -1, 1.0, nn);
  if (e == hipSuccess) e = launch_convert_f32(s, t.T64, t.T32, F * nn * 2);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  (void)hipFree(tmp);
  LCHECK(e, "lattice tables");
  // per-frequency "bodies" and blocks for the batched products
  std::vector<BodyDev> fb(F);
  std::vector<BlockDev> fk(F);
  std::vector<GemmTask> ft;
  for (int64_t x = 0; x < F; ++x) {
    fb[x] = BodyDev{};
    fb[x].off = x * nb;
    fb[x].n = nb;
    fb[x].block = (int32_t)x;
    fk[x] = BlockDev{0, nb, x * nn};
    for (int r0 = 0; r0 < nb; r0 += 64) ft.push_back(GemmTask{(int32_t)x, r0});
  }
  std::vector<int32_t> frow((size_t)F * nb);
  for (int64_t r = 0; r < F * nb; ++r) frow[r] = (int32_t)(r / nb);
  LCHECK(hipMalloc(&t.d_fbodies, F * sizeof(BodyDev)), "lattice tables");
  LCHECK(hipMalloc(&t.d_fblocks, F * sizeof(BlockDev)), "lattice tables");
  LCHECK(hipMalloc(&t.d_frow, frow.size() * 4), "lattice tables");
  LCHECK(hipMalloc(&t.d_ftasks, ft.size() * sizeof(GemmTask)), "lattice tables");
  LCHECK(hipMalloc(&t.d_site_node, nsite * 8), "lattice tables");
  LCHECK(hipMemcpy(t.d_fbodies, fb.data(), F * sizeof(BodyDev), hipMemcpyHostToDevice), "copy");
  LCHECK(hipMemcpy(t.d_fblocks, fk.data(), F * sizeof(BlockDev), hipMemcpyHostToDevice), "copy");
  LCHECK(hipMemcpy(t.d_frow, frow.data(), frow.size() * 4, hipMemcpyHostToDevice), "copy");
  LCHECK(hipMemcpy(t.d_ftasks, ft.data(), ft.size() * sizeof(GemmTask), hipMemcpyHostToDevice), "copy");
  LCHECK(hipMemcpy(t.d_site_node, site_node.data(), nsite * 8, hipMemcpyHostToDevice), "copy");
  t.nftasks = (int)ft.size();
  for (int a = 0; a < 3; ++a) {
    t.dims[a] = n[a];
    t.L[a] = L[a];
  }
  t.F = F;
  t.nb = nb;
  t.active = true;
  if (dims_out)
    for (int a = 0; a < 3; ++a) dims_out[a] = n[a];
  return QAX_OK;
}

// out (+)= inter-body sum of mu by the frequency tables; work holds
// 2 F n_b nrhs complex128.
hipError_t launch_lattice_apply(qax_problem* p, int prec, const double* mu, double* out, int nrhs,
                                double* work, bool accumulate) {
  const auto& t = p->lat;
  hipStream_t s = p->stream;
  const int64_t E = (int64_t)t.nb * nrhs;
  double2* W1 = (double2*)work;
  double2* W2 = W1 + t.F * E;
  const int P = t.dims[0], Q = t.dims[1], R = t.dims[2];
  const int L0 = t.L[0], L1 = t.L[1], L2 = t.L[2];
  const bool f32 = prec != QAX_FP64;
  // forward transform of the density, zero-padded to the period
  const int s1[3] = {P, Q, L2}, s2[3] = {P, L1, L2}, s3[3] = {L0, L1, L2};
  hipError_t e = dft_axis(s, (const double2*)mu, t.d_site_node, W1, nullptr, nrhs, false, s1, 2, R,
                          L2, -1, 1.0, E);
  if (e == hipSuccess) e = dft_axis(s, W1, nullptr, W2, nullptr, 0, false, s2, 1, Q, L1, -1, 1.0, E);
  if (e == hipSuccess) e = dft_axis(s, W2, nullptr, W1, nullptr, 0, false, s3, 0, P, L0, -1, 1.0, E);
  if (e != hipSuccess) return e;
  // one product per frequency
  const int kind = f32 ? QAX_K_LATTICE_F32 : QAX_K_LATTICE_F64;
  const void* pool = f32 ? (const void*)t.T32 : (const void*)t.T64;
  timing_begin(p, kind);
  if (nrhs >= 4)
    e = launch_gemm_tables(s, t.d_ftasks, t.nftasks, t.d_fbodies, t.d_fblocks, pool, f32,
                           (const double*)W1, nrhs, (double*)W2, false);
  else
    e = launch_gemv_tables(s, t.d_fbodies, t.d_fblocks, t.d_frow, pool, f32, t.F * t.nb, t.nb,
                           (const double*)W1, nrhs, (double*)W2, false);
  timing_end(p, kind);
  if (e != hipSuccess) return e;
  // inverse transform, kept only on the array's own sites
  const int u1[3] = {P, L1, L2}, u2[3] = {P, Q, L2}, u3[3] = {P, Q, R};
  e = dft_axis(s, W2, nullptr, W1, nullptr, 0, false, u1, 0, L0, L0, 1, 1.0, E);
  if (e == hipSuccess) e = dft_axis(s, W1, nullptr, W2, nullptr, 0, false, u2, 1, L1, L1, 1, 1.0, E);
  if (e == hipSuccess)
    e = dft_axis(s, W2, nullptr, (double2*)out, t.d_site_node, nrhs, accumulate, u3, 2, L2, L2, 1,
                 1.0 / (double)t.F, E);
  return e;
}

}  // namespace qax
