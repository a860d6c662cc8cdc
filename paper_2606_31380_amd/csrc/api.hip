// Host runtime and C interface of libqax (see include/qax.h).
//
// The solver of Section 6 (GMRES with the block-diagonal preconditioner built
// from the self blocks) is written right-preconditioned: with M = blockdiag(B_b),
// A M^-1 v = v + D_off (M^-1 v), so one Krylov step costs one block-inverse
// apply and one inter-body pair sum.  Every (problem, right-hand side) pair is
// an independent GMRES run; all runs advance in lockstep so that their applies
// share one pair-sum launch.  Restarts recompute the true residual b - A x in
// FP64 (self blocks + FP64 pair sum); with QAX_MIXED the Krylov steps use the
// FP32 pair sum and the FP32 inverse blocks, so each restart is one step of
// FP64 iterative refinement.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "internal.h"
#include "krylov.h"

namespace qax {
hipError_t launch_dense_system(qax_problem* p, double* A);
hipError_t launch_dense_solve(qax_problem* p, double* A, const double* b, int nrhs, double* x,
                              double* work);
size_t dense_solve_work_bytes(int64_t N);
size_t invert_matrices_work_bytes(int count, int nmax, int64_t total_elems, bool f32);
hipError_t launch_invert_matrices(qax_problem* p, bool f32, int count, const int32_t* orders,
                                  double* mats, double* work);
size_t invert_blocks_work_bytes(qax_problem* p);
}  // namespace qax

using namespace qax;
using cplx = std::complex<double>;

namespace {

struct Buffers {
  std::map<std::string, std::pair<void*, size_t>> m;
};
std::map<const qax_problem*, Buffers>& registry() {
  static std::map<const qax_problem*, Buffers> r;
  return r;
}

}  // namespace

namespace qax {

qax_status fail(qax_problem* p, qax_status s, const std::string& msg) {
  if (p) p->err = msg;
  return s;
}

qax_status hip_check(qax_problem* p, hipError_t e, const char* what) {
  if (e == hipSuccess) return QAX_OK;
  std::string m = std::string(what) + ": " + hipGetErrorString(e);
  return fail(p, e == hipErrorOutOfMemory ? QAX_ERR_NOMEM : QAX_ERR_DEVICE, m);
}

// Grow-only named device buffer owned by the handle.
static void* dbuf(qax_problem* p, const char* name, size_t bytes, qax_status* st) {
  auto& b = registry()[p].m[name];
  if (b.second >= bytes && b.first) return b.first;
  if (b.first) (void)hipFree(b.first);
  b.first = nullptr;
  b.second = 0;
  void* ptr = nullptr;
  hipError_t e = hipMalloc(&ptr, std::max<size_t>(bytes, 256));
  if (e != hipSuccess) {
    *st = hip_check(p, e, name);
    return nullptr;
  }
  b.first = ptr;
  b.second = bytes;
  return ptr;
}

void* scratch(qax_problem* p, size_t bytes, qax_status* st) { return dbuf(p, "scratch", bytes, st); }

// A rebuild of the same geometry asks for the same sizes again: buffers it
// released are handed back instead of freed and allocated anew (all work on
// them is ordered on the handle's stream).
void dev_drop_spare(qax_problem* p) {
  for (auto& kv : p->spare) (void)hipFree(kv.second);
  p->spare.clear();
}

hipError_t dev_alloc(qax_problem* p, void** ptr, size_t bytes) {
  bytes = std::max<size_t>(bytes, 256);
  auto it = p->spare.find(bytes);
  if (it != p->spare.end()) {
    *ptr = it->second;
    p->spare.erase(it);
    p->live[*ptr] = bytes;
    return hipSuccess;
  }
  hipError_t e = hipMalloc(ptr, bytes);
  if (e == hipErrorOutOfMemory && !p->spare.empty()) {
    (void)hipGetLastError();
    dev_drop_spare(p);
    e = hipMalloc(ptr, bytes);
  }
  if (e == hipSuccess) p->live[*ptr] = bytes;
  return e;
}

void dev_release(qax_problem* p, void* q) {
  if (!q) return;
  auto it = p->live.find(q);
  if (it == p->live.end()) {
    (void)hipFree(q);
    return;
  }
  p->spare.emplace(it->second, q);
  p->live.erase(it);
}

static hipEvent_t take_event(qax_problem* p) {
  if (!p->event_pool.empty()) {
    hipEvent_t e = p->event_pool.back();
    p->event_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

void timing_begin(qax_problem* p, int kind) {
  if (!p->timing) return;
  qax_problem::Pending pe{kind, take_event(p), nullptr};
  if (pe.a) (void)hipEventRecord(pe.a, p->stream);
  p->pending.push_back(pe);
}

void timing_end(qax_problem* p, int kind) {
  if (!p->timing) return;
  for (auto it = p->pending.rbegin(); it != p->pending.rend(); ++it) {
    if (it->kind == kind && it->b == nullptr) {
      it->b = take_event(p);
      if (it->b) (void)hipEventRecord(it->b, p->stream);
      return;
    }
  }
}

void collect_timing(qax_problem* p) {
  for (auto& pe : p->pending) {
    float ms = 0.0f;
    if (pe.a && pe.b && hipEventElapsedTime(&ms, pe.a, pe.b) == hipSuccess) {
      p->t_launches[pe.kind] += 1;
      p->t_ms[pe.kind] += ms;
    }
    if (pe.a) p->event_pool.push_back(pe.a);
    if (pe.b) p->event_pool.push_back(pe.b);
  }
  p->pending.clear();
}

}  // namespace qax

#define QCHECK(expr, what)                                   \
  do {                                                       \
    qax_status _s = hip_check(p, (expr), what);              \
    if (_s != QAX_OK) return _s;                             \
  } while (0)

#define QBUF(var, type, name, bytes)                         \
  type* var = nullptr;                                       \
  do {                                                       \
    qax_status _s = QAX_OK;                                  \
    var = (type*)dbuf(p, name, (bytes), &_s);                \
    if (!var) return _s;                                     \
  } while (0)

static int cu_count(int dev) {
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return 256;
  return prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
}

static bool is_finite(double v) { return std::isfinite(v); }

// ---------------------------------------------------------------- lifecycle
extern "C" qax_status qax_create(int device, void* hip_stream, qax_problem** out) {
  if (!out) return QAX_ERR_ARG;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return QAX_ERR_DEVICE;
  if (hipSetDevice(device) != hipSuccess) return QAX_ERR_DEVICE;
  qax_problem* p = new (std::nothrow) qax_problem();
  if (!p) return QAX_ERR_NOMEM;
  p->device = device;
  p->stream = (hipStream_t)hip_stream;
  // device address of the allocation-free far field's workspace on this GPU
  if (noalloc_init(device) != hipSuccess) {
    delete p;
    return QAX_ERR_DEVICE;
  }
  *out = p;
  return QAX_OK;
}

// The reciprocal pair sums' blocks and plans (a function of the node ranges
// of the bodies and problems and of the wavenumbers only).
static void free_pair_plans(qax_problem* p) {
  dev_release(p, p->sym.d_bmem);
  p->sym.d_bmem = nullptr;
  for (int pi = 0; pi < 2; ++pi) (void)release_sym_plan(p, pi);
  p->sym.blocks.clear();
  p->sym.key.clear();
}

static void free_geometry(qax_problem* p, bool keep_plans = false) {
  void* ptrs[] = {p->d_bodies, p->d_blocks, p->d_node_body, p->d_pos,  p->d_aw,
                  p->d_loc32,  p->d_aw32,   p->d_gl,        p->d_B,    p->d_Binv,
                  p->d_Binv32, p->d_tasks64, p->d_tasks32, p->d_ew, p->d_ew32, p->d_B32,
                  p->d_pinfo};
  for (void* q : ptrs) dev_release(p, q);
  p->d_bodies = nullptr; p->d_blocks = nullptr; p->d_node_body = nullptr;
  p->d_pos = nullptr; p->d_aw = nullptr; p->d_loc32 = nullptr; p->d_aw32 = nullptr;
  p->d_gl = nullptr; p->d_B = nullptr; p->d_Binv = nullptr; p->d_Binv32 = nullptr;
  p->d_B32 = nullptr; p->d_pinfo = nullptr;
  p->d_tasks64 = nullptr; p->d_tasks32 = nullptr;
  p->d_ew = nullptr; p->d_ew32 = nullptr;
  dev_release(p, p->d_gemm_tasks);
  p->d_gemm_tasks = nullptr;
  if (!keep_plans) free_pair_plans(p);
  free_sym_apply(p);
  p->gemm_tasks.clear();
  lattice_free(p);
}

extern "C" void qax_destroy(qax_problem* p) {
  if (!p) return;
  (void)hipSetDevice(p->device);
  if (p->stream) (void)hipStreamSynchronize(p->stream);
  else (void)hipDeviceSynchronize();
  for (hipGraphExec_t g : p->graphs)
    if (g) (void)hipGraphExecDestroy(g);
  p->graphs.clear();
  if (p->h_flags) (void)hipHostFree(p->h_flags);
  p->h_flags = nullptr;
  if (p->h_stage) (void)hipHostFree(p->h_stage);
  p->h_stage = nullptr;
  if (p->cap_stream) (void)hipStreamDestroy(p->cap_stream);
  p->cap_stream = nullptr;
  free_geometry(p);
  dev_drop_spare(p);
  collect_timing(p);
  for (hipEvent_t e : p->event_pool) (void)hipEventDestroy(e);
  auto it = registry().find(p);
  if (it != registry().end()) {
    for (auto& kv : it->second.m)
      if (kv.second.first) (void)hipFree(kv.second.first);
    registry().erase(it);
  }
  delete p;
}

extern "C" const char* qax_last_error(const qax_problem* p) { return p ? p->err.c_str() : "null handle"; }

static qax_status sync(qax_problem* p, const char* what) {
  qax_status st = hip_check(p, hipStreamSynchronize(p->stream), what);
  if (st == QAX_OK && !p->pending.empty()) collect_timing(p);
  return st;
}

extern "C" qax_status qax_set_formulation(qax_problem* p, int32_t formulation, double eta) {
  if (!p) return QAX_ERR_ARG;
  if ((formulation != QAX_DOUBLE_LAYER && formulation != QAX_COMBINED_FIELD &&
       formulation != QAX_SINGLE_LAYER) || !is_finite(eta))
    return fail(p, QAX_ERR_ARG, "qax_set_formulation: bad formulation or eta");
  p->formulation = formulation;
  p->eta_param = eta;
  if (p->state < 1) return QAX_OK;
  // built handle: couplings, weights and task tables follow; blocks and the
  // lattice tables are stale
  QCHECK(hipSetDevice(p->device), "hipSetDevice");
  QCHECK(hipStreamSynchronize(p->stream), "sync");
  lattice_free(p);
  for (auto& d : p->hbodies) d.eta = p->eta_of(d.k);
  QCHECK(hipMemcpyAsync(p->d_bodies, p->hbodies.data(), sizeof(BodyDev) * p->hbodies.size(),
                        hipMemcpyHostToDevice, p->stream), "copy bodies");
  QCHECK(launch_node_weights(p), "node weights");
  const int cus = cu_count(p->device);
  QCHECK(upload_pair_plan(p, QAX_FP64, cus), "pair-sum plan");
  QCHECK(upload_pair_plan(p, QAX_MIXED, cus), "pair-sum plan");
  p->state = std::min(p->state, 1);
  return sync(p, "qax_set_formulation");
}

extern "C" qax_status qax_lattice(qax_problem* p, int32_t enable, int32_t* dims) {
  if (!p) return QAX_ERR_ARG;
  if (p->state < 1) return fail(p, QAX_ERR_STATE, "qax_lattice: build first");
  QCHECK(hipSetDevice(p->device), "hipSetDevice");
  QCHECK(hipStreamSynchronize(p->stream), "sync");
  lattice_free(p);
  ++p->generation;
  if (!enable) return QAX_OK;
  const qax_status st = lattice_enable(p, dims);
  if (st != QAX_OK) lattice_free(p);
  return st;
}

extern "C" qax_status qax_set_graphs(qax_problem* p, int32_t enable) {
  if (!p) return QAX_ERR_ARG;
  p->use_graphs = enable != 0;
  return QAX_OK;
}

extern "C" qax_status qax_set_timing(qax_problem* p, int32_t enable) {
  if (!p) return QAX_ERR_ARG;
  QCHECK(hipSetDevice(p->device), "hipSetDevice");
  QCHECK(hipStreamSynchronize(p->stream), "sync");
  collect_timing(p);
  p->timing = enable != 0;
  for (int i = 0; i < QAX_K_COUNT; ++i) {
    p->t_launches[i] = 0;
    p->t_ms[i] = 0.0;
  }
  return QAX_OK;
}

extern "C" qax_status qax_timing(const qax_problem* pc, int32_t kernel, int64_t* launches, double* total_ms) {
  qax_problem* p = const_cast<qax_problem*>(pc);
  if (!p || kernel < 0 || kernel >= QAX_K_COUNT || !launches || !total_ms) return QAX_ERR_ARG;
  QCHECK(hipSetDevice(p->device), "hipSetDevice");
  QCHECK(hipStreamSynchronize(p->stream), "sync");
  collect_timing(p);
  *launches = p->t_launches[kernel];
  *total_ms = p->t_ms[kernel];
  return QAX_OK;
}

// ---------------------------------------------------------------- build
static void rotation(double t1, double t2, double* R) {
  const double c1 = std::cos(t1), s1 = std::sin(t1), c2 = std::cos(t2), s2 = std::sin(t2);
  // Rz(t1) Ry(t2)
  const double Rz[9] = {c1, -s1, 0, s1, c1, 0, 0, 0, 1};
  const double Ry[9] = {c2, 0, s2, 0, 1, 0, -s2, 0, c2};
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double s = 0;
      for (int k = 0; k < 3; ++k) s += Rz[3 * i + k] * Ry[3 * k + j];
      R[3 * i + j] = s;
    }
}

extern "C" qax_status qax_build(qax_problem* p, const qax_body* bodies, int32_t n_bodies,
                                const double* k_per_problem, int32_t n_problems) {
  if (!p) return QAX_ERR_ARG;
  if (!bodies || n_bodies <= 0 || !k_per_problem || n_problems <= 0)
    return fail(p, QAX_ERR_ARG, "qax_build: empty body list or wavenumbers");
  for (int i = 0; i < n_problems; ++i)
    if (!is_finite(k_per_problem[i]) || k_per_problem[i] < 0)
      return fail(p, QAX_ERR_ARG, "qax_build: wavenumbers must be finite and >= 0");
  int prev = 0;
  for (int i = 0; i < n_bodies; ++i) {
    const qax_body& b = bodies[i];
    if (b.shape < 0 || b.shape > QAX_CONCH) return fail(p, QAX_ERR_ARG, "qax_build: unknown shape");
    if (b.n_panels < 1 || b.n_panels > 32) return fail(p, QAX_ERR_ARG, "qax_build: n_panels must be in [1, 32]");
    if (b.n_ref < 0 || b.n_ref > 8 || (b.n_ref > 0 && b.n_panels < 2))
      return fail(p, QAX_ERR_ARG, "qax_build: n_ref must be in [0, 8], with n_panels >= 2 when refined");
    if (b.n_theta < 4 || b.n_theta > 64 || (b.n_theta & 1))
      return fail(p, QAX_ERR_ARG, "qax_build: n_theta must be even in [4, 64]");
    if ((int64_t)(b.n_panels + 2 * b.n_ref) * GL_ORDER * b.n_theta > 8192)
      return fail(p, QAX_ERR_ARG, "qax_build: more than 8192 nodes in one body");
    if (b.problem < 0 || b.problem >= n_problems || b.problem < prev || b.problem > prev + 1)
      return fail(p, QAX_ERR_ARG, "qax_build: problems must be contiguous and increasing");
    if (i == 0 && b.problem != 0) return fail(p, QAX_ERR_ARG, "qax_build: first body must be in problem 0");
    prev = b.problem;
    const double vals[] = {b.a, b.c, b.kappa, b.theta1, b.theta2, b.centre[0], b.centre[1], b.centre[2]};
    for (double v : vals)
      if (!is_finite(v)) return fail(p, QAX_ERR_ARG, "qax_build: non-finite body parameter");
    if (b.shape >= QAX_QUASI_ELLIPSOID) {
      if (b.a <= 0 || b.kappa != 0.0)
        return fail(p, QAX_ERR_ARG, "qax_build: shapes 3-5 need a > 0 and kappa = 0");
      continue;
    }
    if (b.a <= 0 || b.c <= 0 || b.kappa < 0) return fail(p, QAX_ERR_ARG, "qax_build: bad shape parameters");
    const double zmax = b.shape == QAX_PEANUT ? b.a * (1 + b.c) : b.c;
    if (b.shape == QAX_PEANUT && b.c >= 1.0) return fail(p, QAX_ERR_ARG, "qax_build: peanut needs c < 1");
    if (b.kappa * zmax >= 1.0) return fail(p, QAX_ERR_ARG, "qax_build: kappa * max|z| must be < 1");
  }
  if (prev != n_problems - 1) return fail(p, QAX_ERR_ARG, "qax_build: a problem has no bodies");
  QCHECK(hipSetDevice(p->device), "hipSetDevice");
  // the pair-sum plans are kept when the new geometry has the same node
  // ranges and wavenumbers (a rebuild of moved or reshaped bodies)
  free_geometry(p, true);
  p->state = 0;
  p->n_bodies = n_bodies;
  p->n_problems = n_problems;
  p->bodies.assign(bodies, bodies + n_bodies);
  p->k.assign(k_per_problem, k_per_problem + n_problems);
  p->off.assign(n_bodies + 1, 0);
  p->prob_body0.assign(n_problems + 1, n_bodies);
  p->hbodies.assign(n_bodies, BodyDev{});
  p->hblocks.clear();
  // distinct self blocks: equal shape, parameters, discretisation and k
  std::map<std::vector<double>, int> key2blk;
  int64_t elems = 0;
  for (int i = 0; i < n_bodies; ++i) {
    const qax_body& b = bodies[i];
    const int n = (b.n_panels + 2 * b.n_ref) * GL_ORDER * b.n_theta;
    p->off[i + 1] = p->off[i] + n;
    if (i == 0 || bodies[i - 1].problem != b.problem) p->prob_body0[b.problem] = i;
    BodyDev& d = p->hbodies[i];
    d.shape = b.shape; d.n_panels = b.n_panels + 2 * b.n_ref; d.n_theta = b.n_theta;
    d.problem = b.problem;
    d.n_uni = b.n_panels; d.n_ref = b.n_ref;
    d.off = p->off[i]; d.n = n;
    d.a = b.a; d.c = b.c; d.kappa = b.kappa;
    rotation(b.theta1, b.theta2, d.R);
    for (int a = 0; a < 3; ++a) d.cen[a] = b.centre[a];
    d.k = k_per_problem[b.problem];
    d.eta = p->eta_of(d.k);
    std::vector<double> key = {(double)b.shape, b.a, b.shape >= QAX_QUASI_ELLIPSOID ? 0.0 : b.c,
                               b.kappa, (double)b.n_panels, (double)b.n_ref, (double)b.n_theta,
                               d.k, d.eta};
    auto it = key2blk.find(key);
    if (it == key2blk.end()) {
      BlockDev bk;
      bk.rep_body = i;
      bk.n = n;
      bk.elem_off = elems;
      elems += (int64_t)n * n;
      key2blk[key] = (int)p->hblocks.size();
      d.block = (int)p->hblocks.size();
      p->hblocks.push_back(bk);
    } else {
      d.block = it->second;
    }
  }
  p->prob_body0[n_problems] = n_bodies;
  {
    std::vector<int64_t> key(p->off.begin(), p->off.end());
    key.insert(key.end(), p->prob_body0.begin(), p->prob_body0.end());
    for (double kv : p->k) {
      int64_t b;
      std::memcpy(&b, &kv, 8);
      key.push_back(b);
    }
    if (key != p->sym.key) {
      QCHECK(hipStreamSynchronize(p->stream), "sync");
      free_pair_plans(p);
      p->sym.key = key;
    }
  }
  p->N = p->off[n_bodies];
  p->block_elems = elems;
  const int64_t N = p->N;
  QCHECK(dev_alloc(p, (void**)&p->d_bodies, sizeof(BodyDev) * n_bodies), "alloc bodies");
  QCHECK(dev_alloc(p, (void**)&p->d_blocks, sizeof(BlockDev) * p->hblocks.size()), "alloc blocks");
  QCHECK(dev_alloc(p, (void**)&p->d_node_body, sizeof(int32_t) * N), "alloc node_body");
  QCHECK(dev_alloc(p, (void**)&p->d_pos, sizeof(double) * 3 * N), "alloc pos");
  QCHECK(dev_alloc(p, (void**)&p->d_aw, sizeof(double) * 3 * N), "alloc aw");
  QCHECK(dev_alloc(p, (void**)&p->d_loc32, sizeof(float) * 4 * N), "alloc loc32");
  QCHECK(dev_alloc(p, (void**)&p->d_aw32, sizeof(float) * 4 * N), "alloc aw32");
  QCHECK(dev_alloc(p, (void**)&p->d_ew, sizeof(double) * N), "alloc ew");
  QCHECK(dev_alloc(p, (void**)&p->d_ew32, sizeof(float) * N), "alloc ew32");
  QCHECK(dev_alloc(p, (void**)&p->d_gl, sizeof(double) * 3 * GL_ORDER), "alloc gl");
  QCHECK(dev_alloc(p, (void**)&p->d_pinfo, sizeof(int64_t) * (2 * n_problems + 1)), "alloc pinfo");
  {
    std::vector<int64_t> pinfo(2 * (size_t)n_problems + 1);
    for (int pr = 0; pr <= n_problems; ++pr) pinfo[pr] = p->off[p->prob_body0[pr]];
    for (int pr = 0; pr < n_problems; ++pr) std::memcpy(&pinfo[n_problems + 1 + pr], &p->k[pr], 8);
    QCHECK(hipMemcpyAsync(p->d_pinfo, pinfo.data(), pinfo.size() * 8, hipMemcpyHostToDevice, p->stream),
           "copy pinfo");
    QCHECK(hipStreamSynchronize(p->stream), "sync");
  }
  double gl[3 * GL_ORDER];   // nodes, weights, barycentric weights on [-1, 1]
  gauss_legendre_host(GL_ORDER, gl, gl + GL_ORDER);
  for (int l = 0; l < GL_ORDER; ++l) {
    double prod = 1.0;
    for (int m = 0; m < GL_ORDER; ++m)
      if (m != l) prod *= gl[l] - gl[m];
    gl[2 * GL_ORDER + l] = 1.0 / prod;
  }
  QCHECK(hipMemcpyAsync(p->d_gl, gl, sizeof(gl), hipMemcpyHostToDevice, p->stream), "copy gl");
  QCHECK(hipMemcpyAsync(p->d_bodies, p->hbodies.data(), sizeof(BodyDev) * n_bodies,
                        hipMemcpyHostToDevice, p->stream), "copy bodies");
  QCHECK(hipMemcpyAsync(p->d_blocks, p->hblocks.data(), sizeof(BlockDev) * p->hblocks.size(),
                        hipMemcpyHostToDevice, p->stream), "copy blocks");
  QCHECK(launch_build_nodes(p), "build_nodes");
  QCHECK(launch_node_weights(p), "node weights");
  const int cus = cu_count(p->device);
  QCHECK(upload_pair_plan(p, QAX_FP64, cus), "pair-sum plan");
  QCHECK(upload_pair_plan(p, QAX_MIXED, cus), "pair-sum plan");
  qax_status st = sync(p, "qax_build");
  if (st != QAX_OK) return st;
  p->state = 1;
  p->err.clear();
  return QAX_OK;
}

extern "C" qax_status qax_size(const qax_problem* p, int64_t* n_unknowns, int64_t* body_offsets) {
  if (!p || !n_unknowns) return QAX_ERR_ARG;
  if (p->state < 1) return QAX_ERR_STATE;
  *n_unknowns = p->N;
  if (body_offsets) std::memcpy(body_offsets, p->off.data(), sizeof(int64_t) * (p->n_bodies + 1));
  return QAX_OK;
}

extern "C" qax_status qax_nodes(const qax_problem* pc, double* d_pos, double* d_aw) {
  qax_problem* p = const_cast<qax_problem*>(pc);
  if (!p || !d_pos || !d_aw) return QAX_ERR_ARG;
  if (p->state < 1) return fail(p, QAX_ERR_STATE, "qax_nodes: call qax_build first");
  QCHECK(hipSetDevice(p->device), "hipSetDevice");
  for (int c = 0; c < 3; ++c) {
    QCHECK(hipMemcpy2DAsync(d_pos + c, 24, p->d_pos + c * p->N, 8, 8, p->N,
                            hipMemcpyDeviceToDevice, p->stream), "copy pos");
    QCHECK(hipMemcpy2DAsync(d_aw + c, 24, p->d_aw + c * p->N, 8, 8, p->N,
                            hipMemcpyDeviceToDevice, p->stream), "copy aw");
  }
  return sync(p, "qax_nodes");
}

// ---------------------------------------------------------------- self blocks
// The FP64 inverse blocks, made on first use after each assembly (the mixed
// path only needs the FP32 inverse, which assembly makes).  Not to be called
// inside a stream capture.
static qax_status ensure_inverse64(qax_problem* p) {
  if (p->inv64_ready) return QAX_OK;
  QBUF(work, double, "gj_work", invert_blocks_work_bytes(p));
  QCHECK(launch_invert_blocks64(p, work), "invert_blocks (FP64)");
  QCHECK(hipStreamSynchronize(p->stream), "sync");
  p->inv64_ready = true;
  return QAX_OK;
}

extern "C" qax_status qax_assemble_self(qax_problem* p, double* t_setup_s) {
  if (!p) return QAX_ERR_ARG;
  if (p->state < 1) return fail(p, QAX_ERR_STATE, "qax_assemble_self: call qax_build first");
  QCHECK(hipSetDevice(p->device), "hipSetDevice");
  QCHECK(hipStreamSynchronize(p->stream), "sync");
  auto t0 = std::chrono::steady_clock::now();
  if (!p->d_B) {
    QCHECK(dev_alloc(p, (void**)&p->d_B, (size_t)p->block_elems * 16), "alloc self blocks");
    QCHECK(dev_alloc(p, (void**)&p->d_Binv, (size_t)p->block_elems * 16), "alloc inverse blocks");
    QCHECK(dev_alloc(p, (void**)&p->d_Binv32, (size_t)p->block_elems * 8), "alloc inverse blocks fp32");
    QCHECK(dev_alloc(p, (void**)&p->d_B32, (size_t)p->block_elems * 8), "alloc self blocks fp32");
  }
  QCHECK(setup_sym_apply(p), "reduced inverses");
  QCHECK(launch_assemble_self(p), "assemble_self");
  QBUF(work, double, "gj_work", invert_blocks_work_bytes(p));
  if (p->factor_prec == QAX_FP64) {
    QCHECK(launch_factor_blocks64(p, work), "invert_blocks (FP64)");
  } else {
    QCHECK(launch_invert_blocks(p, work), "invert_blocks");
  }
  qax_status st = sync(p, "qax_assemble_self");
  if (st != QAX_OK) return st;
  p->inv64_ready = p->factor_prec == QAX_FP64;
  auto t1 = std::chrono::steady_clock::now();
  if (t_setup_s) *t_setup_s = std::chrono::duration<double>(t1 - t0).count();
  p->state = 2;
  ++p->generation;
  return QAX_OK;
}

extern "C" qax_status qax_set_factorization(qax_problem* p, qax_prec prec) {
  if (!p) return QAX_ERR_ARG;
  if (prec != QAX_FP64 && prec != QAX_MIXED)
    return fail(p, QAX_ERR_ARG, "qax_set_factorization: precision must be QAX_FP64 or QAX_MIXED");
  if (p->factor_prec != prec && p->state >= 2) p->state = 1;   // blocks must be factored again
  p->factor_prec = prec;
  return QAX_OK;
}

extern "C" qax_status qax_self_block(const qax_problem* pc, int32_t body, int32_t inverse, void* d_out) {
  qax_problem* p = const_cast<qax_problem*>(pc);
  if (!p || !d_out) return QAX_ERR_ARG;
  if (p->state < 2) return fail(p, QAX_ERR_STATE, "qax_self_block: call qax_assemble_self first");
  if (body < 0 || body >= p->n_bodies) return fail(p, QAX_ERR_ARG, "qax_self_block: bad body index");
  QCHECK(hipSetDevice(p->device), "hipSetDevice");
  if (inverse) {
    const qax_status st = ensure_inverse64(p);
    if (st != QAX_OK) return st;
  }
  const BlockDev& K = p->hblocks[p->hbodies[body].block];
  const double* src = (inverse ? p->d_Binv : p->d_B) + 2 * K.elem_off;
  QCHECK(hipMemcpyAsync(d_out, src, (size_t)K.n * K.n * 16, hipMemcpyDeviceToDevice, p->stream),
         "copy block");
  return sync(p, "qax_self_block");
}

// ---------------------------------------------------------------- applies
static qax_status check_vec_call(qax_problem* p, const void* a, const void* b, int nrhs, int need) {
  if (!a || !b || nrhs < 1 || nrhs > 256) return fail(p, QAX_ERR_ARG, "null vector or nrhs out of [1, 256]");
  if (p->state < need) return fail(p, QAX_ERR_STATE, need == 1 ? "call qax_build first" : "call qax_assemble_self first");
  return QAX_OK;
}

static qax_status pair_sum_into(qax_problem* p, int prec, const double* mu, double* out, int nrhs,
                                bool accumulate) {
  QBUF(partial, double, "pair_partial", pair_work_bytes(p, prec, nrhs));
  QCHECK(launch_pair_sum(p, prec, mu, out, nrhs, partial, accumulate), "pair_sum");
  return QAX_OK;
}

extern "C" qax_status qax_pair_sum(qax_problem* p, qax_prec prec, const void* d_mu, void* d_out,
                                   int32_t nrhs) {
  if (!p) return QAX_ERR_ARG;
  qax_status st = check_vec_call(p, d_mu, d_out, nrhs, 1);
  if (st != QAX_OK) return st;
  if (prec != QAX_FP64 && prec != QAX_MIXED) return fail(p, QAX_ERR_ARG, "bad precision");
  QCHECK(hipSetDevice(p->device), "hipSetDevice");
  st = pair_sum_into(p, prec, (const double*)d_mu, (double*)d_out, nrhs, false);
  if (st != QAX_OK) return st;
  return sync(p, "qax_pair_sum");
}

extern "C" qax_status qax_block_apply(qax_problem* p, int32_t inverse, qax_prec prec, const void* d_v,
                                      void* d_out, int32_t nrhs) {
  if (!p) return QAX_ERR_ARG;
  qax_status st = check_vec_call(p, d_v, d_out, nrhs, 2);
  if (st != QAX_OK) return st;
  QCHECK(hipSetDevice(p->device), "hipSetDevice");
  if (inverse && prec == QAX_FP64) {
    st = ensure_inverse64(p);
    if (st != QAX_OK) return st;
  }
  QCHECK(launch_block_apply(p, inverse, prec, (const double*)d_v, (double*)d_out, nrhs, false),
         "block_apply");
  return sync(p, "qax_block_apply");
}

static qax_status apply_full(qax_problem* p, int prec, const double* mu, double* out, int nrhs) {
  QCHECK(launch_block_apply(p, 0, QAX_FP64, mu, out, nrhs, false), "block_apply");
  return pair_sum_into(p, prec, mu, out, nrhs, true);
}

extern "C" qax_status qax_apply(qax_problem* p, qax_prec prec, const void* d_mu, void* d_out,
                                int32_t nrhs) {
  if (!p) return QAX_ERR_ARG;
  qax_status st = check_vec_call(p, d_mu, d_out, nrhs, 2);
  if (st != QAX_OK) return st;
  QCHECK(hipSetDevice(p->device), "hipSetDevice");
  st = apply_full(p, prec, (const double*)d_mu, (double*)d_out, nrhs);
  if (st != QAX_OK) return st;
  return sync(p, "qax_apply");
}

static qax_status upload_dirs(qax_problem* p, const double* dirs, int nrhs, double** d_dirs) {
  const size_t cnt = (size_t)p->n_problems * nrhs * 3;
  for (size_t i = 0; i < cnt; ++i)
    if (!is_finite(dirs[i])) return fail(p, QAX_ERR_ARG, "non-finite direction");
  QBUF(dd, double, "dirs", cnt * 8);
  QCHECK(hipMemcpyAsync(dd, dirs, cnt * 8, hipMemcpyHostToDevice, p->stream), "copy dirs");
  *d_dirs = dd;
  return QAX_OK;
}

extern "C" qax_status qax_rhs(qax_problem* p, const double* dirs, int32_t nrhs, void* d_out) {
  if (!p) return QAX_ERR_ARG;
  qax_status st = check_vec_call(p, dirs, d_out, nrhs, 1);
  if (st != QAX_OK) return st;
  QCHECK(hipSetDevice(p->device), "hipSetDevice");
  double* dd = nullptr;
  st = upload_dirs(p, dirs, nrhs, &dd);
  if (st != QAX_OK) return st;
  QCHECK(launch_rhs(p, dd, nrhs, (double*)d_out), "rhs");
  return sync(p, "qax_rhs");
}

extern "C" qax_status qax_farfield(qax_problem* p, const void* d_mu, int32_t nrhs, const double* xhat,
                                   int32_t n_dirs, void* d_u_inf) {
  if (!p) return QAX_ERR_ARG;
  qax_status st = check_vec_call(p, d_mu, d_u_inf, nrhs, 1);
  if (st != QAX_OK) return st;
  if (!xhat || n_dirs < 1) return fail(p, QAX_ERR_ARG, "qax_farfield: no directions");
  for (int i = 0; i < 3 * n_dirs; ++i)
    if (!is_finite(xhat[i])) return fail(p, QAX_ERR_ARG, "qax_farfield: non-finite direction");
  QCHECK(hipSetDevice(p->device), "hipSetDevice");
  // items: each direction, paired with a later one that is its exact
  // negation (bitwise, open-addressing table over the 24-byte keys)
  std::vector<int2> items;
  items.reserve(n_dirs);
  {
    const uint64_t* bits = (const uint64_t*)xhat;
    auto hash = [&](uint64_t a, uint64_t b, uint64_t c) {
      uint64_t h = a * 0x9E3779B97F4A7C15ULL;
      h ^= (b + 0x632BE59BD9B4E019ULL + (h << 6) + (h >> 2));
      h ^= (c + 0x94D049BB133111EBULL + (h << 6) + (h >> 2));
      return h ^ (h >> 29);
    };
    size_t cap = 1;
    while (cap < 2 * (size_t)n_dirs) cap <<= 1;
    std::vector<int32_t> table(cap, -1);
    for (int i = 0; i < n_dirs; ++i) {
      size_t h = hash(bits[3 * i], bits[3 * i + 1], bits[3 * i + 2]) & (cap - 1);
      while (table[h] >= 0) h = (h + 1) & (cap - 1);
      table[h] = i;
    }
    const uint64_t sg = 0x8000000000000000ULL;
    std::vector<char> used(n_dirs, 0);
    for (int i = 0; i < n_dirs; ++i) {
      if (used[i]) continue;
      used[i] = 1;
      const uint64_t a = bits[3 * i] ^ sg, b = bits[3 * i + 1] ^ sg, c = bits[3 * i + 2] ^ sg;
      int partner = -1;
      for (size_t h = hash(a, b, c) & (cap - 1); table[h] >= 0; h = (h + 1) & (cap - 1)) {
        const int q = table[h];
        if (!used[q] && bits[3 * q] == a && bits[3 * q + 1] == b && bits[3 * q + 2] == c) {
          partner = q;
          break;
        }
      }
      if (partner >= 0) used[partner] = 1;
      items.push_back(make_int2(i, partner));
    }
  }
  const int nitems = (int)items.size();
  const int slots = farfield_slots((int64_t)nitems * p->n_problems, cu_count(p->device));
  const int np = p->n_problems;
  const size_t up = (size_t)n_dirs * 24 + (size_t)nitems * sizeof(int2);
  QBUF(dx, double, "xhat", up);
  QBUF(part, double, "ff_partial", (size_t)slots * np * n_dirs * nrhs * 16);
  int2* ditems = (int2*)(dx + 3 * (size_t)n_dirs);
  // directions and items through pinned staging: one asynchronous copy
  if (p->h_stage_bytes < up) {
    if (p->h_stage) (void)hipHostFree(p->h_stage);
    p->h_stage = nullptr;
    p->h_stage_bytes = 0;
    QCHECK(hipHostMalloc(&p->h_stage, up, hipHostMallocDefault), "pinned staging");
    p->h_stage_bytes = up;
  }
  std::memcpy(p->h_stage, xhat, (size_t)n_dirs * 24);
  std::memcpy((char*)p->h_stage + (size_t)n_dirs * 24, items.data(), (size_t)nitems * sizeof(int2));
  QCHECK(hipMemcpyAsync(dx, p->h_stage, up, hipMemcpyHostToDevice, p->stream), "copy directions");
  QCHECK(launch_farfield(p, (const double*)d_mu, nrhs, dx, n_dirs, ditems, nitems, p->d_pinfo, slots, part,
                         (double*)d_u_inf),
         "farfield");
  return sync(p, "qax_farfield");
}

extern "C" qax_status qax_nearfield(qax_problem* p, const void* d_mu, int32_t nrhs, const double* pts,
                                    int64_t n_pts, int32_t problem, void* d_u) {
  if (!p) return QAX_ERR_ARG;
  qax_status st = check_vec_call(p, d_mu, d_u, nrhs, 1);
  if (st != QAX_OK) return st;
  if (!pts || n_pts < 1 || n_pts > (int64_t)1 << 28) return fail(p, QAX_ERR_ARG, "qax_nearfield: no points");
  if (problem < 0 || problem >= p->n_problems) return fail(p, QAX_ERR_ARG, "qax_nearfield: bad problem index");
  std::vector<double> soa((size_t)n_pts * 3);
  for (int64_t i = 0; i < n_pts; ++i)
    for (int c = 0; c < 3; ++c) {
      const double v = pts[3 * i + c];
      if (!is_finite(v)) return fail(p, QAX_ERR_ARG, "qax_nearfield: non-finite point");
      soa[(size_t)c * n_pts + i] = v;
    }
  QCHECK(hipSetDevice(p->device), "hipSetDevice");
  const int slots = nearfield_slots(n_pts, cu_count(p->device));
  QBUF(dp, double, "nf_points", soa.size() * 8);
  QBUF(part, double, "nf_partial", (size_t)slots * n_pts * nrhs * 16);
  QCHECK(hipMemcpyAsync(dp, soa.data(), soa.size() * 8, hipMemcpyHostToDevice, p->stream), "copy points");
  QCHECK(launch_nearfield(p, (const double*)d_mu, nrhs, dp, n_pts, problem, slots, part, (double*)d_u),
         "nearfield");
  return sync(p, "qax_nearfield");
}

extern "C" qax_status qax_modal_modes(qax_problem* p, int32_t n_pts, const double* d_r,
                                      const double* d_rt, const double* d_c, const double* d_chim1,
                                      const double* d_rmrt, double k, int32_t nmax, void* d_A,
                                      void* d_B) {
  if (!p) return QAX_ERR_ARG;
  if (n_pts < 1 || nmax < 0 || nmax > 160 || !d_r || !d_rt || !d_c || !d_chim1 || !d_rmrt || !d_A || !d_B)
    return fail(p, QAX_ERR_ARG, "qax_modal_modes: bad arguments");
  if (!is_finite(k) || k < 0) return fail(p, QAX_ERR_ARG, "qax_modal_modes: bad k");
  QCHECK(hipSetDevice(p->device), "hipSetDevice");
  QCHECK(launch_modal_modes(p->stream, n_pts, d_r, d_rt, d_c, d_chim1, d_rmrt, k, nmax,
                            (double*)d_A, (double*)d_B), "modal_modes");
  return sync(p, "qax_modal_modes");
}

// ---------------------------------------------------------------- dense solve
extern "C" qax_status qax_invert(qax_problem* p, qax_prec prec, int32_t count, const int32_t* orders,
                                 void* d_mats) {
  if (!p) return QAX_ERR_ARG;
  if (prec != QAX_FP64 && prec != QAX_MIXED) return fail(p, QAX_ERR_ARG, "qax_invert: bad precision");
  if (count < 0 || (count > 0 && (!orders || !d_mats)))
    return fail(p, QAX_ERR_ARG, "qax_invert: bad count or null pointer");
  if (count == 0) return QAX_OK;
  int nmax = 0;
  int64_t total = 0;
  for (int i = 0; i < count; ++i) {
    if (orders[i] < 1 || orders[i] > 8192)
      return fail(p, QAX_ERR_ARG, "qax_invert: matrix orders must be in [1, 8192]");
    nmax = std::max(nmax, (int)orders[i]);
    total += (int64_t)orders[i] * orders[i];
  }
  QCHECK(hipSetDevice(p->device), "hipSetDevice");
  const bool f32 = prec == QAX_MIXED;
  QBUF(work, double, "invert_work", invert_matrices_work_bytes(count, nmax, total, f32));
  QCHECK(launch_invert_matrices(p, f32, count, orders, (double*)d_mats, work), "invert");
  return sync(p, "qax_invert");
}

extern "C" qax_status qax_solve_dense(qax_problem* p, const double* dirs, int32_t nrhs, void* d_mu_out) {
  if (!p) return QAX_ERR_ARG;
  qax_status st = check_vec_call(p, dirs, d_mu_out, nrhs, 2);
  if (st != QAX_OK) return st;
  if (p->N > 8192) return fail(p, QAX_ERR_ARG, "qax_solve_dense: N > 8192");
  QCHECK(hipSetDevice(p->device), "hipSetDevice");
  const int64_t N = p->N;
  QBUF(A, double, "dense_A", (size_t)N * N * 16);
  QBUF(b, double, "dense_b", (size_t)N * nrhs * 16);
  QBUF(work, double, "dense_work", dense_solve_work_bytes(N));
  double* dd = nullptr;
  st = upload_dirs(p, dirs, nrhs, &dd);
  if (st != QAX_OK) return st;
  QCHECK(launch_rhs(p, dd, nrhs, b), "rhs");
  QCHECK(launch_dense_system(p, A), "dense_system");
  QCHECK(launch_dense_solve(p, A, b, nrhs, (double*)d_mu_out, work), "dense_solve");
  return sync(p, "qax_solve_dense");
}

// ---------------------------------------------------------------- GMRES

static qax_status setup_krylov(qax_problem* p, int nrhs, int mmax, Krylov& K) {
  K.stream = p->stream;
  K.N = p->N;
  K.nrhs = nrhs;
  K.nprob = p->n_problems;
  const int64_t chunk_nodes = std::max<int64_t>(64, 8192 / nrhs);
  std::vector<Chunk> ch;
  std::vector<int32_t> pc0(p->n_problems + 1, 0);
  for (int pr = 0; pr < p->n_problems; ++pr) {
    pc0[pr] = (int32_t)ch.size();
    const int64_t n0 = p->off[p->prob_body0[pr]], n1 = p->off[p->prob_body0[pr + 1]];
    for (int64_t a = n0; a < n1; a += chunk_nodes) ch.push_back(Chunk{a, std::min(n1, a + chunk_nodes)});
  }
  pc0[p->n_problems] = (int32_t)ch.size();
  K.nchunks = (int)ch.size();
  std::vector<int32_t> nprob(p->N);
  for (int b = 0; b < p->n_bodies; ++b)
    for (int64_t n = p->off[b]; n < p->off[b + 1]; ++n) nprob[n] = p->hbodies[b].problem;
  QBUF(dch, Chunk, "kry_chunks", ch.size() * sizeof(Chunk));
  QBUF(dpc, int32_t, "kry_pc0", pc0.size() * 4);
  QBUF(dnp, int32_t, "kry_nprob", (size_t)p->N * 4);
  QBUF(dpart, double, "kry_partial", (size_t)(mmax + 2) * ch.size() * nrhs * 16);
  QCHECK(hipMemcpyAsync(dch, ch.data(), ch.size() * sizeof(Chunk), hipMemcpyHostToDevice, p->stream), "copy");
  QCHECK(hipMemcpyAsync(dpc, pc0.data(), pc0.size() * 4, hipMemcpyHostToDevice, p->stream), "copy");
  QCHECK(hipMemcpyAsync(dnp, nprob.data(), (size_t)p->N * 4, hipMemcpyHostToDevice, p->stream), "copy");
  QCHECK(hipStreamSynchronize(p->stream), "sync");
  K.d_chunks = dch;
  K.d_prob_chunk0 = dpc;
  K.d_node_prob = dnp;
  K.d_partial = dpart;
  return QAX_OK;
}

// Solve with the plane-wave right-hand sides of `dirs` (host) or, when dirs is
// null, the caller's device right-hand side d_rhs.
// Smallest residual reduction one mixed refinement cycle aims at.  The FP32
// operator (FP32 pair sum, FP32 copy of the inverse) is accurate to a few
// 1e-7 per apply, and the implicit GMRES residual stops tracking the true one
// near 1e-6 of the cycle's right-hand side; a cycle pushed further only adds
// steps that the next FP64 residual undoes.  Restarting costs no steps here
// (the preconditioned operator is the identity plus a compact part, so GMRES
// converges at a nearly fixed rate): on the 1000-body workload at 1e-6 a first
// cycle aimed at 5e-7 took 39 FP32 steps in all, one aimed at 3e-6 ... 1e-3
// took 36, as many as the FP64 solver.  With the inverse computed in FP32
// (accurate to ~1e-5) a cycle cannot gain more than that.
static double mixed_cycle_floor(const qax_problem* p) {
  return p->factor_prec == QAX_FP64 ? 1e-5 : 2e-5;
}

static qax_status solve_core(qax_problem* p, qax_prec prec, const double* dirs, const double* d_rhs,
                             int32_t nrhs, double tol, int32_t maxit, void* d_mu_out, qax_info* info) {
  qax_status st = check_vec_call(p, dirs ? (const void*)dirs : (const void*)d_rhs, d_mu_out, nrhs, 2);
  if (st != QAX_OK) return st;
  if (prec != QAX_FP64 && prec != QAX_MIXED) return fail(p, QAX_ERR_ARG, "bad precision");
  if (!(tol > 0) || !is_finite(tol) || maxit < 1) return fail(p, QAX_ERR_ARG, "qax_solve: bad tol / maxit");
  QCHECK(hipSetDevice(p->device), "hipSetDevice");
  QCHECK(hipStreamSynchronize(p->stream), "sync");
  // set-up outside the solve time: the FP64 preconditioner on first FP64 use
  if (prec == QAX_FP64 && (st = ensure_inverse64(p)) != QAX_OK) return st;
  auto t0 = std::chrono::steady_clock::now();

  const int64_t N = p->N;
  const int64_t vs = N * nrhs * 2;  // doubles per vector
  const int nseg = p->n_problems * nrhs;
  const int m = std::min<int>(maxit, nrhs > 8 ? 40 : 100);
  Krylov K;
  st = setup_krylov(p, nrhs, m, K);
  if (st != QAX_OK) return st;
  QBUF(V, double, "kry_V", (size_t)(m + 1) * vs * 8);
  QBUF(w, double, "kry_w", (size_t)vs * 8);
  QBUF(t, double, "kry_t", (size_t)vs * 8);
  QBUF(r, double, "kry_r", (size_t)vs * 8);
  QBUF(b, double, "kry_b", (size_t)vs * 8);
  QBUF(hd, double, "kry_h", (size_t)(2 * m + 4) * nseg * 16);
  double* x = (double*)d_mu_out;
  if (dirs) {
    double* dd = nullptr;
    st = upload_dirs(p, dirs, nrhs, &dd);
    if (st != QAX_OK) return st;
    QCHECK(launch_rhs(p, dd, nrhs, b), "rhs");
  } else {
    QCHECK(hipMemcpyAsync(b, d_rhs, (size_t)vs * 8, hipMemcpyDeviceToDevice, p->stream), "copy rhs");
  }
  QCHECK(hipMemsetAsync(x, 0, (size_t)vs * 8, p->stream), "zero x");

  const int inner_prec = prec;
  std::vector<cplx> hh((size_t)(2 * m + 4) * nseg);
  auto fetch = [&](int rows) -> qax_status {
    QCHECK(hipMemcpyAsync(hh.data(), hd, (size_t)rows * nseg * 16, hipMemcpyDeviceToHost, p->stream),
           "copy h");
    return sync(p, "gmres");
  };
  // least-squares state on the device
  GivensState G;
  {
    QBUF(gH, double2, "kry_gH", (size_t)nseg * m * (m + 1) * 16);
    QBUF(gcs, double, "kry_gcs", (size_t)nseg * m * 8);
    QBUF(gsn, double2, "kry_gsn", (size_t)nseg * m * 16);
    QBUF(gg, double2, "kry_gg", (size_t)nseg * (m + 1) * 16);
    QBUF(gpar, double, "kry_gpar", (size_t)nseg * 16 + 256);
    QBUF(gfz, int32_t, "kry_gfrozen", (size_t)nseg * 12 + (size_t)(m + 1) * 4);
    QBUF(gscl, double2, "kry_gscl", (size_t)nseg * 16);
    G.H = gH;
    G.cs = gcs;
    G.sn = gsn;
    G.g = gg;
    G.beta = gpar;
    G.tin = gpar + nseg;
    G.frozen = gfz;
    G.active = gfz + nseg;
    G.kconv = gfz + 2 * nseg;
    G.notdone = gfz + 3 * nseg;
    G.scl = gscl;
  }
  QBUF(ydev, double2, "kry_y", (size_t)m * nseg * 16);
  // pair-sum workspace sized before any capture (no allocation inside a
  // graph), large enough for the FP64 residual's pair sum too, so that the
  // shared buffer is never reallocated under the captured steps
  QBUF(ppart, double, "pair_partial",
       std::max(pair_work_bytes(p, inner_prec, nrhs), pair_work_bytes(p, QAX_FP64, nrhs)));
  if (p->h_flags_n < m + 1) {
    if (p->h_flags) (void)hipHostFree(p->h_flags);
    p->h_flags = nullptr;
    p->h_flags_n = 0;
    QCHECK(hipHostMalloc((void**)&p->h_flags, (size_t)(m + 1) * 4, hipHostMallocDefault), "pinned flags");
    p->h_flags_n = m + 1;
  }
  // ||b|| per segment
  K.dots(b, 0, 1, b, hd);
  if ((st = fetch(1)) != QAX_OK) return st;
  std::vector<double> bnorm(nseg);
  for (int s = 0; s < nseg; ++s) bnorm[s] = std::sqrt(std::max(hh[s].real(), 0.0));

  // One Arnoldi step j for all segments: z = M^-1 v_j, w = v_j + D_off z
  // (mixed, cycles that must reduce the residual by more than 1e3: w = B z +
  // D_off z with the FP32 copies, since the FP32 inverse is only accurate to
  // ~1e-5 and B M^-1 v = v would cap the cycle's gain there),
  // classical Gram-Schmidt twice, |w|^2, the Givens update on the device,
  // v_{j+1} = w / h_{j+1,j}, and the step's count of unconverged segments
  // copied to pinned host memory.  Enqueued directly, or captured once per j
  // into an executable graph and replayed.
  double* h1 = hd;
  double* h2 = hd + (size_t)(m + 2) * nseg * 2;
  bool exact_op = false;
  auto enqueue_step = [&](int j) -> hipError_t {
    double* Vj = V + (size_t)j * vs;
    double* Vn = V + (size_t)(j + 1) * vs;
    p->seg_active = G.active;   // operator work of stopped segments is skipped
    hipError_t e = launch_block_apply(p, 1, inner_prec, Vj, t, nrhs, false);
    if (exact_op) {
      if (e == hipSuccess) e = launch_block_apply(p, 0, QAX_MIXED, t, w, nrhs, false);
      if (e == hipSuccess) e = launch_pair_sum(p, inner_prec, t, w, nrhs, ppart, true);
    } else {
      if (e == hipSuccess) e = launch_pair_sum(p, inner_prec, t, w, nrhs, ppart, false);
    }
    p->seg_active = nullptr;
    if (e != hipSuccess) return e;
    if (!exact_op) K.axpby(1.0, w, 1.0, Vj, w);
    K.dots(V, vs, j + 1, w, h1);
    K.orth(V, vs, j + 1, h1, w);
    K.dots(V, vs, j + 1, w, h2);
    K.orth(V, vs, j + 1, h2, w);
    K.dots(w, 0, 1, w, h2 + (size_t)(j + 1) * nseg * 2);
    K.givens(nseg, j, m, h1, h2, h2 + (size_t)(j + 1) * nseg * 2, G);
    K.scale(w, (const double*)G.scl, Vn);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    return hipMemcpyAsync(p->h_flags + j, G.notdone + j, 4, hipMemcpyDeviceToHost, p->stream);
  };
  const bool graphs = p->use_graphs && !p->timing;
  if (nrhs >= 4) QCHECK(ensure_gemm_tasks(p), "block GEMM tiles");
  if (graphs) {
    char key[512];
    std::snprintf(key, sizeof(key), "%llu %d %d %d %d %p %p %p %p %p %p %p %p %p %p %p %p",
                  (unsigned long long)p->generation, inner_prec, nrhs, m, nseg, (void*)V, (void*)w,
                  (void*)t, (void*)hd, (void*)ppart, (void*)G.H, (void*)G.g, (void*)G.scl,
                  (void*)G.notdone, (void*)p->h_flags, (void*)K.d_partial, (void*)K.d_chunks);
    if (p->graph_key != key) {
      for (hipGraphExec_t g : p->graphs)
        if (g) (void)hipGraphExecDestroy(g);
      p->graphs.clear();
      p->graph_key = key;
    }
    // one graph per step index and operator form
    if ((int)p->graphs.size() < 2 * m) p->graphs.resize(2 * m, nullptr);
  }
  auto run_step = [&](int j) -> qax_status {
    if (!graphs) {
      QCHECK(enqueue_step(j), "gmres step");
      return QAX_OK;
    }
    const int gi = (exact_op ? m : 0) + j;
    if (!p->graphs[gi]) {
      // capture on the handle's own stream (the caller's may be the legacy
      // default stream, which cannot be captured); replays go to the caller's
      if (!p->cap_stream)
        QCHECK(hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking), "capture stream");
      const hipStream_t user = p->stream;
      QCHECK(hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal), "begin capture");
      p->stream = K.stream = p->cap_stream;
      const hipError_t e = enqueue_step(j);
      p->stream = K.stream = user;
      hipGraph_t gr = nullptr;
      const hipError_t e2 = hipStreamEndCapture(p->cap_stream, &gr);
      if (e != hipSuccess && gr) (void)hipGraphDestroy(gr);
      QCHECK(e, "gmres step (capture)");
      QCHECK(e2, "end capture");
      hipGraphExec_t ex = nullptr;
      const hipError_t e3 = hipGraphInstantiate(&ex, gr, nullptr, nullptr, 0);
      (void)hipGraphDestroy(gr);
      QCHECK(e3, "instantiate graph");
      p->graphs[gi] = ex;
    }
    QCHECK(hipGraphLaunch(p->graphs[gi], p->stream), "graph launch");
    return QAX_OK;
  };

  int total_its = 0, outer = 0;
  double relres = 1.0;
  std::vector<double> rn(nseg);
  qax_status result = QAX_ERR_NOCONV;
  while (true) {
    // true residual r = b - A x  (FP64)
    if (outer == 0) {
      QCHECK(hipMemcpyAsync(r, b, (size_t)vs * 8, hipMemcpyDeviceToDevice, p->stream), "copy");
    } else {
      st = apply_full(p, QAX_FP64, x, w, nrhs);
      if (st != QAX_OK) return st;
      K.axpby(1.0, b, -1.0, w, r);
    }
    K.dots(r, 0, 1, r, hd);
    if ((st = fetch(1)) != QAX_OK) return st;
    relres = 0.0;
    for (int s = 0; s < nseg; ++s) {
      rn[s] = std::sqrt(std::max(hh[s].real(), 0.0));
      const double rel = bnorm[s] > 0 ? rn[s] / bnorm[s] : 0.0;
      relres = std::max(relres, rel);
    }
    if (relres <= tol) {
      result = QAX_OK;
      break;
    }
    if (total_its >= maxit) break;
    // inner right-preconditioned GMRES cycle on A d = r: per-segment start
    std::vector<double> par(2 * nseg);
    std::vector<int32_t> fz(3 * nseg + m + 1, 0);   // frozen, active, kconv, notdone
    std::vector<cplx> g0((size_t)nseg * (m + 1), 0.0), scl(nseg);
    double min_need = 1.0;
    for (int s = 0; s < nseg; ++s) {
      const bool frozen = !(rn[s] > 0) || (bnorm[s] > 0 && rn[s] <= tol * bnorm[s]);
      // the inner cycle's reduction: half the way below the target
      const double need = bnorm[s] > 0 && rn[s] > 0 ? 0.5 * tol * bnorm[s] / rn[s] : 1.0;
      if (!frozen) min_need = std::min(min_need, need);
      par[s] = rn[s];
      par[nseg + s] = prec == QAX_MIXED ? std::max(need, mixed_cycle_floor(p)) : need;
      fz[s] = frozen ? 1 : 0;
      fz[nseg + s] = frozen ? 0 : 1;
      g0[(size_t)s * (m + 1)] = rn[s];
      scl[s] = frozen ? 0.0 : 1.0 / rn[s];
    }
    QCHECK(hipMemcpyAsync(G.beta, par.data(), par.size() * 8, hipMemcpyHostToDevice, p->stream), "copy");
    QCHECK(hipMemcpyAsync(G.frozen, fz.data(), fz.size() * 4, hipMemcpyHostToDevice, p->stream), "copy");
    QCHECK(hipMemcpyAsync(G.g, g0.data(), g0.size() * 16, hipMemcpyHostToDevice, p->stream), "copy");
    QCHECK(hipMemcpyAsync(G.scl, scl.data(), nseg * 16, hipMemcpyHostToDevice, p->stream), "copy");
    K.scale(r, (const double*)G.scl, V);
    // with the FP32-computed inverse the first cycle aims at the FP32 floor
    // anyway; later ones that must gain more than 1e3 use the exact operator
    // form (the rounded FP64 inverse needs no such form)
    exact_op = prec == QAX_MIXED && p->factor_prec != QAX_FP64 && outer > 0 && min_need < 1e-3;
    int j = 0;
    for (; j < m && total_its < maxit; ++j) {
      if ((st = run_step(j)) != QAX_OK) return st;
      if ((st = sync(p, "gmres")) != QAX_OK) return st;
      ++total_its;
      if (p->h_flags[j] == 0) {
        ++j;
        break;
      }
    }
    // d = M^-1 V y;  x += d
    K.back_solve(nseg, j, m, G, (double*)ydev);
    K.combine(V, vs, j, (const double*)ydev, t, false);
    QCHECK(launch_block_apply(p, 1, inner_prec, t, x, nrhs, true), "precond");
    ++outer;
  }
  if ((st = sync(p, "qax_solve")) != QAX_OK) return st;
  auto t1 = std::chrono::steady_clock::now();
  if (info) {
    info->iters = total_its;
    info->outer_iters = outer;
    info->rel_res = relres;
    info->t_setup_s = 0.0;
    info->t_solve_s = std::chrono::duration<double>(t1 - t0).count();
  }
  if (result != QAX_OK)
    return fail(p, QAX_ERR_NOCONV, "qax_solve: tolerance not reached within maxit iterations");
  return QAX_OK;
}

// ---------------------------------------------------------------- autotuner
namespace {

// The fastest of `reps` launches (after one warm-up launch when `warm`).
template <typename F>
static double time_best(qax_problem* p, int reps, F&& launch, hipError_t* err, bool warm = true) {
  hipEvent_t a = nullptr, b = nullptr;
  *err = hipEventCreate(&a);
  if (*err == hipSuccess) *err = hipEventCreate(&b);
  double best = 1e300;
  if (*err == hipSuccess && warm) *err = launch();
  if (*err == hipSuccess) *err = hipStreamSynchronize(p->stream);
  for (int r = 0; r < reps && *err == hipSuccess; ++r) {
    *err = hipEventRecord(a, p->stream);
    if (*err == hipSuccess) *err = launch();
    if (*err == hipSuccess) *err = hipEventRecord(b, p->stream);
    if (*err == hipSuccess) *err = hipEventSynchronize(b);
    float ms = 0.0f;
    if (*err == hipSuccess) *err = hipEventElapsedTime(&ms, a, b);
    if (*err == hipSuccess) best = std::min(best, (double)ms);
  }
  if (a) (void)hipEventDestroy(a);
  if (b) (void)hipEventDestroy(b);
  return best;
}

static std::string tune_key(qax_problem* p, int nrhs_max) {
  hipDeviceProp_t prop;
  std::string dev = "unknown";
  if (hipGetDeviceProperties(&prop, p->device) == hipSuccess) {
    dev = prop.gcnArchName;
    dev += "/" + std::to_string(prop.multiProcessorCount) + "cu";
  }
  int nmax = 0;
  for (auto& b : p->hblocks) nmax = std::max(nmax, b.n);
  for (char& c : dev)
    if (c == ' ' || c == '|') c = '_';
  return "qax-tune v2 dev=" + dev + " N=" + std::to_string(p->N) + " bodies=" +
         std::to_string(p->n_bodies) + " problems=" + std::to_string(p->n_problems) +
         " nmax=" + std::to_string(nmax) + " nrhs_max=" + std::to_string(nrhs_max) +
         " assembled=" + std::to_string(p->state >= 2 ? 1 : 0);
}

static std::string tune_value(const qax::Tune& t) {
  char buf[512];
  std::snprintf(buf, sizeof(buf),
                "pair_tpb=%d,%d pair_mult=%d,%d pair_nrc=%d,%d,%d,%d;%d,%d,%d,%d gemv_vec=%d,%d "
                "pair_ms=%.6g,%.6g default_ms=%.6g,%.6g sym_s=%d,%d",
                t.pair_tpb[0], t.pair_tpb[1], t.pair_mult[0], t.pair_mult[1], t.pair_nrc[0][0],
                t.pair_nrc[0][1], t.pair_nrc[0][2], t.pair_nrc[0][3], t.pair_nrc[1][0],
                t.pair_nrc[1][1], t.pair_nrc[1][2], t.pair_nrc[1][3], t.gemv_vec[0], t.gemv_vec[1],
                t.pair_ms[0], t.pair_ms[1], t.default_pair_ms[0], t.default_pair_ms[1], t.sym_s[0],
                t.sym_s[1]);
  return buf;
}

static int clamp_nrc(int prec, int tpb, int nrc) {
  while (nrc > 1 && !pair_config_ok(prec, tpb, nrc)) nrc /= 2;
  return nrc;
}

static bool parse_tune(const std::string& v, qax::Tune& t) {
  qax::Tune o;
  const int n = std::sscanf(v.c_str(),
                            "pair_tpb=%d,%d pair_mult=%d,%d pair_nrc=%d,%d,%d,%d;%d,%d,%d,%d "
                            "gemv_vec=%d,%d pair_ms=%lf,%lf default_ms=%lf,%lf sym_s=%d,%d",
                            &o.pair_tpb[0], &o.pair_tpb[1], &o.pair_mult[0], &o.pair_mult[1],
                            &o.pair_nrc[0][0], &o.pair_nrc[0][1], &o.pair_nrc[0][2],
                            &o.pair_nrc[0][3], &o.pair_nrc[1][0], &o.pair_nrc[1][1],
                            &o.pair_nrc[1][2], &o.pair_nrc[1][3], &o.gemv_vec[0], &o.gemv_vec[1],
                            &o.pair_ms[0], &o.pair_ms[1], &o.default_pair_ms[0],
                            &o.default_pair_ms[1], &o.sym_s[0], &o.sym_s[1]);
  if (n != 20) return false;
  for (int pi = 0; pi < 2; ++pi)
    if (o.sym_s[pi] < 0 || o.sym_s[pi] > qax::SYM_SMAX) return false;
  for (int pi = 0; pi < 2; ++pi) {
    const int prec = pi == 0 ? QAX_FP64 : QAX_MIXED;
    if (!pair_config_ok(prec, o.pair_tpb[pi], 1) || o.pair_mult[pi] < 1 || o.pair_mult[pi] > 64)
      return false;
    for (int c = 0; c < 4; ++c) {
      o.pair_nrc[pi][c] = clamp_nrc(prec, o.pair_tpb[pi], o.pair_nrc[pi][c]);
      if (!pair_config_ok(prec, o.pair_tpb[pi], o.pair_nrc[pi][c])) return false;
    }
  }
  if (o.gemv_vec[0] != 1 && o.gemv_vec[0] != 2) return false;
  if (o.gemv_vec[1] != 1 && o.gemv_vec[1] != 2 && o.gemv_vec[1] != 4) return false;
  t = o;
  return true;
}

static std::vector<std::string> read_lines(const char* path) {
  std::vector<std::string> out;
  if (!path) return out;
  FILE* f = std::fopen(path, "r");
  if (!f) return out;
  char buf[2048];
  while (std::fgets(buf, sizeof(buf), f)) {
    std::string s(buf);
    while (!s.empty() && (s.back() == '\n' || s.back() == '\r')) s.pop_back();
    if (!s.empty()) out.push_back(s);
  }
  std::fclose(f);
  return out;
}

}  // namespace

extern "C" qax_status qax_autotune(qax_problem* p, int32_t nrhs_max, const char* cache_path) {
  if (!p) return QAX_ERR_ARG;
  if (p->state < 1) return fail(p, QAX_ERR_STATE, "qax_autotune: call qax_build first");
  if (nrhs_max < 1 || nrhs_max > 1024) return fail(p, QAX_ERR_ARG, "qax_autotune: nrhs_max out of range");
  QCHECK(hipSetDevice(p->device), "hipSetDevice");
  QCHECK(hipStreamSynchronize(p->stream), "sync");
  const int cus = cu_count(p->device);
  const std::string key = tune_key(p, nrhs_max);
  // cached result for this device and problem signature
  std::vector<std::string> lines = read_lines(cache_path);
  for (const std::string& l : lines) {
    const size_t bar = l.find(" | ");
    if (bar == std::string::npos || l.compare(0, bar, key) != 0) continue;
    qax::Tune t;
    if (parse_tune(l.substr(bar + 3), t)) {
      t.tuned = true;
      t.from_cache = true;
      p->tune = t;
      QCHECK(upload_pair_plan(p, QAX_FP64, cus), "pair-sum plan");
      QCHECK(upload_pair_plan(p, QAX_MIXED, cus), "pair-sum plan");
      return QAX_OK;
    }
  }
  const bool was_timing = p->timing;
  p->timing = false;
  // the launch choices concern the direct pair sum: lattice tables off while tuning
  struct LatticeOff {
    qax_problem* q;
    bool on;
    explicit LatticeOff(qax_problem* h) : q(h), on(h->lat.active) { h->lat.active = false; }
    ~LatticeOff() { q->lat.active = on; }
  } lattice_off(p);
  struct SymOn {   // the reciprocal kernel is back on however tuning ends
    qax_problem* q;
    ~SymOn() { q->sym.enabled = true; }
  } sym_on{p};
  QBUF(mu, double, "tune_mu", (size_t)p->N * nrhs_max * 16);
  QBUF(out, double, "tune_out", (size_t)p->N * nrhs_max * 16);
  QCHECK(hipMemsetAsync(mu, 0, (size_t)p->N * nrhs_max * 16, p->stream), "zero");
  qax::Tune t = p->tune;
  const qax::Tune defaults;
  hipError_t err = hipSuccess;
  for (int pi = 0; pi < 2; ++pi) {
    const int prec = pi == 0 ? QAX_FP64 : QAX_MIXED;
    // the per-target kernel's choices are timed with the reciprocal FP32
    // kernel off (it serves one right-hand side whenever it applies)
    p->sym.enabled = false;
    auto run = [&](int nrhs) -> hipError_t {
      qax_status s = QAX_OK;
      double* part = (double*)dbuf(p, "pair_partial", pair_work_bytes(p, prec, nrhs), &s);
      if (!part) return hipErrorOutOfMemory;
      return launch_pair_sum(p, prec, mu, out, nrhs, part, false);
    };
    const int lo[4] = {2, 5, 9, 17}, rep[4] = {4, 8, 16, 64};
    auto nrc_ok = [&](int tpb, int nrc, int c, int nrhs) {
      return pair_config_ok(prec, tpb, nrc) && nrc <= 2 * nrhs && !(c > 0 && nrc < 4);
    };
    double best = 1e300;
    int btpb = t.pair_tpb[pi], bmult = t.pair_mult[pi];
    // one right-hand side with the reciprocal kernel serving every such pair
    // sum: the per-target kernel's choices are never used, nothing to time
    const bool recip_only = nrhs_max == 1 && p->sym.ok && p->form() != 2;
    if (recip_only) {
      btpb = defaults.pair_tpb[pi];
      bmult = defaults.pair_mult[pi];
    } else if (nrhs_max == 1) {
      // workgroup size and source-chunk schedule for one right-hand side
      for (int tpb : {128, 256, 512}) {
        for (int mult : {4, 8, 16}) {
          p->tune.pair_tpb[pi] = tpb;
          p->tune.pair_mult[pi] = mult;
          QCHECK(upload_pair_plan(p, prec, cus), "pair-sum plan");
          const double ms = time_best(p, 2, [&] { return run(1); }, &err);
          QCHECK(err, "autotune pair sum");
          if (ms < best) {
            best = ms;
            btpb = tpb;
            bmult = mult;
          }
        }
      }
    } else {
      // several right-hand sides: workgroup size and right-hand sides per
      // pass together for the largest class, then the schedule
      const int ctop = qax::nrhs_class(nrhs_max), nr = std::min(nrhs_max, rep[ctop]);
      int bn = t.pair_nrc[pi][ctop];
      for (int tpb : {128, 256, 512}) {
        p->tune.pair_tpb[pi] = tpb;
        p->tune.pair_mult[pi] = defaults.pair_mult[pi];
        QCHECK(upload_pair_plan(p, prec, cus), "pair-sum plan");
        for (int nrc : {2, 4, 8, 16, 32}) {
          if (!nrc_ok(tpb, nrc, ctop, nr)) continue;
          p->tune.pair_nrc[pi][ctop] = nrc;
          const double ms = time_best(p, 1, [&] { return run(nr); }, &err, false);
          QCHECK(err, "autotune pair sum (several right-hand sides)");
          if (ms < best) {
            best = ms;
            btpb = tpb;
            bn = nrc;
          }
        }
      }
      p->tune.pair_tpb[pi] = btpb;
      p->tune.pair_nrc[pi][ctop] = t.pair_nrc[pi][ctop] = bn;
      bmult = defaults.pair_mult[pi];
      for (int mult : {4, 16}) {
        p->tune.pair_mult[pi] = mult;
        QCHECK(upload_pair_plan(p, prec, cus), "pair-sum plan");
        const double ms = time_best(p, 1, [&] { return run(nr); }, &err, false);
        QCHECK(err, "autotune pair sum (several right-hand sides)");
        if (ms < best) {
          best = ms;
          bmult = mult;
        }
      }
    }
    p->tune.pair_tpb[pi] = t.pair_tpb[pi] = btpb;
    p->tune.pair_mult[pi] = t.pair_mult[pi] = bmult;
    for (int c = 0; c < 4; ++c)
      p->tune.pair_nrc[pi][c] = t.pair_nrc[pi][c] = clamp_nrc(prec, btpb, t.pair_nrc[pi][c]);
    // single-right-hand-side times of the choice and of the default (report)
    if (recip_only) {
      // the reciprocal kernel: block pairs per super-task side (1, 2, 4, 8;
      // default chosen by the work per compute unit), timed on this problem
      p->tune.pair_tpb[pi] = btpb;
      p->tune.pair_mult[pi] = bmult;
      p->sym.enabled = true;
      const int s_def = sym_default_s(p, cus);
      double best_s = 1e300;
      int bs = s_def;
      for (int sv : {s_def, 1, 2, 4, 8}) {
        if (sv == s_def && best_s < 1e300) continue;
        p->tune.sym_s[pi] = sv;
        QCHECK(upload_pair_plan(p, prec, cus), "pair-sum plan");
        const double ms = time_best(p, 2, [&] { return run(1); }, &err);
        QCHECK(err, "autotune pair sum (reciprocal)");
        if (sv == s_def) t.default_pair_ms[pi] = ms;
        if (ms < best_s) {
          best_s = ms;
          bs = sv;
        }
      }
      p->tune.sym_s[pi] = t.sym_s[pi] = bs;
      QCHECK(upload_pair_plan(p, prec, cus), "pair-sum plan");
      t.pair_ms[pi] = best_s;
    } else {
      p->tune.pair_tpb[pi] = defaults.pair_tpb[pi];
      p->tune.pair_mult[pi] = defaults.pair_mult[pi];
      QCHECK(upload_pair_plan(p, prec, cus), "pair-sum plan");
      t.default_pair_ms[pi] = time_best(p, 2, [&] { return run(1); }, &err);
      QCHECK(err, "autotune pair sum");
      p->tune.pair_tpb[pi] = btpb;
      p->tune.pair_mult[pi] = bmult;
      QCHECK(upload_pair_plan(p, prec, cus), "pair-sum plan");
      p->sym.enabled = true;
      t.pair_ms[pi] = time_best(p, 2, [&] { return run(1); }, &err);
      QCHECK(err, "autotune pair sum");
    }
    // right-hand sides per pass for the other classes that nrhs_max reaches
    for (int c = 0; c < 4; ++c) {
      if (nrhs_max < lo[c] || (nrhs_max > 1 && c == qax::nrhs_class(nrhs_max))) continue;
      const int nrhs = std::min(nrhs_max, rep[c]);
      double bc = 1e300;
      int bn = t.pair_nrc[pi][c];
      for (int nrc : {2, 4, 8, 16, 32}) {
        if (!nrc_ok(btpb, nrc, c, nrhs)) continue;
        p->tune.pair_nrc[pi][c] = nrc;
        const double ms = time_best(p, 1, [&] { return run(nrhs); }, &err, false);
        QCHECK(err, "autotune pair sum (several right-hand sides)");
        if (ms < bc) {
          bc = ms;
          bn = nrc;
        }
      }
      p->tune.pair_nrc[pi][c] = t.pair_nrc[pi][c] = bn;
    }
  }
  // block apply, one right-hand side (after assembly)
  if (p->state >= 2) {
    for (int pi = 0; pi < 2; ++pi) {
      const int prec = pi == 0 ? QAX_FP64 : QAX_MIXED;
      double best = 1e300;
      int bv = t.gemv_vec[pi];
      for (int vec : {1, 2, 4}) {
        if (pi == 0 && vec == 4) continue;
        p->tune.gemv_vec[pi] = vec;
        // FP64: timed on B (same layout and bytes as the FP64 inverse, which
        // may not have been made yet)
        const int inv = prec == QAX_FP64 ? 0 : 1;
        const double ms = time_best(p, 3, [&] { return launch_block_apply(p, inv, prec, mu, out, 1, false); }, &err);
        QCHECK(err, "autotune block apply");
        if (ms < best) {
          best = ms;
          bv = vec;
        }
      }
      p->tune.gemv_vec[pi] = t.gemv_vec[pi] = bv;
    }
  }
  p->timing = was_timing;
  t.tuned = true;
  t.from_cache = false;
  p->tune = t;
  if (cache_path) {
    std::vector<std::string> keep;
    for (const std::string& l : lines)
      if (l.compare(0, key.size() + 3, key + " | ") != 0) keep.push_back(l);
    keep.push_back(key + " | " + tune_value(t));
    FILE* f = std::fopen(cache_path, "w");
    if (f) {
      for (const std::string& l : keep) std::fprintf(f, "%s\n", l.c_str());
      std::fclose(f);
    }
  }
  return sync(p, "qax_autotune");
}

extern "C" qax_status qax_tuning(const qax_problem* pc, qax_tuning_info* out) {
  if (!pc || !out) return QAX_ERR_ARG;
  const qax::Tune& t = pc->tune;
  out->tuned = t.tuned ? 1 : 0;
  out->from_cache = t.from_cache ? 1 : 0;
  for (int pi = 0; pi < 2; ++pi) {
    out->pair_tpb[pi] = t.pair_tpb[pi];
    out->pair_slot_mult[pi] = t.pair_mult[pi];
    for (int c = 0; c < 4; ++c) out->pair_nrc[pi][c] = t.pair_nrc[pi][c];
    out->gemv_vec[pi] = t.gemv_vec[pi];
    out->pair_ms[pi] = t.pair_ms[pi];
    out->default_pair_ms[pi] = t.default_pair_ms[pi];
    out->pair_sym_s[pi] = pc->sym.plan[pi].s;
  }
  return QAX_OK;
}

extern "C" qax_status qax_set_tuning(qax_problem* p, const qax_tuning_info* in) {
  if (!p || !in) return QAX_ERR_ARG;
  if (p->state < 1) return fail(p, QAX_ERR_STATE, "qax_set_tuning: call qax_build first");
  qax::Tune t = p->tune;
  for (int pi = 0; pi < 2; ++pi) {
    const int prec = pi == 0 ? QAX_FP64 : QAX_MIXED;
    if (!pair_config_ok(prec, in->pair_tpb[pi], 1) || in->pair_slot_mult[pi] < 1 ||
        in->pair_slot_mult[pi] > 64)
      return fail(p, QAX_ERR_ARG, "qax_set_tuning: unsupported pair-sum choice");
    for (int c = 0; c < 4; ++c)
      if (!pair_config_ok(prec, in->pair_tpb[pi], in->pair_nrc[pi][c]))
        return fail(p, QAX_ERR_ARG, "qax_set_tuning: unsupported right-hand sides per pass");
    t.pair_tpb[pi] = in->pair_tpb[pi];
    t.pair_mult[pi] = in->pair_slot_mult[pi];
    for (int c = 0; c < 4; ++c) t.pair_nrc[pi][c] = in->pair_nrc[pi][c];
  }
  if ((in->gemv_vec[0] != 1 && in->gemv_vec[0] != 2) ||
      (in->gemv_vec[1] != 1 && in->gemv_vec[1] != 2 && in->gemv_vec[1] != 4))
    return fail(p, QAX_ERR_ARG, "qax_set_tuning: unsupported block-apply choice");
  t.gemv_vec[0] = in->gemv_vec[0];
  t.gemv_vec[1] = in->gemv_vec[1];
  for (int pi = 0; pi < 2; ++pi) {
    if (in->pair_sym_s[pi] < 0 || in->pair_sym_s[pi] > qax::SYM_SMAX)
      return fail(p, QAX_ERR_ARG, "qax_set_tuning: reciprocal super-task size out of [0, 8]");
    t.sym_s[pi] = in->pair_sym_s[pi];
  }
  QCHECK(hipSetDevice(p->device), "hipSetDevice");
  QCHECK(hipStreamSynchronize(p->stream), "sync");
  p->tune = t;
  const int cus = cu_count(p->device);
  QCHECK(upload_pair_plan(p, QAX_FP64, cus), "pair-sum plan");
  QCHECK(upload_pair_plan(p, QAX_MIXED, cus), "pair-sum plan");
  return QAX_OK;
}

// ---------------------------------------------------------------- block GMRES
// One Krylov space for all right-hand sides of a problem (block size p =
// nrhs): block Arnoldi with classical block Gram-Schmidt twice and a
// Cholesky QR done twice for the new block, the block upper Hessenberg
// least-squares problem min ||E1 R0 - Hbar Y|| by Householder reflections on
// the host (one reflection of length p + 1 per column), restarted, right
// preconditioned like the lockstep solver; QAX_MIXED is again FP64 iterative
// refinement around an inner cycle with the FP32 operator.

// G = R^H R for Hermitian G (p x p, row-major); R upper triangular.  False
// when a pivot is not positive beyond the rounding of its column.
static bool chol_upper(const std::vector<cplx>& G, int p, std::vector<cplx>& R) {
  R.assign((size_t)p * p, 0.0);
  for (int j = 0; j < p; ++j) {
    cplx s = G[(size_t)j * p + j];
    for (int k = 0; k < j; ++k) s -= std::conj(R[(size_t)k * p + j]) * R[(size_t)k * p + j];
    const double d = s.real();
    if (!(d > 1e-26 * std::max(G[(size_t)j * p + j].real(), 1e-300))) return false;
    const double r = std::sqrt(d);
    R[(size_t)j * p + j] = r;
    for (int i = j + 1; i < p; ++i) {
      cplx t = G[(size_t)j * p + i];
      for (int k = 0; k < j; ++k) t -= std::conj(R[(size_t)k * p + j]) * R[(size_t)k * p + i];
      R[(size_t)j * p + i] = t / r;
    }
  }
  return true;
}

// Inverse of an upper triangular p x p matrix (row-major).
static std::vector<cplx> inv_upper(const std::vector<cplx>& R, int p) {
  std::vector<cplx> X((size_t)p * p, 0.0);
  for (int c = 0; c < p; ++c) {
    X[(size_t)c * p + c] = 1.0 / R[(size_t)c * p + c];
    for (int r = c - 1; r >= 0; --r) {
      cplx t = 0.0;
      for (int k = r + 1; k <= c; ++k) t += R[(size_t)r * p + k] * X[(size_t)k * p + c];
      X[(size_t)r * p + c] = -t / R[(size_t)r * p + r];
    }
  }
  return X;
}

// Least-squares state of a block GMRES cycle: the block Hessenberg matrix
// (column-major, (m + 1) p rows), the transformed right-hand side E1 R0, and
// one Householder reflection per column acting on rows c .. c + p.
struct BlockLS {
  int p = 0, m = 0, rows = 0;
  std::vector<cplx> H, G, V, tau;
  void init(int p_, int m_, const std::vector<cplx>& R0) {
    p = p_;
    m = m_;
    rows = (m + 1) * p;
    H.assign((size_t)rows * m * p, 0.0);
    G.assign((size_t)rows * p, 0.0);
    V.assign((size_t)m * p * (p + 1), 0.0);
    tau.assign((size_t)m * p, 0.0);
    for (int b = 0; b < p; ++b)
      for (int a = 0; a < p; ++a) G[(size_t)a * rows + b] = R0[(size_t)b * p + a];
  }
  // y <- (I - conj(tau_c) v_c v_c^H) y on rows c .. c + p of a column
  void reflect(int c, cplx* y) const {
    const cplx* v = &V[(size_t)c * (p + 1)];
    cplx w = 0.0;
    for (int t = 0; t <= p; ++t) w += std::conj(v[t]) * y[c + t];
    w *= std::conj(tau[c]);
    for (int t = 0; t <= p; ++t) y[c + t] -= w * v[t];
  }
  // block column j from blocks hblk[i][b][a] (i <= j + 1); res: residual
  // norm of every right-hand side after the step
  void add_column(int j, const std::vector<cplx>& hblk, std::vector<double>& res) {
    for (int a = 0; a < p; ++a) {
      cplx* col = &H[(size_t)(j * p + a) * rows];
      for (int r = 0; r < (j + 2) * p; ++r) col[r] = hblk[(size_t)(r / p) * p * p + (size_t)(r % p) * p + a];
      for (int c = 0; c < j * p; ++c) reflect(c, col);
    }
    for (int a = 0; a < p; ++a) {
      const int c = j * p + a;
      cplx* col = &H[(size_t)c * rows];
      // reflection with (I - tau v v^H)^H (alpha, x) = (beta, 0), beta real
      const cplx alpha = col[c];
      double xn2 = 0.0;
      for (int t = 1; t <= p; ++t) xn2 += std::norm(col[c + t]);
      cplx* v = &V[(size_t)c * (p + 1)];
      v[0] = 1.0;
      if (xn2 == 0.0 && alpha.imag() == 0.0) {
        tau[c] = 0.0;
        for (int t = 1; t <= p; ++t) v[t] = 0.0;
      } else {
        const double beta = -std::copysign(std::sqrt(std::norm(alpha) + xn2), alpha.real());
        tau[c] = (beta - alpha) / beta;
        const cplx scl = 1.0 / (alpha - beta);
        for (int t = 1; t <= p; ++t) v[t] = col[c + t] * scl;
        col[c] = beta;
        for (int t = 1; t <= p; ++t) col[c + t] = 0.0;
      }
      for (int a2 = a + 1; a2 < p; ++a2) reflect(c, &H[(size_t)(j * p + a2) * rows]);
      for (int r = 0; r < p; ++r) reflect(c, &G[(size_t)r * rows]);
    }
    res.assign(p, 0.0);
    for (int r = 0; r < p; ++r) {
      double s2 = 0.0;
      for (int t = 0; t < p; ++t) s2 += std::norm(G[(size_t)r * rows + (j + 1) * p + t]);
      res[r] = std::sqrt(s2);
    }
  }
  // Y (k p x p, row-major) = T^-1 G[0 .. k p) with T the leading triangle
  void solve(int k, std::vector<cplx>& Y) const {
    const int n = k * p;
    Y.assign((size_t)n * p, 0.0);
    for (int r = 0; r < p; ++r) {
      for (int i = n - 1; i >= 0; --i) {
        cplx t = G[(size_t)r * rows + i];
        for (int c = i + 1; c < n; ++c) t -= H[(size_t)c * rows + i] * Y[(size_t)c * p + r];
        Y[(size_t)i * p + r] = t / H[(size_t)i * rows + i];
      }
    }
  }
};

static qax_status solve_block(qax_problem* p, qax_prec prec, const double* dirs, const double* d_rhs,
                              int32_t nrhs, double tol, int32_t maxit, void* d_mu_out, qax_info* info) {
  qax_status st = check_vec_call(p, dirs ? (const void*)dirs : (const void*)d_rhs, d_mu_out, nrhs, 2);
  if (st != QAX_OK) return st;
  if (prec != QAX_FP64 && prec != QAX_MIXED) return fail(p, QAX_ERR_ARG, "bad precision");
  if (!(tol > 0) || !is_finite(tol) || maxit < 1) return fail(p, QAX_ERR_ARG, "qax_solve: bad tol / maxit");
  if (p->n_problems != 1) return fail(p, QAX_ERR_ARG, "block GMRES solves one problem per handle");
  if (nrhs > 64) return fail(p, QAX_ERR_ARG, "block GMRES takes at most 64 right-hand sides");
  QCHECK(hipSetDevice(p->device), "hipSetDevice");
  QCHECK(hipStreamSynchronize(p->stream), "sync");
  if (prec == QAX_FP64 && (st = ensure_inverse64(p)) != QAX_OK) return st;
  auto t0 = std::chrono::steady_clock::now();
  const int P = nrhs;
  const int64_t N = p->N;
  const int64_t vs = N * P * 2;   // doubles per block
  const int m = std::min<int>(maxit, 40);
  Krylov K;
  st = setup_krylov(p, P, m, K);
  if (st != QAX_OK) return st;
  QBUF(V, double, "bk_V", (size_t)(m + 1) * vs * 8);
  QBUF(W, double, "kry_w", (size_t)vs * 8);
  QBUF(T, double, "kry_t", (size_t)vs * 8);
  QBUF(R, double, "kry_r", (size_t)vs * 8);
  QBUF(B, double, "kry_b", (size_t)vs * 8);
  QBUF(hd, double, "bk_h", (size_t)(m + 1) * P * P * 16);
  QBUF(cd, double, "bk_c", (size_t)(m + 1) * P * P * 16);
  QBUF(dpart, double, "bk_dots", block_dots_work_bytes(N, m + 1));
  const int inner_prec = prec;
  QBUF(ppart, double, "pair_partial",
       std::max(pair_work_bytes(p, inner_prec, P), pair_work_bytes(p, QAX_FP64, P)));
  double* X = (double*)d_mu_out;
  if (dirs) {
    double* dd = nullptr;
    st = upload_dirs(p, dirs, P, &dd);
    if (st != QAX_OK) return st;
    QCHECK(launch_rhs(p, dd, P, B), "rhs");
  } else {
    QCHECK(hipMemcpyAsync(B, d_rhs, (size_t)vs * 8, hipMemcpyDeviceToDevice, p->stream), "copy rhs");
  }
  QCHECK(hipMemsetAsync(X, 0, (size_t)vs * 8, p->stream), "zero x");
  std::vector<cplx> hh((size_t)(m + 1) * P * P);
  // Gram matrix of a block (or nb blocks against w) to the host
  auto gram = [&](const double* Vb, int nb, const double* w) -> qax_status {
    QCHECK(launch_block_dots(p->stream, Vb, vs, nb, w, N, P, dpart, hd), "block dots");
    QCHECK(hipMemcpyAsync(hh.data(), hd, (size_t)nb * P * P * 16, hipMemcpyDeviceToHost, p->stream),
           "copy h");
    return sync(p, "block gmres");
  };
  auto upload_c = [&](const std::vector<cplx>& c) -> qax_status {
    QCHECK(hipMemcpyAsync(cd, c.data(), c.size() * 16, hipMemcpyHostToDevice, p->stream), "copy c");
    return QAX_OK;
  };
  // Cholesky QR twice: src (N x P) = dst Rq, dst orthonormal; false on
  // numerical rank deficiency
  std::vector<cplx> Gm, R1, R2, Rq;
  auto cholqr2 = [&](const double* src, double* dst, bool* ok) -> qax_status {
    *ok = false;
    qax_status s2 = gram(src, 1, src);
    if (s2 != QAX_OK) return s2;
    Gm.assign(hh.begin(), hh.begin() + (size_t)P * P);
    if (!chol_upper(Gm, P, R1)) return QAX_OK;
    if ((s2 = upload_c(inv_upper(R1, P))) != QAX_OK) return s2;
    QCHECK(launch_block_update(p->stream, src, vs, 1, cd, P, N, 1.0, 0.0, nullptr, T), "block update");
    if ((s2 = gram(T, 1, T)) != QAX_OK) return s2;
    Gm.assign(hh.begin(), hh.begin() + (size_t)P * P);
    if (!chol_upper(Gm, P, R2)) return QAX_OK;
    if ((s2 = upload_c(inv_upper(R2, P))) != QAX_OK) return s2;
    QCHECK(launch_block_update(p->stream, T, vs, 1, cd, P, N, 1.0, 0.0, nullptr, dst), "block update");
    Rq.assign((size_t)P * P, 0.0);
    for (int r = 0; r < P; ++r)
      for (int c = r; c < P; ++c) {
        cplx t = 0.0;
        for (int k = r; k <= c; ++k) t += R2[(size_t)r * P + k] * R1[(size_t)k * P + c];
        Rq[(size_t)r * P + c] = t;
      }
    *ok = true;
    return QAX_OK;
  };

  std::vector<double> bn(P), rn(P), need(P), res;
  if ((st = gram(B, 1, B)) != QAX_OK) return st;
  for (int c = 0; c < P; ++c) bn[c] = std::sqrt(std::max(hh[(size_t)c * P + c].real(), 0.0));
  int total_its = 0, outer = 0;
  double relres = 1.0;
  qax_status result = QAX_ERR_NOCONV;
  BlockLS ls;
  std::vector<cplx> hblk, Y;
  while (true) {
    if (outer == 0) {
      QCHECK(hipMemcpyAsync(R, B, (size_t)vs * 8, hipMemcpyDeviceToDevice, p->stream), "copy");
    } else {
      st = apply_full(p, QAX_FP64, X, W, P);
      if (st != QAX_OK) return st;
      K.axpby(1.0, B, -1.0, W, R);
    }
    if ((st = gram(R, 1, R)) != QAX_OK) return st;
    relres = 0.0;
    bool done = true;
    for (int c = 0; c < P; ++c) {
      rn[c] = std::sqrt(std::max(hh[(size_t)c * P + c].real(), 0.0));
      const double rel = bn[c] > 0 ? rn[c] / bn[c] : 0.0;
      relres = std::max(relres, rel);
      done = done && rel <= tol;
    }
    if (done) {
      result = QAX_OK;
      break;
    }
    if (total_its >= maxit) break;
    const double floor32 = mixed_cycle_floor(p);
    for (int c = 0; c < P; ++c) {
      const double nd = rn[c] > 0 ? 0.5 * tol * bn[c] / rn[c] : 1.0;
      need[c] = prec == QAX_MIXED ? std::max(nd, floor32) : nd;
    }
    bool ok = false;
    if ((st = cholqr2(R, V, &ok)) != QAX_OK) return st;
    if (!ok) return fail(p, QAX_ERR_NOCONV, "block GMRES: residual block of numerically deficient rank");
    ls.init(P, m, Rq);
    int k = 0;
    for (int j = 0; j < m && total_its < maxit; ++j) {
      double* Vj = V + (size_t)j * vs;
      QCHECK(launch_block_apply(p, 1, inner_prec, Vj, T, P, false), "block apply");
      QCHECK(launch_pair_sum(p, inner_prec, T, W, P, ppart, false), "pair sum");
      K.axpby(1.0, W, 1.0, Vj, W);
      // block Gram-Schmidt twice against V_0 .. V_j
      hblk.assign((size_t)(j + 2) * P * P, 0.0);
      for (int pass = 0; pass < 2; ++pass) {
        if ((st = gram(V, j + 1, W)) != QAX_OK) return st;
        for (size_t e = 0; e < (size_t)(j + 1) * P * P; ++e) hblk[e] += hh[e];
        QCHECK(launch_block_update(p->stream, V, vs, j + 1, hd, P, N, -1.0, 1.0, W, W), "block update");
      }
      ++total_its;
      k = j + 1;
      bool okq = false;
      if ((st = cholqr2(W, V + (size_t)(j + 1) * vs, &okq)) != QAX_OK) return st;
      if (okq)
        for (int r = 0; r < P; ++r)
          for (int c = 0; c < P; ++c) hblk[(size_t)(j + 1) * P * P + (size_t)r * P + c] = Rq[(size_t)r * P + c];
      ls.add_column(j, hblk, res);
      bool conv = true;
      for (int c = 0; c < P; ++c) conv = conv && res[c] <= need[c] * rn[c];
      if (conv || !okq) break;   // converged, or the new block is in the span
    }
    // d = M^-1 V Y;  x += d
    ls.solve(k, Y);
    if ((st = upload_c(Y)) != QAX_OK) return st;
    QCHECK(launch_block_update(p->stream, V, vs, k, cd, P, N, 1.0, 0.0, nullptr, T), "block combine");
    QCHECK(launch_block_apply(p, 1, inner_prec, T, X, P, true), "precond");
    ++outer;
  }
  if ((st = sync(p, "qax_solve")) != QAX_OK) return st;
  auto t1 = std::chrono::steady_clock::now();
  if (info) {
    info->iters = total_its;
    info->outer_iters = outer;
    info->rel_res = relres;
    info->t_setup_s = 0.0;
    info->t_solve_s = std::chrono::duration<double>(t1 - t0).count();
  }
  if (result != QAX_OK)
    return fail(p, QAX_ERR_NOCONV, "qax_solve: tolerance not reached within maxit iterations");
  return QAX_OK;
}

extern "C" qax_status qax_set_solver(qax_problem* p, int32_t solver) {
  if (!p) return QAX_ERR_ARG;
  if (solver != QAX_SOLVER_LOCKSTEP && solver != QAX_SOLVER_BLOCK)
    return fail(p, QAX_ERR_ARG, "qax_set_solver: QAX_SOLVER_LOCKSTEP or QAX_SOLVER_BLOCK");
  p->solver = solver;
  return QAX_OK;
}

extern "C" qax_status qax_solve(qax_problem* p, qax_prec prec, const double* dirs, int32_t nrhs,
                                double tol, int32_t maxit, void* d_mu_out, qax_info* info) {
  if (!p) return QAX_ERR_ARG;
  if (!dirs) return fail(p, QAX_ERR_ARG, "qax_solve: null directions");
  if (p->solver == QAX_SOLVER_BLOCK && nrhs > 1)
    return solve_block(p, prec, dirs, nullptr, nrhs, tol, maxit, d_mu_out, info);
  return solve_core(p, prec, dirs, nullptr, nrhs, tol, maxit, d_mu_out, info);
}

extern "C" qax_status qax_solve_rhs(qax_problem* p, qax_prec prec, const void* d_rhs, int32_t nrhs,
                                    double tol, int32_t maxit, void* d_mu_out, qax_info* info) {
  if (!p) return QAX_ERR_ARG;
  if (!d_rhs) return fail(p, QAX_ERR_ARG, "qax_solve_rhs: null right-hand side");
  if (d_rhs == d_mu_out) return fail(p, QAX_ERR_ARG, "qax_solve_rhs: rhs and solution must not alias");
  if (p->solver == QAX_SOLVER_BLOCK && nrhs > 1)
    return solve_block(p, prec, nullptr, (const double*)d_rhs, nrhs, tol, maxit, d_mu_out, info);
  return solve_core(p, prec, nullptr, (const double*)d_rhs, nrhs, tol, maxit, d_mu_out, info);
}
