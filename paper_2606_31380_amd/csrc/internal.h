// Internal declarations shared by the HIP translation units of libqax.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <map>
#include <string>
#include <vector>

#include "../../include/qax.h"

namespace qax {

constexpr int GL_ORDER = 16;
constexpr double PI = 3.14159265358979323846;
constexpr double TWO_PI = 6.28318530717958647692;
constexpr double FOUR_PI = 12.5663706143591729539;

// Per-body record on the device.
struct BodyDev {
  int32_t shape, n_panels, n_theta, problem;   // n_panels: after refinement
  int32_t n_uni, n_ref;                        // uniform panels, refinements per pole
  int64_t off;        // first node
  int32_t n;          // nodes
  int32_t block;      // distinct self-block index
  double a, c, kappa;
  double R[9];        // rotation, row-major
  double cen[3];
  double k;           // wavenumber of the body's problem
  double eta;         // combined-field coupling (0: double layer only)
};

// Distinct self block.
struct BlockDev {
  int32_t rep_body;   // representative body (its shape parameters)
  int32_t n;          // order
  int64_t elem_off;   // offset (in complex elements) in the block pools
};

// A chunk of pair-sum work: targets [t0, t1) against source bodies
// [b0, b1) of the same problem, writing partial slot `slot`.
struct PairTask {
  int64_t t0;
  int32_t nt;
  int32_t b0, b1;
  int32_t slot;
  int32_t tbody_lo, tbody_hi;  // bodies spanned by the targets
  double k;
  double eta;                  // combined-field coupling of the problem (0: none)
};

// Reciprocal pair sums (one right-hand side): each problem's node range is
// cut into blocks of SYM_T consecutive nodes (a block may straddle bodies); a
// super-task is a square of up to SYM_SMAX x SYM_SMAX block pairs (I, J),
// I <= J, of one problem, evaluated by one workgroup.  Its target-side sums go
// to ni slots from part[toff], its source-side sums to nj slots from
// part[soff] (SYM_T complex128 values per slot).
constexpr int SYM_T = 256;
constexpr int SYM_SMAX = 8;
// largest workspace of one launch of the reciprocal kernels, complex128
// values (960 MB; twice as many complex64 slots of the FP32 kernel); more
// super-tasks are split into several launches
constexpr int64_t SYM_SLOT_CAP = 60000000;
struct SymBlock {
  int64_t n0;          // first node
  int32_t n;           // nodes, 1 .. SYM_T
  int32_t problem;
};
struct SymSuper {
  int32_t i0, ni, j0, nj;  // block rows [i0, i0 + ni) x columns [j0, j0 + nj)
  int32_t diag;            // rows == columns: block pairs with J >= I only
  int32_t problem;
  double k;
  uint64_t skip;           // bit ii * SYM_SMAX + jj: both blocks inside one body
  int64_t toff, soff;      // first target / source slot
};

// Row tile of the several-RHS block apply: 64 rows of one body from row0.
struct GemmTask {
  int32_t body;
  int32_t row0;
};

// One right-hand side through the symmetry-reduced inverses (every block
// mirror-symmetric): segment c of a body, the rows of its reduced inverse
// M_c^-1 (order n) applied to the segment of the reduced vector at voff.
struct SymSeg {
  int64_t voff;      // first entry of the segment in the reduced vectors (node offset of the body + start)
  int64_t moff;      // complex offset of M_c^-1 in the reduced pools
  int32_t n;         // order
  int32_t problem;
};
// A symmetric body for the vector transforms.
struct SymBody {
  int64_t off;       // first node
  int32_t ns, nth;   // Gauss-Legendre nodes along the curve, azimuths
  int32_t problem;
};

// Work item of the self-block assembly: one target row x one near panel.
struct SelfTask {
  int32_t block;   // distinct block
  int32_t row;     // target row within the block
  int32_t panel;   // source panel
};

}  // namespace qax

namespace qax {
// Launch choices of the tunable kernels (defaults until qax_autotune runs).
// Index 0: FP64 pair sum / FP64 blocks, 1: FP32 pair sum / FP32 inverse copy.
struct Tune {
  int pair_tpb[2] = {256, 256};    // targets per workgroup (= source tile in LDS)
  int pair_mult[2] = {8, 8};       // workgroups per CU aimed at by the source-chunk split
  int pair_nrc[2][4] = {{4, 8, 8, 8}, {4, 8, 16, 16}};  // RHS per pass, nrhs in 2-4, 5-8, 9-16, >16
  int gemv_vec[2] = {1, 1};        // complex elements per lane and load, one RHS
  int sym_s[2] = {0, 0};           // reciprocal pair sum: block pairs per super-task side (0: default)
  bool tuned = false, from_cache = false;
  double pair_ms[2] = {0.0, 0.0}, default_pair_ms[2] = {0.0, 0.0};
};
inline int nrhs_class(int nrhs) { return nrhs <= 4 ? 0 : nrhs <= 8 ? 1 : nrhs <= 16 ? 2 : 3; }
}  // namespace qax

struct qax_problem {
  int device = 0;
  hipStream_t stream = nullptr;
  std::string err;
  int state = 0;  // 0 created, 1 built, 2 assembled
  int formulation = QAX_DOUBLE_LAYER;
  double eta_param = 0.0;          // > 0 fixed coupling, <= 0 k of each problem
  // per-node single-layer weight factor: eta (combined field), 1 (single layer), 0
  double eta_of(double k) const {
    if (formulation == QAX_SINGLE_LAYER) return 1.0;
    return formulation == QAX_COMBINED_FIELD ? (eta_param > 0 ? eta_param : k) : 0.0;
  }
  // kernel variant: 0 double layer, 1 combined field, 2 single layer
  int form() const { return formulation == QAX_COMBINED_FIELD ? 1 : formulation == QAX_SINGLE_LAYER ? 2 : 0; }

  int32_t n_bodies = 0, n_problems = 0;
  std::vector<qax_body> bodies;
  std::vector<double> k;
  std::vector<int64_t> off;           // n_bodies + 1
  std::vector<int64_t> prob_body0;    // n_problems + 1 (body index range)
  std::vector<qax::BodyDev> hbodies;
  std::vector<qax::BlockDev> hblocks;
  int64_t N = 0;
  int64_t block_elems = 0;            // sum of n^2 over distinct blocks

  // device buffers released by a rebuild, kept for the next allocation of
  // the same size (freed by qax_destroy, or when an allocation fails)
  std::multimap<size_t, void*> spare;
  std::map<void*, size_t> live;
  // pinned host staging for uploads of call arguments (grow-only; every call
  // that uses it synchronises before returning)
  void* h_stage = nullptr;
  size_t h_stage_bytes = 0;

  // device geometry
  qax::BodyDev* d_bodies = nullptr;
  qax::BlockDev* d_blocks = nullptr;
  int32_t* d_node_body = nullptr;
  double* d_pos = nullptr;      // SoA: x[N], y[N], z[N]
  double* d_aw = nullptr;       // SoA
  float* d_loc32 = nullptr;     // float4 per node: local offset from the body centre, |y'|^2
  float* d_aw32 = nullptr;      // float4 per node: aw, aw . (local offset)
  double* d_ew = nullptr;       // per node eta |aw| (combined field; 0 otherwise)
  float* d_ew32 = nullptr;
  double* d_gl = nullptr;       // 16 GL nodes, weights, barycentric weights on [-1, 1]
  int64_t* d_pinfo = nullptr;   // problems' first nodes (n_problems + 1), then their k (as bits)

  // self blocks (complex128 / complex64 pools)
  double* d_B = nullptr;
  double* d_Binv = nullptr;
  bool inv64_ready = false;     // d_Binv holds the inverse of the current blocks
  // precision of the factorisation made by qax_assemble_self: QAX_FP64 (the
  // FP64 inverse, rounded to FP32 for the mixed path) or QAX_MIXED (B rounded
  // to FP32 and inverted in FP32; the FP64 inverse made on first use)
  int factor_prec = QAX_FP64;
  int solver = QAX_SOLVER_LOCKSTEP;   // several right-hand sides: lockstep or block GMRES
  float* d_Binv32 = nullptr;
  float* d_B32 = nullptr;       // B rounded to FP32 (the mixed path's operator blocks)
  bool b32_ready = false;       // d_B32 holds the current blocks (rounded on first use after an FP64 factorisation)
  // every block mirror-symmetric: the inverses also as their four reduced
  // blocks (complex128 valid with inv64_ready, complex64 after every
  // assembly), and the tables of the one-right-hand-side apply through them
  struct SymApply {
    bool on = false;
    double* d_Minv = nullptr;
    float* d_Minv32 = nullptr;
    int64_t elems = 0;                 // complex entries of the reduced pools
    void* d_mem = nullptr;             // the tables and the reduced vectors
    qax::SymSeg* d_segs = nullptr;
    int2* d_groups = nullptr;          // (segment, first row) of 16-row groups
    qax::SymBody* d_bodies = nullptr;
    double* d_u = nullptr;             // reduced input vector (N complex)
    double* d_w = nullptr;             // reduced output vector (N complex)
    int n_groups = 0, n_bodies = 0;
  } symap;

  // pair-sum task tables per precision
  std::vector<qax::PairTask> tasks64, tasks32;
  qax::PairTask* d_tasks64 = nullptr;
  qax::PairTask* d_tasks32 = nullptr;
  int32_t slots64 = 1, slots32 = 1;
  int32_t plan_tpb[2] = {0, 0};       // workgroup size the task tables were planned for
  // reciprocal pair sums (one right-hand side, k > 0 in every problem,
  // double layer or combined field): node blocks, and per precision the
  // super-tasks, their launches and the per-launch reduction lists
  struct Sym {
    bool ok = false;                  // every problem has k > 0
    bool enabled = true;              // off while the per-target kernel is tuned
    std::vector<qax::SymBlock> blocks;
    std::vector<int32_t> prob_blk0;   // first block of each problem (n_problems + 1)
    std::vector<int32_t> blk_body_lo, blk_body_hi;
    std::vector<int64_t> key;         // node ranges, problem bounds and k the plans were made for
    void* d_bmem = nullptr;           // blocks and the block of each node
    qax::SymBlock* d_blocks = nullptr;
    int32_t* d_node_block = nullptr;
    struct Plan {
      int s = 0;                      // super-task size (block pairs per side)
      std::vector<qax::SymSuper> supers;
      std::vector<int64_t> launch_super;   // super-task range of each launch
      std::vector<int64_t> lptr;           // per launch: n_blocks + 1 list offsets
      std::vector<int64_t> list;           // slot offsets
      int64_t max_slots = 0;               // complex values of the largest launch
      void* d_mem = nullptr;
      qax::SymSuper* d_supers = nullptr;
      int64_t* d_lptr = nullptr;
      int64_t* d_list = nullptr;
    } plan[2];                        // [0] FP64, [1] FP32
  } sym;
  qax::Tune tune;

  // block-Toeplitz apply of the inter-body sum on a regular array of
  // identical bodies (tables per frequency of the circulant embedding)
  struct Lattice {
    bool active = false;
    int dims[3] = {1, 1, 1};            // P, Q, R
    int L[3] = {1, 1, 1};               // 2P - 1, 2Q - 1, 2R - 1
    int64_t F = 0;                      // L0 L1 L2 frequencies
    int nb = 0;                         // nodes per body
    double* T64 = nullptr;              // F x nb x nb complex128
    float* T32 = nullptr;               // complex64 copy
    qax::BodyDev* d_fbodies = nullptr;  // one "body" per frequency (batched products)
    qax::BlockDev* d_fblocks = nullptr;
    int32_t* d_frow = nullptr;          // row -> frequency
    qax::GemmTask* d_ftasks = nullptr;
    int nftasks = 0;
    int64_t* d_site_node = nullptr;     // first node of the body at each site
  } lat;

  // block GEMM row tiles (several right-hand sides)
  std::vector<qax::GemmTask> gemm_tasks;
  void* d_gemm_tasks = nullptr;
  // scratch
  void* d_scratch = nullptr;
  size_t scratch_bytes = 0;

  // captured GMRES steps: one executable graph per Arnoldi step index, valid
  // while `graph_key` (buffers, sizes, launch choices) is unchanged
  bool use_graphs = true;
  const int32_t* seg_active = nullptr;  // set while a lockstep solve enqueues its steps
  uint64_t generation = 0;            // bumped by build, assembly and tuning changes
  std::string graph_key;
  std::vector<hipGraphExec_t> graphs;
  hipStream_t cap_stream = nullptr;   // the handle's own stream for captures
  int32_t* h_flags = nullptr;         // pinned host copies of the per-step counters
  int h_flags_n = 0;

  // kernel timing
  bool timing = false;
  struct Pending {
    int kind;
    hipEvent_t a, b;
  };
  std::vector<Pending> pending;
  std::vector<hipEvent_t> event_pool;
  int64_t t_launches[QAX_K_COUNT] = {0};
  double t_ms[QAX_K_COUNT] = {0};
};

namespace qax {

// timing: begin/end bracket a launch of kernel `kind` on p->stream;
// collect_timing() folds completed brackets into the counters (call after a
// stream synchronisation).
void timing_begin(qax_problem* p, int kind);
void timing_end(qax_problem* p, int kind);
void collect_timing(qax_problem* p);

// error helpers
qax_status fail(qax_problem* p, qax_status s, const std::string& msg);
qax_status hip_check(qax_problem* p, hipError_t e, const char* what);
void* scratch(qax_problem* p, size_t bytes, qax_status* st);

// geometry.hip
void gauss_legendre_host(int n, double* x, double* w);
hipError_t launch_build_nodes(qax_problem* p);
hipError_t launch_node_weights(qax_problem* p);

// lattice.hip
void lattice_free(qax_problem* p);
qax_status lattice_enable(qax_problem* p, int32_t* dims);
hipError_t launch_lattice_apply(qax_problem* p, int prec, const double* mu, double* out, int nrhs,
                                double* work, bool accumulate);
size_t lattice_work_bytes(const qax_problem* p, int nrhs);

// dense.hip: block-diagonal products over explicit tables
hipError_t launch_gemv_tables(hipStream_t s, const BodyDev* bodies, const BlockDev* blocks,
                              const int32_t* node_body, const void* pool, bool f32, int64_t rows,
                              int order, const double* v, int nrhs, double* out, bool accumulate);
hipError_t launch_gemm_tables(hipStream_t s, const GemmTask* tasks, int ntasks,
                              const BodyDev* bodies, const BlockDev* blocks, const void* pool,
                              bool f32, const double* v, int nrhs, double* out, bool accumulate);

// pairsum.hip
// Device allocation through the handle's cache of released buffers.
hipError_t dev_alloc(qax_problem* p, void** ptr, size_t bytes);
void dev_release(qax_problem* p, void* ptr);
void dev_drop_spare(qax_problem* p);
size_t pair_work_bytes(const qax_problem* p, int prec, int nrhs);
hipError_t launch_pair_sum(qax_problem* p, int prec, const double* mu, double* out, int nrhs,
                           double* partial, bool accumulate);
void plan_pair_sum(qax_problem* p, int prec, int cu_count);
// plan_pair_sum + device copy of the task table (synchronous).
hipError_t upload_pair_plan(qax_problem* p, int prec, int cu_count);
// reciprocal pair sums: plan for precision index pi (0 FP64, 1 FP32) with
// super-tasks of s x s block pairs (s <= 0: the default for this problem)
hipError_t plan_sym(qax_problem* p, int pi, int s, int cu_count);
hipError_t release_sym_plan(qax_problem* p, int pi);
int sym_default_s(const qax_problem* p, int cu_count);
// launch choices the kernels support (LDS within 64 KB)
bool pair_config_ok(int prec, int tpb, int nrc);
int nearfield_slots(int64_t M, int cu_count);
hipError_t launch_nearfield(qax_problem* p, const double* mu, int nrhs, const double* pts, int64_t M,
                            int problem, int slots, double* partial, double* u);
hipError_t ensure_gemm_tasks(qax_problem* p);

// dense.hip
hipError_t launch_block_apply(qax_problem* p, int inverse, int prec, const double* v, double* out,
                              int nrhs, bool accumulate);
hipError_t launch_invert_blocks(qax_problem* p, double* work);     // FP32 inverse (mixed path)
hipError_t launch_invert_blocks64(qax_problem* p, double* work);   // FP64 inverse
hipError_t launch_factor_blocks64(qax_problem* p, double* work);   // FP64 inverse + FP32 roundings
// every block mirror-symmetric: reduced inverses and the one-right-hand-side
// apply through them (no-op otherwise); freed with the geometry
hipError_t setup_sym_apply(qax_problem* p);
void free_sym_apply(qax_problem* p);
hipError_t launch_convert_f32(hipStream_t s, const double* src, float* dst, int64_t count);
hipError_t launch_dense_offdiag(qax_problem* p, double* A);

// selfblock.hip
hipError_t launch_assemble_self(qax_problem* p);
hipError_t launch_modal_modes(hipStream_t s, int n, const double* r, const double* rt,
                              const double* c, const double* chim1, const double* rmrt, double k,
                              int nmax, double* A, double* B);

// krylov.hip
hipError_t launch_rhs(qax_problem* p, const double* dirs_dev, int nrhs, double* out);
int farfield_slots(int64_t M, int cu_count);
// block GMRES products over N x p blocks (p <= 64, node-major, columns
// fastest; vstride: doubles between consecutive blocks):
// out[i][b][a] = sum_n conj(V_i[n][b]) W[n][a] for i < nb (partial:
// block_dots_work_bytes(N, nb)), and
// out = beta base + alpha sum_i V_i C_i (C: nb x p x p, row-major p x p each)
size_t block_dots_work_bytes(int64_t N, int nb_max);
hipError_t launch_block_dots(hipStream_t s, const double* V, int64_t vstride, int nb, const double* W,
                             int64_t N, int p, double* partial, double* out);
hipError_t launch_block_update(hipStream_t s, const double* V, int64_t vstride, int nb, const double* C,
                               int p, int64_t N, double alpha, double beta, const double* base,
                               double* out);
// the far field's allocation-free workspace: its device address on `device`
// (current), taken once per device
hipError_t noalloc_init(int device);
hipError_t launch_farfield(qax_problem* p, const double* mu, int nrhs, const double* xhat_dev,
                           int ndir, const int2* items_dev, int nitems, const int64_t* pinfo_dev,
                           int slots, double* partial, double* out);

}  // namespace qax
