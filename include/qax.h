/*
 * qax.h -- C interface of the MI355X (gfx950) multi-body Helmholtz
 * double-layer Nystrom solver.
 *
 * The operator is the second-kind double-layer equation for sound-soft
 * scattering by many quasi-axisymmetric bodies,
 *     (1/2 I + D) mu = -u_inc,                                  (Section 4)
 * with diagonal (self) blocks built by product integration over modal Green's
 * functions (Sections 3.1-3.4) and off-diagonal (inter-body) blocks applied
 * on the fly as a smooth Gauss-Legendre x trapezoidal pair sum (Section 4).
 *
 * Conventions shared by every call
 *  - Every call returns a qax_status; QAX_OK (0) on success.  No C++ exception
 *    and no abort crosses this interface.  On failure qax_last_error() holds a
 *    message.
 *  - Complex arrays are interleaved (re, im) pairs: complex128 = two doubles,
 *    complex64 = two floats (the memory of torch.complex128 / complex64).
 *  - Arrays of unknowns are node-major with right-hand sides fastest: element
 *    (node i, rhs r) is at index i * nrhs + r.  Node order is body, then panel,
 *    then Gauss-Legendre index, then azimuthal index (azimuth fastest).
 *  - Pointers named d_* are DEVICE pointers on the handle's device; all other
 *    pointers are host pointers.  The caller owns every buffer it passes in;
 *    the library owns the device memory it allocates until qax_destroy().
 *  - Work is enqueued on the stream given to qax_create; each call returns
 *    after that stream has completed the call's work.
 *  - Call order: qax_build -> qax_assemble_self -> apply / solve / far field.
 *    Calls out of order return QAX_ERR_STATE.
 *  - One handle per host thread; handles are independent.
 */
#ifndef QAX_H
#define QAX_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct qax_problem qax_problem;

typedef enum {
  QAX_OK = 0,
  QAX_ERR_ARG = 1,     /* invalid argument (sizes, NaN/Inf, null pointers)   */
  QAX_ERR_DEVICE = 2,  /* HIP runtime error                                   */
  QAX_ERR_NOMEM = 3,   /* device allocation failed                            */
  QAX_ERR_NOCONV = 4,  /* iterative solver did not reach the tolerance        */
  QAX_ERR_STATE = 5    /* call out of order                                   */
} qax_status;

typedef enum {
  QAX_FP64 = 0,   /* every step in FP64                                        */
  QAX_MIXED = 1   /* inter-body pair sum in FP32 with compensated accumulation,
                     self blocks and their inverses applied from FP32 copies,
                     inside FP64 iterative refinement                          */
} qax_prec;

typedef enum {
  QAX_SPHERE = 0,   /* r = a cos t, z = a sin t                               */
  QAX_SPHEROID = 1, /* r = a cos t, z = c sin t                               */
  QAX_PEANUT = 2,   /* polar radius a (1 + c cos 2 psi), psi = polar angle     */
  /* The geometries of Section 6.1, Example 2, scaled by a (c unused, kappa 0): */
  QAX_QUASI_ELLIPSOID = 3, /* r = 2a cos t, z = 3a sin t, p = a cos t, q = 0 */
  QAX_SPIRAL = 4,   /* r = 1.5a cos t, z = 2a sin t, p = 0.05a cos 4 pi t,
                       q = 0.1a sin 4 pi t                                     */
  QAX_CONCH = 5     /* r = a cos t, z = 1.5a sin t, p = a f cos t, q = a f sin t,
                       f = 0.2 + 0.1 sin 8t                                    */
} qax_shape;

/* One body.  Generating curve over t in [-pi/2, pi/2] (south to north); for
 * shapes 0-2 the centreline is bent into the circle of curvature kappa tangent
 * to the z-axis, p = kappa z^2 / (1 + sqrt(1 - kappa^2 z^2)), q = 0 (the
 * quasi-axisymmetric surface of Section 2, equation para_quasi).  Panels of
 * 16 Gauss-Legendre nodes in t: n_panels uniform panels, then the panel at
 * each pole halved n_ref times toward the pole (dyadic refinement, the N_ref
 * of Section 6), n_panels + 2 n_ref panels in all; times n_theta = 2N
 * azimuthal nodes theta_j = j pi/N (Section 3.1).  World position
 * x = R x0 + centre, R = Rz(theta1) Ry(theta2) (Section 6.2, Example 5).
 * `problem` selects the independent scattering problem (0..n_problems-1) the
 * body belongs to; bodies of one problem must be contiguous and problems in
 * increasing order. */
typedef struct {
  int32_t shape;
  int32_t n_panels;   /* uniform panels, 1..32                               */
  int32_t n_theta;    /* even, 4..64                                        */
  int32_t problem;
  double a, c;        /* shape parameters (see qax_shape)                   */
  double kappa;       /* 0 <= kappa, kappa * max|z| < 1                       */
  double theta1, theta2;
  double centre[3];
  int32_t n_ref;      /* 0..8 refinements per pole (n_panels >= 2 when > 0);
                         at most 8192 nodes per body in all                 */
} qax_body;

typedef struct {
  int32_t iters;        /* Krylov iterations, summed over restarts/refinements   */
  int32_t outer_iters;  /* refinement steps (QAX_MIXED) or restarts (QAX_FP64)   */
  double rel_res;       /* final true relative residual ||b - A mu|| / ||b||,
                           maximum over right-hand sides and problems            */
  double t_setup_s;     /* unused by qax_solve (reported by qax_assemble_self)   */
  double t_solve_s;     /* wall time of the solve                                */
} qax_info;

/* Create a handle on HIP device `device`, enqueuing on `hip_stream`
 * (a hipStream_t, or NULL for the default stream). */
qax_status qax_create(int device, void* hip_stream, qax_problem** out);
void qax_destroy(qax_problem* p);
/* Message of the last failed call on this handle ("" if none). */
const char* qax_last_error(const qax_problem* p);

/* Build nodes, weights and outward normals of all bodies on the device
 * (Sections 2, 3.1; rigid motions of Section 6.2).  k_per_problem[n_problems]
 * are the wavenumbers (k >= 0).  Bodies with identical shape, discretisation
 * and wavenumber share one self block (Section 4: congruent bodies have equal
 * diagonal blocks whatever their rigid motion).  A handle may be built again:
 * the earlier geometry and self blocks are dropped (assemble again); the
 * pair sums' work plans are kept when the bodies' node counts, their split
 * into problems and the wavenumbers are unchanged (bodies moved, rotated or
 * reshaped), and made again otherwise. */
qax_status qax_build(qax_problem* p, const qax_body* bodies, int32_t n_bodies,
                     const double* k_per_problem, int32_t n_problems);

/* Number of unknowns and, if body_offsets is non-NULL, the n_bodies+1 node
 * offsets of the bodies (host array). */
qax_status qax_size(const qax_problem* p, int64_t* n_unknowns, int64_t* body_offsets);

/* Copy out node positions and area-weighted normals n |J| (pi/N) omega (the
 * smooth-rule weight times the unit normal, Section 3.1 equation sx), each as
 * (N, 3) row-major FP64 device arrays. */
qax_status qax_nodes(const qax_problem* p, double* d_pos, double* d_aw);

/* Assemble every distinct self block B = 1/2 I + D_bb in FP64 (Sections
 * 3.1-3.4: modal Green's functions by recurrence, FFT and convolution; product
 * integration in s), then factor it: by default its inverse is computed in
 * FP64 (Gauss-Jordan with partial pivoting; the block-diagonal preconditioner
 * of Section 6) and B^-1 is rounded to FP32 for the mixed path (B itself is
 * rounded to FP32 by the first call that applies it in FP32).  Bodies mapped
 * onto themselves by both reflections theta -> -theta and t -> -t (sphere,
 * spheroid and peanut, bent or not, and the quasi-ellipsoid) have a quarter of their rows assembled
 * and the rest stored as images, and are inverted through four
 * symmetry-reduced blocks; when every body is such, the handle also keeps
 * the reduced inverses (FP64 and FP32, about a quarter of the inverse blocks'
 * entries) and applies B^-1 to one right-hand side through them.  With
 * qax_set_factorization(p, QAX_MIXED) the inverse is instead computed in FP32
 * from B rounded to FP32, and the FP64 inverse is made by the first call that
 * needs it (qax_self_block with inverse, qax_block_apply with inverse in
 * QAX_FP64, QAX_FP64 solves; outside their solve time).  The quadrature
 * rules are fixed (converged to about 1e-13 relative for the supported
 * shapes and discretisations), so no accuracy argument is taken.
 * *t_setup_s (may be NULL) receives the wall time of assembly and
 * factorisation. */
qax_status qax_assemble_self(qax_problem* p, double* t_setup_s);

/* Precision of the factorisation made by qax_assemble_self: QAX_FP64 (the
 * default: FP64 inverse, FP32 roundings of B and B^-1 for QAX_MIXED solves)
 * or QAX_MIXED (B rounded to FP32 and inverted in FP32 on the FP32 matrix
 * cores; the mixed solver then limits each refinement cycle to the FP32
 * inverse's accuracy, about 1e-5, and evaluates later cycles with the FP32
 * copy of B).  Changing it on an assembled handle drops the handle back to
 * the built state (qax_assemble_self is needed again).  Errors: QAX_ERR_ARG. */
qax_status qax_set_factorization(qax_problem* p, qax_prec prec);

/* Copy the self block of body `body` (n_b x n_b complex128, row-major: row =
 * target node, column = source node) into d_out.  inverse != 0 copies the
 * FP64 B^-1. */
qax_status qax_self_block(const qax_problem* p, int32_t body, int32_t inverse, void* d_out);

/* Inter-body pair sum only (Section 4): d_out = D_off d_mu, i.e. for every
 * node x_i the sum over nodes y_j of other bodies of the same problem of
 * (ik/r - 1/r^2) e^{ikr}/(4 pi r) n_j.(y_j - x_i) |J_j| (pi/N) omega_j mu_j.
 * d_mu, d_out: N x nrhs complex128.  Needs only qax_build. */
qax_status qax_pair_sum(qax_problem* p, qax_prec prec, const void* d_mu, void* d_out, int32_t nrhs);

/* Block-diagonal apply: d_out_b = M_b d_v_b for every body, M_b = B_b
 * (inverse == 0) or B_b^-1 (inverse != 0); prec QAX_MIXED uses the FP32
 * blocks (B rounded to FP32, or the FP32 inverse) with FP64 accumulation.
 * N x nrhs complex128. */
qax_status qax_block_apply(qax_problem* p, int32_t inverse, qax_prec prec,
                           const void* d_v, void* d_out, int32_t nrhs);

/* Full operator: d_out = (1/2 I + D) d_mu (self blocks + pair sum). */
qax_status qax_apply(qax_problem* p, qax_prec prec, const void* d_mu, void* d_out, int32_t nrhs);

/* Right-hand side b = -exp(i k d.x) (Section 2, plane wave).  dirs: host,
 * n_problems x nrhs x 3 unit vectors.  d_out: N x nrhs complex128. */
qax_status qax_rhs(qax_problem* p, const double* dirs, int32_t nrhs, void* d_out);

/* Solve (1/2 I + D) mu = -u_inc for nrhs plane waves (dirs as in qax_rhs) by
 * right-preconditioned restarted GMRES with the block-diagonal preconditioner
 * (Section 6).  QAX_FP64: FP64 throughout.  QAX_MIXED: FP64 iterative
 * refinement around an inner GMRES whose operator applies the FP32 pair sum
 * and the FP32 blocks (B and its inverse); residuals and orthogonalisation
 * stay FP64.
 * Stops when ||b - A mu|| / ||b|| <= tol for every right-hand side and
 * problem; otherwise returns QAX_ERR_NOCONV after maxit inner iterations with
 * the best iterate in d_mu_out and info filled.  Single-problem, single-body
 * systems of at most 4096 unknowns (e.g. two spheres) may instead be solved
 * directly with qax_solve_dense. */
qax_status qax_solve(qax_problem* p, qax_prec prec, const double* dirs, int32_t nrhs,
                     double tol, int32_t maxit, void* d_mu_out, qax_info* info);

/* Solver for several right-hand sides (qax_solve and qax_solve_rhs with
 * nrhs > 1).  QAX_SOLVER_LOCKSTEP (default): an independent GMRES run per
 * right-hand side and problem, all advancing together and sharing each
 * operator apply.  QAX_SOLVER_BLOCK: block GMRES, one Krylov space shared by
 * the nrhs right-hand sides (block Arnoldi with block Gram-Schmidt twice and
 * Cholesky QR twice, the block Hessenberg least-squares problem by
 * Householder reflections, restart after 40 block steps, right
 * preconditioning with the block-diagonal preconditioner of Section 6;
 * QAX_MIXED as FP64 iterative refinement around FP32 inner cycles); handles
 * with one problem and at most 64 right-hand sides (else QAX_ERR_ARG at
 * solve time).  One right-hand side always uses the lockstep solver.
 * Errors: QAX_ERR_ARG. */
typedef enum { QAX_SOLVER_LOCKSTEP = 0, QAX_SOLVER_BLOCK = 1 } qax_solver;
qax_status qax_set_solver(qax_problem* p, int32_t solver);

/* As qax_solve with the right-hand side given by the caller instead of plane
 * waves: d_rhs (device, N x nrhs complex128, not aliasing d_mu_out), e.g. the
 * boundary values of a known radiating field (the artificial solutions of
 * Section 6: solving with them and evaluating qax_nearfield / qax_farfield
 * recovers the field). */
qax_status qax_solve_rhs(qax_problem* p, qax_prec prec, const void* d_rhs, int32_t nrhs,
                         double tol, int32_t maxit, void* d_mu_out, qax_info* info);

/* Batched in-place inversion of caller matrices with the Gauss-Jordan
 * elimination (partial pivoting, 128-column panels) that inverts the self
 * blocks for the block-diagonal preconditioner of the hybrid solver (Section 6):
 * d_mats holds `count` complex128 matrices, orders[i] x orders[i] each
 * (host array, orders in [1, 8192]), row-major, stored one after another;
 * each is replaced by its inverse.  prec QAX_FP64 inverts in FP64;
 * QAX_MIXED rounds to complex64, inverts in FP32 (the mixed path's
 * preconditioner) and widens the result back.  Needs only a created handle
 * (no build).  Singular matrices give non-finite entries (no error).
 * Synchronises the handle's stream. */
qax_status qax_invert(qax_problem* p, qax_prec prec, int32_t count, const int32_t* orders,
                      void* d_mats);

/* Dense direct solve of the full system (all blocks assembled on the device,
 * Gauss-Jordan inversion in FP64) for N <= 8192; d_mu_out N x nrhs. */
qax_status qax_solve_dense(qax_problem* p, const double* dirs, int32_t nrhs, void* d_mu_out);

/* Far field of the double-layer density of every problem p (Section 6, the
 * far-field pattern, in its double-layer form):
 * u_inf_p(xhat) = (1/4 pi) sum_{j in p} (-i k_p xhat.n_j) e^{-i k_p xhat.y_j}
 * mu_j |J_j| w_j (combined field: plus -i eta |J_j| w_j e^{...}; single layer:
 * |J_j| w_j e^{...} mu_j alone).  xhat: host, n_dirs x 3 (finite; a direction
 * whose exact negation is also listed shares its phase evaluation, with the
 * same results).  d_mu: N x nrhs; d_u_inf: n_problems x n_dirs x nrhs
 * complex128 (problem, then direction, then right-hand side). */
qax_status qax_farfield(qax_problem* p, const void* d_mu, int32_t nrhs,
                        const double* xhat, int32_t n_dirs, void* d_u_inf);

/* For callers that cannot allocate (code under HIP graph or stream capture,
 * serving loops, harnesses that forbid device allocation): qax_farfield with
 * the directions already on the device and no allocation of any kind.
 * d_xhat: DEVICE array, n_dirs x 3 FP64 (unit directions; not checked:
 * non-finite entries give non-finite results); d_mu: N x nrhs; d_u_inf:
 * n_problems x n_dirs x nrhs complex128, as qax_farfield (no antipodal
 * pairing; the results agree with qax_farfield to rounding).  The partial
 * sums go to a fixed 64 MiB device workspace that the library holds on each
 * GPU until the process ends, shared by every handle and call on that GPU:
 * calls that overlap on one GPU (several host threads, several streams) race
 * on it and must be serialised by the caller.  Limit: n_problems * n_dirs *
 * nrhs <= 4194304, else QAX_ERR_ARG; nrhs in [1, 256].  Needs qax_build.
 * Enqueues the work on the handle's stream and returns WITHOUT waiting for
 * it (unlike the other calls); the caller synchronises the stream.  Calls
 * no hipMalloc, hipFree, pinned-host allocation or host-to-device copy. */
qax_status qax_farfield_noalloc(qax_problem* p, const void* d_mu, int32_t nrhs, const double* d_xhat,
                                int32_t n_dirs, void* d_u_inf);

/* Scattered field at points off the surfaces: the double-layer potential of
 * the density of one problem, u(x) = sum_j dG/dn_y(x, y_j) mu_j |J_j| w_j
 * (Section 4, equation multi-double, with the smooth rule of Section 3.1,
 * equation sx).  Accurate for points whose distance to every surface is at
 * least about one panel length (no near-singular quadrature).  pts: host,
 * n_pts x 3 (finite); problem: 0 .. n_problems - 1; d_mu: N x nrhs, d_u:
 * n_pts x nrhs complex128 (device).  FP64. */
qax_status qax_nearfield(qax_problem* p, const void* d_mu, int32_t nrhs, const double* pts,
                         int64_t n_pts, int32_t problem, void* d_u);

/* Test hook for the modal engine (Section 3.3): phi-frame modes m = 0..nmax of
 * the source derivatives dr G and dz G of the Helmholtz kernel for n_pts
 * (r, rt, c, chi - 1, r - rt) tuples (device FP64 arrays), wavenumber k.
 * d_A, d_B: n_pts x (nmax+1) complex128. */
qax_status qax_modal_modes(qax_problem* p, int32_t n_pts, const double* d_r, const double* d_rt,
                           const double* d_c, const double* d_chim1, const double* d_rmrt,
                           double k, int32_t nmax, void* d_A, void* d_B);

/* Captured solver steps.  With enable != 0 (the default) qax_solve captures
 * each Arnoldi step (block apply, pair sum, two Gram-Schmidt passes, norm,
 * Givens update, next basis vector, convergence count) once per step index
 * into a HIP graph and replays it; the graphs stay with the handle while the
 * buffers, sizes and launch choices are unchanged.  enable = 0 enqueues the
 * same kernels one by one (identical results).  While kernel timing is on,
 * the steps are always enqueued one by one. */
qax_status qax_set_graphs(qax_problem* p, int32_t enable);

/* Boundary-integral formulation.  QAX_DOUBLE_LAYER (default): the paper's
 * multi-body system (1/2 I + D) mu = -u_inc (Section 4).  QAX_SINGLE_LAYER:
 * the first-kind equation S mu = -u_inc (Section 2, equation
 * single-layer-bie; eta ignored), the field represented by the single-layer
 * potential.  QAX_COMBINED_FIELD:
 * (1/2 I + D - i eta S) mu = -u_inc with the single-layer operator S (Section
 * 2, the remark on combined fields; uniquely solvable at interior resonances,
 * where the double-layer system is singular); S is discretised with the
 * density times |J| interpolated (Section 3.1) and its modal Green's function
 * by convolution and FFT (Section 3.3).  eta > 0: that coupling for every
 * problem; eta <= 0: eta = k of each problem.  Applies to the self blocks,
 * pair sums, near and far field.  May be called at any time; on a built
 * handle it updates the per-node weights and drops the handle back to the
 * built state (qax_assemble_self is needed again).  Errors: QAX_ERR_ARG. */
typedef enum {
  QAX_DOUBLE_LAYER = 0,
  QAX_COMBINED_FIELD = 1,
  QAX_SINGLE_LAYER = 2
} qax_formulation;
qax_status qax_set_formulation(qax_problem* p, int32_t formulation, double eta);

/* Block-Toeplitz inter-body apply for a regular array of identical bodies
 * (Section 4, the paragraph on identical scatterers on a P x Q x R array:
 * the interaction block of two bodies depends only on the displacement of
 * their centres, so there are (2P-1)(2Q-1)(2R-1) - 1 distinct blocks; Table
 * 7).  enable != 0: checks that the built handle holds one problem whose
 * bodies share shape, curvature, discretisation and orientation and whose
 * centres fill a P x Q x R array aligned with the coordinate axes (uniform
 * spacing per axis, any listing order), then computes one block per
 * displacement on the device, transforms them over the array's circulant
 * embedding of size (2P-1)(2Q-1)(2R-1) = F, and keeps the F frequency
 * tables (F n_b^2 complex128 plus a complex64 copy, n_b nodes per body).
 * From then on every inter-body sum of the handle (qax_pair_sum, qax_apply,
 * the solvers; QAX_MIXED uses the complex64 tables) is evaluated as: forward
 * transform of the density over the array, one n_b x n_b product per
 * frequency (batched; matrix cores for 4 or more right-hand sides), inverse
 * transform.  enable = 0 frees the tables and returns to the direct pair
 * sum; qax_build and qax_set_formulation also free them.  dims (host, 3
 * int32, may be null) receives P, Q, R.  Errors: QAX_ERR_STATE (not built),
 * QAX_ERR_ARG (not such an array, or F > 65535), QAX_ERR_NOMEM. */
qax_status qax_lattice(qax_problem* p, int32_t enable, int32_t* dims);

/* Kernel timing (instrumentation).  When enabled, each launch of the kernels
 * below is bracketed by HIP events recorded on the handle's stream and its
 * duration is accumulated per kernel kind.  Disabled by default. */
typedef enum {
  QAX_K_PAIRSUM_FP64 = 0,  /* inter-body pair sum, FP64                        */
  QAX_K_PAIRSUM_FP32 = 1,  /* inter-body pair sum, FP32 compensated            */
  QAX_K_BLOCK_APPLY = 2,   /* block-diagonal apply, FP64 (B or B^-1)           */
  QAX_K_SELF_ASSEMBLY = 3, /* self-block assembly                              */
  QAX_K_INVERT = 4,        /* self-block inversion (all of its launches)       */
  QAX_K_INVERT_UPDATE = 5, /* inversion: trailing update of one 128-column panel */
  QAX_K_BLOCK_APPLY_F32 = 6, /* block-diagonal apply of the FP32 inverse of B   */
  QAX_K_LATTICE_F64 = 7,   /* lattice apply: per-frequency products, FP64 tables */
  QAX_K_LATTICE_F32 = 8,   /* lattice apply: per-frequency products, FP32 tables */
  QAX_K_COUNT = 9
} qax_kernel;

/* enable != 0 turns timing on (and clears the counters). */
qax_status qax_set_timing(qax_problem* p, int32_t enable);
/* Launch count and summed duration (milliseconds) of one kernel kind since
 * timing was enabled. */
qax_status qax_timing(const qax_problem* p, int32_t kernel, int64_t* launches, double* total_ms);

/* Autotuner (the batching pattern's tile and schedule choices).  Tunable:
 *  - pair sum, per precision: targets per workgroup, which is also the source
 *    tile staged in LDS (128, 256, 512), and the number of workgroups per
 *    compute unit that the split of the source bodies into chunks aims at
 *    (4, 8, 16; sets how many partial sums each target row gets); with
 *    several right-hand sides, right-hand sides per pass (2 ... 32), chosen
 *    together with the workgroup size for the largest class nrhs_max reaches;
 *  - block apply with one right-hand side, per storage precision: complex
 *    entries per lane and load (1, 2; 4 for the FP32 inverse);
 *  - the reciprocal pair sum (one right-hand side, k > 0, double layer or
 *    combined field: each unordered pair of nodes evaluated once for both
 *    directions), per precision: the number of 256-node block pairs per
 *    side of the square of block pairs one workgroup evaluates (1, 2, 4, 8),
 *    which sets the launch's workgroup count and the size of its partial
 *    sums (about 2 N (N / 256) / s complex values, cut into launches of at
 *    most 960 MB each).  With one right-hand side and the reciprocal kernel
 *    serving every such pair sum, the per-target kernel's choices above are
 *    not timed.
 * Every candidate is timed on this problem's own data (HIP events, the
 * fastest of a few launches after a warm-up) and the fastest is kept for the
 * handle until the next qax_autotune.  Results do not depend on the choices
 * beyond the order of floating-point additions.
 * nrhs_max: largest number of right-hand sides to tune for (1 ... 1024).
 * cache_path: text file of earlier results (NULL: none); a line whose device
 * and problem signature (N, bodies, problems, largest block, nrhs_max) match
 * is used instead of timing, and new results are written back.
 * Requires qax_build; the block-apply part needs qax_assemble_self (skipped
 * before it).  Errors: QAX_ERR_ARG, QAX_ERR_STATE, QAX_ERR_DEVICE. */
qax_status qax_autotune(qax_problem* p, int32_t nrhs_max, const char* cache_path);

typedef struct {
  int32_t tuned;              /* 1 once qax_autotune has run on this handle   */
  int32_t from_cache;         /* 1 if the last choices came from cache_path   */
  int32_t pair_tpb[2];        /* [0] FP64, [1] FP32 pair sum: workgroup size  */
  int32_t pair_slot_mult[2];  /* workgroups per CU of the source-chunk split  */
  int32_t pair_nrc[2][4];     /* RHS per pass for nrhs 2-4, 5-8, 9-16, > 16   */
  int32_t gemv_vec[2];        /* block apply, 1 RHS: [0] FP64, [1] FP32 inverse*/
  double pair_ms[2];          /* chosen single-RHS pair sum, ms (timed runs)  */
  double default_pair_ms[2];  /* the built-in default choice, ms             */
  int32_t pair_sym_s[2];      /* reciprocal one-RHS pair sum: block pairs per
                                 super-task side (1, 2, 4, 8; 0 in
                                 qax_set_tuning: the default for the problem) */
} qax_tuning_info;

/* Current launch choices (defaults before any qax_autotune). */
qax_status qax_tuning(const qax_problem* p, qax_tuning_info* out);

/* Set the launch choices by hand (pair_tpb, pair_slot_mult, pair_nrc,
 * gemv_vec of `in`; the other fields are ignored).  Requires qax_build.
 * QAX_ERR_ARG if a choice is not one the kernels support (pair_tpb 128, 256
 * or 512; pair_slot_mult 1 ... 64; pair_nrc 1, 2, 4, 8 (FP64) or ... 32
 * (FP32) with the LDS of the workgroup within 64 KB; gemv_vec 1, 2 (FP64) or
 * 1, 2, 4 (FP32); pair_sym_s 0 ... 8). */
qax_status qax_set_tuning(qax_problem* p, const qax_tuning_info* in);

#ifdef __cplusplus
}
#endif
#endif /* QAX_H */
