// Segmented GMRES vector operations (device kernels in krylov.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace qax {

// A contiguous node range inside one problem.
struct Chunk {
  int64_t n0, n1;
};

// Least-squares state of every segment's GMRES cycle, on the device (restart
// length m, nseg segments).
struct GivensState {
  double2* H = nullptr;       // rotated Hessenberg columns: segment s, column j at (s m + j)(m + 1)
  double* cs = nullptr;       // nseg x m rotation cosines
  double2* sn = nullptr;      // nseg x m rotation sines
  double2* g = nullptr;       // nseg x (m + 1) rotated right-hand side (g_0 = beta)
  double* beta = nullptr;     // nseg: residual norm at the start of the cycle
  double* tin = nullptr;      // nseg: relative tolerance of the cycle
  int32_t* frozen = nullptr;  // nseg: 1 = segment not iterated in this cycle
  double2* scl = nullptr;     // nseg: scale of the next basis vector (0 for stopped ones)
  int32_t* notdone = nullptr; // m: per step, number of segments still above tolerance
  int32_t* active = nullptr;  // nseg: 1 while the segment is iterated (0: frozen or converged)
  int32_t* kconv = nullptr;   // nseg: steps taken when the segment converged (0: not yet)
};

// Launch helpers over N x nrhs complex vectors whose segments are
// (problem, right-hand side) pairs.  Segmented scalars are stored as
// [m][nprob][nrhs] complex128.  `vstride` arguments are the distance between
// consecutive vectors of V in doubles.
struct Krylov {
  hipStream_t stream = nullptr;
  int64_t N = 0;
  int nrhs = 1;
  int nprob = 1;
  int nchunks = 0;
  Chunk* d_chunks = nullptr;
  int32_t* d_prob_chunk0 = nullptr;
  int32_t* d_node_prob = nullptr;
  double* d_partial = nullptr;   // m_max x nchunks x nrhs complex

  // h[i] = V_i^H w for i < m (segmented)
  void dots(const double* V, int64_t vstride, int m, const double* w, double* h);
  // w -= sum_i V_i h[i]
  void orth(const double* V, int64_t vstride, int m, const double* h, double* w);
  // out (+)= sum_i V_i y[i]
  void combine(const double* V, int64_t vstride, int m, const double* y, double* out, bool accumulate);
  // out = a * s (segment scale)
  void scale(const double* a, const double* s, double* out);
  // out = alpha a + beta b
  void axpby(double alpha, const double* a, double beta, const double* b, double* out);
  // step j of every segment's least-squares problem from the two Gram-Schmidt
  // passes h1, h2 (rows 0..j) and |w|^2 (hn2): new Givens rotation, residual
  // estimate, next-vector scale, and the count of unconverged segments
  void givens(int nseg, int j, int m, const double* h1, const double* h2, const double* hn2,
              const GivensState& G);
  // y[i][s] (i < k) = solution of the rotated triangular system of segment s
  void back_solve(int nseg, int k, int m, const GivensState& G, double* y);
};

}  // namespace qax
