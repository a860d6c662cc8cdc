// Segmented GMRES vector operations (device kernels in krylov.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace qax {

// A contiguous node range inside one problem.
struct Chunk {
  int64_t n0, n1;
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
};

}  // namespace qax
