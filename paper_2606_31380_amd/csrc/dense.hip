// Dense block work: the block-diagonal apply of the self blocks (Section 4,
// equation linearsys, diagonal blocks D_tt plus 1/2 I), their inversion for the
// block-diagonal preconditioner (Section 6, the hybrid-solver paragraph: "LU
// factorization of the single-body self-interaction matrix"), and the dense
// assembly of the whole system for the direct solve.
//
// Block apply with one right-hand side is bound by HBM bandwidth: every matrix
// element is read once, rows are streamed by one wavefront each with
// coalesced 16-byte (FP64 complex) or 8-byte (FP32 complex) loads, and the
// input slice comes from L2.  FP32 storage is accumulated in FP64.
//
// Inversion: blocked Gauss-Jordan elimination with partial pivoting, in place,
// batched over matrices of different orders (see gj_invert).
#include <hip/hip_runtime.h>

#include "fastmath.h"
#include "internal.h"
#include "shapes.h"

namespace qax {

// ---------------------------------------------------------------- block apply
// LPR lanes per row (64: one wavefront per row; 32 or 16 for short rows, two
// or four rows per wavefront); each lane loads VEC consecutive complex entries
// per step (block orders are multiples of 16).
template <typename MT, int NRC, int VEC, int LPR = 64>
__global__ __launch_bounds__(256) void block_gemv_kernel(
    const BodyDev* __restrict__ bodies, const BlockDev* __restrict__ blocks,
    const int32_t* __restrict__ node_body, const MT* __restrict__ pool, int64_t N,
    const double2* __restrict__ v, int nrhs, double2* __restrict__ out, int accumulate,
    const int32_t* __restrict__ seg_active) {
  typedef MT vec_t __attribute__((ext_vector_type(2 * VEC)));
  const int lane = threadIdx.x & (LPR - 1);
  const int64_t row = (int64_t)blockIdx.x * (256 / LPR) + (threadIdx.x / LPR);
  const int rc0 = blockIdx.y * NRC;
  if (row >= N) return;
  const int b = node_body[row];
  const BodyDev& B = bodies[b];
  if (seg_active) {
    // converged lockstep segments: their input is zero, so is the output
    bool any = false;
    for (int r = rc0; r < rc0 + NRC && r < nrhs; ++r) any = any || seg_active[B.problem * nrhs + r] != 0;
    if (!any) {
      if (lane == 0 && !accumulate)
        for (int r = rc0; r < rc0 + NRC && r < nrhs; ++r) out[row * nrhs + r] = make_double2(0.0, 0.0);
      return;
    }
  }
  const BlockDev& K = blocks[B.block];
  const int n = K.n;
  const int lr = (int)(row - B.off);
  const MT* a = pool + 2 * (K.elem_off + (int64_t)lr * n);
  const double2* vb = v + B.off * nrhs;
  double ar[NRC], ai[NRC];
#pragma unroll
  for (int r = 0; r < NRC; ++r) { ar[r] = 0.0; ai[r] = 0.0; }
  for (int j0 = lane * VEC; j0 < n; j0 += LPR * VEC) {
    const vec_t av = *(const vec_t*)(a + 2 * j0);
#pragma unroll
    for (int q = 0; q < VEC; ++q) {
      const double mr = (double)av[2 * q], mi = (double)av[2 * q + 1];
      const int j = j0 + q;
#pragma unroll
      for (int r = 0; r < NRC; ++r) {
        if (rc0 + r < nrhs) {
          const double2 x = vb[(int64_t)j * nrhs + rc0 + r];
          ar[r] += mr * x.x - mi * x.y;
          ai[r] += mr * x.y + mi * x.x;
        }
      }
    }
  }
#pragma unroll
  for (int r = 0; r < NRC; ++r) {
#pragma unroll
    for (int off = LPR / 2; off > 0; off >>= 1) {
      ar[r] += __shfl_xor(ar[r], off);
      ai[r] += __shfl_xor(ai[r], off);
    }
  }
  if (lane == 0) {
#pragma unroll
    for (int r = 0; r < NRC; ++r) {
      if (rc0 + r < nrhs) {
        const int64_t e = row * nrhs + rc0 + r;
        double2 o = accumulate ? out[e] : make_double2(0.0, 0.0);
        o.x += ar[r];
        o.y += ai[r];
        out[e] = o;
      }
    }
  }
}

// FP32 matrix, one right-hand side: GV_ROWS rows of one block per workgroup
// (four per wavefront), the block's input vector staged in LDS in chunks of
// GV_CH entries and shared by those rows.  The matrix streams from HBM once;
// the FP64 vector (twice the bytes of an FP32 matrix entry) is read once per
// GV_ROWS rows instead of once per row.  Blocks (orders multiples of 16) and
// their offsets are multiples of GV_ROWS, so a workgroup never spans two.
constexpr int GV_ROWS = 16, GV_CH = 1024;

template <int VEC>
__global__ __launch_bounds__(256) void block_gemv_f32_lds_kernel(
    const BodyDev* __restrict__ bodies, const BlockDev* __restrict__ blocks,
    const int32_t* __restrict__ node_body, const float* __restrict__ pool, int64_t N,
    const double2* __restrict__ v, double2* __restrict__ out, int accumulate,
    const int32_t* __restrict__ seg_active) {
  typedef float vec_t __attribute__((ext_vector_type(2 * VEC)));
  __shared__ double2 vs[GV_CH];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t row0 = (int64_t)blockIdx.x * GV_ROWS;
  if (row0 >= N) return;
  const BodyDev& B = bodies[node_body[row0]];
  if (seg_active && seg_active[B.problem] == 0) {
    // a converged lockstep segment: its input is zero, so is the output
    if (!accumulate && threadIdx.x < GV_ROWS) out[row0 + threadIdx.x] = make_double2(0.0, 0.0);
    return;
  }
  const BlockDev& K = blocks[B.block];
  const int n = K.n;
  const double2* vb = v + B.off;
  double ar[GV_ROWS / 4], ai[GV_ROWS / 4];
#pragma unroll
  for (int q = 0; q < GV_ROWS / 4; ++q) { ar[q] = 0.0; ai[q] = 0.0; }
  for (int c0 = 0; c0 < n; c0 += GV_CH) {
    const int cn = min(GV_CH, n - c0);
    __syncthreads();
    for (int q = threadIdx.x; q < cn; q += 256) vs[q] = vb[c0 + q];
    __syncthreads();
    // the wavefront's rows side by side: their loads in flight together and
    // each staged entry of the vector read once for all of them
    const float* a = pool + 2 * (K.elem_off + (row0 + wave * (GV_ROWS / 4) - B.off) * n + c0);
    for (int j0 = lane * VEC; j0 < cn; j0 += 64 * VEC) {
      vec_t av[GV_ROWS / 4];
#pragma unroll
      for (int rr = 0; rr < GV_ROWS / 4; ++rr) av[rr] = *(const vec_t*)(a + 2 * ((int64_t)rr * n + j0));
#pragma unroll
      for (int q = 0; q < VEC; ++q) {
        const double2 x = vs[j0 + q];
#pragma unroll
        for (int rr = 0; rr < GV_ROWS / 4; ++rr) {
          const double mr = (double)av[rr][2 * q], mi = (double)av[rr][2 * q + 1];
          ar[rr] = fma(mr, x.x, fma(-mi, x.y, ar[rr]));
          ai[rr] = fma(mr, x.y, fma(mi, x.x, ai[rr]));
        }
      }
    }
  }
#pragma unroll
  for (int rr = 0; rr < GV_ROWS / 4; ++rr) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      ar[rr] += __shfl_xor(ar[rr], off);
      ai[rr] += __shfl_xor(ai[rr], off);
    }
    if (lane == 0) {
      const int64_t row = row0 + wave * (GV_ROWS / 4) + rr;
      double2 o = accumulate ? out[row] : make_double2(0.0, 0.0);
      o.x += ar[rr];
      o.y += ai[rr];
      out[row] = o;
    }
  }
}

template <int VEC>
static void gemv_f32_lds_launch(hipStream_t s, const BodyDev* bodies, const BlockDev* blocks,
                                const int32_t* node_body, const float* pool, int64_t N,
                                const double* v, double* out, bool acc, const int32_t* seg_active) {
  hipLaunchKernelGGL((block_gemv_f32_lds_kernel<VEC>), dim3((unsigned)((N + GV_ROWS - 1) / GV_ROWS)),
                     dim3(256), 0, s, bodies, blocks, node_body, pool, N, (const double2*)v,
                     (double2*)out, acc ? 1 : 0, seg_active);
}

template <typename MT, int NRC, int VEC>
static void gemv_launch(qax_problem* p, const MT* pool, const double* v, double* out, int nrhs,
                        bool acc) {
  dim3 grid((unsigned)((p->N + 3) / 4), (unsigned)((nrhs + NRC - 1) / NRC));
  hipLaunchKernelGGL((block_gemv_kernel<MT, NRC, VEC>), grid, dim3(256), 0, p->stream, p->d_bodies,
                     p->d_blocks, p->d_node_body, pool, p->N, (const double2*)v, nrhs,
                     (double2*)out, acc ? 1 : 0, p->seg_active);
}

hipError_t launch_block_gemm(qax_problem* p, int inverse, int prec, const double* v, double* out,
                             int nrhs, bool accumulate);

static void launch_sym_apply(qax_problem* p, int prec, const double* v, double* out, bool accumulate);

// B rounded to FP32 on first use after an FP64 factorisation (the FP32
// factorisation makes it; solves with the FP64 factorisation never read it).
static hipError_t ensure_b32(qax_problem* p) {
  if (p->b32_ready) return hipSuccess;
  hipError_t e = launch_convert_f32(p->stream, p->d_B, p->d_B32, 2 * p->block_elems);
  if (e == hipSuccess) p->b32_ready = true;
  return e;
}

hipError_t launch_block_apply(qax_problem* p, int inverse, int prec, const double* v, double* out,
                              int nrhs, bool accumulate) {
  const int kind = prec == QAX_MIXED ? QAX_K_BLOCK_APPLY_F32 : QAX_K_BLOCK_APPLY;
  if (!inverse && prec == QAX_MIXED) {
    hipError_t e = ensure_b32(p);
    if (e != hipSuccess) return e;
  }
  if (inverse && nrhs == 1 && p->symap.on && (prec == QAX_MIXED || p->inv64_ready)) {
    // every block mirror-symmetric: through the four reduced inverses
    timing_begin(p, kind);
    launch_sym_apply(p, prec, v, out, accumulate);
    timing_end(p, kind);
    return hipGetLastError();
  }
  if (nrhs >= 4) {
    // several right-hand sides: batched complex GEMM on the matrix cores
    timing_begin(p, kind);
    hipError_t e = launch_block_gemm(p, inverse, prec, v, out, nrhs, accumulate);
    timing_end(p, kind);
    return e;
  }
  timing_begin(p, kind);
  if (prec == QAX_MIXED) {
    const float* pool = inverse ? p->d_Binv32 : p->d_B32;
    if (nrhs > 1) gemv_launch<float, 4, 1>(p, pool, v, out, nrhs, accumulate);
    else if (p->tune.gemv_vec[1] == 4)
      gemv_f32_lds_launch<4>(p->stream, p->d_bodies, p->d_blocks, p->d_node_body, pool, p->N, v, out,
                             accumulate, p->seg_active);
    else if (p->tune.gemv_vec[1] == 2)
      gemv_f32_lds_launch<2>(p->stream, p->d_bodies, p->d_blocks, p->d_node_body, pool, p->N, v, out,
                             accumulate, p->seg_active);
    else
      gemv_f32_lds_launch<1>(p->stream, p->d_bodies, p->d_blocks, p->d_node_body, pool, p->N, v, out,
                             accumulate, p->seg_active);
  } else {
    const double* pool = inverse ? p->d_Binv : p->d_B;
    if (nrhs > 1) gemv_launch<double, 4, 1>(p, pool, v, out, nrhs, accumulate);
    else if (p->tune.gemv_vec[0] == 2) gemv_launch<double, 1, 2>(p, pool, v, out, nrhs, accumulate);
    else gemv_launch<double, 1, 1>(p, pool, v, out, nrhs, accumulate);
  }
  timing_end(p, kind);
  return hipGetLastError();
}

// ---------------------------------------------------------------- block apply, several RHS (MFMA)
// Y_b = M_b V_b for every body with V, Y node-major (RHS fastest).  The
// complex product is the real product A' B' with A' = M_b viewed as a real
// n x 2n matrix (interleaved storage, read in place) and B' the 2n x 2nrhs
// expansion of V: B'[2j] = (Re V_j0, Im V_j0, ...), B'[2j+1] = (-Im V_j0,
// Re V_j0, ...), built while staging V in LDS.  64 x 64 real output tiles per
// workgroup of 4 wavefronts (32 x 32 each = 2 x 2 MFMA 16x16 tiles), K steps
// of 16 staged through LDS; MFMA 16x16x4 in FP64 (B) or FP32 (FP32 inverse).
template <typename T>
struct MfmaAcc;
template <>
struct MfmaAcc<double> {
  typedef __attribute__((__vector_size__(4 * sizeof(double)))) double v4;
  static __device__ __forceinline__ v4 mma(double a, double b, v4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  // D[i][j] of the 16 x 16 tile: lane j + 16 (i % 4), element i / 4
  static __device__ __forceinline__ int row(int lane, int e) { return (lane >> 4) + 4 * e; }
};
template <>
struct MfmaAcc<float> {
  typedef __attribute__((__vector_size__(4 * sizeof(float)))) float v4;
  static __device__ __forceinline__ v4 mma(float a, float b, v4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  // D[i][j] of the 16 x 16 tile: lane j + 16 (i / 4), element i % 4
  static __device__ __forceinline__ int row(int lane, int e) { return 4 * (lane >> 4) + e; }
};

template <typename T>
__global__ __launch_bounds__(256) void block_gemm_kernel(
    const GemmTask* __restrict__ tasks, const BodyDev* __restrict__ bodies,
    const BlockDev* __restrict__ blocks, const T* __restrict__ pool,
    const double* __restrict__ v, int nrhs, double* __restrict__ out, int accumulate) {
  typedef typename MfmaAcc<T>::v4 v4;
  const GemmTask task = tasks[blockIdx.x];
  const BodyDev& Bd = bodies[task.body];
  const BlockDev& K = blocks[Bd.block];
  const int n = K.n;
  const int ncol = 2 * nrhs;                  // real columns of V and Y
  const int c0 = blockIdx.y * 64;
  const int row0 = task.row0;
  const T* A = pool + 2 * K.elem_off;         // real n x 2n, row stride 2n
  const double* Vb = v + 2 * Bd.off * nrhs;   // real n x 2 nrhs
  double* Yb = out + 2 * Bd.off * nrhs;
  __shared__ T As[16][64 + 1];
  __shared__ T Bs[16][64 + 1];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
  v4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int e = 0; e < 4; ++e) acc[a][b][e] = 0;
  for (int k0 = 0; k0 < 2 * n; k0 += 16) {
    // A tile: rows row0..row0+63, real columns k0..k0+15
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = tid + 256 * q;
      const int rr = e >> 4, kk = e & 15;
      const int i = row0 + rr;
      As[kk][rr] = (i < n) ? A[(int64_t)i * 2 * n + k0 + kk] : (T)0;
    }
    // B' tile: real rows k0..k0+15 (complex rows k0/2..k0/2+7), columns c0..c0+63
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int e = tid + 256 * q;             // 512 = 8 complex rows x 64 columns
      const int jr = e >> 6, cc = e & 63;
      const int c = c0 + cc;
      const int j = k0 / 2 + jr;
      T re = 0, alt = 0;
      if (c < ncol) {
        const double x = Vb[(int64_t)j * ncol + c];
        const double y = Vb[(int64_t)j * ncol + (c ^ 1)];
        re = (T)x;
        alt = (c & 1) ? (T)y : (T)(-y);        // row 2j+1: (-Im, Re) pairs
      }
      Bs[2 * jr][cc] = re;
      Bs[2 * jr + 1][cc] = alt;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 16; kk += 4) {
      const int kr = kk + (lane >> 4), ci = lane & 15;
      T af[2], bf[2];
#pragma unroll
      for (int a = 0; a < 2; ++a) af[a] = As[kr][wr + 16 * a + ci];
#pragma unroll
      for (int b = 0; b < 2; ++b) bf[b] = Bs[kr][wc + 16 * b + ci];
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = MfmaAcc<T>::mma(af[a], bf[b], acc[a][b]);
    }
    __syncthreads();
  }
  // accumulator element e of the lane holds column lane % 16 of the tile
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int i = row0 + wr + 16 * a + MfmaAcc<T>::row(lane, e);
        const int c = c0 + wc + 16 * b + (lane & 15);
        if (i < n && c < ncol) {
          double* y = Yb + (int64_t)i * ncol + c;
          *y = (accumulate ? *y : 0.0) + (double)acc[a][b][e];
        }
      }
}

// Row tiles of the block GEMM (built once per geometry; synchronous copy, so
// not to be first called inside a stream capture).
hipError_t ensure_gemm_tasks(qax_problem* p) {
  if (!p->gemm_tasks.empty()) return hipSuccess;
  for (int b = 0; b < p->n_bodies; ++b)
    for (int r0 = 0; r0 < p->hbodies[b].n; r0 += 64) p->gemm_tasks.push_back(GemmTask{b, r0});
  hipError_t e = dev_alloc(p, &p->d_gemm_tasks, p->gemm_tasks.size() * sizeof(GemmTask));
  if (e != hipSuccess) {
    p->gemm_tasks.clear();
    return e;
  }
  return hipMemcpy(p->d_gemm_tasks, p->gemm_tasks.data(), p->gemm_tasks.size() * sizeof(GemmTask),
                   hipMemcpyHostToDevice);
}

hipError_t launch_block_gemm(qax_problem* p, int inverse, int prec, const double* v, double* out,
                             int nrhs, bool accumulate) {
  hipError_t e = ensure_gemm_tasks(p);
  if (e != hipSuccess) return e;
  dim3 grid((unsigned)p->gemm_tasks.size(), (unsigned)((2 * nrhs + 63) / 64));
  const GemmTask* t = (const GemmTask*)p->d_gemm_tasks;
  if (prec == QAX_MIXED)
    hipLaunchKernelGGL(block_gemm_kernel<float>, grid, dim3(256), 0, p->stream, t, p->d_bodies,
                       p->d_blocks, inverse ? p->d_Binv32 : p->d_B32, v, nrhs, out, accumulate ? 1 : 0);
  else
    hipLaunchKernelGGL(block_gemm_kernel<double>, grid, dim3(256), 0, p->stream, t, p->d_bodies,
                       p->d_blocks, inverse ? p->d_Binv : p->d_B, v, nrhs, out, accumulate ? 1 : 0);
  return hipGetLastError();
}

// Block-diagonal products over caller-built tables (the lattice apply's
// per-frequency matrices): rows = sum of the orders, every order a multiple
// of 16.
template <typename MT, int NRC, int VEC, int LPR>
static void gemv_tables_launch(hipStream_t s, const BodyDev* bodies, const BlockDev* blocks,
                               const int32_t* node_body, const void* pool, int64_t rows,
                               const double2* v, int nrhs, double2* out, int acc) {
  dim3 grid((unsigned)((rows + 256 / LPR - 1) / (256 / LPR)), (unsigned)((nrhs + NRC - 1) / NRC));
  hipLaunchKernelGGL((block_gemv_kernel<MT, NRC, VEC, LPR>), grid, dim3(256), 0, s, bodies, blocks,
                     node_body, (const MT*)pool, rows, v, nrhs, out, acc, nullptr);
}

template <typename MT, int NRC, int VEC>
static void gemv_tables_lpr(hipStream_t s, const BodyDev* bodies, const BlockDev* blocks,
                            const int32_t* node_body, const void* pool, int64_t rows, int order,
                            const double2* v, int nrhs, double2* out, int acc) {
  // short rows: up to four loads per lane, several rows per wavefront
  if (order <= 64 * VEC)
    gemv_tables_launch<MT, NRC, VEC, 16>(s, bodies, blocks, node_body, pool, rows, v, nrhs, out, acc);
  else if (order <= 128 * VEC)
    gemv_tables_launch<MT, NRC, VEC, 32>(s, bodies, blocks, node_body, pool, rows, v, nrhs, out, acc);
  else
    gemv_tables_launch<MT, NRC, VEC, 64>(s, bodies, blocks, node_body, pool, rows, v, nrhs, out, acc);
}

hipError_t launch_gemv_tables(hipStream_t s, const BodyDev* bodies, const BlockDev* blocks,
                              const int32_t* node_body, const void* pool, bool f32, int64_t rows,
                              int order, const double* v, int nrhs, double* out, bool accumulate) {
  const double2* vv = (const double2*)v;
  double2* oo = (double2*)out;
  const int acc = accumulate ? 1 : 0;
  if (f32) {
    if (nrhs == 1 && order > 128 * 2)
      gemv_f32_lds_launch<2>(s, bodies, blocks, node_body, (const float*)pool, rows, v, out, accumulate,
                             nullptr);
    else if (nrhs == 1) gemv_tables_lpr<float, 1, 2>(s, bodies, blocks, node_body, pool, rows, order, vv, nrhs, oo, acc);
    else gemv_tables_lpr<float, 4, 1>(s, bodies, blocks, node_body, pool, rows, order, vv, nrhs, oo, acc);
  } else {
    if (nrhs == 1) gemv_tables_lpr<double, 1, 1>(s, bodies, blocks, node_body, pool, rows, order, vv, nrhs, oo, acc);
    else gemv_tables_lpr<double, 4, 1>(s, bodies, blocks, node_body, pool, rows, order, vv, nrhs, oo, acc);
  }
  return hipGetLastError();
}

hipError_t launch_gemm_tables(hipStream_t s, const GemmTask* tasks, int ntasks,
                              const BodyDev* bodies, const BlockDev* blocks, const void* pool,
                              bool f32, const double* v, int nrhs, double* out, bool accumulate) {
  dim3 grid((unsigned)ntasks, (unsigned)((2 * nrhs + 63) / 64));
  if (f32)
    hipLaunchKernelGGL(block_gemm_kernel<float>, grid, dim3(256), 0, s, tasks, bodies, blocks,
                       (const float*)pool, v, nrhs, out, accumulate ? 1 : 0);
  else
    hipLaunchKernelGGL(block_gemm_kernel<double>, grid, dim3(256), 0, s, tasks, bodies, blocks,
                       (const double*)pool, v, nrhs, out, accumulate ? 1 : 0);
  return hipGetLastError();
}

// ---------------------------------------------------------------- conversion
__global__ void convert_f32_kernel(const double* __restrict__ src, float* __restrict__ dst,
                                   int64_t count) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < count) dst[e] = (float)src[e];
}

hipError_t launch_convert_f32(hipStream_t s, const double* src, float* dst, int64_t count) {
  hipLaunchKernelGGL(convert_f32_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s,
                     src, dst, count);
  return hipGetLastError();
}

// B rounded to FP32 into both the FP32 blocks and the buffer the FP32
// inverse is made in (one read of the FP64 blocks); two values per thread.
__global__ void convert_f32_twice_kernel(const double2* __restrict__ src, float2* __restrict__ d0,
                                         float2* __restrict__ d1, int64_t pairs) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= pairs) return;
  const double2 v = src[e];
  const float2 f = make_float2((float)v.x, (float)v.y);
  d0[e] = f;
  d1[e] = f;
}

__global__ void convert_f64_kernel(const float* __restrict__ src, double* __restrict__ dst,
                                   int64_t count) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < count) dst[e] = (double)src[e];
}

// ---------------------------------------------------------------- Gauss-Jordan
struct MatDesc {
  int64_t elem_off;  // complex elements
  int32_t n;
};

// Complex element type of the inversion: FP64 (V) or FP32 (float2).
template <typename T>
struct Cx;
template <>
struct Cx<double> {
  typedef double2 V;
  static __device__ __forceinline__ double2 make(double a, double b) { return make_double2(a, b); }
};
template <>
struct Cx<float> {
  typedef float2 V;
  static __device__ __forceinline__ float2 make(float a, float b) { return make_float2(a, b); }
};

// Undo the row interchanges as column interchanges, last step first.
template <typename T>
__global__ void gj_unpivot_kernel(const MatDesc* __restrict__ mats, typename Cx<T>::V* __restrict__ pool,
                                  const int32_t* __restrict__ piv, int nmax) {
  typedef typename Cx<T>::V V;
  const MatDesc M = mats[blockIdx.y];
  const int n = M.n;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  V* row = pool + M.elem_off + (int64_t)i * n;
  const int32_t* pv = piv + (int64_t)blockIdx.y * nmax;
  for (int k = n - 1; k >= 0; --k) {
    const int p = pv[k];
    if (p != k) {
      const V t = row[k];
      row[k] = row[p];
      row[p] = t;
    }
  }
}

// ---------------------------------------------------------------- blocked Gauss-Jordan
// Panels of GJB columns.  For the panel [k0, k0+w): (1) one workgroup per
// matrix runs the unblocked elimination with partial pivoting restricted to the
// panel columns (pivot rows >= k); (2) the panel's row interchanges are applied
// to every other column and the panel rows are copied to W; (3) every other
// column is updated, A[i][j] = (i in panel ? 0 : A[i][j]) + sum_p A[i][k0+p] W[p][j]
// (the block form of the same row operations).  Column interchanges undo the
// row interchanges at the end.
constexpr int GJB = 128;

// Wavefront maximum of a 64-bit key by DPP row shifts and row broadcasts
// (lane 15 of each row of 16 ends with its row's maximum, lane 63 with the
// wavefront's), read back from lane 63.
template <int CTRL, int ROWM>
__device__ __forceinline__ unsigned long long dpp_u64(unsigned long long v) {
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)v, CTRL, ROWM, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(v >> 32), CTRL, ROWM, 0xf, false);
  return ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo;
}
__device__ __forceinline__ unsigned long long max_u64(unsigned long long a, unsigned long long b) {
  return a > b ? a : b;
}
__device__ __forceinline__ unsigned long long readlane_u64(unsigned long long v, int l) {
  const unsigned lo = __builtin_amdgcn_readlane((int)(unsigned)v, l);
  const unsigned hi = __builtin_amdgcn_readlane((int)(unsigned)(v >> 32), l);
  return ((unsigned long long)hi << 32) | lo;
}
template <bool WHOLE_WAVE>
__device__ __forceinline__ unsigned long long dpp_max_u64(unsigned long long v) {
  v = max_u64(v, dpp_u64<0x111, 0xf>(v));   // row_shr:1
  v = max_u64(v, dpp_u64<0x112, 0xf>(v));   // row_shr:2
  v = max_u64(v, dpp_u64<0x114, 0xf>(v));   // row_shr:4
  v = max_u64(v, dpp_u64<0x118, 0xf>(v));   // row_shr:8
  if (!WHOLE_WAVE) return readlane_u64(v, 15);
  v = max_u64(v, dpp_u64<0x142, 0xa>(v));   // row_bcast:15 into rows 1, 3
  v = max_u64(v, dpp_u64<0x143, 0xc>(v));   // row_bcast:31 into rows 2, 3
  return readlane_u64(v, 63);
}

// Pivot row of column k: the row i in [k, n) of largest |a_ik|^2 (compared
// after rounding to FP32 in the FP64 elimination: candidates within FP32
// rounding of each other are equally good pivots), ties to the lower row.
// col[r] is the thread's entry in row tid + 1024 r.  One 64-bit key per
// thread (the FP32 magnitude bits, which order like the non-negative values,
// then the complemented row) reduced by DPP within each wavefront and over
// the 16 wavefronts through LDS.
template <typename T, int R>
__device__ __forceinline__ int leaf_pivot(const typename Cx<T>::V (&col)[R], int tid, int k, int n,
                                          unsigned long long* red_k) {
  const int lane = tid & 63, wave = tid >> 6;
  unsigned long long key = 0;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int i = tid + 1024 * r;
    const float m = (float)(col[r].x * col[r].x + col[r].y * col[r].y);
    const unsigned long long ki = ((unsigned long long)__float_as_uint(m) << 32) | (unsigned)~i;
    if (i >= k && i < n) key = max_u64(key, ki);
  }
  key = dpp_max_u64<true>(key);
  if (lane == 0) red_k[wave] = key;
  __syncthreads();
  key = dpp_max_u64<false>(red_k[lane & 15]);
  return (int)~(unsigned)key;
}

// Unblocked elimination with partial pivoting on the columns [c0, c0 + wcols)
// only (pivot rows >= k; row interchanges applied to these columns only), one
// workgroup of 1024 threads per matrix with the columns held in registers:
// thread t owns rows t + 1024 r, r < R, and WL <= 16 / R columns.  Per column:
// the pivot row (leaf_pivot), then one LDS exchange that carries both the
// pivot row scaled by its owner and the row it displaces, and the rank-1
// elimination of the other rows: two barriers per column.  The column loop is
// unrolled by groups of U columns only (at most 4 in FP32, 1 in FP64; the
// body stays small in the instruction cache): the group is always register
// columns [0, U) and the register columns rotate by U after each group, so
// they end in their original order.
template <typename T, int R, int WL>
__global__ __launch_bounds__(1024) void gjr_leaf_kernel(const MatDesc* __restrict__ mats,
                                                        typename Cx<T>::V* __restrict__ pool, int c0,
                                                        int wcols, int32_t* __restrict__ piv,
                                                        int nmax) {
  typedef typename Cx<T>::V V;
  const MatDesc M = mats[blockIdx.x];
  const int n = M.n;
  if (c0 >= n) return;
  V* A = pool + M.elem_off;
  const int w = min(c0 + wcols, n) - c0;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  __shared__ unsigned long long red_k[16];
  __shared__ V swap_buf[WL];
  __shared__ V rowk[WL];
  // staging of a full-width panel through LDS: wave q moves its 64 rows
  // 1024 r + 64 q + [0, 64) with 16-byte loads and stores that cover whole
  // row segments (LPR lanes per row), padded by 16 bytes per row so the
  // per-lane row reads spread over the banks
  constexpr int LPR = WL * (int)sizeof(V) / 16;   // 16-byte chunks per row
  constexpr int SROW = LPR + 1;
  constexpr int RPI = 64 / LPR;                   // rows per wave instruction
  constexpr int VPC = 16 / (int)sizeof(V);        // complex per chunk
  __shared__ float4 stage[16 * 64 * SROW];
  float4* st = stage + wave * 64 * SROW;
  const bool staged = w == WL && (M.elem_off + c0) % VPC == 0 && n % VPC == 0;
  V a[R][WL];
  if (staged) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
#pragma unroll
      for (int q = 0; q < LPR; ++q) {
        const int rr = q * RPI + lane / LPR, ch = lane % LPR;
        const int i = 1024 * r + 64 * wave + rr;
        st[rr * SROW + ch] = i < n ? reinterpret_cast<const float4*>(A + (int64_t)i * n + c0)[ch]
                                   : make_float4(0.f, 0.f, 0.f, 0.f);
      }
      __syncthreads();
      const V* row = reinterpret_cast<const V*>(st + lane * SROW);
#pragma unroll
      for (int c = 0; c < WL; ++c) a[r][c] = row[c];
      __syncthreads();
    }
  } else {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int i = tid + 1024 * r;
#pragma unroll
      for (int c = 0; c < WL; ++c)
        a[r][c] = (i < n && c < w) ? A[(int64_t)i * n + c0 + c] : Cx<T>::make(0.0, 0.0);
    }
  }
  // columns of one unrolled group; the register columns rotate by U after
  // each group (WL / U groups in all)
  constexpr int U = sizeof(T) == 8 ? 1 : (WL < 4 ? WL : 4);
#pragma unroll 1
  for (int g0 = 0; g0 < WL; g0 += U) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int kk = g0 + u;
      if (kk < w) {   // (uniform)
        const int k = c0 + kk;
        V col[R];
#pragma unroll
        for (int r = 0; r < R; ++r) col[r] = a[r][u];
        const int pr = leaf_pivot<T, R>(col, tid, k, n, red_k);
        if (tid == 0) piv[(int64_t)blockIdx.x * nmax + k] = pr;
        // one exchange through LDS: the owner of row pr publishes the scaled
        // pivot row (it becomes row k), the owner of row k its old row (it
        // becomes row pr)
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const int i = tid + 1024 * r;
          if (i == pr) {
            const V d = a[r][u];
            const T den = d.x * d.x + d.y * d.y;
            const V inv = Cx<T>::make(d.x / den, -d.y / den);
#pragma unroll
            for (int c = 0; c < WL; ++c) {
              const V x = (c == u) ? Cx<T>::make(1.0, 0.0) : a[r][c];
              rowk[c] = Cx<T>::make(fma(x.x, inv.x, -x.y * inv.y), fma(x.x, inv.y, x.y * inv.x));
            }
          }
          if (i == k && pr != k)
#pragma unroll
            for (int c = 0; c < WL; ++c) swap_buf[c] = a[r][c];
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const int i = tid + 1024 * r;
          if (i == k) {
#pragma unroll
            for (int c = 0; c < WL; ++c) a[r][c] = rowk[c];
          } else if (i < n) {
            if (i == pr)
#pragma unroll
              for (int c = 0; c < WL; ++c) a[r][c] = swap_buf[c];
            const V f = a[r][u];
#pragma unroll
            for (int c = 0; c < WL; ++c) {
              // x - f rk, with x = 0 in the pivot column
              const V x = (c == u) ? Cx<T>::make(0.0, 0.0) : a[r][c];
              const V rk = rowk[c];
              a[r][c] = Cx<T>::make(fma(-f.x, rk.x, fma(f.y, rk.y, x.x)), fma(-f.x, rk.y, fma(-f.y, rk.x, x.y)));
            }
          }
        }
      }
    }
    // rotate: the next group to register columns [0, U)
#pragma unroll
    for (int r = 0; r < R; ++r) {
      V t[WL];
#pragma unroll
      for (int c = 0; c < WL; ++c) t[c] = a[r][(c + U) % WL];
#pragma unroll
      for (int c = 0; c < WL; ++c) a[r][c] = t[c];
    }
  }
  if (staged) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      V* row = reinterpret_cast<V*>(st + lane * SROW);
#pragma unroll
      for (int c = 0; c < WL; ++c) row[c] = a[r][c];
      __syncthreads();
#pragma unroll
      for (int q = 0; q < LPR; ++q) {
        const int rr = q * RPI + lane / LPR, ch = lane % LPR;
        const int i = 1024 * r + 64 * wave + rr;
        if (i < n) reinterpret_cast<float4*>(A + (int64_t)i * n + c0)[ch] = st[rr * SROW + ch];
      }
      __syncthreads();
    }
  } else {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int i = tid + 1024 * r;
      if (i < n)
#pragma unroll
        for (int c = 0; c < WL; ++c)
          if (c < w) A[(int64_t)i * n + c0 + c] = a[r][c];
    }
  }
}

// Recursive panel factorization helpers: the row operations of the columns
// [s0, s0 + ws) (already eliminated) applied to the sibling columns
// [d0, d0 + wd): (1) their row interchanges, then the pivot rows copied to W;
// (2) A[i][d0+j] = (i in [s0, s0+ws) ? 0 : A[i][d0+j]) + sum_p A[i][s0+p] W[p][j].
//
// (1) without a chain of dependent swaps: the interchanges P_k (rows k and
// piv[k], k = s0, ..., s0 + ws - 1, in that order) leave in row p the row
// sigma(p) = P_s0(P_s0+1(... P_last(p))), so each touched row p (the ws panel
// rows and every other pivot row, once) is gathered from sigma(p) through LDS
// and stored back, 16 columns at a time.  ws, wd <= 64.
constexpr int GJN_SWAP_TPB = 256;
template <typename T>
__global__ __launch_bounds__(GJN_SWAP_TPB) void gjn_swap_copy_kernel(
    const MatDesc* __restrict__ mats, typename Cx<T>::V* __restrict__ pool, int s0, int ws, int d0,
    int wd, const int32_t* __restrict__ piv, int nmax, typename Cx<T>::V* __restrict__ W) {
  typedef typename Cx<T>::V V;
  const MatDesc M = mats[blockIdx.x];
  const int n = M.n;
  if (s0 >= n) return;
  V* A = pool + M.elem_off;
  V* Wm = W + (int64_t)blockIdx.x * GJB * GJB;
  const int send = min(s0 + ws, n), wsv = send - s0;
  const int wdv = min(d0 + wd, n) - d0;
  const int32_t* pv = piv + (int64_t)blockIdx.x * nmax;
  const int tid = threadIdx.x;
  __shared__ int ps[64];
  __shared__ int dst[128], src[128];   // touched rows (-1: none) and their sources
  __shared__ V buf[128][16];
  if (tid < wsv) ps[tid] = pv[s0 + tid];
  __syncthreads();
  if (tid < 2 * wsv) {
    int p;
    bool use = true;
    if (tid < wsv) {
      p = s0 + tid;                       // a panel row
    } else {
      const int q = tid - wsv;            // pivot row q, unless in the panel or seen before
      p = ps[q];
      use = p < s0 || p >= send;
      for (int q2 = 0; q2 < q; ++q2) use = use && ps[q2] != p;
    }
    int sg = p;
    for (int kk = wsv - 1; kk >= 0; --kk) {
      const int k = s0 + kk, pr = ps[kk];
      sg = sg == k ? pr : (sg == pr ? k : sg);
    }
    dst[tid] = use ? p : -1;
    src[tid] = sg;
  }
  __syncthreads();
  const int np = 2 * wsv;
  for (int c0 = 0; c0 < wdv; c0 += 16) {
    const int cn = min(16, wdv - c0);
    for (int e = tid; e < np * 16; e += GJN_SWAP_TPB) {
      const int q = e >> 4, c = e & 15;
      if (c < cn && dst[q] >= 0) buf[q][c] = A[(int64_t)src[q] * n + d0 + c0 + c];
    }
    __syncthreads();
    for (int e = tid; e < np * 16; e += GJN_SWAP_TPB) {
      const int q = e >> 4, c = e & 15;
      if (c < cn && dst[q] >= 0) {
        A[(int64_t)dst[q] * n + d0 + c0 + c] = buf[q][c];
        if (q < wsv) Wm[q * GJB + c0 + c] = buf[q][c];
      }
    }
    __syncthreads();
  }
}

template <typename T>
__global__ __launch_bounds__(256) void gjn_update_kernel(const MatDesc* __restrict__ mats,
                                                         typename Cx<T>::V* __restrict__ pool, int s0,
                                                         int ws, int d0, int wd,
                                                         const typename Cx<T>::V* __restrict__ W) {
  typedef typename Cx<T>::V V;
  const MatDesc M = mats[blockIdx.y];
  const int n = M.n;
  if (s0 >= n) return;
  const int send = min(s0 + ws, n);
  const int wsv = send - s0;
  const int wdv = min(d0 + wd, n) - d0;
  const int rows = 256 / wd;
  if ((int)blockIdx.x * rows >= n || wdv <= 0) return;   // no row of this matrix (uniform)
  __shared__ V Ws[32][32];   // halves of at most 32 columns (wider ones: gjm_update_kernel)
  const V* Wm = W + (int64_t)blockIdx.y * GJB * GJB;
  for (int e = threadIdx.x; e < wsv * wdv; e += 256) Ws[e / wdv][e % wdv] = Wm[(e / wdv) * GJB + e % wdv];
  __syncthreads();
  const int i = blockIdx.x * rows + threadIdx.x / wd;
  const int j = threadIdx.x % wd;
  if (i >= n || j >= wdv) return;
  V* A = pool + M.elem_off;
  const V* ar = A + (int64_t)i * n + s0;
  V acc = Cx<T>::make(0.0, 0.0);
  for (int p = 0; p < wsv; ++p) {
    const V a = ar[p], w = Ws[p][j];
    acc.x = fma(a.x, w.x, fma(-a.y, w.y, acc.x));
    acc.y = fma(a.x, w.y, fma(a.y, w.x, acc.y));
  }
  V* cptr = A + (int64_t)i * n + d0 + j;
  const bool prow = i >= s0 && i < send;
  const V base = prow ? Cx<T>::make(0.0, 0.0) : *cptr;
  *cptr = Cx<T>::make(base.x + acc.x, base.y + acc.y);
}

// Row interchanges of the panel applied to the other columns, then the panel
// rows copied to W (w x n per matrix).
template <typename T>
__global__ __launch_bounds__(256) void gjb_swap_copy_kernel(const MatDesc* __restrict__ mats,
                                                            typename Cx<T>::V* __restrict__ pool,
                                                            int k0, const int32_t* __restrict__ piv,
                                                            int nmax, typename Cx<T>::V* __restrict__ W) {
  typedef typename Cx<T>::V V;
  const MatDesc M = mats[blockIdx.y];
  const int n = M.n;
  if (k0 >= n || (int)blockIdx.x * 64 >= n) return;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int j = blockIdx.x * 64 + lane;
  const int kend = min(k0 + GJB, n);
  V* A = pool + M.elem_off;
  V* Wm = W + (int64_t)blockIdx.y * GJB * nmax;
  const bool in_panel = j >= k0 && j < kend;
  // the interchanges, in order, on the workgroup's 64 columns (first wavefront)
  if (wv == 0 && j < n && !in_panel) {
    const int32_t* pv = piv + (int64_t)blockIdx.y * nmax;
    for (int k = k0; k < kend; ++k) {
      const int pr = pv[k];
      if (pr != k) {
        const V t = A[(int64_t)k * n + j];
        A[(int64_t)k * n + j] = A[(int64_t)pr * n + j];
        A[(int64_t)pr * n + j] = t;
      }
    }
  }
  __syncthreads();
  // the panel rows into W, every fourth row per wavefront
  if (j < n) {
#pragma unroll 8
    for (int k = k0 + wv; k < kend; k += 4)
      Wm[(int64_t)(k - k0) * nmax + j] = in_panel ? Cx<T>::make(0.0, 0.0) : A[(int64_t)k * n + j];
  }
}

// A[i][j] = (i in panel ? 0 : A[i][j]) + sum_p A[i][k0+p] W[p][j] for j outside
// the panel, on the matrix cores: the complex product as a real one,
// [Re a, Im a] x [[Re w, Im w], [-Im w, Re w]], with v_mfma_f64_16x16x4f64
// (v_mfma_f32_16x16x4f32 in FP32, four workgroups per CU).  64 x 64 complex
// output tile per workgroup (64 x 128 real); each of the four wavefronts owns
// 32 rows x 64 real columns (2 x 4 MFMA tiles); the panel columns and rows
// are staged through LDS 16 complex columns at a time.
// The eliminated columns are [k0, k0 + ws); the output columns start at
// jbase (tiles of 64); row p of W holds the pivot row's entries of the output
// columns from wcol0 on (leading dimension ldw, matrix stride wstride): the
// trailing update of a panel (jbase = wcol0 = 0, W is GJB x nmax) and, inside
// the recursive panel factorization, the update of one half by the other
// (W is the half's pivot rows, GJB x GJB).
// FP64: three wavefronts per SIMD (at most 168 registers, no accumulator
// registers; the 51.7 KB of LDS also allows three workgroups per CU), 7.5 %
// faster than the two the unconstrained allocation gave (153 + 64 AGPRs).
template <typename T>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 4 : 3))) void gjm_update_kernel(const MatDesc* __restrict__ mats,
                                                         typename Cx<T>::V* __restrict__ pool, int k0, int ws,
                                                         const typename Cx<T>::V* __restrict__ W, int ldw,
                                                         int64_t wstride, int jbase, int wcol0) {
  typedef typename Cx<T>::V V;
  typedef typename MfmaAcc<T>::v4 v4;
  const MatDesc M = mats[blockIdx.z];
  const int n = M.n;
  if (k0 >= n) return;
  const int kend = min(k0 + ws, n);
  const int w = kend - k0;
  const int i0 = blockIdx.y * 64, j0 = jbase + blockIdx.x * 64;
  if (i0 >= n || j0 >= n) return;
  if (j0 >= k0 && j0 + 64 <= kend) return;  // tile inside the panel columns
  V* A = pool + M.elem_off;
  const V* Wm = W + (int64_t)blockIdx.z * wstride;
  // A chunk as rows x real k, B chunk as real k x real columns; the row
  // strides keep both the 8-byte writes and the operand reads of a
  // half-wavefront (16 rows or columns x two k) on distinct banks
  constexpr int AS = sizeof(T) == 4 ? 34 : 33;
  constexpr int BS = sizeof(T) == 4 ? 144 : 136;
  __shared__ T As[64][AS];
  __shared__ T Bs[32][BS];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = (wave >> 1) * 32, wc = (wave & 1) * 64;
  // accumulators start from the tile of A (zero on the panel rows and for
  // entries outside the matrix or inside the panel columns, which are not stored)
  v4 acc[2][4];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int i = i0 + wr + 16 * x + MfmaAcc<T>::row(lane, e);
      const bool prow = i >= k0 && i < kend;
#pragma unroll
      for (int y = 0; y < 4; ++y) {
        const int c = wc + 16 * y + (lane & 15);
        const int j = j0 + (c >> 1);
        const bool keep = i < n && j < n && !(j >= k0 && j < kend) && !prow;
        acc[x][y][e] = keep ? ((const T*)(A + (int64_t)i * n + j))[c & 1] : (T)0;
      }
    }
  // panel columns of A and rows of W, 16 at a time, the next chunk loaded into
  // registers while the current one is multiplied
  V ra[4], rw[4];
  auto load_chunk = [&](int p0) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = tid + 256 * q;
      const int rr = e >> 4, pp = e & 15;
      const int i = i0 + rr, pc = p0 + pp;
      ra[q] = (i < n && pc < w) ? A[(int64_t)i * n + k0 + pc] : Cx<T>::make(0.0, 0.0);
      const int pw = e >> 6, jj = e & 63;
      const int j = j0 + jj, pcw = p0 + pw;
      rw[q] = (j < n && pcw < w) ? Wm[(int64_t)pcw * ldw + (j - wcol0)] : Cx<T>::make(0.0, 0.0);
    }
  };
  load_chunk(0);
  for (int p0 = 0; p0 < w; p0 += 16) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = tid + 256 * q;
      const int rr = e >> 4, pp = e & 15;
      As[rr][2 * pp] = ra[q].x;
      As[rr][2 * pp + 1] = ra[q].y;
      const int pw = e >> 6, jj = e & 63;
      Bs[2 * pw][2 * jj] = rw[q].x;
      Bs[2 * pw][2 * jj + 1] = rw[q].y;
      Bs[2 * pw + 1][2 * jj] = -rw[q].y;
      Bs[2 * pw + 1][2 * jj + 1] = rw[q].x;
    }
    __syncthreads();
    if (p0 + 16 < w) load_chunk(p0 + 16);
#pragma unroll
    for (int kk = 0; kk < 32; kk += 4) {
      const int kr = kk + (lane >> 4), ci = lane & 15;
      T af[2], bf[4];
#pragma unroll
      for (int x = 0; x < 2; ++x) af[x] = As[wr + 16 * x + ci][kr];
#pragma unroll
      for (int y = 0; y < 4; ++y) bf[y] = Bs[kr][wc + 16 * y + ci];
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y) acc[x][y] = MfmaAcc<T>::mma(af[x], bf[y], acc[x][y]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int i = i0 + wr + 16 * x + MfmaAcc<T>::row(lane, e);
      if (i >= n) continue;
#pragma unroll
      for (int y = 0; y < 4; ++y) {
        const int c = wc + 16 * y + (lane & 15);   // real column in the tile
        const int j = j0 + (c >> 1);
        if (j >= n || (j >= k0 && j < kend)) continue;
        ((T*)(A + (int64_t)i * n + j))[c & 1] = acc[x][y][e];
      }
    }
}

// FP32 variant of the same update with three real products per complex one:
// with P = Re a Re w, Q = Im a Im w and S = (Re a + Im a)(Re w + Im w), the
// product is P - Q + i (S - P - Q), so the three 64 x 64 real products
// replace the 64 x 128 x 2 real product above (a quarter fewer MFMA
// operations).  Each wavefront owns 32 rows x 32 complex columns (2 x 2 tiles
// of each product); the tile of A is read when the sums are stored.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void gjm3_update_kernel(
    const MatDesc* __restrict__ mats, float2* __restrict__ pool, int k0, int ws,
    const float2* __restrict__ W, int ldw, int64_t wstride, int jbase, int wcol0) {
  typedef MfmaAcc<float>::v4 v4;
  const MatDesc M = mats[blockIdx.z];
  const int n = M.n;
  if (k0 >= n) return;
  const int kend = min(k0 + ws, n);
  const int w = kend - k0;
  const int i0 = blockIdx.y * 64, j0 = jbase + blockIdx.x * 64;
  if (i0 >= n || j0 >= n) return;
  if (j0 >= k0 && j0 + 64 <= kend) return;  // tile inside the panel columns
  float2* A = pool + M.elem_off;
  const float2* Wm = W + (int64_t)blockIdx.z * wstride;
  // Re, Im and Re + Im of the A chunk (rows x k) and of the W chunk (k x
  // columns); row strides 18 and 80 keep the operand reads of a
  // half-wavefront (16 rows or columns x two k) on distinct banks
  __shared__ float As[3][64][18];
  __shared__ float Bs[3][16][80];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
  v4 P[2][2], Q[2][2], S[2][2];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int e = 0; e < 4; ++e) P[x][y][e] = Q[x][y][e] = S[x][y][e] = 0.0f;
  float2 ra[4], rw[4];
  auto load_chunk = [&](int p0) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = tid + 256 * q;
      const int rr = e >> 4, pp = e & 15;
      const int i = i0 + rr, pc = p0 + pp;
      ra[q] = (i < n && pc < w) ? A[(int64_t)i * n + k0 + pc] : make_float2(0.0f, 0.0f);
      const int pw = e >> 6, jj = e & 63;
      const int j = j0 + jj, pcw = p0 + pw;
      rw[q] = (j < n && pcw < w) ? Wm[(int64_t)pcw * ldw + (j - wcol0)] : make_float2(0.0f, 0.0f);
    }
  };
  load_chunk(0);
  for (int p0 = 0; p0 < w; p0 += 16) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = tid + 256 * q;
      const int rr = e >> 4, pp = e & 15;
      As[0][rr][pp] = ra[q].x;
      As[1][rr][pp] = ra[q].y;
      As[2][rr][pp] = ra[q].x + ra[q].y;
      const int pw = e >> 6, jj = e & 63;
      Bs[0][pw][jj] = rw[q].x;
      Bs[1][pw][jj] = rw[q].y;
      Bs[2][pw][jj] = rw[q].x + rw[q].y;
    }
    __syncthreads();
    if (p0 + 16 < w) load_chunk(p0 + 16);
#pragma unroll
    for (int kk = 0; kk < 16; kk += 4) {
      const int kr = kk + (lane >> 4), ci = lane & 15;
#pragma unroll
      for (int m = 0; m < 3; ++m) {
        float af[2], bf[2];
#pragma unroll
        for (int x = 0; x < 2; ++x) af[x] = As[m][wr + 16 * x + ci][kr];
#pragma unroll
        for (int y = 0; y < 2; ++y) bf[y] = Bs[m][kr][wc + 16 * y + ci];
#pragma unroll
        for (int x = 0; x < 2; ++x)
#pragma unroll
          for (int y = 0; y < 2; ++y) {
            if (m == 0) P[x][y] = MfmaAcc<float>::mma(af[x], bf[y], P[x][y]);
            else if (m == 1) Q[x][y] = MfmaAcc<float>::mma(af[x], bf[y], Q[x][y]);
            else S[x][y] = MfmaAcc<float>::mma(af[x], bf[y], S[x][y]);
          }
      }
    }
    __syncthreads();
  }
  // A[i][j] = (i in panel ? 0 : A[i][j]) + P - Q + i (S - P - Q), for j
  // outside the panel columns
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int i = i0 + wr + 16 * x + MfmaAcc<float>::row(lane, e);
      if (i >= n) continue;
      const bool prow = i >= k0 && i < kend;
#pragma unroll
      for (int y = 0; y < 2; ++y) {
        const int j = j0 + wc + 16 * y + (lane & 15);
        if (j >= n || (j >= k0 && j < kend)) continue;
        float2* dst = A + (int64_t)i * n + j;
        const float2 a = prow ? make_float2(0.0f, 0.0f) : *dst;
        const float p = P[x][y][e], qv = Q[x][y][e];
        *dst = make_float2(a.x + (p - qv), a.y + (S[x][y][e] - (p + qv)));
      }
    }
}

// The matrix-core update for either element type (FP32: three products).
template <typename T>
static void launch_gjm(dim3 grid, hipStream_t s, const MatDesc* d_mats, typename Cx<T>::V* pool,
                       int k0, int ws, const typename Cx<T>::V* W, int ldw, int64_t wstride,
                       int jbase, int wcol0) {
  if constexpr (sizeof(T) == 4)
    hipLaunchKernelGGL(gjm3_update_kernel, grid, dim3(256), 0, s, d_mats, pool, k0, ws, W, ldw,
                       wstride, jbase, wcol0);
  else
    hipLaunchKernelGGL(gjm_update_kernel<T>, grid, dim3(256), 0, s, d_mats, pool, k0, ws, W, ldw,
                       wstride, jbase, wcol0);
}

// Leaf shape of the recursive panel factorization for matrices of order <= nmax:
// R rows per thread (1024 threads), WL = min(8, 16 / R) columns.
static int gj_leaf_rows(int nmax) {
  int r = 1;
  while (1024 * r < nmax) r *= 2;
  return r;
}

// FP32 leaves hold twice the columns in the same registers (fewer recursion
// steps per panel)
template <typename T>
static int gj_leaf_cols(int nmax) {
  const int c = gj_leaf_rows(nmax) == 1 ? 8 : 16 / gj_leaf_rows(nmax);
  return sizeof(T) == 4 ? 2 * c : c;
}

template <typename T>
static void launch_leaf(hipStream_t s, typename Cx<T>::V* pool, const MatDesc* d_mats, int batch,
                        int nmax, int c0, int w, int32_t* piv) {
  switch (gj_leaf_rows(nmax)) {
    case 1:
      hipLaunchKernelGGL((gjr_leaf_kernel<T, 1, sizeof(T) == 4 ? 16 : 8>), dim3(batch), dim3(1024), 0, s, d_mats, pool, c0, w, piv, nmax);
      break;
    case 2:
      hipLaunchKernelGGL((gjr_leaf_kernel<T, 2, sizeof(T) == 4 ? 16 : 8>), dim3(batch), dim3(1024), 0, s, d_mats, pool, c0, w, piv, nmax);
      break;
    case 4:
      hipLaunchKernelGGL((gjr_leaf_kernel<T, 4, sizeof(T) == 4 ? 8 : 4>), dim3(batch), dim3(1024), 0, s, d_mats, pool, c0, w, piv, nmax);
      break;
    default:
      hipLaunchKernelGGL((gjr_leaf_kernel<T, 8, sizeof(T) == 4 ? 4 : 2>), dim3(batch), dim3(1024), 0, s, d_mats, pool, c0, w, piv, nmax);
      break;
  }
}

// The row operations of the eliminated half [s0, s0 + h) applied to its
// sibling half [d0, d0 + h): halves of 64 columns or more on the matrix cores
// (one column of 64-wide tiles per 64 columns), narrower ones on the vector
// ALUs.
template <typename T>
static void launch_half_update(hipStream_t s, typename Cx<T>::V* pool, const MatDesc* d_mats, int batch,
                               int nmax, int s0, int h, int d0, typename Cx<T>::V* Wn,
                               unsigned rows_blocks) {
  if (h >= 64) {
    const unsigned tiles = (unsigned)((nmax + 63) / 64);
    launch_gjm<T>(dim3((unsigned)(h / 64), tiles, batch), s, d_mats, pool, s0, h, Wn, GJB,
                  (int64_t)GJB * GJB, d0, d0);
  } else {
    hipLaunchKernelGGL(gjn_update_kernel<T>, dim3(rows_blocks, batch), dim3(256), 0, s, d_mats, pool,
                       s0, h, d0, h, Wn);
  }
}

// Factor the panel columns [c0, c0 + w) (w a power of two, <= GJB) by halves:
// left half, its row operations on the right half, right half, its row
// operations on the left half; leaves of gj_leaf_cols columns run unblocked.
template <typename T>
static void gj_factor_panel(hipStream_t s, typename Cx<T>::V* pool, const MatDesc* d_mats, int batch,
                            int nmax, int c0, int w, int32_t* piv, typename Cx<T>::V* Wn) {
  if (w <= gj_leaf_cols<T>(nmax)) {
    launch_leaf<T>(s, pool, d_mats, batch, nmax, c0, w, piv);
    return;
  }
  const int h = w / 2;
  const unsigned rows_blocks = (unsigned)((nmax + (256 / h) - 1) / (256 / h));
  gj_factor_panel<T>(s, pool, d_mats, batch, nmax, c0, h, piv, Wn);
  hipLaunchKernelGGL(gjn_swap_copy_kernel<T>, dim3(batch), dim3(GJN_SWAP_TPB), 0, s, d_mats, pool, c0, h,
                     c0 + h, h, piv, nmax, Wn);
  launch_half_update<T>(s, pool, d_mats, batch, nmax, c0, h, c0 + h, Wn, rows_blocks);
  gj_factor_panel<T>(s, pool, d_mats, batch, nmax, c0 + h, h, piv, Wn);
  hipLaunchKernelGGL(gjn_swap_copy_kernel<T>, dim3(batch), dim3(GJN_SWAP_TPB), 0, s, d_mats, pool, c0 + h, h,
                     c0, h, piv, nmax, Wn);
  launch_half_update<T>(s, pool, d_mats, batch, nmax, c0 + h, h, c0, Wn, rows_blocks);
}

// In-place inversion of `batch` matrices of complex T (interleaved, pool in
// units of T) described on the device by `mats` (orders up to nmax, at most
// 8192), on p->stream.  work: see gj_work_bytes.  With timed set, the trailing
// updates are timed on p's counters.
template <typename T>
hipError_t gj_invert(qax_problem* p, T* pool, const MatDesc* d_mats, int batch, int nmax,
                     double* work, bool timed) {
  typedef typename Cx<T>::V V;
  if (nmax > 8192) return hipErrorInvalidValue;
  const hipStream_t s = p->stream;
  V* W = (V*)work;
  int32_t* piv = (int32_t*)(W + (int64_t)GJB * nmax * batch);
  const size_t piv_bytes = (((size_t)nmax * batch * sizeof(int32_t)) + 255) / 256 * 256;
  V* Wn = (V*)((char*)piv + piv_bytes);
  const unsigned tiles = (unsigned)((nmax + 63) / 64);
  for (int k0 = 0; k0 < nmax; k0 += GJB) {
    gj_factor_panel<T>(s, (V*)pool, d_mats, batch, nmax, k0, GJB, piv, Wn);
    hipLaunchKernelGGL(gjb_swap_copy_kernel<T>, dim3((nmax + 63) / 64, batch), dim3(256), 0, s,
                       d_mats, (V*)pool, k0, piv, nmax, W);
    if (timed) timing_begin(p, QAX_K_INVERT_UPDATE);
    launch_gjm<T>(dim3(tiles, tiles, batch), s, d_mats, (V*)pool, k0, GJB, W, nmax,
                  (int64_t)GJB * nmax, 0, 0);
    if (timed) timing_end(p, QAX_K_INVERT_UPDATE);
  }
  hipLaunchKernelGGL(gj_unpivot_kernel<T>, dim3((nmax + 255) / 256, batch), dim3(256), 0, s, d_mats,
                     (V*)pool, piv, nmax);
  return hipGetLastError();
}

size_t gj_work_bytes(int batch, int nmax) {
  return (size_t)nmax * batch * sizeof(double2) * GJB +
         (((size_t)nmax * batch * sizeof(int32_t)) + 255) / 256 * 256 +
         (size_t)batch * GJB * GJB * sizeof(double2);
}

// Caller matrices: `count` complex128 matrices of the given orders stored one
// after another (row-major), inverted in place; FP64, or (mixed) rounded to
// FP32, inverted in FP32 and widened back.  work: invert_matrices_work_bytes.
size_t invert_matrices_work_bytes(int count, int nmax, int64_t total_elems, bool f32) {
  return ((count * sizeof(MatDesc) + 255) / 256) * 256 + gj_work_bytes(count, nmax) +
         (f32 ? (size_t)total_elems * 8 : 0);
}

hipError_t launch_invert_matrices(qax_problem* p, bool f32, int count, const int32_t* orders,
                                  double* mats, double* work) {
  std::vector<MatDesc> md(count);
  int nmax = 0;
  int64_t off = 0;
  for (int i = 0; i < count; ++i) {
    md[i].elem_off = off;
    md[i].n = orders[i];
    nmax = std::max(nmax, orders[i]);
    off += (int64_t)orders[i] * orders[i];
  }
  MatDesc* d_md = (MatDesc*)work;
  double* w2 = (double*)((char*)work + ((count * sizeof(MatDesc) + 255) / 256) * 256);
  hipError_t e = hipMemcpyAsync(d_md, md.data(), count * sizeof(MatDesc), hipMemcpyHostToDevice,
                                p->stream);
  if (e != hipSuccess) return e;
  if (!f32) return gj_invert<double>(p, mats, d_md, count, nmax, w2, false);
  float* pool = (float*)((char*)w2 + gj_work_bytes(count, nmax));
  if ((e = launch_convert_f32(p->stream, mats, pool, 2 * off)) != hipSuccess) return e;
  if ((e = gj_invert<float>(p, pool, d_md, count, nmax, w2, false)) != hipSuccess) return e;
  hipLaunchKernelGGL(convert_f64_kernel, dim3((unsigned)((2 * off + 255) / 256)), dim3(256), 0,
                     p->stream, pool, mats, 2 * off);
  return hipGetLastError();
}

// ---------------------------------------------------------------- mirror-symmetric blocks
// The self block of a mirror-symmetric body (mirror_symmetric) commutes with
// the node permutations of the reflections R_h (theta -> -theta) and R_t
// (t -> -t).  Orbit o = (s, j), s < n_s / 2, j <= N: its nodes g(o) for the
// group elements g = R_h^a R_t^b (two nodes where j is 0 or N, which R_h
// fixes).  With the characters chi_c(g) = (-1)^(c_h a + c_t b), c = c_h + 2 c_t,
// B splits into four blocks
//   M_c[o1, o2] = sum over the distinct nodes g(o2) of chi_c(g) B[o1, g(o2)]
// (orbits with j = 0 or N only in the blocks with c_h = 0), of orders
// (n_s / 2)(N + 1) and (n_s / 2)(N - 1), and
//   B^-1[g1(o1), g2(o2)] = (1 / |orbit of o2|) sum_c chi_c(g1) chi_c(g2) M_c^-1[o1, o2]
// over the blocks that hold both orbits: four inversions of about a quarter
// of the order, 1/16 of the elimination work.  Orbit index in block c:
// s (N + 1) + j for c_h = 0, s (N - 1) + j - 1 for c_h = 1.
struct SymInvDesc {
  int64_t b_off;      // complex offset of B and B^-1 in the block pools
  int64_t m_off[4];   // complex offset of M_c in the reduced pool
  int32_t ns, nth;    // Gauss-Legendre nodes along the curve, azimuths
};

struct SymInvRow {
  int32_t blk;   // index into the descriptors
  int32_t o1;    // orbit of the row, numbered s (N + 1) + j
};

// Host plan: descriptors, one row item per orbit of every symmetric block,
// the reduced matrices and the blocks inverted as they are.
struct SymInvPlan {
  std::vector<SymInvDesc> desc;
  std::vector<SymInvRow> rows;
  std::vector<MatDesc> red, plain;
  int nmax_red = 0, nmax_plain = 0;
  int64_t red_elems = 0;
  size_t off_red = 0, off_plain = 0, off_desc = 0, off_rows = 0, off_gj = 0, off_pool = 0, bytes = 0;
};

static size_t align256(size_t b) { return (b + 255) / 256 * 256; }

static void plan_sym_inverse(const qax_problem* p, size_t elem_bytes, SymInvPlan& P) {
  for (const BlockDev& bk : p->hblocks) {
    const BodyDev& B = p->hbodies[bk.rep_body];
    if (!mirror_symmetric(B.shape)) {
      P.plain.push_back(MatDesc{bk.elem_off, bk.n});
      P.nmax_plain = std::max(P.nmax_plain, bk.n);
      continue;
    }
    const int nth = B.n_theta, N = nth / 2, ns = bk.n / nth, half = ns / 2;
    SymInvDesc d;
    d.b_off = bk.elem_off;
    d.ns = ns;
    d.nth = nth;
    for (int c = 0; c < 4; ++c) {
      const int m = half * ((c & 1) ? N - 1 : N + 1);
      d.m_off[c] = P.red_elems;
      P.red_elems += (int64_t)m * m;
      P.red.push_back(MatDesc{d.m_off[c], m});
      P.nmax_red = std::max(P.nmax_red, m);
    }
    const int blk = (int)P.desc.size();
    P.desc.push_back(d);
    for (int o = 0; o < half * (N + 1); ++o) P.rows.push_back(SymInvRow{blk, o});
  }
  P.off_red = 0;
  P.off_plain = align256(P.red.size() * sizeof(MatDesc));
  P.off_desc = P.off_plain + align256(P.plain.size() * sizeof(MatDesc));
  P.off_rows = P.off_desc + align256(P.desc.size() * sizeof(SymInvDesc));
  P.off_gj = P.off_rows + align256(P.rows.size() * sizeof(SymInvRow));
  const size_t gj = std::max(P.red.empty() ? 0 : gj_work_bytes((int)P.red.size(), P.nmax_red),
                             P.plain.empty() ? 0 : gj_work_bytes((int)P.plain.size(), P.nmax_plain));
  P.off_pool = P.off_gj + align256(gj);
  // the reduced blocks live in the workspace unless the handle keeps them
  P.bytes = P.off_pool + (p->symap.on ? 0 : (size_t)P.red_elems * elem_bytes);
}

// M_c from B for one orbit row (o1) per workgroup, columns o2 over the threads.
template <typename T>
__global__ __launch_bounds__(256) void sym_reduce_kernel(const SymInvRow* __restrict__ rows,
                                                         const SymInvDesc* __restrict__ descs,
                                                         const double2* __restrict__ B,
                                                         typename Cx<T>::V* __restrict__ M) {
  const SymInvRow R = rows[blockIdx.x];
  const SymInvDesc D = descs[R.blk];
  const int nth = D.nth, N = nth / 2, ns = D.ns, n = ns * nth, half = ns / 2;
  const int np = N + 1, nm = N - 1;
  const int s1 = R.o1 / np, j1 = R.o1 % np;
  const bool fix1 = j1 == 0 || j1 == N;
  const double2* brow = B + D.b_off + (int64_t)(s1 * nth + j1) * n;
  const int64_t r0 = (int64_t)R.o1 * (half * np), r1 = (int64_t)(s1 * nm + j1 - 1) * (half * nm);
  for (int o2 = threadIdx.x; o2 < half * np; o2 += blockDim.x) {
    const int s2 = o2 / np, j2 = o2 % np, s2m = ns - 1 - s2;
    const double2 b0 = brow[s2 * nth + j2], bt = brow[s2m * nth + j2];
    const bool fix2 = j2 == 0 || j2 == N;
    double2 bh = make_double2(0.0, 0.0), bht = make_double2(0.0, 0.0);
    if (!fix2) {
      bh = brow[s2 * nth + nth - j2];
      bht = brow[s2m * nth + nth - j2];
    }
    // c_h = 0: b0 + bh +- (bt + bht)
    const double2 e0 = make_double2(b0.x + bh.x, b0.y + bh.y), et = make_double2(bt.x + bht.x, bt.y + bht.y);
    M[D.m_off[0] + r0 + o2] = Cx<T>::make((T)(e0.x + et.x), (T)(e0.y + et.y));
    M[D.m_off[2] + r0 + o2] = Cx<T>::make((T)(e0.x - et.x), (T)(e0.y - et.y));
    if (!fix1 && !fix2) {
      // c_h = 1: b0 - bh +- (bt - bht)
      const double2 d0 = make_double2(b0.x - bh.x, b0.y - bh.y), dt = make_double2(bt.x - bht.x, bt.y - bht.y);
      const int64_t c1 = s2 * nm + j2 - 1;
      M[D.m_off[1] + r1 + c1] = Cx<T>::make((T)(d0.x + dt.x), (T)(d0.y + dt.y));
      M[D.m_off[3] + r1 + c1] = Cx<T>::make((T)(d0.x - dt.x), (T)(d0.y - dt.y));
    }
  }
}

// B^-1 from the inverses M_c^-1: every pair of images of (o1, o2).
template <typename T>
__global__ __launch_bounds__(256) void sym_expand_kernel(const SymInvRow* __restrict__ rows,
                                                         const SymInvDesc* __restrict__ descs,
                                                         const typename Cx<T>::V* __restrict__ M,
                                                         typename Cx<T>::V* __restrict__ Binv) {
  typedef typename Cx<T>::V V;
  const SymInvRow R = rows[blockIdx.x];
  const SymInvDesc D = descs[R.blk];
  const int nth = D.nth, N = nth / 2, ns = D.ns, n = ns * nth, half = ns / 2;
  const int np = N + 1, nm = N - 1;
  const int s1 = R.o1 / np, j1 = R.o1 % np;
  const bool fix1 = j1 == 0 || j1 == N;
  const int64_t r0 = (int64_t)R.o1 * (half * np), r1 = (int64_t)(s1 * nm + j1 - 1) * (half * nm);
  // rows of the images: [a_t][a_h] (a_h = 1 only where R_h moves the orbit)
  V* rw[2][2];
  for (int at = 0; at < 2; ++at)
    for (int ah = 0; ah < 2; ++ah) {
      const int s = at ? ns - 1 - s1 : s1, j = ah ? (nth - j1) % nth : j1;
      rw[at][ah] = Binv + D.b_off + (int64_t)(s * nth + j) * n;
    }
  for (int o2 = threadIdx.x; o2 < half * np; o2 += blockDim.x) {
    const int s2 = o2 / np, j2 = o2 % np;
    const bool fix2 = j2 == 0 || j2 == N;
    const V m0 = M[D.m_off[0] + r0 + o2], m2 = M[D.m_off[2] + r0 + o2];
    V m1 = Cx<T>::make(0, 0), m3 = Cx<T>::make(0, 0);
    if (!fix1 && !fix2) {
      const int64_t c1 = s2 * nm + j2 - 1;
      m1 = M[D.m_off[1] + r1 + c1];
      m3 = M[D.m_off[3] + r1 + c1];
    }
    const T w = fix2 ? (T)0.5 : (T)0.25;
    // same t image (p_t = +1): m0 + m2 +- (m1 + m3); other: m0 - m2 +- (m1 - m3)
    const V ap = Cx<T>::make((m0.x + m2.x) * w, (m0.y + m2.y) * w);
    const V am = Cx<T>::make((m0.x - m2.x) * w, (m0.y - m2.y) * w);
    const V cp = Cx<T>::make((m1.x + m3.x) * w, (m1.y + m3.y) * w);
    const V cm = Cx<T>::make((m1.x - m3.x) * w, (m1.y - m3.y) * w);
    const int col[2] = {s2 * nth, (ns - 1 - s2) * nth};   // column slice of the t images
    const int jj[2] = {j2, (nth - j2) % nth};
    for (int at = 0; at < 2; ++at)
      for (int ah = 0; ah < (fix1 ? 1 : 2); ++ah)
        for (int bt = 0; bt < 2; ++bt) {
          const V a = at == bt ? ap : am, c = at == bt ? cp : cm;
          for (int bh = 0; bh < (fix2 ? 1 : 2); ++bh) {
            const T sg = ah == bh ? (T)1 : (T)-1;
            rw[at][ah][col[bt] + jj[bh]] = Cx<T>::make(a.x + sg * c.x, a.y + sg * c.y);
          }
        }
  }
}

// ---- one right-hand side through the reduced inverses (every block
// mirror-symmetric).  With v = sum_c sum_o u_c[o] e_c(o), e_c(o) the vector
// with chi_c(g) at the nodes g(o) of orbit o,
//   u_c[o] = |orbit|^-1 sum over the distinct nodes g(o) of chi_c(g) v[g(o)],
// B^-1 v = sum_c sum_o (M_c^-1 u_c)[o] e_c(o).  Per body the reduced vectors
// hold the four segments c = 0, 1, 2, 3 (lengths (n_s/2)(N + 1),
// (n_s/2)(N - 1), (n_s/2)(N + 1), (n_s/2)(N - 1)) at the body's node offset.
__global__ __launch_bounds__(256) void sym_vec_reduce_kernel(const SymBody* __restrict__ bodies,
                                                             const double2* __restrict__ v,
                                                             double2* __restrict__ u,
                                                             const int32_t* __restrict__ seg_active) {
  const SymBody B = bodies[blockIdx.x];
  if (seg_active && seg_active[B.problem] == 0) return;
  const int nth = B.nth, N = nth / 2, ns = B.ns, half = ns / 2, np = N + 1, nm = N - 1;
  const int64_t lp = (int64_t)half * np, lm = (int64_t)half * nm;
  const double2* vb = v + B.off;
  double2* ub = u + B.off;
  for (int o = threadIdx.x; o < half * np; o += blockDim.x) {
    const int s = o / np, j = o % np, sm = ns - 1 - s;
    const double2 a = vb[s * nth + j], at = vb[sm * nth + j];
    if (j == 0 || j == N) {
      ub[o] = make_double2(0.5 * (a.x + at.x), 0.5 * (a.y + at.y));
      ub[lp + lm + o] = make_double2(0.5 * (a.x - at.x), 0.5 * (a.y - at.y));
    } else {
      const double2 ah = vb[s * nth + nth - j], aht = vb[sm * nth + nth - j];
      const int64_t o1 = (int64_t)s * nm + j - 1;
      ub[o] = make_double2(0.25 * (a.x + ah.x + at.x + aht.x), 0.25 * (a.y + ah.y + at.y + aht.y));
      ub[lp + o1] = make_double2(0.25 * (a.x - ah.x + at.x - aht.x), 0.25 * (a.y - ah.y + at.y - aht.y));
      ub[lp + lm + o] = make_double2(0.25 * (a.x + ah.x - at.x - aht.x), 0.25 * (a.y + ah.y - at.y - aht.y));
      ub[2 * lp + lm + o1] =
          make_double2(0.25 * (a.x - ah.x - at.x + aht.x), 0.25 * (a.y - ah.y - at.y + aht.y));
    }
  }
}

// w = M_c^-1 u per segment: 16 rows per workgroup (four per wavefront), the
// segment's input staged in LDS, FP64 accumulation (as block_gemv_f32_lds_kernel).
template <typename MT, int VEC>
__global__ __launch_bounds__(256) void sym_seg_gemv_kernel(const SymSeg* __restrict__ segs,
                                                           const int2* __restrict__ groups,
                                                           const MT* __restrict__ pool,
                                                           const double2* __restrict__ u,
                                                           double2* __restrict__ w,
                                                           const int32_t* __restrict__ seg_active) {
  typedef MT vec_t __attribute__((ext_vector_type(2 * VEC)));
  __shared__ double2 vs[GV_CH];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int2 G = groups[blockIdx.x];
  const SymSeg S = segs[G.x];
  if (seg_active && seg_active[S.problem] == 0) return;
  const int n = S.n, r0 = G.y + wave * (GV_ROWS / 4);
  const double2* ub = u + S.voff;
  double ar[GV_ROWS / 4], ai[GV_ROWS / 4];
#pragma unroll
  for (int q = 0; q < GV_ROWS / 4; ++q) { ar[q] = 0.0; ai[q] = 0.0; }
  for (int c0 = 0; c0 < n; c0 += GV_CH) {
    const int cn = min(GV_CH, n - c0);
    __syncthreads();
    for (int q = threadIdx.x; q < cn; q += 256) vs[q] = ub[c0 + q];
    __syncthreads();
    const MT* a = pool + 2 * (S.moff + (int64_t)r0 * n + c0);
    for (int j0 = lane * VEC; j0 < cn; j0 += 64 * VEC) {
      vec_t av[GV_ROWS / 4];
#pragma unroll
      for (int rr = 0; rr < GV_ROWS / 4; ++rr) {
        if (r0 + rr < n) av[rr] = *(const vec_t*)(a + 2 * ((int64_t)rr * n + j0));
        else av[rr] = (vec_t)0;
      }
#pragma unroll
      for (int q = 0; q < VEC; ++q) {
        const double2 x = vs[j0 + q];
#pragma unroll
        for (int rr = 0; rr < GV_ROWS / 4; ++rr) {
          const double mr = (double)av[rr][2 * q], mi = (double)av[rr][2 * q + 1];
          ar[rr] = fma(mr, x.x, fma(-mi, x.y, ar[rr]));
          ai[rr] = fma(mr, x.y, fma(mi, x.x, ai[rr]));
        }
      }
    }
  }
#pragma unroll
  for (int rr = 0; rr < GV_ROWS / 4; ++rr) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      ar[rr] += __shfl_xor(ar[rr], off);
      ai[rr] += __shfl_xor(ai[rr], off);
    }
    if (lane == 0 && r0 + rr < n) w[S.voff + r0 + rr] = make_double2(ar[rr], ai[rr]);
  }
}

// y (+)= sum_c chi_c(g) w_c[o] at the nodes g(o).
__global__ __launch_bounds__(256) void sym_vec_expand_kernel(const SymBody* __restrict__ bodies,
                                                             const double2* __restrict__ w,
                                                             double2* __restrict__ y, int accumulate,
                                                             const int32_t* __restrict__ seg_active) {
  const SymBody B = bodies[blockIdx.x];
  const int nth = B.nth, N = nth / 2, ns = B.ns, half = ns / 2, np = N + 1, nm = N - 1;
  double2* yb = y + B.off;
  if (seg_active && seg_active[B.problem] == 0) {
    // a converged lockstep segment: its input is zero, so is the output
    if (!accumulate)
      for (int e = threadIdx.x; e < ns * nth; e += blockDim.x) yb[e] = make_double2(0.0, 0.0);
    return;
  }
  const int64_t lp = (int64_t)half * np, lm = (int64_t)half * nm;
  const double2* wb = w + B.off;
  auto put = [&](int e, double re, double im) {
    double2 o = accumulate ? yb[e] : make_double2(0.0, 0.0);
    o.x += re;
    o.y += im;
    yb[e] = o;
  };
  for (int o = threadIdx.x; o < half * np; o += blockDim.x) {
    const int s = o / np, j = o % np, sm = ns - 1 - s;
    const double2 m0 = wb[o], m2 = wb[lp + lm + o];
    if (j == 0 || j == N) {
      put(s * nth + j, m0.x + m2.x, m0.y + m2.y);
      put(sm * nth + j, m0.x - m2.x, m0.y - m2.y);
    } else {
      const int64_t o1 = (int64_t)s * nm + j - 1;
      const double2 m1 = wb[lp + o1], m3 = wb[2 * lp + lm + o1];
      put(s * nth + j, m0.x + m1.x + m2.x + m3.x, m0.y + m1.y + m2.y + m3.y);
      put(sm * nth + j, m0.x + m1.x - m2.x - m3.x, m0.y + m1.y - m2.y - m3.y);
      put(s * nth + nth - j, m0.x - m1.x + m2.x - m3.x, m0.y - m1.y + m2.y - m3.y);
      put(sm * nth + nth - j, m0.x - m1.x - m2.x + m3.x, m0.y - m1.y - m2.y + m3.y);
    }
  }
}

static void launch_sym_apply(qax_problem* p, int prec, const double* v, double* out, bool accumulate) {
  auto& A = p->symap;
  hipLaunchKernelGGL(sym_vec_reduce_kernel, dim3((unsigned)A.n_bodies), dim3(256), 0, p->stream, A.d_bodies,
                     (const double2*)v, (double2*)A.d_u, p->seg_active);
  if (prec == QAX_MIXED)
    hipLaunchKernelGGL((sym_seg_gemv_kernel<float, 4>), dim3((unsigned)A.n_groups), dim3(256), 0, p->stream,
                       A.d_segs, A.d_groups, A.d_Minv32, (const double2*)A.d_u, (double2*)A.d_w, p->seg_active);
  else
    hipLaunchKernelGGL((sym_seg_gemv_kernel<double, 2>), dim3((unsigned)A.n_groups), dim3(256), 0, p->stream,
                       A.d_segs, A.d_groups, A.d_Minv, (const double2*)A.d_u, (double2*)A.d_w, p->seg_active);
  hipLaunchKernelGGL(sym_vec_expand_kernel, dim3((unsigned)A.n_bodies), dim3(256), 0, p->stream, A.d_bodies,
                     (const double2*)A.d_w, (double2*)out, accumulate ? 1 : 0, p->seg_active);
}

// Symmetric blocks: B -> M_c (reduced pool), inverted there, B^-1 (FP64 into
// d_Binv, FP32 into d_Binv32); the others inverted in place in the inverse
// pool of their precision.  The inverse pool of a non-symmetric block holds
// a copy of B (FP64) or B rounded to FP32 on entry.
template <typename T>
static hipError_t invert_blocks_sym(qax_problem* p, const SymInvPlan& P, char* work,
                                    typename Cx<T>::V* inv_pool) {
  const hipStream_t s = p->stream;
  MatDesc* d_red = (MatDesc*)(work + P.off_red);
  MatDesc* d_plain = (MatDesc*)(work + P.off_plain);
  SymInvDesc* d_desc = (SymInvDesc*)(work + P.off_desc);
  SymInvRow* d_rows = (SymInvRow*)(work + P.off_rows);
  double* gjw = (double*)(work + P.off_gj);
  T* pool = (T*)(work + P.off_pool);
  if (p->symap.on) pool = sizeof(T) == 8 ? (T*)p->symap.d_Minv : (T*)p->symap.d_Minv32;
  hipError_t e = hipSuccess;
  if (!P.red.empty()) {
    e = hipMemcpyAsync(d_red, P.red.data(), P.red.size() * sizeof(MatDesc), hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
      e = hipMemcpyAsync(d_desc, P.desc.data(), P.desc.size() * sizeof(SymInvDesc), hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
      e = hipMemcpyAsync(d_rows, P.rows.data(), P.rows.size() * sizeof(SymInvRow), hipMemcpyHostToDevice, s);
  }
  if (e == hipSuccess && !P.plain.empty())
    e = hipMemcpyAsync(d_plain, P.plain.data(), P.plain.size() * sizeof(MatDesc), hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return e;
  timing_begin(p, QAX_K_INVERT);
  if (!P.red.empty()) {
    hipLaunchKernelGGL(sym_reduce_kernel<T>, dim3((unsigned)P.rows.size()), dim3(256), 0, s, d_rows,
                       d_desc, (const double2*)p->d_B, (typename Cx<T>::V*)pool);
    e = hipGetLastError();
    if (e == hipSuccess) e = gj_invert<T>(p, pool, d_red, (int)P.red.size(), P.nmax_red, gjw, true);
    if (e == hipSuccess) {
      hipLaunchKernelGGL(sym_expand_kernel<T>, dim3((unsigned)P.rows.size()), dim3(256), 0, s, d_rows,
                         d_desc, (const typename Cx<T>::V*)pool, inv_pool);
      e = hipGetLastError();
    }
  }
  if (e == hipSuccess && !P.plain.empty())
    e = gj_invert<T>(p, (T*)inv_pool, d_plain, (int)P.plain.size(), P.nmax_plain, gjw, true);
  timing_end(p, QAX_K_INVERT);
  return e;
}

// Every distinct self block inverted in FP32 for the mixed path (matrix cores
// at the FP32 rate); the FP64 inverse is made on demand by
// launch_invert_blocks64.
hipError_t launch_invert_blocks(qax_problem* p, double* work) {
  p->inv64_ready = false;
  SymInvPlan P;
  plan_sym_inverse(p, sizeof(float2), P);
  // block_elems complex elements = block_elems (re, im) pairs; B rounded to
  // FP32 (and into the inverse pool where a block is inverted as it is)
  p->b32_ready = true;
  if (P.plain.empty()) {
    hipError_t e = launch_convert_f32(p->stream, p->d_B, (float*)p->d_B32, 2 * p->block_elems);
    if (e != hipSuccess) return e;
  } else {
    hipLaunchKernelGGL(convert_f32_twice_kernel, dim3((unsigned)((p->block_elems + 255) / 256)),
                       dim3(256), 0, p->stream, (const double2*)p->d_B, (float2*)p->d_B32,
                       (float2*)p->d_Binv32, p->block_elems);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return invert_blocks_sym<float>(p, P, (char*)work, (float2*)p->d_Binv32);
}

// Factorisation in FP64 for both paths: the FP64 inverse (below), then B^-1
// rounded to FP32 for the mixed path.
hipError_t launch_factor_blocks64(qax_problem* p, double* work) {
  hipError_t e = launch_invert_blocks64(p, work);
  if (e != hipSuccess) return e;
  if (p->symap.on) {
    e = launch_convert_f32(p->stream, p->symap.d_Minv, p->symap.d_Minv32, 2 * p->symap.elems);
    if (e != hipSuccess) return e;
  }
  // B^-1 rounded to FP32 (the mixed path's preconditioner); B itself on
  // first use (ensure_b32)
  p->b32_ready = false;
  return launch_convert_f32(p->stream, p->d_Binv, (float*)p->d_Binv32, 2 * p->block_elems);
}

// FP64 inverse: symmetric blocks through their four reduced blocks, the
// others copied into Binv and inverted in place.
hipError_t launch_invert_blocks64(qax_problem* p, double* work) {
  SymInvPlan P;
  plan_sym_inverse(p, sizeof(double2), P);
  if (P.red.empty()) {
    hipError_t e = hipMemcpyAsync(p->d_Binv, p->d_B, (size_t)p->block_elems * 16,
                                  hipMemcpyDeviceToDevice, p->stream);
    if (e != hipSuccess) return e;
  } else {
    for (const MatDesc& m : P.plain) {
      hipError_t e = hipMemcpyAsync(p->d_Binv + 2 * m.elem_off, p->d_B + 2 * m.elem_off,
                                    (size_t)m.n * m.n * 16, hipMemcpyDeviceToDevice, p->stream);
      if (e != hipSuccess) return e;
    }
  }
  return invert_blocks_sym<double>(p, P, (char*)work, (double2*)p->d_Binv);
}

// The reduced inverses and the tables of the one-right-hand-side apply, when
// every block is mirror-symmetric (after qax_build, before the first
// factorisation).
void free_sym_apply(qax_problem* p) {
  auto& A = p->symap;
  dev_release(p, A.d_Minv);
  dev_release(p, A.d_Minv32);
  dev_release(p, A.d_mem);
  A = qax_problem::SymApply{};
}

hipError_t setup_sym_apply(qax_problem* p) {
  if (p->symap.on) return hipSuccess;
  for (const BlockDev& bk : p->hblocks)
    if (!mirror_symmetric(p->hbodies[bk.rep_body].shape)) return hipSuccess;
  if (p->hblocks.empty()) return hipSuccess;
  SymInvPlan P;
  plan_sym_inverse(p, sizeof(double2), P);   // m_off of every block (all symmetric: desc = block)
  std::vector<SymSeg> segs;
  std::vector<int2> groups;
  std::vector<SymBody> bodies;
  for (int b = 0; b < p->n_bodies; ++b) {
    const BodyDev& B = p->hbodies[b];
    const SymInvDesc& D = P.desc[B.block];
    const int nth = B.n_theta, N = nth / 2, ns = D.ns, half = ns / 2;
    bodies.push_back(SymBody{B.off, ns, nth, B.problem});
    int64_t start = 0;
    for (int c = 0; c < 4; ++c) {
      const int m = half * ((c & 1) ? N - 1 : N + 1);
      const int si = (int)segs.size();
      segs.push_back(SymSeg{B.off + start, D.m_off[c], m, B.problem});
      for (int r = 0; r < m; r += GV_ROWS) groups.push_back(make_int2(si, r));
      start += m;
    }
  }
  auto& A = p->symap;
  A.elems = P.red_elems;
  A.n_groups = (int)groups.size();
  A.n_bodies = (int)bodies.size();
  const size_t bs = align256(segs.size() * sizeof(SymSeg)), bg = align256(groups.size() * sizeof(int2)),
               bb = align256(bodies.size() * sizeof(SymBody)), bv = align256((size_t)p->N * 16);
  hipError_t e = dev_alloc(p, (void**)&A.d_Minv, (size_t)A.elems * 16);
  if (e == hipSuccess) e = dev_alloc(p, (void**)&A.d_Minv32, (size_t)A.elems * 8);
  if (e == hipSuccess) e = dev_alloc(p, &A.d_mem, bs + bg + bb + 2 * bv);
  if (e != hipSuccess) {
    free_sym_apply(p);
    return e;
  }
  char* m = (char*)A.d_mem;
  A.d_segs = (SymSeg*)m;
  A.d_groups = (int2*)(m + bs);
  A.d_bodies = (SymBody*)(m + bs + bg);
  A.d_u = (double*)(m + bs + bg + bb);
  A.d_w = (double*)(m + bs + bg + bb + bv);
  e = hipMemcpyAsync(A.d_segs, segs.data(), segs.size() * sizeof(SymSeg), hipMemcpyHostToDevice, p->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(A.d_groups, groups.data(), groups.size() * sizeof(int2), hipMemcpyHostToDevice, p->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(A.d_bodies, bodies.data(), bodies.size() * sizeof(SymBody), hipMemcpyHostToDevice,
                       p->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
  if (e != hipSuccess) {
    free_sym_apply(p);
    return e;
  }
  A.on = true;
  return hipSuccess;
}

size_t invert_blocks_work_bytes(qax_problem* p) {
  SymInvPlan P64, P32;
  plan_sym_inverse(p, sizeof(double2), P64);
  plan_sym_inverse(p, sizeof(float2), P32);
  return std::max(P64.bytes, P32.bytes);
}

// ---------------------------------------------------------------- dense system
constexpr double INV_FOUR_PI_D = 0.0795774715459476678844;

// Off-diagonal entries A[i][j] (different bodies, same problem) of the full
// system; entries of a body with itself are left untouched.
__global__ void dense_offdiag_kernel(const BodyDev* __restrict__ bodies,
                                     const int32_t* __restrict__ node_body,
                                     const double* __restrict__ pos, const double* __restrict__ aw,
                                     int64_t N, double2* __restrict__ A) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t i = blockIdx.y;
  if (j >= N) return;
  const int bi = node_body[i], bj = node_body[j];
  if (bi == bj) return;
  if (bodies[bi].problem != bodies[bj].problem) {
    A[i * N + j] = make_double2(0.0, 0.0);
    return;
  }
  const double k = bodies[bi].k;
  const double dx = pos[j] - pos[i], dy = pos[N + j] - pos[N + i], dz = pos[2 * N + j] - pos[2 * N + i];
  const double r2 = dx * dx + dy * dy + dz * dz;
  const double ir = rsqrt(r2);
  const double r = r2 * ir;
  double s, c;
  sincos_cw(k * r, &s, &c);
  const double sc = (aw[j] * dx + aw[N + j] * dy + aw[2 * N + j] * dz) * ir * ir * ir * INV_FOUR_PI_D;
  A[i * N + j] = make_double2(-(c + k * r * s) * sc, (k * r * c - s) * sc);
}

// Copy each body's self block into its diagonal block of the dense matrix.
__global__ void dense_diag_kernel(const BodyDev* __restrict__ bodies,
                                  const BlockDev* __restrict__ blocks,
                                  const int32_t* __restrict__ node_body,
                                  const double2* __restrict__ pool, int64_t N,
                                  double2* __restrict__ A) {
  const int64_t i = blockIdx.y;
  const int b = node_body[i];
  const BodyDev& B = bodies[b];
  const BlockDev& K = blocks[B.block];
  const int jl = blockIdx.x * blockDim.x + threadIdx.x;
  if (jl >= K.n) return;
  const int il = (int)(i - B.off);
  A[i * N + B.off + jl] = pool[K.elem_off + (int64_t)il * K.n + jl];
}

hipError_t launch_dense_system(qax_problem* p, double* A) {
  hipLaunchKernelGGL(dense_offdiag_kernel, dim3((unsigned)((p->N + 255) / 256), (unsigned)p->N),
                     dim3(256), 0, p->stream, p->d_bodies, p->d_node_body, p->d_pos, p->d_aw, p->N,
                     (double2*)A);
  int nmax = 0;
  for (auto& b : p->hblocks) nmax = std::max(nmax, b.n);
  hipLaunchKernelGGL(dense_diag_kernel, dim3((unsigned)((nmax + 255) / 256), (unsigned)p->N),
                     dim3(256), 0, p->stream, p->d_bodies, p->d_blocks, p->d_node_body,
                     (const double2*)p->d_B, p->N, (double2*)A);
  return hipGetLastError();
}

// x = Ainv b for a dense N x N inverse and N x nrhs right-hand sides.
__global__ void dense_matvec_kernel(const double2* __restrict__ A, int64_t N,
                                    const double2* __restrict__ b, int nrhs,
                                    double2* __restrict__ x) {
  const int lane = threadIdx.x & 63;
  const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int r = blockIdx.y;
  if (row >= N) return;
  double ar = 0.0, ai = 0.0;
  for (int64_t j = lane; j < N; j += 64) {
    const double2 a = A[row * N + j];
    const double2 v = b[j * nrhs + r];
    ar += a.x * v.x - a.y * v.y;
    ai += a.x * v.y + a.y * v.x;
  }
  for (int off = 32; off > 0; off >>= 1) {
    ar += __shfl_xor(ar, off);
    ai += __shfl_xor(ai, off);
  }
  if (lane == 0) x[row * nrhs + r] = make_double2(ar, ai);
}

hipError_t launch_dense_solve(qax_problem* p, double* A, const double* b, int nrhs, double* x,
                              double* work) {
  MatDesc md{0, (int32_t)p->N};
  MatDesc* d_md = (MatDesc*)work;
  double* w2 = (double*)((char*)work + 256);
  hipError_t e = hipMemcpyAsync(d_md, &md, sizeof(MatDesc), hipMemcpyHostToDevice, p->stream);
  if (e != hipSuccess) return e;
  e = gj_invert<double>(p, A, d_md, 1, (int)p->N, w2, false);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(dense_matvec_kernel, dim3((unsigned)((p->N + 3) / 4), (unsigned)nrhs),
                     dim3(256), 0, p->stream, (const double2*)A, p->N, (const double2*)b, nrhs,
                     (double2*)x);
  return hipGetLastError();
}

size_t dense_solve_work_bytes(int64_t N) { return 256 + gj_work_bytes(1, (int)N); }

}  // namespace qax
