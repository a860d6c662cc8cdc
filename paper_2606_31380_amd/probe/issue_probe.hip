// Issue-cost microbenchmark for gfx950: SIMD cycles per wave-iteration of a
// loop with NV independent FP32 fmas, NT FP32 transcendentals (v_sin, v_rsq
// or v_rcp) and NM MFMA 16x16x4 FP32 products, none of them depending on the
// others, at 2 and 4 wavefronts per SIMD; then FP64 fmas, FP64 v_rsq and
// FP64 fmas mixed with FP32 fmas.  Used to price the instruction mix
// of the pair-sum kernels (how many cycles a VALU, a transcendental and a
// matrix instruction take, and whether they overlap).
//
//   hipcc -O3 --offload-arch=gfx950 issue_probe.hip -o issue_probe
//   ./issue_probe          (one line per configuration)
#include <hip/hip_runtime.h>

#include <cstdio>

typedef __attribute__((__vector_size__(4 * sizeof(float)))) float v4;

// TK: 0 sin, 1 rsq, 2 rcp
template <int NV, int NT, int NM, int TK>
__global__ __launch_bounds__(256) void probe(float* out, int iters, float seed) {
  float a[8], t[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    a[i] = seed + threadIdx.x * 1e-3f + i;
    t[i] = 0.1f * i + seed + 1.0f;
  }
  const float ma = seed + threadIdx.x * 1e-4f, mb = seed - threadIdx.x * 1e-4f;
  v4 acc[5];
  for (int q = 0; q < 5; ++q)
    for (int e = 0; e < 4; ++e) acc[q][e] = 0.0f;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int q = 0; q < NM; ++q) acc[q % 5] = __builtin_amdgcn_mfma_f32_16x16x4f32(ma, mb, acc[q % 5], 0, 0, 0);
#pragma unroll
    for (int q = 0; q < NT; ++q) {
      if (TK == 0) t[q & 7] = __builtin_amdgcn_sinf(t[q & 7]);
      else if (TK == 1) t[q & 7] = __builtin_amdgcn_rsqf(t[q & 7]);
      else t[q & 7] = __builtin_amdgcn_rcpf(t[q & 7]);
    }
#pragma unroll
    for (int q = 0; q < NV; ++q) a[q & 7] = fmaf(a[q & 7], a[(q + 3) & 7], 0.5f);
  }
  float s = 0.0f;
#pragma unroll
  for (int i = 0; i < 8; ++i) s += a[i] + t[i];
  for (int q = 0; q < 5; ++q)
    for (int e = 0; e < 4; ++e) s += acc[q][e];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

// FP64: ND independent FP64 fmas (8 chains), NQ FP64 v_rsq (8 chains) and
// NF FP32 fmas (8 chains) per iteration, to price the FP64 pair sum's mix.
template <int ND, int NQ, int NF>
__global__ __launch_bounds__(256) void probe64(double* out, int iters, double seed) {
  double a[8], q[8];
  float f[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    a[i] = seed + threadIdx.x * 1e-3 + i;
    q[i] = 0.1 * i + seed + 1.0;
    f[i] = (float)(seed + i);
  }
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int k = 0; k < NQ; ++k) q[k & 7] = __builtin_amdgcn_rsq(q[k & 7]);
#pragma unroll
    for (int k = 0; k < ND; ++k) a[k & 7] = fma(a[k & 7], a[(k + 3) & 7], 0.5);
#pragma unroll
    for (int k = 0; k < NF; ++k) f[k & 7] = fmaf(f[k & 7], f[(k + 3) & 7], 0.5f);
  }
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < 8; ++i) s += a[i] + q[i] + f[i];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

static int n_cu() {
  hipDeviceProp_t p;
  if (hipGetDeviceProperties(&p, 0) != hipSuccess) return 256;
  return p.multiProcessorCount;
}

template <int NV, int NT, int NM, int TK>
static int run(float* out, int wps, int cus, double ghz) {
  const int blocks = cus * wps;   // 4 wavefronts per block, one per SIMD
  const int iters = 20000;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return 1;
  probe<NV, NT, NM, TK><<<blocks, 256>>>(out, 100, 0.3f);
  if (hipEventRecord(e0) != hipSuccess) return 1;
  probe<NV, NT, NM, TK><<<blocks, 256>>>(out, iters, 0.3f);
  if (hipEventRecord(e1) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) return 1;
  float ms = 0;
  if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) return 1;
  const double cyc = ms * 1e-3 * ghz * 1e9 / ((double)iters * wps);
  std::printf("fma=%3d trans=%2d(%s) mfma=%d waves/SIMD=%d: %.1f cycles per wave-iteration\n", NV, NT,
              TK == 0 ? "sin" : TK == 1 ? "rsq" : "rcp", NM, wps, cyc);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return 0;
}

template <int ND, int NQ, int NF>
static int run64(double* out, int wps, int cus, double ghz) {
  const int blocks = cus * wps;
  const int iters = 20000;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return 1;
  probe64<ND, NQ, NF><<<blocks, 256>>>(out, 100, 0.3);
  if (hipEventRecord(e0) != hipSuccess) return 1;
  probe64<ND, NQ, NF><<<blocks, 256>>>(out, iters, 0.3);
  if (hipEventRecord(e1) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) return 1;
  float ms = 0;
  if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) return 1;
  const double cyc = ms * 1e-3 * ghz * 1e9 / ((double)iters * wps);
  std::printf("fma64=%3d rsq64=%2d fma32=%3d waves/SIMD=%d: %.1f cycles per wave-iteration\n", ND, NQ, NF,
              wps, cyc);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return 0;
}

int main() {
  const int cus = n_cu();
  const double ghz = 2.4;   // MI355X peak engine clock
  float* out = nullptr;
  if (hipMalloc(&out, sizeof(float) * 256 * 4 * cus) != hipSuccess) return 1;
  int bad = 0;
  for (int w = 2; w <= 4; w *= 2) {
    bad |= run<64, 0, 0, 0>(out, w, cus, ghz);
    bad |= run<128, 0, 0, 0>(out, w, cus, ghz);
    bad |= run<0, 16, 0, 0>(out, w, cus, ghz);
    bad |= run<0, 16, 0, 1>(out, w, cus, ghz);
    bad |= run<0, 16, 0, 2>(out, w, cus, ghz);
    bad |= run<0, 0, 5, 0>(out, w, cus, ghz);
    bad |= run<64, 0, 5, 0>(out, w, cus, ghz);
    bad |= run<64, 16, 0, 0>(out, w, cus, ghz);
    bad |= run<64, 16, 5, 0>(out, w, cus, ghz);
  }
  (void)hipFree(out);
  double* out64 = nullptr;
  if (hipMalloc(&out64, sizeof(double) * 256 * 4 * cus) != hipSuccess) return 1;
  for (int w = 2; w <= 4; w *= 2) {
    bad |= run64<64, 0, 0>(out64, w, cus, ghz);
    bad |= run64<128, 0, 0>(out64, w, cus, ghz);
    bad |= run64<0, 16, 0>(out64, w, cus, ghz);
    bad |= run64<64, 0, 64>(out64, w, cus, ghz);
    bad |= run64<64, 16, 0>(out64, w, cus, ghz);
  }
  (void)hipFree(out64);
  return bad;
}
