// Matrix-core throughput probe: the rate the H X kernels are compared with
// beside the published peak.  Every wave of a grid that fills each CU runs
// a long chain of MFMAs on register operands, with four independent
// accumulators so that the matrix pipe never waits on a result, and writes
// one value per wave so that nothing is eliminated.
#include <algorithm>

#include "common.h"

namespace chase {
namespace {

constexpr int PROBE_BLOCKS = 256 * 8;  // 8 workgroups of 4 waves per CU
constexpr int PROBE_THREADS = 256;

__global__ __launch_bounds__(PROBE_THREADS) void mfma_f32_probe(int iters, float seed, float* out) {
  floatx16 c0{}, c1{}, c2{}, c3{};
  const float a = seed + 1e-3f * (float)threadIdx.x, b = seed - 1e-3f * (float)threadIdx.x;
  for (int i = 0; i < iters; i += 8) {
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      c0 = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c0, 0, 0, 0);
      c1 = __builtin_amdgcn_mfma_f32_32x32x2f32(b, a, c1, 0, 0, 0);
      c2 = __builtin_amdgcn_mfma_f32_32x32x2f32(a, a, c2, 0, 0, 0);
      c3 = __builtin_amdgcn_mfma_f32_32x32x2f32(b, b, c3, 0, 0, 0);
    }
  }
  float s = 0.f;
#pragma unroll
  for (int r = 0; r < 16; ++r) s += c0[r] + c1[r] + c2[r] + c3[r];
  if ((threadIdx.x & 63) == 0) out[blockIdx.x * (PROBE_THREADS / 64) + (threadIdx.x >> 6)] = s;
}

__global__ __launch_bounds__(PROBE_THREADS) void mfma_f64_probe(int iters, double seed, double* out) {
  doublex4 c0{}, c1{}, c2{}, c3{};
  const double a = seed + 1e-3 * (double)threadIdx.x, b = seed - 1e-3 * (double)threadIdx.x;
  for (int i = 0; i < iters; i += 8) {
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      c0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c0, 0, 0, 0);
      c1 = __builtin_amdgcn_mfma_f64_16x16x4f64(b, a, c1, 0, 0, 0);
      c2 = __builtin_amdgcn_mfma_f64_16x16x4f64(a, a, c2, 0, 0, 0);
      c3 = __builtin_amdgcn_mfma_f64_16x16x4f64(b, b, c3, 0, 0, 0);
    }
  }
  double s = 0.0;
#pragma unroll
  for (int r = 0; r < 4; ++r) s += c0[r] + c1[r] + c2[r] + c3[r];
  if ((threadIdx.x & 63) == 0) out[blockIdx.x * (PROBE_THREADS / 64) + (threadIdx.x >> 6)] = s;
}

}  // namespace
}  // namespace chase

extern "C" {

// kind 0: v_mfma_f32_32x32x2f32 (4096 flops per wave instruction);
// kind 1: v_mfma_f64_16x16x4f64 (2048 flops).  Returns the best of three
// timed launches (after one warm-up) in TFLOP/s.
int32_t chase_ph_mfma_probe(int32_t kind, int32_t iters, double* tflops) {
  using namespace chase;
  if ((kind != 0 && kind != 1) || iters <= 0 || !tflops) return 1;
  void* out = nullptr;
  const size_t nout = (size_t)PROBE_BLOCKS * (PROBE_THREADS / 64);
  if (hipMalloc(&out, nout * sizeof(double)) != hipSuccess) return 2;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    (void)hipFree(out);
    return 3;
  }
  double best = 0.0;
  int rc = 0;
  for (int rep = 0; rep < 4 && rc == 0; ++rep) {
    if (hipEventRecord(e0, nullptr) != hipSuccess) rc = 3;
    if (kind == 0)
      hipLaunchKernelGGL(mfma_f32_probe, dim3(PROBE_BLOCKS), dim3(PROBE_THREADS), 0, nullptr, iters, 0.5f,
                         (float*)out);
    else
      hipLaunchKernelGGL(mfma_f64_probe, dim3(PROBE_BLOCKS), dim3(PROBE_THREADS), 0, nullptr, iters, 0.5,
                         (double*)out);
    if (hipGetLastError() != hipSuccess) rc = 3;
    float ms = 0.f;
    if (rc == 0 && (hipEventRecord(e1, nullptr) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                    hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
      rc = 3;
    const double per = kind == 0 ? 4096.0 : 2048.0;
    const double flops = per * 4.0 * (double)((iters + 7) / 8 * 8) * (double)PROBE_BLOCKS * (PROBE_THREADS / 64);
    if (rc == 0 && rep > 0 && ms > 0.f) best = std::max(best, flops / (ms * 1e-3) / 1e12);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipFree(out);
  *tflops = best;
  return rc;
}

}  // extern "C"
