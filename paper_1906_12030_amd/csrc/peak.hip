// MFMA throughput microbenchmark: the matrix-core peak the contraction
// kernels are measured against, on the card at hand (clock and power state
// included).  Each wave keeps eight independent accumulator chains on one
// MFMA shape with register operands only (no memory traffic in the loop).
#include <hip/hip_runtime.h>

#include "engine.h"

namespace mera {

namespace {

typedef float f4_t __attribute__((ext_vector_type(4)));
typedef double d4_t __attribute__((ext_vector_type(4)));
typedef __bf16 bf8_t __attribute__((ext_vector_type(8)));

constexpr int kChains = 8;

// P = 0: v_mfma_f32_16x16x32_bf16 (16384 flop), 1: v_mfma_f32_16x16x4_f32
// (2048 flop), 2: v_mfma_f64_16x16x4_f64 (2048 flop).
template <int P>
__global__ __launch_bounds__(256) void k_mfma_peak(float* out, int iters) {
  const int lane = threadIdx.x & 63;
  float s = 0.f;
  if constexpr (P == 0) {
    bf8_t a, b;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      a[e] = (__bf16)(0.001f * (lane + e));
      b[e] = (__bf16)(0.002f * (lane - e));
    }
    f4_t acc[kChains];
#pragma unroll
    for (int c = 0; c < kChains; ++c) acc[c] = f4_t{0.f, 0.f, 0.f, 0.f};
    for (int it = 0; it < iters; ++it)
#pragma unroll
      for (int c = 0; c < kChains; ++c) acc[c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[c], 0, 0, 0);
#pragma unroll
    for (int c = 0; c < kChains; ++c) s += acc[c][0] + acc[c][3];
  } else if constexpr (P == 1) {
    const float a = 0.001f * lane, b = 0.002f * lane;
    f4_t acc[kChains];
#pragma unroll
    for (int c = 0; c < kChains; ++c) acc[c] = f4_t{0.f, 0.f, 0.f, 0.f};
    for (int it = 0; it < iters; ++it)
#pragma unroll
      for (int c = 0; c < kChains; ++c) acc[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[c], 0, 0, 0);
#pragma unroll
    for (int c = 0; c < kChains; ++c) s += acc[c][0] + acc[c][3];
  } else {
    const double a = 0.001 * lane, b = 0.002 * lane;
    d4_t acc[kChains];
#pragma unroll
    for (int c = 0; c < kChains; ++c) acc[c] = d4_t{0.0, 0.0, 0.0, 0.0};
    for (int it = 0; it < iters; ++it)
#pragma unroll
      for (int c = 0; c < kChains; ++c) acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[c], 0, 0, 0);
#pragma unroll
    for (int c = 0; c < kChains; ++c) s += (float)(acc[c][0] + acc[c][3]);
  }
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;  // keeps the chains live
}

}  // namespace

hipError_t run_mfma_peak(int precision, float* out, int blocks, int iters, hipStream_t s) {
  switch (precision) {
    case 0: hipLaunchKernelGGL(k_mfma_peak<0>, dim3(blocks), dim3(256), 0, s, out, iters); break;
    case 1: hipLaunchKernelGGL(k_mfma_peak<1>, dim3(blocks), dim3(256), 0, s, out, iters); break;
    case 2: hipLaunchKernelGGL(k_mfma_peak<2>, dim3(blocks), dim3(256), 0, s, out, iters); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

double mfma_peak_flops_per_wave_iter(int precision) {
  return kChains * (precision == 0 ? 16.0 * 16 * 32 * 2 : 16.0 * 16 * 4 * 2);
}

}  // namespace mera
