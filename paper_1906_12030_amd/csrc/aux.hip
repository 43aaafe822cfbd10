// Bandwidth-bound helper kernels: conversions, scaled copies, deterministic
// FP64 reductions, and the symmetrise-and-renormalise step of the fixed point.
#include <hip/hip_runtime.h>

#include "engine.h"
#include "tc_common.h"

namespace mera {

namespace {

constexpr int kBlock = 256;

int grid_for(int64_t n, int per_thread = 4) {
  int64_t g = (n + (int64_t)kBlock * per_thread - 1) / ((int64_t)kBlock * per_thread);
  if (g < 1) g = 1;
  if (g > 65535 * 8) g = 65535 * 8;
  return (int)g;
}

__global__ void k_to_f32(const double* __restrict__ x, float* __restrict__ y, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    y[i] = (float)x[i];
}

// Split tensor of (float) x: one thread per 32-byte group of 8 elements (the
// padding of a last, partial group is written as zeros).
__global__ void k_to_split(const double* __restrict__ x, uint16_t* __restrict__ y, int64_t n) {
  typedef uint16_t h8_t __attribute__((ext_vector_type(8)));
  const int64_t groups = (n + 7) >> 3;
  for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < groups;
       g += (int64_t)gridDim.x * blockDim.x) {
    h8_t h, l;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int64_t i = 8 * g + e;
      const float v = i < n ? (float)x[i] : 0.f;
      h[e] = bf16_bits(v);
      l[e] = bf16_bits(v - bf16_value(h[e]));
    }
    *reinterpret_cast<h8_t*>(y + 16 * g) = h;
    *reinterpret_cast<h8_t*>(y + 16 * g + 8) = l;
  }
}

// Split tensor of a d^6 density x[i j k I J K] written as y[j k J K i I]: a
// transpose of the d^2 x d^4 matrix (rows (i, I), columns (j, k, J, K)) in
// 64 x 64 tiles through LDS, so that the loads run along the columns (the
// innermost J K of x) and the stores along the rows (the innermost i I of y).
// The padding of a last, partial group (d odd) is never read.
__global__ __launch_bounds__(256) void k_rho_to_split_perm(const double* __restrict__ x,
                                                           uint16_t* __restrict__ y, int32_t d) {
  __shared__ float t[64][65];
  const int64_t d2 = (int64_t)d * d, d3 = d2 * d, d4 = d3 * d, d5 = d4 * d;
  const int64_t c0 = (int64_t)blockIdx.x * 64;
  const int64_t r0 = (int64_t)blockIdx.y * 64;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  const int64_t c = c0 + tx;
  if (c < d4) {
    const int64_t coff = (c / d2) * d3 + c % d2;
#pragma unroll 4
    for (int q = 0; q < 16; ++q) {
      const int rl = ty + 4 * q;
      const int64_t r = r0 + rl;
      if (r < d2) t[rl][tx] = (float)x[(r / d) * d5 + (r % d) * d2 + coff];
    }
  }
  __syncthreads();
  const int64_t r = r0 + tx;
  if (r < d2) {
#pragma unroll 4
    for (int q = 0; q < 16; ++q) {
      const int cl = ty + 4 * q;
      const int64_t cc = c0 + cl;
      if (cc < d4) split_store(y, cc * d2 + r, t[tx][cl]);
    }
  }
}

__global__ void k_scale(const double* __restrict__ x, double* __restrict__ y, double a, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    y[i] = a * x[i];
}

__global__ void k_fill(double* __restrict__ y, double v, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    y[i] = v;
}

__global__ void k_axpby(const double* __restrict__ x, double* __restrict__ y, double a, double b,
                        int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    y[i] = a * x[i] + b * y[i];
}

__global__ void k_scale_rsqrt(const double* __restrict__ x, double* __restrict__ y,
                              const double* __restrict__ nrm2, int64_t n) {
  const double a = 1.0 / sqrt(*nrm2);
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    y[i] = a * x[i];
}

// Block-level tree sum in a fixed order (deterministic for a fixed launch shape).
__device__ double block_sum(double v) {
  __shared__ double sh[kBlock];
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int s = kBlock / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  return sh[0];
}

// First pass: each of kReduceBlocks blocks sums a fixed, strided subset.
// n is the element count for kinds 0,1,4 and the matrix order for kinds 2,3.
__global__ void k_reduce_partial(int kind, const double* __restrict__ x,
                                 const double* __restrict__ y, int64_t n,
                                 double* __restrict__ partial) {
  double acc = 0.0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t start = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (kind == 0) {
    for (int64_t i = start; i < n; i += stride) acc += x[i] * y[i];
  } else if (kind == 1) {
    for (int64_t i = start; i < n; i += stride) {
      const double d = x[i] - y[i];
      acc += d * d;
    }
  } else if (kind == 2) {
    for (int64_t i = start; i < n; i += stride) acc += x[i * n + i];
  } else if (kind == 3) {
    // sum_ij x[i,j] y[j,i]: thread walks rows i of x (coalesced) and columns of y
    const int64_t total = n * n;
    for (int64_t t = start; t < total; t += stride) {
      const int64_t i = t / n, j = t - i * n;
      acc += x[t] * y[j * n + i];
    }
  } else {
    for (int64_t i = start; i < n; i += stride) acc += x[i] * x[i];
  }
  const double s = block_sum(acc);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

__global__ void k_reduce_final(const double* __restrict__ partial, int nparts,
                               double* __restrict__ out) {
  double acc = 0.0;
  for (int i = threadIdx.x; i < nparts; i += blockDim.x) acc += partial[i];
  const double s = block_sum(acc);
  if (threadIdx.x == 0) *out = s;
}

// y = (x + x^T) * 0.5 / tr, tiled through LDS so both reads are coalesced.
constexpr int kT = 32;
__global__ void k_sym_normalize(const double* __restrict__ x, double* __restrict__ y, int64_t n,
                                const double* __restrict__ trace) {
  __shared__ double tile[kT][kT + 1];
  const double a = 0.5 / (*trace);
  const int64_t bi = (int64_t)blockIdx.y * kT, bj = (int64_t)blockIdx.x * kT;
  const int tx = threadIdx.x, ty = threadIdx.y;  // 32 x 8
  // load the transposed block x[bj.., bi..] into tile
  for (int r = ty; r < kT; r += 8) {
    const int64_t row = bj + r, col = bi + tx;
    tile[r][tx] = (row < n && col < n) ? x[row * n + col] : 0.0;
  }
  __syncthreads();
  for (int r = ty; r < kT; r += 8) {
    const int64_t row = bi + r, col = bj + tx;
    if (row < n && col < n) y[row * n + col] = a * (x[row * n + col] + tile[tx][r]);
  }
}

// Single-workgroup sum_ij x[i,j] y[j,i] (fixed order; meant for small n).
__global__ void k_trace_product_1blk(const double* __restrict__ x, const double* __restrict__ y,
                                     int64_t n, double* __restrict__ out) {
  double acc = 0.0;
  const int64_t total = n * n;
  for (int64_t t = threadIdx.x; t < total; t += blockDim.x) {
    const int64_t i = t / n, j = t - i * n;
    acc += x[t] * y[j * n + i];
  }
  const double s = block_sum(acc);
  if (threadIdx.x == 0) *out = s;
}

__global__ void k_sqrt_ratio(const double* __restrict__ a, const double* __restrict__ b,
                             double* __restrict__ out) {
  if (threadIdx.x == 0) *out = sqrt(*a / *b);
}

}  // namespace

hipError_t launch_trace_product_small(const double* x, const double* y, int64_t n, double* out,
                                      hipStream_t s) {
  hipLaunchKernelGGL(k_trace_product_1blk, dim3(1), dim3(kBlock), 0, s, x, y, n, out);
  return hipGetLastError();
}
hipError_t launch_sqrt_ratio(const double* a, const double* b, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_sqrt_ratio, dim3(1), dim3(64), 0, s, a, b, out);
  return hipGetLastError();
}

hipError_t launch_to_f32(const double* x, float* y, int64_t n, bool split, hipStream_t s) {
  if (split)
    hipLaunchKernelGGL(k_to_split, dim3(grid_for((n + 7) / 8, 1)), dim3(kBlock), 0, s, x,
                       reinterpret_cast<uint16_t*>(y), n);
  else
    hipLaunchKernelGGL(k_to_f32, dim3(grid_for(n)), dim3(kBlock), 0, s, x, y, n);
  return hipGetLastError();
}
hipError_t launch_rho_to_split_perm(const double* x, float* y, int32_t d, hipStream_t s) {
  const int64_t d2 = (int64_t)d * d;
  const dim3 grid((unsigned)((d2 * d2 + 63) / 64), (unsigned)((d2 + 63) / 64));
  hipLaunchKernelGGL(k_rho_to_split_perm, grid, dim3(256), 0, s, x, reinterpret_cast<uint16_t*>(y), d);
  return hipGetLastError();
}
hipError_t launch_scale(const double* x, double* y, double a, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_scale, dim3(grid_for(n)), dim3(kBlock), 0, s, x, y, a, n);
  return hipGetLastError();
}
hipError_t launch_fill(double* y, double v, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_fill, dim3(grid_for(n)), dim3(kBlock), 0, s, y, v, n);
  return hipGetLastError();
}
hipError_t launch_axpby(const double* x, double* y, double a, double b, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_axpby, dim3(grid_for(n)), dim3(kBlock), 0, s, x, y, a, b, n);
  return hipGetLastError();
}
hipError_t launch_scale_by_rsqrt(const double* x, double* y, const double* nrm2_d, int64_t n,
                                 hipStream_t s) {
  hipLaunchKernelGGL(k_scale_rsqrt, dim3(grid_for(n)), dim3(kBlock), 0, s, x, y, nrm2_d, n);
  return hipGetLastError();
}
hipError_t launch_reduce(int kind, const double* x, const double* y, int64_t n, double* partial,
                         double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_reduce_partial, dim3(kReduceBlocks), dim3(kBlock), 0, s, kind, x, y, n,
                     partial);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(kBlock), 0, s, partial, kReduceBlocks, out);
  return hipGetLastError();
}
hipError_t launch_sym_normalize(const double* x, double* y, int64_t n, const double* trace_d,
                                hipStream_t s) {
  dim3 grid((unsigned)((n + kT - 1) / kT), (unsigned)((n + kT - 1) / kT));
  hipLaunchKernelGGL(k_sym_normalize, grid, dim3(kT, 8), 0, s, x, y, n, trace_d);
  return hipGetLastError();
}

}  // namespace mera
