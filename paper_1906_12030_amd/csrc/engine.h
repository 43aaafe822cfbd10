// Internal interface of the MI355X contraction engine and auxiliary kernels.
// Not part of the public C ABI (include/mera.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>

namespace mera {

// Arithmetic of one contraction.
//   F64: double operands, FP64 MFMA (v_mfma_f64_16x16x4f64).
//   F32: float operands, FP32 MFMA (v_mfma_f32_16x16x4f32).
//   B3 : operands and FP32 intermediates stored as split tensors (bf16 hi of
//        the FP32 value and bf16 lo of the remainder, the halves of 8
//        consecutive elements grouped; see split_hi in tc_common.h), three BF16
//        MFMA products (hi*hi + hi*lo + lo*hi) accumulated in FP32.
enum class Arith : int { F64 = 0, F32 = 1, B3 = 2 };

// Sizes of the index labels used by contraction specs (one char per label).
struct LabelDims {
  int64_t d[128];
  LabelDims() {
    for (auto& x : d) x = 0;
  }
  void set(const char* labels, int64_t v) {
    for (const char* p = labels; *p; ++p) d[(unsigned char)*p] = v;
  }
};

// C[lc] = alpha * sum_{shared labels} A[la] * B[lb] + beta * C[lc].
// Each operand is dense row-major in the order of its label string.  Labels
// shared by A and B and absent from C are summed; labels of C come from exactly
// one of A and B.  A and B hold double for F64, float for F32 and split
// tensors for B3 (32-byte aligned); C holds double when c_f64 and otherwise
// float (F32) or a split tensor (B3).  K must be at least 1.  Returns hipSuccess or the launch
// error.  `flops` (nullable) is increased by 2*M*N*K.  `scratch` (device,
// nullable) of scratch_elems doubles lets the engine split long k ranges over
// several workgroups (partial sums reduced in a fixed order) when the output
// alone has too few tiles to fill the GPU.  `cdims` (nullable) gives the leg
// sizes of the tensor C is a slice of: C's strides come from cdims while the
// extents of the contraction come from dims (C then points at the slice start).
hipError_t contract(Arith ar, const LabelDims& dims, const void* A, const char* la, const void* B,
                    const char* lb, void* C, const char* lc, bool c_f64, double alpha, double beta,
                    hipStream_t stream, double* flops = nullptr, double* scratch = nullptr,
                    size_t scratch_elems = 0, const LabelDims* cdims = nullptr);

// Flop count of the same contraction without launching anything.
double contract_flops(const LabelDims& dims, const char* la, const char* lb, const char* lc);

// The kernel contract() would choose for the same labels and sizes, as one
// line ("b3x192 m=... n=... k=... tiles=MxN splits=S store=m4", store n4/n1 =
// vector/element stores along n, m4/m1 along m; "unsupported" for label sets
// contract() rejects).  Host only, assumes 16-byte aligned operands.
std::string contract_plan(Arith ar, const LabelDims& dims, const char* la, const char* lb,
                          const char* lc, bool c_f64, size_t scratch_elems,
                          const LabelDims* cdims = nullptr);

// ---- MFMA throughput microbenchmark (peak.hip) ----
// kind 0: bf16 16x16x32, 1: f32 16x16x4, 2: f64 16x16x4; `out` holds
// blocks*256 floats; flops of one launch = blocks*4 waves*iters*per_wave_iter.
hipError_t run_mfma_peak(int kind, float* out, int blocks, int iters, hipStream_t s);
double mfma_peak_flops_per_wave_iter(int kind);

// ---- auxiliary kernels (aux.hip) ----
// y[i] = (float) x[i]; with split, y is the split tensor of (float) x (see
// split_hi in tc_common.h; 32 * ceil(n / 8) bytes)
hipError_t launch_to_f32(const double* x, float* y, int64_t n, bool split, hipStream_t s);
// y = split tensor of the d^6 density x[i j k I J K], stored as y[j k J K i I]
hipError_t launch_rho_to_split_perm(const double* x, float* y, int32_t d, hipStream_t s);
// y[i] = a * x[i]
hipError_t launch_scale(const double* x, double* y, double a, int64_t n, hipStream_t s);
// fill y with value
hipError_t launch_fill(double* y, double v, int64_t n, hipStream_t s);
// partial sums for deterministic reductions: out[b] = sum over block b
// kind 0: sum_i x[i]*y[i];  kind 1: sum_i (x[i]-y[i])^2 ; kind 2: trace of n x n matrix x;
// kind 3: sum_ij x[i,j]*y[j,i] (trace of product); kind 4: sum x[i]^2
// The result lands in out[0] after the second pass; partial needs kReduceBlocks doubles.
constexpr int kReduceBlocks = 1024;
hipError_t launch_reduce(int kind, const double* x, const double* y, int64_t n, double* partial,
                         double* out, hipStream_t s);
// *out = sum_ij x[i,j] y[j,i] in one workgroup (small n; no scratch needed)
hipError_t launch_trace_product_small(const double* x, const double* y, int64_t n, double* out,
                                      hipStream_t s);
// *out = sqrt(*a / *b)
hipError_t launch_sqrt_ratio(const double* a, const double* b, double* out, hipStream_t s);
// y = (x + x^T) * (0.5 / (*trace_d)) for an n x n matrix (x, y distinct)
hipError_t launch_sym_normalize(const double* x, double* y, int64_t n, const double* trace_d,
                                hipStream_t s);
// y = a * x + b * y
hipError_t launch_axpby(const double* x, double* y, double a, double b, int64_t n, hipStream_t s);
// y = x * (1 / sqrt(*nrm2_d)) (nrm2_d holds a squared norm)
hipError_t launch_scale_by_rsqrt(const double* x, double* y, const double* nrm2_d, int64_t n,
                                 hipStream_t s);

// ---- symmetric eigenvalues (symeig.hip) ----
// Eigenvalues of the symmetric part of the n x n row-major matrix `a`, largest
// first, clamped at zero from below (used for singular values from X^T Y).
// Destroys `a`; dg and off hold n doubles each.  1 <= n <= kSymEigMaxOrder.
constexpr int64_t kSymEigMaxOrder = 4080;
hipError_t launch_sym_eigvals_desc(double* a, int64_t n, double* dg, double* off, double* out,
                                   hipStream_t s);

}  // namespace mera
