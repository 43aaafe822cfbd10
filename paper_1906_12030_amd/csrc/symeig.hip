// Eigenvalues of a real symmetric matrix on the device, for the singular values
// returned by the SVD (polar) update (Sec. II.C, Fig. 5): at convergence of the
// polar iteration, X^T Y = V S V^T is symmetric positive semidefinite and its
// eigenvalues are the singular values of Y.
//
// Two steps, both textbook (Golub & Van Loan, "Matrix Computations", Sec. 8.3.1
// Householder tridiagonalisation and Sec. 8.4.1 Sturm-sequence bisection):
//   1. one workgroup reduces the n x n matrix (in place, row-major) to symmetric
//      tridiagonal form T = Q^T A Q with n - 2 Householder reflections; the
//      trailing block is updated as a whole (both triangles), so every read of a
//      column is a coalesced read of a row;
//   2. one thread per eigenvalue bisects the Gershgorin interval of T with the
//      Sturm count (number of eigenvalues below x) until the interval is a few
//      ulps of the matrix scale wide.
#include <hip/hip_runtime.h>

#include <cfloat>
#include <cmath>

#include "engine.h"

namespace mera {
namespace {

constexpr int kTriThreads = 1024;

// Sum over the workgroup; every thread gets the total.  `red` holds one double
// per wave plus one for the total.  Starts and ends with a barrier.
__device__ double block_sum(double v, double* red) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) s += red[i];  // fixed order
    red[kTriThreads / 64] = s;
  }
  __syncthreads();
  return red[kTriThreads / 64];
}

// a: n x n, symmetrised then overwritten; dg[n] diagonal, off[n-1] off-diagonal of T.
// Dynamic LDS: 2n + kTriThreads/64 + 1 doubles.
__global__ __launch_bounds__(kTriThreads) void k_tridiagonalize(double* __restrict__ a, int n,
                                                                double* __restrict__ dg,
                                                                double* __restrict__ off) {
  extern __shared__ double sm[];
  double* v = sm;
  double* q = sm + n;
  double* red = sm + 2 * n;
  const int tid = threadIdx.x;
  const int nt = blockDim.x;
  const int64_t nn = (int64_t)n * n;
  // a <- (a + a^T) / 2
  for (int64_t idx = tid; idx < nn; idx += nt) {
    const int i = (int)(idx / n), j = (int)(idx % n);
    if (j > i) {
      const double s = 0.5 * (a[idx] + a[(int64_t)j * n + i]);
      a[idx] = s;
      a[(int64_t)j * n + i] = s;
    }
  }
  __syncthreads();
  for (int k = 0; k + 2 < n; ++k) {
    const int m = n - k - 1;  // order of the trailing block a[k+1.., k+1..]
    const int b = k + 1;
    // x = column k below the diagonal = row k right of it (symmetry)
    double ss = 0.0;
    for (int i = tid; i < m; i += nt) {
      const double x = a[(int64_t)k * n + b + i];
      v[i] = x;
      ss += x * x;
    }
    const double nrm2 = block_sum(ss, red);
    const double x0 = v[0];
    if (nrm2 == 0.0) {  // already tridiagonal in this column (uniform branch)
      if (tid == 0) {
        dg[k] = a[(int64_t)k * n + k];
        off[k] = 0.0;
      }
      __syncthreads();
      continue;
    }
    // reflection H = I - tau v v^T with v = x - alpha e1 maps x to alpha e1
    const double alpha = x0 >= 0.0 ? -sqrt(nrm2) : sqrt(nrm2);
    const double tau = 1.0 / (nrm2 - alpha * x0);  // 2 / v^T v
    __syncthreads();  // every thread has read v[0]
    if (tid == 0) v[0] = x0 - alpha;
    __syncthreads();
    // p = tau * A v (columns read as rows), then q = p - (tau/2)(v^T p) v
    double pv = 0.0;
    for (int i = tid; i < m; i += nt) {
      double acc = 0.0;
      const double* col = a + (int64_t)b * n + b + i;
      for (int j = 0; j < m; ++j) acc += col[(int64_t)j * n] * v[j];
      acc *= tau;
      q[i] = acc;
      pv += acc * v[i];
    }
    const double kk = 0.5 * tau * block_sum(pv, red);
    for (int i = tid; i < m; i += nt) q[i] -= kk * v[i];
    __syncthreads();
    // A <- A - v q^T - q v^T on the trailing block
    for (int i = tid; i < m; i += nt) {
      const double vi = v[i], qi = q[i];
      double* col = a + (int64_t)b * n + b + i;
      for (int j = 0; j < m; ++j) col[(int64_t)j * n] -= v[j] * qi + q[j] * vi;
    }
    if (tid == 0) {
      dg[k] = a[(int64_t)k * n + k];
      off[k] = alpha;
    }
    __syncthreads();
  }
  if (tid == 0) {
    if (n >= 2) {
      dg[n - 2] = a[(int64_t)(n - 2) * n + n - 2];
      off[n - 2] = a[(int64_t)(n - 1) * n + n - 2];
    }
    dg[n - 1] = a[nn - 1];
  }
}

// Number of eigenvalues of T below x (Sturm sequence of the LDL^T pivots).
__device__ int sturm_count(const double* dg, const double* off, int n, double x, double pivmin) {
  int c = 0;
  double p = dg[0] - x;
  if (fabs(p) < pivmin) p = -pivmin;
  c += p < 0.0;
  for (int i = 1; i < n; ++i) {
    p = dg[i] - x - off[i - 1] * off[i - 1] / p;
    if (fabs(p) < pivmin) p = -pivmin;
    c += p < 0.0;
  }
  return c;
}

// out[j] = j-th largest eigenvalue of T, clamped at zero from below.
__global__ void k_bisect_desc(const double* __restrict__ dg, const double* __restrict__ off, int n,
                              double* __restrict__ out) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  double lo = DBL_MAX, hi = -DBL_MAX, emax = 0.0;
  for (int i = 0; i < n; ++i) {  // Gershgorin discs
    const double r = (i > 0 ? fabs(off[i - 1]) : 0.0) + (i + 1 < n ? fabs(off[i]) : 0.0);
    lo = fmin(lo, dg[i] - r);
    hi = fmax(hi, dg[i] + r);
    if (i + 1 < n) emax = fmax(emax, off[i] * off[i]);
  }
  const double scale = fmax(fabs(lo), fabs(hi));
  const double pivmin = DBL_MIN * fmax(1.0, emax);
  const double atol = 4.0 * DBL_EPSILON * scale + pivmin;
  lo -= atol;
  hi += atol;
  const int target = n - 1 - j;  // ascending index
  for (int it = 0; it < 2048 && hi - lo > atol; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (sturm_count(dg, off, n, mid, pivmin) > target)
      hi = mid;
    else
      lo = mid;
  }
  out[j] = fmax(0.5 * (lo + hi), 0.0);
}

}  // namespace

hipError_t launch_sym_eigvals_desc(double* a, int64_t n, double* dg, double* off, double* out,
                                   hipStream_t s) {
  if (n < 1 || n > kSymEigMaxOrder) return hipErrorInvalidValue;
  const size_t lds = sizeof(double) * (2 * (size_t)n + kTriThreads / 64 + 1);
  hipLaunchKernelGGL(k_tridiagonalize, dim3(1), dim3(kTriThreads), lds, s, a, (int)n, dg, off);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_bisect_desc, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, dg, off, (int)n, out);
  return hipGetLastError();
}

}  // namespace mera
