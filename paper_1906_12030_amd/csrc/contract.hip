// Tensor-contraction engine for gfx950 (MI355X).
//
// Every pairwise contraction of the MERA schedules is run as one GEMM
//   C[m, n] = alpha * sum_k A[m, k] B[k, n] + beta * C[m, n]
// where m, n, k are multi-indices (groups of tensor legs).  Because the legs of
// each group belong to different operands, every address is separable:
//   addr_A(m, k) = offA(m) + offA(k),  addr_B(k, n) = offB(k) + offB(n),
//   addr_C(m, n) = offC(m) + offC(n),
// with each offset a sum of (leg index * leg stride) over the legs of its group.
// The kernel therefore reads the permuted tensors in place (no transposes):
// tiles are gathered from HBM with row offsets computed once per tile and
// k offsets once per k-step, staged through LDS, and multiplied on MFMA.  The
// epilogue scatters the tile back with the same separable offsets.
//
// Tiling: 256 threads = 4 wave64, 128x128 output tile per workgroup, 64x64 per
// wave as 4x4 MFMA 16x16 blocks, k-step 16 (F64/F32).  Two LDS stages; the
// next k-step's global loads are issued before the current step's MFMAs.
// Workgroups are remapped so that each of the 8 XCDs (each with its own L2)
// receives a contiguous range of tiles, ordered in groups of G tile rows so
// that neighbouring workgroups share A and B panels in L2.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "engine.h"
#include "tc_common.h"

namespace mera {

// ---------------------------------------------------------------------------
// F64 / F32 MFMA kernel
// ---------------------------------------------------------------------------
typedef double d4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));

template <typename T>
struct Mfma;

template <>
struct Mfma<double> {
  typedef d4_t acc_t;
  static __device__ __forceinline__ acc_t mac(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  // row (within the 16x16 block) of accumulator register r for this lane
  static __device__ __forceinline__ int row(int lane, int r) { return (lane >> 4) + 4 * r; }
};

template <>
struct Mfma<float> {
  typedef f4_t acc_t;
  static __device__ __forceinline__ acc_t mac(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};

template <typename T, int V>
struct VecLoad;
template <typename T>
struct VecLoad<T, 1> {
  static __device__ __forceinline__ void load(const T* p, T* out) { out[0] = *p; }
};
template <>
struct VecLoad<double, 2> {
  static __device__ __forceinline__ void load(const double* p, double* out) {
    typedef double v2 __attribute__((ext_vector_type(2)));
    v2 v = *reinterpret_cast<const v2*>(p);
    out[0] = v.x;
    out[1] = v.y;
  }
};
template <>
struct VecLoad<float, 4> {
  static __device__ __forceinline__ void load(const float* p, float* out) {
    typedef float v4 __attribute__((ext_vector_type(4)));
    v4 v = *reinterpret_cast<const v4*>(p);
    out[0] = v.x;
    out[1] = v.y;
    out[2] = v.z;
    out[3] = v.w;
  }
};

constexpr int kThreads = 256;
constexpr int kBM = 128;
constexpr int kBN = 128;
constexpr int kBK = 16;
constexpr int kPad = 4;

template <typename T, typename TC, bool A_KC, int VA, bool B_NC, int VB>
__global__ __launch_bounds__(kThreads) void tc_mfma_kernel(TcArgs p) {
  typedef typename Mfma<T>::acc_t acc_t;
  __shared__ T As[2][kBK][kBM + kPad];
  __shared__ T Bs[2][kBK][kBN + kPad];

  int tm, tn;
  if (!tile_of_block(p, tm, tn)) return;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = (wave >> 1) * 64;
  const int wn = (wave & 1) * 64;
  const uint32_t m0 = (uint32_t)tm * kBM;
  const uint32_t n0 = (uint32_t)tn * kBN;
  const T* __restrict__ A = static_cast<const T*>(p.a);
  const T* __restrict__ B = static_cast<const T*>(p.b);

  // ---- loader geometry for A ----
  // A_KC: each thread loads VA consecutive k of one row; else VA consecutive rows at one k.
  constexpr int A_TPR = A_KC ? kBK / VA : kBM / VA;          // threads per row (KC) or per k-line
  constexpr int A_RPP = kThreads / A_TPR;                     // rows (KC) or k-lines per pass
  constexpr int A_NP = A_KC ? kBM / A_RPP : kBK / A_RPP;      // passes
  constexpr int B_TPR = B_NC ? kBN / VB : kBK / VB;
  constexpr int B_RPP = kThreads / B_TPR;
  constexpr int B_NP = B_NC ? kBK / B_RPP : kBN / B_RPP;
  static_assert(A_NP >= 1 && B_NP >= 1, "tile geometry");

  const int a_line = tid / A_TPR;
  const int a_vec = (tid % A_TPR) * VA;
  const int b_line = tid / B_TPR;
  const int b_vec = (tid % B_TPR) * VB;

  int64_t a_off[A_KC ? A_NP : 1];
  bool a_ok[A_KC ? A_NP : 1];
  if (A_KC) {
#pragma unroll
    for (int i = 0; i < A_NP; ++i) {
      const uint32_t m = m0 + a_line + i * A_RPP;
      a_ok[i] = m < (uint32_t)p.M;
      a_off[i] = a_ok[i] ? goff<false>(p.gm, m) : 0;
    }
  } else {
    const uint32_t m = m0 + a_vec;
    a_ok[0] = m < (uint32_t)p.M;
    a_off[0] = a_ok[0] ? goff<false>(p.gm, m) : 0;
  }
  int64_t b_off[B_NC ? 1 : B_NP];
  bool b_ok[B_NC ? 1 : B_NP];
  if (B_NC) {
    const uint32_t n = n0 + b_vec;
    b_ok[0] = n < (uint32_t)p.N;
    b_off[0] = b_ok[0] ? goff<false>(p.gn, n) : 0;
  } else {
#pragma unroll
    for (int i = 0; i < B_NP; ++i) {
      const uint32_t n = n0 + b_line + i * B_RPP;
      b_ok[i] = n < (uint32_t)p.N;
      b_off[i] = b_ok[i] ? goff<false>(p.gn, n) : 0;
    }
  }

  T ra[A_NP][VA];
  T rb[B_NP][VB];

  auto load_tiles = [&](uint32_t k0) {
    if (A_KC) {
      const uint32_t k = k0 + a_vec;
      const bool kok = k < (uint32_t)p.K;
      const int64_t ko = kok ? goff<false>(p.gk, k) : 0;
#pragma unroll
      for (int i = 0; i < A_NP; ++i) {
        if (kok && a_ok[i]) {
          VecLoad<T, VA>::load(A + a_off[i] + ko, ra[i]);
        } else {
#pragma unroll
          for (int v = 0; v < VA; ++v) ra[i][v] = T(0);
        }
      }
    } else {
#pragma unroll
      for (int i = 0; i < A_NP; ++i) {
        const uint32_t k = k0 + a_line + i * A_RPP;
        if (k < (uint32_t)p.K && a_ok[0]) {
          VecLoad<T, VA>::load(A + a_off[0] + goff<false>(p.gk, k), ra[i]);
        } else {
#pragma unroll
          for (int v = 0; v < VA; ++v) ra[i][v] = T(0);
        }
      }
    }
    if (B_NC) {
#pragma unroll
      for (int i = 0; i < B_NP; ++i) {
        const uint32_t k = k0 + b_line + i * B_RPP;
        if (k < (uint32_t)p.K && b_ok[0]) {
          VecLoad<T, VB>::load(B + b_off[0] + goff<true>(p.gk, k), rb[i]);
        } else {
#pragma unroll
          for (int v = 0; v < VB; ++v) rb[i][v] = T(0);
        }
      }
    } else {
      const uint32_t k = k0 + b_vec;
      const bool kok = k < (uint32_t)p.K;
      const int64_t ko = kok ? goff<true>(p.gk, k) : 0;
#pragma unroll
      for (int i = 0; i < B_NP; ++i) {
        if (kok && b_ok[i]) {
          VecLoad<T, VB>::load(B + b_off[i] + ko, rb[i]);
        } else {
#pragma unroll
          for (int v = 0; v < VB; ++v) rb[i][v] = T(0);
        }
      }
    }
  };

  auto store_tiles = [&](int buf) {
    if (A_KC) {
#pragma unroll
      for (int i = 0; i < A_NP; ++i)
#pragma unroll
        for (int v = 0; v < VA; ++v) As[buf][a_vec + v][a_line + i * A_RPP] = ra[i][v];
    } else {
#pragma unroll
      for (int i = 0; i < A_NP; ++i)
#pragma unroll
        for (int v = 0; v < VA; ++v) As[buf][a_line + i * A_RPP][a_vec + v] = ra[i][v];
    }
    if (B_NC) {
#pragma unroll
      for (int i = 0; i < B_NP; ++i)
#pragma unroll
        for (int v = 0; v < VB; ++v) Bs[buf][b_line + i * B_RPP][b_vec + v] = rb[i][v];
    } else {
#pragma unroll
      for (int i = 0; i < B_NP; ++i)
#pragma unroll
        for (int v = 0; v < VB; ++v) Bs[buf][b_vec + v][b_line + i * B_RPP] = rb[i][v];
    }
  };

  acc_t acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = acc_t{0, 0, 0, 0};

  const int nk = (p.K + kBK - 1) / kBK;
  load_tiles(0);
  store_tiles(0);
  __syncthreads();
  const int lr = lane & 15;
  const int lk = lane >> 4;
  for (int kt = 0; kt < nk; ++kt) {
    const int cur = kt & 1;
    if (kt + 1 < nk) load_tiles((uint32_t)(kt + 1) * kBK);
#pragma unroll
    for (int ks = 0; ks < kBK / 4; ++ks) {
      T a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = As[cur][ks * 4 + lk][wm + i * 16 + lr];
#pragma unroll
      for (int j = 0; j < 4; ++j) b[j] = Bs[cur][ks * 4 + lk][wn + j * 16 + lr];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = Mfma<T>::mac(a[i], b[j], acc[i][j]);
    }
    if (kt + 1 < nk) store_tiles(cur ^ 1);
    __syncthreads();
  }

  // ---- epilogue: scatter with separable offsets ----
  TC* __restrict__ C = static_cast<TC*>(p.c);
  int64_t coff[4];
  bool cok[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const uint32_t n = n0 + wn + j * 16 + lr;
    cok[j] = n < (uint32_t)p.N;
    coff[j] = cok[j] ? goff<true>(p.gn, n) : 0;
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const uint32_t m = m0 + wm + i * 16 + Mfma<T>::row(lane, r);
      if (m >= (uint32_t)p.M) continue;
      const int64_t ro = goff<true>(p.gm, m);
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        if (!cok[j]) continue;
        TC* dst = C + ro + coff[j];
        double v = p.alpha * (double)acc[i][j][r];
        if (p.beta != 0.0) v += p.beta * (double)(*dst);
        *dst = (TC)v;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Host planner
// ---------------------------------------------------------------------------
namespace {

struct Plan {
  std::string mlab, nlab, klab;  // group legs, outer..inner
  bool swapped = false;
};

int64_t stride_in(const std::string& lab, char c, const LabelDims& dims) {
  int64_t s = 1;
  for (int i = (int)lab.size() - 1; i >= 0; --i) {
    if (lab[i] == c) return s;
    s *= dims.d[(unsigned char)lab[i]];
  }
  return -1;
}

bool contains(const std::string& s, char c) { return s.find(c) != std::string::npos; }

// Build a group from legs (outer..inner) with strides in operands X and Y,
// merging neighbours that are contiguous in both.
bool build_group(const std::string& legs, const std::string& lx, const std::string& ly,
                 const LabelDims& dims, Group& g, int64_t& total) {
  std::vector<int64_t> sz, sx, sy;
  for (char c : legs) {
    sz.push_back(dims.d[(unsigned char)c]);
    sx.push_back(stride_in(lx, c, dims));
    sy.push_back(stride_in(ly, c, dims));
  }
  // merge from inner to outer
  std::vector<int64_t> msz, msx, msy;
  for (int i = (int)sz.size() - 1; i >= 0; --i) {
    if (!msz.empty() && sx[i] == msx.back() * msz.back() && sy[i] == msy.back() * msz.back()) {
      msz.back() *= sz[i];
    } else {
      msz.push_back(sz[i]);
      msx.push_back(sx[i]);
      msy.push_back(sy[i]);
    }
  }
  std::reverse(msz.begin(), msz.end());
  std::reverse(msx.begin(), msx.end());
  std::reverse(msy.begin(), msy.end());
  if (msz.empty()) {  // empty group: a single dim of size 1
    msz.push_back(1);
    msx.push_back(0);
    msy.push_back(0);
  }
  if ((int)msz.size() > kMaxDims) return false;
  g.nd = (int)msz.size();
  total = 1;
  for (int i = 0; i < kMaxDims; ++i) {
    g.size[i] = i < g.nd ? (int32_t)msz[i] : 1;
    g.sx[i] = i < g.nd ? msx[i] : 0;
    g.sy[i] = i < g.nd ? msy[i] : 0;
    if (i < g.nd) total *= msz[i];
  }
  return total < (int64_t(1) << 31);
}

template <typename T, typename TC, bool AKC, int VA, bool BNC, int VB>
hipError_t launch_one(const TcArgs& a, int blocks, hipStream_t s) {
  hipLaunchKernelGGL((tc_mfma_kernel<T, TC, AKC, VA, BNC, VB>), dim3(blocks), dim3(kThreads), 0, s,
                     a);
  return hipGetLastError();
}

template <typename T, typename TC>
hipError_t dispatch(const TcArgs& a, int blocks, bool akc, bool va, bool bnc, bool vb,
                    hipStream_t s) {
  constexpr int W = 16 / sizeof(T);
  if (akc) {
    if (bnc) {
      if (va)
        return vb ? launch_one<T, TC, true, W, true, W>(a, blocks, s)
                  : launch_one<T, TC, true, W, true, 1>(a, blocks, s);
      return vb ? launch_one<T, TC, true, 1, true, W>(a, blocks, s)
                : launch_one<T, TC, true, 1, true, 1>(a, blocks, s);
    }
    if (va)
      return vb ? launch_one<T, TC, true, W, false, W>(a, blocks, s)
                : launch_one<T, TC, true, W, false, 1>(a, blocks, s);
    return vb ? launch_one<T, TC, true, 1, false, W>(a, blocks, s)
              : launch_one<T, TC, true, 1, false, 1>(a, blocks, s);
  }
  if (bnc) {
    if (va)
      return vb ? launch_one<T, TC, false, W, true, W>(a, blocks, s)
                : launch_one<T, TC, false, W, true, 1>(a, blocks, s);
    return vb ? launch_one<T, TC, false, 1, true, W>(a, blocks, s)
              : launch_one<T, TC, false, 1, true, 1>(a, blocks, s);
  }
  if (va)
    return vb ? launch_one<T, TC, false, W, false, W>(a, blocks, s)
              : launch_one<T, TC, false, W, false, 1>(a, blocks, s);
  return vb ? launch_one<T, TC, false, 1, false, W>(a, blocks, s)
            : launch_one<T, TC, false, 1, false, 1>(a, blocks, s);
}

// Vector width usable along the unit-stride leg `inner` of operand `lab`:
// every other stride and the leg size must be multiples of W.
bool vec_ok(const std::string& lab, char inner, const LabelDims& dims, int W) {
  if (lab.empty() || lab.back() != inner) return false;
  return dims.d[(unsigned char)inner] % W == 0;
}

}  // namespace

double contract_flops(const LabelDims& dims, const char* la_, const char* lb_, const char* lc_) {
  std::string la(la_), lb(lb_), lc(lc_);
  double f = 2.0;
  std::string seen;
  for (const std::string* s : {&la, &lb, &lc})
    for (char c : *s)
      if (!contains(seen, c)) {
        seen.push_back(c);
        f *= (double)dims.d[(unsigned char)c];
      }
  return f;
}

hipError_t contract(Arith ar, const LabelDims& dims, const void* A, const char* la_, const void* B,
                    const char* lb_, void* C, const char* lc_, bool c_f64, double alpha,
                    double beta, hipStream_t stream, double* flops) {
  std::string la(la_), lb(lb_), lc(lc_);
  // C's innermost leg must come from "B" so that stores run along n.
  if (!lc.empty() && contains(la, lc.back()) && !contains(lb, lc.back())) {
    std::swap(la, lb);
    std::swap(A, B);
  }
  std::string mlab, nlab, klab;
  for (char c : lc) {
    const bool ia = contains(la, c), ib = contains(lb, c);
    if (ia == ib) return hipErrorInvalidValue;  // batch legs / orphan legs unsupported
    (ia ? mlab : nlab).push_back(c);
  }
  for (char c : la) {
    if (contains(lc, c)) continue;
    if (!contains(lb, c)) return hipErrorInvalidValue;  // summed leg of a single operand
    klab.push_back(c);
  }
  for (char c : lb)
    if (!contains(lc, c) && !contains(la, c)) return hipErrorInvalidValue;
  // order m legs as in A when A's innermost leg is an m leg (loads along m)
  const bool a_last_m = !la.empty() && contains(mlab, la.back());
  if (a_last_m) {
    std::string o;
    for (char c : la)
      if (contains(mlab, c)) o.push_back(c);
    mlab = o;
  }
  // order k legs by the operand whose innermost leg is a k leg (A first)
  const bool a_last_k = !la.empty() && contains(klab, la.back());
  const bool b_last_k = !lb.empty() && contains(klab, lb.back());
  if (!a_last_k && b_last_k) {
    std::string o;
    for (char c : lb)
      if (contains(klab, c)) o.push_back(c);
    klab = o;
  }
  TcArgs args;
  std::memset(&args, 0, sizeof(args));
  int64_t M, N, K;
  if (!build_group(mlab, la, lc, dims, args.gm, M)) return hipErrorInvalidValue;
  if (!build_group(nlab, lb, lc, dims, args.gn, N)) return hipErrorInvalidValue;
  if (!build_group(klab, la, lb, dims, args.gk, K)) return hipErrorInvalidValue;
  if (flops) *flops += 2.0 * (double)M * (double)N * (double)K;
  if (M == 0 || N == 0) return hipSuccess;
  args.a = A;
  args.b = B;
  args.c = C;
  args.M = (int32_t)M;
  args.N = (int32_t)N;
  args.K = (int32_t)K;
  args.alpha = alpha;
  args.beta = beta;
  // loader modes: contiguous leg of A along k (else along m); of B along n (else along k)
  const bool akc = a_last_k && args.gk.sx[args.gk.nd - 1] == 1;
  const bool amc = a_last_m && args.gm.sx[args.gm.nd - 1] == 1;
  const bool bnc = !lb.empty() && contains(nlab, lb.back()) && args.gn.sx[args.gn.nd - 1] == 1;
  const bool bkc = b_last_k && args.gk.sy[args.gk.nd - 1] == 1;
  const int elem = (ar == Arith::F64) ? 8 : 4;
  const int W = 16 / elem;
  bool A_KC = akc || !amc;  // generic layouts fall back to element loads along k
  bool B_NC = bnc || !bkc;
  bool va = A_KC ? (akc && vec_ok(la, la.back(), dims, W) && args.gk.size[args.gk.nd - 1] % W == 0)
                 : (vec_ok(la, la.back(), dims, W) && args.gm.size[args.gm.nd - 1] % W == 0);
  bool vb = B_NC ? (bnc && vec_ok(lb, lb.back(), dims, W) && args.gn.size[args.gn.nd - 1] % W == 0)
                 : (vec_ok(lb, lb.back(), dims, W) && args.gk.size[args.gk.nd - 1] % W == 0);
  if (reinterpret_cast<uintptr_t>(A) % 16) va = false;
  if (reinterpret_cast<uintptr_t>(B) % 16) vb = false;
  args.tiles_m = (int32_t)((M + kBM - 1) / kBM);
  args.tiles_n = (int32_t)((N + kBN - 1) / kBN);
  const int64_t total = (int64_t)args.tiles_m * args.tiles_n;
  args.per_xcd = (int32_t)((total + 7) / 8);
  args.group_m = 8;
  const int blocks = args.per_xcd * 8;
  if (ar == Arith::F64) {
    if (!c_f64) return hipErrorInvalidValue;
    return dispatch<double, double>(args, blocks, A_KC, va, B_NC, vb, stream);
  }
  if (ar == Arith::F32) {
    return c_f64 ? dispatch<float, double>(args, blocks, A_KC, va, B_NC, vb, stream)
                 : dispatch<float, float>(args, blocks, A_KC, va, B_NC, vb, stream);
  }
  return launch_contract_b3(args, A_KC, va, B_NC, vb, c_f64, stream);
}

}  // namespace mera
