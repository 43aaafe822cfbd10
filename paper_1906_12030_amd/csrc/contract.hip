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
#include <cmath>
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

constexpr int kBM = 128;
constexpr int kBN = 128;
constexpr int kBK = 16;
constexpr int kPad = 4;

template <typename T, typename TC, bool A_KC, int VA, bool B_NC, int VB, bool KAL>
__global__ __launch_bounds__(kThreads) void tc_mfma_kernel(TcArgs p) {
  typedef typename Mfma<T>::acc_t acc_t;
  constexpr int kStage = kBK * (kBM + kPad);  // elements of one operand stage
  __shared__ __attribute__((aligned(16))) char smem[4 * kStage * sizeof(T)];
  T (*As)[kBK][kBM + kPad] = reinterpret_cast<T (*)[kBK][kBM + kPad]>(smem);
  T (*Bs)[kBK][kBN + kPad] = reinterpret_cast<T (*)[kBK][kBN + kPad]>(smem + 2 * kStage * sizeof(T));

  int tm, tn, split;
  if (!tile_of_block(p, tm, tn, split)) return;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = (wave >> 1) * 64;
  const int wn = (wave & 1) * 64;
  const uint32_t m0 = (uint32_t)tm * kBM;
  const uint32_t n0 = (uint32_t)tn * kBN;
  const uint32_t kbeg = (uint32_t)split * (uint32_t)p.kchunk;
  const uint32_t kend = min((uint32_t)p.K, kbeg + (uint32_t)p.kchunk);
  const T* __restrict__ A = static_cast<const T*>(p.a);
  const T* __restrict__ B = static_cast<const T*>(p.b);

  TileLoad<T, kBM, kBK, A_KC, VA, KAL, false> la;
  TileLoad<T, kBN, kBK, !B_NC, VB, KAL, true> lb;
  la.init(p.gm, p.gk, m0, (uint32_t)p.M);
  lb.init(p.gn, p.gk, n0, (uint32_t)p.N);

  auto store_tiles = [&](int buf) {
#pragma unroll
    for (int i = 0; i < la.NP; ++i)
#pragma unroll
      for (int v = 0; v < VA; ++v) {
        if (A_KC)
          As[buf][la.vec + v][la.line + i * la.LPP] = la.r[i][v];
        else
          As[buf][la.line + i * la.LPP][la.vec + v] = la.r[i][v];
      }
#pragma unroll
    for (int i = 0; i < lb.NP; ++i)
#pragma unroll
      for (int v = 0; v < VB; ++v) {
        if (B_NC)
          Bs[buf][lb.line + i * lb.LPP][lb.vec + v] = lb.r[i][v];
        else
          Bs[buf][lb.vec + v][lb.line + i * lb.LPP] = lb.r[i][v];
      }
  };

  acc_t acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = acc_t{0, 0, 0, 0};

  const int nk = (int)((kend - kbeg + kBK - 1) / kBK);
  KWalk<kBK> kw;
  if constexpr (KAL) kw.init(p.gk, kbeg);
  // k-tile fetch: carry walk for k-aligned tiles, leg decomposition otherwise
  auto fetch = [&](int kt) {
    if constexpr (KAL) {
      if (kt > 0) kw.next();
      la.load_at(A, kw.oa);
      lb.load_at(B, kw.ob);
    } else {
      la.load(A, p.gk, kbeg + (uint32_t)kt * kBK, kend);
      lb.load(B, p.gk, kbeg + (uint32_t)kt * kBK, kend);
    }
  };
  fetch(0);
  store_tiles(0);
  __syncthreads();
  const int lr = lane & 15;
  const int lk = lane >> 4;
  auto compute = [&](int cur) {
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
  };
  // steady state without branches: prefetch k-tile kt+1 while multiplying tile kt
  for (int kt = 0; kt + 1 < nk; ++kt) {
    const int cur = kt & 1;
    fetch(kt + 1);
    compute(cur);
    store_tiles(cur ^ 1);
    __syncthreads();
  }
  compute((nk - 1) & 1);
  __syncthreads();
  write_tile<T, TC>(p, acc, m0, n0, split, smem,
                    [](int ln, int r) { return Mfma<T>::row(ln, r); });
}

// C = alpha * sum over splits of the partial sums + beta * C
template <typename TC>
__global__ __launch_bounds__(256) void tc_splitk_reduce(TcArgs p) {
  const int64_t mn = (int64_t)p.M * p.N;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < mn;
       t += (int64_t)gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int c = 0; c < p.splits; ++c) s += p.part[c * mn + t];
    const uint32_t m = (uint32_t)(t / p.N), n = (uint32_t)(t - (int64_t)m * p.N);
    TC* C = static_cast<TC*>(p.c);
    const int64_t off = goff<true>(p.gm, (uint32_t)p.m_base + m) + goff<true>(p.gn, n);
    double y = p.alpha * s;
    if (p.beta != 0.0) y += p.beta * load_c(p, C, off);
    store_c(p, C, off, y);
  }
}

// ---------------------------------------------------------------------------
// Host planner
// ---------------------------------------------------------------------------
namespace {

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
                 const LabelDims& dims, const LabelDims& ydims, Group& g, int64_t& total) {
  std::vector<int64_t> sz, sx, sy;
  for (char c : legs) {
    sz.push_back(dims.d[(unsigned char)c]);
    sx.push_back(stride_in(lx, c, dims));
    sy.push_back(stride_in(ly, c, ydims));
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

template <typename T, typename TC, bool AKC, int VA, bool BNC, int VB, bool KAL>
hipError_t launch_one(const TcArgs& a, int blocks, hipStream_t s) {
  hipLaunchKernelGGL((tc_mfma_kernel<T, TC, AKC, VA, BNC, VB, KAL>), dim3(blocks), dim3(kThreads),
                     0, s, a);
  return hipGetLastError();
}

// Instantiated variants: k-aligned tiles with or without vector loads on each
// operand; unaligned tiles with element loads only.
template <typename T, typename TC>
hipError_t dispatch(const TcArgs& a, int blocks, bool akc, bool va, bool bnc, bool vb, bool kal,
                    hipStream_t s) {
  constexpr int W = 16 / sizeof(T);
  if (!kal) {
    if (akc) return bnc ? launch_one<T, TC, true, 1, true, 1, false>(a, blocks, s)
                        : launch_one<T, TC, true, 1, false, 1, false>(a, blocks, s);
    return bnc ? launch_one<T, TC, false, 1, true, 1, false>(a, blocks, s)
               : launch_one<T, TC, false, 1, false, 1, false>(a, blocks, s);
  }
#define MERA_TC_CASE(AK, AV, BN, BV)                                              \
  if (akc == AK && (va ? W : 1) == AV && bnc == BN && (vb ? W : 1) == BV)        \
    return launch_one<T, TC, AK, AV, BN, BV, true>(a, blocks, s);
  MERA_TC_CASE(true, W, true, W)
  MERA_TC_CASE(true, W, true, 1)
  MERA_TC_CASE(true, 1, true, W)
  MERA_TC_CASE(true, 1, true, 1)
  MERA_TC_CASE(true, W, false, W)
  MERA_TC_CASE(true, W, false, 1)
  MERA_TC_CASE(true, 1, false, W)
  MERA_TC_CASE(true, 1, false, 1)
  MERA_TC_CASE(false, W, true, W)
  MERA_TC_CASE(false, W, true, 1)
  MERA_TC_CASE(false, 1, true, W)
  MERA_TC_CASE(false, 1, true, 1)
  MERA_TC_CASE(false, W, false, W)
  MERA_TC_CASE(false, W, false, 1)
  MERA_TC_CASE(false, 1, false, W)
  MERA_TC_CASE(false, 1, false, 1)
#undef MERA_TC_CASE
  return hipErrorInvalidValue;
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

namespace {

// Kernel choice and arguments of one contraction, A on the m side and B on
// the n side.
struct Plan {
  TcArgs args;
  int64_t M = 0, N = 0, K = 0;
  bool A_KC = false, va = false, B_NC = false, vb = false, kal = false;
  bool use_x = false;
  int xbn = 0;
  // large-tile launches with a short last wave: the last tail_tm tile rows run as
  // a second launch split tail_ks ways along k (see plan_tail)
  int tail_tm = 0, tail_ks = 0;
};

// Plans C[lc] = A[la] . B[lb].  `m_store`: C's innermost leg is an m leg,
// which only the large-tile kernel stores efficiently (pl.use_x says whether
// it was chosen).  Stops after the group sizes when M, N or K is zero.
hipError_t make_plan(Arith ar, const LabelDims& dims, const LabelDims& cd, const void* A,
                     const std::string& la, const void* B, const std::string& lb, void* C,
                     const std::string& lc, bool c_f64, double alpha, double beta, double* scratch,
                     size_t scratch_elems, bool m_store, Plan& pl) {
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
  // order m legs as in A when A's innermost leg is an m leg (loads along m);
  // otherwise they keep C's order
  const bool a_last_m = !la.empty() && contains(mlab, la.back());
  if (a_last_m && !m_store) {
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
  TcArgs& args = pl.args;
  std::memset(&args, 0, sizeof(args));
  if (!build_group(mlab, la, lc, dims, cd, args.gm, pl.M)) return hipErrorInvalidValue;
  if (!build_group(nlab, lb, lc, dims, cd, args.gn, pl.N)) return hipErrorInvalidValue;
  if (!build_group(klab, la, lb, dims, dims, args.gk, pl.K)) return hipErrorInvalidValue;
  const int64_t M = pl.M, N = pl.N, K = pl.K;
  if (M == 0 || N == 0 || K == 0) return hipSuccess;
  args.a = A;
  args.b = B;
  args.c = C;
  args.M = (int32_t)M;
  args.N = (int32_t)N;
  args.K = (int32_t)K;
  args.alpha = alpha;
  args.beta = beta;
  // the split-bf16 path keeps its FP32 intermediates as split tensors
  args.csplit = (ar == Arith::B3 && !c_f64) ? 1 : 0;
  // loader modes: contiguous leg of A along k (else along m); of B along n (else along k)
  const bool akc = a_last_k && args.gk.sx[args.gk.nd - 1] == 1;
  const bool amc = a_last_m && args.gm.sx[args.gm.nd - 1] == 1;
  const bool bnc = !lb.empty() && contains(nlab, lb.back()) && args.gn.sx[args.gn.nd - 1] == 1;
  const bool bkc = b_last_k && args.gk.sy[args.gk.nd - 1] == 1;
  const int elem = (ar == Arith::F64) ? 8 : 4;
  const int W = 16 / elem;
  pl.A_KC = akc || !amc;  // generic layouts fall back to element loads along k
  pl.B_NC = bnc || !bkc;
  pl.va = pl.A_KC ? (akc && vec_ok(la, la.back(), dims, W) && args.gk.size[args.gk.nd - 1] % W == 0)
                  : (vec_ok(la, la.back(), dims, W) && args.gm.size[args.gm.nd - 1] % W == 0);
  pl.vb = pl.B_NC ? (bnc && vec_ok(lb, lb.back(), dims, W) && args.gn.size[args.gn.nd - 1] % W == 0)
                  : (vec_ok(lb, lb.back(), dims, W) && args.gk.size[args.gk.nd - 1] % W == 0);
  if (reinterpret_cast<uintptr_t>(A) % 16) pl.va = false;
  if (reinterpret_cast<uintptr_t>(B) % 16) pl.vb = false;
  // k-aligned tiles: the innermost k leg's extent is a multiple of the k-tile
  const int bk = (ar == Arith::B3) ? 32 : 16;
  pl.kal = args.gk.size[args.gk.nd - 1] % bk == 0;
  if (!pl.kal) pl.va = pl.vb = false;
  // Split-bf16 contractions whose operands are both contiguous along k go to
  // the large-tile kernel with direct-to-LDS loads (contract_b3x.hip).
  pl.use_x = ar == Arith::B3 && pl.kal && akc && pl.va && bkc && !bnc && pl.vb &&
             contract_b3x_fits(M, N, K, pl.xbn);
  if (m_store && !pl.use_x) return hipSuccess;  // the caller plans the swapped order
  const int64_t tbm = pl.use_x ? 256 : kBM, tbn = pl.use_x ? pl.xbn : kBN;
  args.tiles_m = (int32_t)((M + tbm - 1) / tbm);
  args.tiles_n = (int32_t)((N + tbn - 1) / tbn);
  const int64_t tiles = (int64_t)args.tiles_m * args.tiles_n;
  // Split k when the output has too few tiles to fill the GPU (two resident
  // workgroups on each of the 256 CUs; one for the large-tile kernel): pick
  // the split count that best fills whole waves of workgroups, with at least
  // 8 k-tiles per split.
  int splits = 1;
  int64_t kchunk = ((K + bk - 1) / bk) * bk;
  if (scratch && scratch_elems > 0) {
    const double kSlots = pl.use_x ? 256.0 : 512.0;
    auto fill = [&](int64_t n) { return (double)n / (std::ceil((double)n / kSlots) * kSlots); };
    double best = fill(tiles);
    for (int s = 2; s <= 16; ++s) {
      const int64_t kc = ((K + s - 1) / s + bk - 1) / bk * bk;
      const int64_t se = (K + kc - 1) / kc;
      if (kc < 8 * bk || se * M * N > (int64_t)scratch_elems) break;
      const double f = fill(tiles * se);
      if (f > best + 0.05) {
        best = f;
        splits = (int)se;
        kchunk = kc;
      }
    }
  }
  args.splits = splits;
  args.kchunk = (int32_t)kchunk;
  args.part = splits > 1 ? scratch : nullptr;
  // 64-wide column spans of the tile are contiguous in the output
  if (splits > 1)
    args.cvec = (N % 64 == 0) ? 1 : 0;
  else
    args.cvec = (args.gn.sy[args.gn.nd - 1] == 1 && args.gn.size[args.gn.nd - 1] % 64 == 0 &&
                 reinterpret_cast<uintptr_t>(C) % 16 == 0)
                    ? 1
                    : 0;
  if (splits == 1) {
    bool v2 = args.gn.sy[args.gn.nd - 1] == 1 && args.gn.size[args.gn.nd - 1] % 2 == 0 &&
              reinterpret_cast<uintptr_t>(C) % 16 == 0;
    for (int d = 0; d < args.gn.nd - 1; ++d) v2 = v2 && args.gn.sy[d] % 2 == 0;
    for (int d = 0; d < args.gm.nd; ++d) v2 = v2 && args.gm.sy[d] % 2 == 0;
    args.cvec2 = v2 ? 1 : 0;
  }
  if (pl.use_x) {
    // the large-tile kernel stores 4 consecutive columns (a multiple of 4
    // from the tile start) as one vector
    if (splits > 1) {
      args.cvec = (N % 4 == 0) ? 1 : 0;
    } else {
      bool nv = args.gn.sy[args.gn.nd - 1] == 1 && args.gn.size[args.gn.nd - 1] % 4 == 0 &&
                reinterpret_cast<uintptr_t>(C) % 16 == 0;
      for (int d = 0; d < args.gn.nd - 1; ++d) nv = nv && args.gn.sy[d] % 4 == 0;
      for (int d = 0; d < args.gm.nd; ++d) nv = nv && args.gm.sy[d] % 4 == 0;
      args.cvec = nv ? 1 : 0;
      bool g8 = args.csplit && args.gn.sy[args.gn.nd - 1] == 1 && args.gn.size[args.gn.nd - 1] % 8 == 0 &&
                reinterpret_cast<uintptr_t>(C) % 32 == 0;
      for (int d = 0; d < args.gn.nd - 1; ++d) g8 = g8 && args.gn.sy[d] % 8 == 0;
      for (int d = 0; d < args.gm.nd; ++d) g8 = g8 && args.gm.sy[d] % 8 == 0;
      args.cgroup8 = g8 ? 1 : 0;
    }
  }
  if (m_store) {
    // four consecutive rows (a multiple of 4 apart from the tile start) are
    // adjacent and 16-byte aligned in C
    bool mv = args.gm.sy[args.gm.nd - 1] == 1 && args.gm.size[args.gm.nd - 1] % 4 == 0 &&
              reinterpret_cast<uintptr_t>(C) % 16 == 0;
    for (int d = 0; d < args.gm.nd - 1; ++d) mv = mv && args.gm.sy[d] % 4 == 0;
    for (int d = 0; d < args.gn.nd; ++d) mv = mv && args.gn.sy[d] % 4 == 0;
    args.cm = mv ? 1 : 2;
  }
  args.per_xcd = (int32_t)((tiles * splits + 7) / 8);
  args.group_m = 8;
  return hipSuccess;
}

// Operand order and plan: the general kernels store along n, so C's innermost
// leg must come from "B"; the large-tile split-bf16 kernel also stores along
// m and then takes the operands in the given order (A = m side).
// Tail of a large-tile launch.  When the tiles fill whole waves of the GPU's
// workgroup slots except for a last wave that fills at most a quarter of them,
// and the k range is long (at least 64 k-tiles), the rows of that last wave run as a second launch
// whose tiles are split along k (at least 8 k-tiles per split) over the free
// slots, with the partial sums reduced in a fixed order afterwards: no CU then
// works through a whole extra tile while the others wait.  Needs scratch for the
// partial sums of the tail rows.
void plan_tail(Plan& pl, bool have_scratch, size_t scratch_elems) {
  const TcArgs& a = pl.args;
  pl.tail_tm = pl.tail_ks = 0;
  if (!pl.use_x || a.splits != 1 || !have_scratch) return;
  const int64_t slots = b3x_slots();
  const int64_t tiles = (int64_t)a.tiles_m * a.tiles_n;
  const int64_t full = tiles / slots * slots, rem = tiles - full;
  if (full == 0 || rem == 0 || 4 * rem > slots || full % a.tiles_n != 0) return;
  const int64_t nk = pl.K / 32;
  if (nk < 64) return;  // short k ranges: the two extra launches would cost what they save
  int64_t ks = std::min<int64_t>(slots / rem, nk / 8);
  if (ks < 2) return;
  const int64_t chunk = (nk + ks - 1) / ks;  // k-tiles per split
  ks = (nk + chunk - 1) / chunk;
  const int64_t tail_tm = rem / a.tiles_n;
  const int64_t rows = pl.M - (int64_t)(a.tiles_m - tail_tm) * 256;
  if (ks < 2 || (size_t)(ks * rows * pl.N) > scratch_elems) return;
  pl.tail_tm = (int)tail_tm;
  pl.tail_ks = (int)ks;
}

hipError_t choose_plan(Arith ar, const LabelDims& dims, const LabelDims& cd, const void* A,
                       const char* la_, const void* B, const char* lb_, void* C, const char* lc_,
                       bool c_f64, double alpha, double beta, double* scratch,
                       size_t scratch_elems, Plan& pl) {
  std::string la(la_), lb(lb_), lc(lc_);
  const bool c_from_a = !lc.empty() && contains(la, lc.back()) && !contains(lb, lc.back());
  if (c_from_a && ar == Arith::B3) {
    const hipError_t e = make_plan(ar, dims, cd, A, la, B, lb, C, lc, c_f64, alpha, beta, scratch,
                                   scratch_elems, true, pl);
    if (e != hipSuccess) return e;
    if (pl.use_x || pl.M == 0 || pl.N == 0 || pl.K == 0) return hipSuccess;
  }
  if (c_from_a) {
    std::swap(la, lb);
    std::swap(A, B);
  }
  pl = Plan();
  return make_plan(ar, dims, cd, A, la, B, lb, C, lc, c_f64, alpha, beta, scratch, scratch_elems,
                   false, pl);
}

}  // namespace

std::string contract_plan(Arith ar, const LabelDims& dims, const char* la, const char* lb,
                          const char* lc, bool c_f64, size_t scratch_elems,
                          const LabelDims* cdims) {
  // host-only: aligned placeholder addresses, never dereferenced
  void* const fake = reinterpret_cast<void*>(uintptr_t(1) << 20);
  Plan pl;
  if (choose_plan(ar, dims, cdims ? *cdims : dims, fake, la, fake, lb, fake, lc, c_f64, 1.0, 0.0,
                  scratch_elems ? static_cast<double*>(fake) : nullptr, scratch_elems,
                  pl) != hipSuccess)
    return "unsupported";
  char buf[160];
  const TcArgs& a = pl.args;
  const char* kern = ar == Arith::F64 ? "f64" : ar == Arith::F32 ? "f32" : pl.use_x ? "b3x" : "b3";
  plan_tail(pl, scratch_elems > 0, scratch_elems);
  std::snprintf(buf, sizeof(buf), "%s%s m=%lld n=%lld k=%lld tiles=%dx%d splits=%d store=%s", kern,
                pl.use_x ? std::to_string(pl.xbn).c_str() : "", (long long)pl.M, (long long)pl.N,
                (long long)pl.K, a.tiles_m, a.tiles_n, a.splits,
                a.cm == 1 ? "m4" : a.cm == 2 ? "m1" : a.cgroup8 ? "n8" : a.cvec ? "n4"
                : (a.cvec2 && ar == Arith::F64) ? "n2" : "n1");
  std::string out(buf);
  if (pl.tail_tm > 0) out += " tail=" + std::to_string(pl.tail_tm) + "x" + std::to_string(pl.tail_ks);
  return out;
}

hipError_t contract(Arith ar, const LabelDims& dims, const void* A, const char* la_, const void* B,
                    const char* lb_, void* C, const char* lc_, bool c_f64, double alpha,
                    double beta, hipStream_t stream, double* flops, double* scratch,
                    size_t scratch_elems, const LabelDims* cdims) {
  Plan pl;
  const hipError_t pe = choose_plan(ar, dims, cdims ? *cdims : dims, A, la_, B, lb_, C, lc_, c_f64,
                                    alpha, beta, scratch, scratch_elems, pl);
  if (pe != hipSuccess) return pe;
  if (flops) *flops += 2.0 * (double)pl.M * (double)pl.N * (double)pl.K;
  if (pl.M == 0 || pl.N == 0) return hipSuccess;
  if (pl.K == 0) return hipErrorInvalidValue;  // the kernels assume at least one k-tile
  const TcArgs& args = pl.args;
  const int blocks = args.per_xcd * 8;
  const int splits = args.splits;
  const bool c64 = c_f64 || splits > 1;  // partial sums are kept in double
  hipError_t e;
  if (ar == Arith::F64) {
    if (!c_f64) return hipErrorInvalidValue;
    e = dispatch<double, double>(args, blocks, pl.A_KC, pl.va, pl.B_NC, pl.vb, pl.kal, stream);
  } else if (ar == Arith::F32) {
    e = c64 ? dispatch<float, double>(args, blocks, pl.A_KC, pl.va, pl.B_NC, pl.vb, pl.kal, stream)
            : dispatch<float, float>(args, blocks, pl.A_KC, pl.va, pl.B_NC, pl.vb, pl.kal, stream);
  } else if (pl.use_x) {
    plan_tail(pl, scratch != nullptr, scratch_elems);
    if (pl.tail_tm == 0) {
      e = launch_contract_b3x(args, pl.xbn, c64, stream);
    } else {
      // the whole waves of tiles: rows [0, head), one tile per slot and wave
      TcArgs head = args;
      head.tiles_m = args.tiles_m - pl.tail_tm;
      head.M = head.tiles_m * 256;
      head.per_xcd = (head.tiles_m * head.tiles_n + 7) / 8;
      e = launch_contract_b3x(head, pl.xbn, c64, stream);
      if (e != hipSuccess) return e;
      // the tail rows, split along k into double partial sums, then reduced
      TcArgs tail = args;
      tail.m_base = head.M;
      tail.M = args.M - head.M;
      tail.tiles_m = pl.tail_tm;
      tail.splits = pl.tail_ks;
      tail.kchunk = (int32_t)((pl.K / 32 + pl.tail_ks - 1) / pl.tail_ks * 32);
      tail.part = scratch;
      tail.cvec = (tail.N % 4 == 0) ? 1 : 0;
      tail.cgroup8 = 0;
      tail.per_xcd = (tail.tiles_m * tail.tiles_n * tail.splits + 7) / 8;
      e = launch_contract_b3x(tail, pl.xbn, true, stream);
      if (e != hipSuccess) return e;
      const int64_t tmn = (int64_t)tail.M * tail.N;
      const int tgrid = (int)std::min<int64_t>((tmn + 255) / 256, 8192);
      if (c_f64)
        hipLaunchKernelGGL(tc_splitk_reduce<double>, dim3(tgrid), dim3(256), 0, stream, tail);
      else
        hipLaunchKernelGGL(tc_splitk_reduce<float>, dim3(tgrid), dim3(256), 0, stream, tail);
      return hipGetLastError();
    }
  } else {
    e = launch_contract_b3(args, pl.A_KC, pl.va, pl.B_NC, pl.vb, pl.kal, c64, stream);
  }
  if (e != hipSuccess || splits == 1) return e;
  const int64_t mn = pl.M * pl.N;
  const int grid = (int)std::min<int64_t>((mn + 255) / 256, 8192);
  if (c_f64)
    hipLaunchKernelGGL(tc_splitk_reduce<double>, dim3(grid), dim3(256), 0, stream, args);
  else
    hipLaunchKernelGGL(tc_splitk_reduce<float>, dim3(grid), dim3(256), 0, stream, args);
  return hipGetLastError();
}

}  // namespace mera
