// Split-bf16 ("3xBF16") contraction kernel for gfx950.
//
// Operands arrive as FP32.  On the way into LDS every value x is split into
//   hi = bf16_rne(x),  lo = bf16_rne(x - hi),
// and the tile product is formed on BF16 MFMA (v_mfma_f32_16x16x32_bf16) as
//   hi_a*hi_b + hi_a*lo_b + lo_a*hi_b      (lo*lo, of relative size 2^-16, is dropped)
// with FP32 accumulation (Henry, Tang and Heinecke, "Leveraging the bfloat16
// artificial intelligence datatype for higher-precision computations",
// ARITH 2019).  The addressing (separable leg offsets, XCD-aware tile order)
// is the same as in the FP64/FP32 kernel of contract.hip.
#include <hip/hip_runtime.h>

#include <cstring>

#include "engine.h"
#include "tc_common.h"

namespace mera {

namespace b3 {

typedef float f4_t __attribute__((ext_vector_type(4)));
typedef __bf16 bf8_t __attribute__((ext_vector_type(8)));

__device__ __forceinline__ void split_bf16(float x, __bf16& hi, __bf16& lo) {
  hi = (__bf16)x;
  lo = (__bf16)(x - (float)hi);
}

constexpr int kBM = 128;
constexpr int kBN = 128;
constexpr int kBK = 32;
constexpr int kPadK = 8;  // bf16 elements of padding per LDS row (keeps 16-lane b128 reads conflict-free)

constexpr int kRow = kBK + kPadK;

// Operand loaders for the split kernel.  LDS holds each operand as
// [row][k] (k fastest) so that an MFMA fragment (8 consecutive k of one row)
// is one 16-byte read.  KC operands (contiguous along k) use TileLoad; operands
// contiguous along their rows (m for A, n for B) are read 16 k per thread at
// one row, so that every global load of a wave covers 64 consecutive rows and
// every LDS write is a 16-byte row segment.
template <bool KC, int V, bool KAL, bool KSecond>
struct B3Load;

template <int V, bool KAL, bool KSecond>
struct B3Load<true, V, KAL, KSecond> {
  TileLoad<float, 128, kBK, true, V, KAL, KSecond> t;
  __device__ __forceinline__ void init(const Group& grow, const Group& gk, uint32_t row0,
                                       uint32_t nrows) {
    t.init(grow, gk, row0, nrows);
  }
  __device__ __forceinline__ void load_at(const float* __restrict__ base, int64_t kb) {
    t.load_at(base, kb);
  }
  __device__ __forceinline__ void load(const float* __restrict__ base, const Group& gk, uint32_t k0,
                                       uint32_t kend) {
    t.load(base, gk, k0, kend);
  }
  __device__ __forceinline__ void store(__bf16 (*H)[kRow], __bf16 (*L)[kRow]) {
#pragma unroll
    for (int i = 0; i < t.NP; ++i)
#pragma unroll
      for (int v = 0; v < V; ++v) {
        __bf16 h, l;
        split_bf16(t.r[i][v], h, l);
        H[t.line + i * t.LPP][t.vec + v] = h;
        L[t.line + i * t.LPP][t.vec + v] = l;
      }
  }
};

template <int V, bool KAL, bool KSecond>
struct B3Load<false, V, KAL, KSecond> {
  static_assert(kThreads == 2 * 128 && kBK == 32, "row loader geometry");
  int row, kg;
  int64_t roff, ks;
  float r[16];
  __device__ __forceinline__ void init(const Group& grow, const Group& gk, uint32_t row0,
                                       uint32_t nrows) {
    row = threadIdx.x & 127;
    kg = threadIdx.x >> 7;
    const uint32_t rr = row0 + row;
    // rows past the end read row 0 (their products are never stored)
    roff = rr < nrows ? goff<false>(grow, rr) : 0;
    ks = KSecond ? gk.sy[gk.nd - 1] : gk.sx[gk.nd - 1];
  }
  __device__ __forceinline__ void load_at(const float* __restrict__ base, int64_t kb) {
    const float* q = base + roff + kb + (int64_t)(kg * 16) * ks;
#pragma unroll
    for (int e = 0; e < 16; ++e) r[e] = q[(int64_t)e * ks];
  }
  __device__ __forceinline__ void load(const float* __restrict__ base, const Group& gk, uint32_t k0,
                                       uint32_t kend) {
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const uint32_t k = k0 + kg * 16 + e;
      r[e] = k < kend ? base[roff + goff<KSecond>(gk, k)] : 0.f;
    }
  }
  __device__ __forceinline__ void store(__bf16 (*H)[kRow], __bf16 (*L)[kRow]) {
    bf8_t h0, h1, l0, l1;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      __bf16 h, l;
      split_bf16(r[e], h, l);
      h0[e] = h;
      l0[e] = l;
      split_bf16(r[e + 8], h, l);
      h1[e] = h;
      l1[e] = l;
    }
    *reinterpret_cast<bf8_t*>(&H[row][kg * 16]) = h0;
    *reinterpret_cast<bf8_t*>(&H[row][kg * 16 + 8]) = h1;
    *reinterpret_cast<bf8_t*>(&L[row][kg * 16]) = l0;
    *reinterpret_cast<bf8_t*>(&L[row][kg * 16 + 8]) = l1;
  }
};

template <typename TC, bool A_KC, int VA, bool B_NC, int VB, bool KAL>
__global__ __launch_bounds__(kThreads) void tc_b3_kernel(TcArgs p) {
  __shared__ __attribute__((aligned(16))) char smem[2 * (kBM + kBN) * kRow * sizeof(__bf16)];
  __bf16 (*Ah)[kRow] = reinterpret_cast<__bf16 (*)[kRow]>(smem);
  __bf16 (*Al)[kRow] = reinterpret_cast<__bf16 (*)[kRow]>(smem + kBM * kRow * sizeof(__bf16));
  __bf16 (*Bh)[kRow] = reinterpret_cast<__bf16 (*)[kRow]>(smem + 2 * kBM * kRow * sizeof(__bf16));
  __bf16 (*Bl)[kRow] =
      reinterpret_cast<__bf16 (*)[kRow]>(smem + (2 * kBM + kBN) * kRow * sizeof(__bf16));

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
  const float* __restrict__ A = static_cast<const float*>(p.a);
  const float* __restrict__ B = static_cast<const float*>(p.b);

  B3Load<A_KC, VA, KAL, false> la;
  B3Load<!B_NC, VB, KAL, true> lb;
  la.init(p.gm, p.gk, m0, (uint32_t)p.M);
  lb.init(p.gn, p.gk, n0, (uint32_t)p.N);

  auto store_tiles = [&]() {
    la.store(Ah, Al);
    lb.store(Bh, Bl);
  };

  f4_t acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = f4_t{0.f, 0.f, 0.f, 0.f};

  const int nk = (int)((kend - kbeg + kBK - 1) / kBK);
  const int lr = lane & 15;
  const int lk = (lane >> 4) * 8;
  KWalk<kBK> kw;
  if constexpr (KAL) kw.init(p.gk, kbeg);
  // k-tile fetch: carry walk for k-aligned tiles, leg decomposition otherwise
  auto fetch = [&](int kt) {
    if constexpr (KAL) {
      if (kt > 0) kw.next(p.gk);
      la.load_at(A, kw.oa);
      lb.load_at(B, kw.ob);
    } else {
      la.load(A, p.gk, kbeg + (uint32_t)kt * kBK, kend);
      lb.load(B, p.gk, kbeg + (uint32_t)kt * kBK, kend);
    }
  };
  fetch(0);
  for (int kt = 0; kt < nk; ++kt) {
    store_tiles();
    __syncthreads();
    if (kt + 1 < nk) {
      fetch(kt + 1);
    }
    bf8_t ah[4], al[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      ah[i] = *reinterpret_cast<const bf8_t*>(&Ah[wm + i * 16 + lr][lk]);
      al[i] = *reinterpret_cast<const bf8_t*>(&Al[wm + i * 16 + lr][lk]);
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const bf8_t bh = *reinterpret_cast<const bf8_t*>(&Bh[wn + j * 16 + lr][lk]);
      const bf8_t bl = *reinterpret_cast<const bf8_t*>(&Bl[wn + j * 16 + lr][lk]);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[i], bh, acc[i][j], 0, 0, 0);
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bl, acc[i][j], 0, 0, 0);
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bh, acc[i][j], 0, 0, 0);
      }
    }
    __syncthreads();
  }

  write_tile<float, TC>(p, acc, m0, n0, split, smem,
                        [](int ln, int r) { return 4 * (ln >> 4) + r; });
}

template <typename TC, bool AKC, int VA, bool BNC, int VB, bool KAL>
hipError_t launch_one(const TcArgs& a, int blocks, hipStream_t s) {
  hipLaunchKernelGGL((tc_b3_kernel<TC, AKC, VA, BNC, VB, KAL>), dim3(blocks), dim3(kThreads), 0, s,
                     a);
  return hipGetLastError();
}

template <typename TC>
hipError_t dispatch(const TcArgs& a, int blocks, bool akc, bool va, bool bnc, bool vb, bool kal,
                    hipStream_t s) {
  if (!kal) {
    if (akc) return bnc ? launch_one<TC, true, 1, true, 1, false>(a, blocks, s)
                        : launch_one<TC, true, 1, false, 1, false>(a, blocks, s);
    return bnc ? launch_one<TC, false, 1, true, 1, false>(a, blocks, s)
               : launch_one<TC, false, 1, false, 1, false>(a, blocks, s);
  }
#define MERA_B3_CASE(AK, AV, BN, BV)                                      \
  if (akc == AK && (AK && va ? 4 : 1) == AV && bnc == BN && (!BN && vb ? 4 : 1) == BV) \
    return launch_one<TC, AK, AV, BN, BV, true>(a, blocks, s);
  MERA_B3_CASE(true, 4, true, 1)
  MERA_B3_CASE(true, 1, true, 1)
  MERA_B3_CASE(true, 4, false, 4)
  MERA_B3_CASE(true, 4, false, 1)
  MERA_B3_CASE(true, 1, false, 4)
  MERA_B3_CASE(true, 1, false, 1)
  MERA_B3_CASE(false, 1, true, 1)
  MERA_B3_CASE(false, 1, false, 4)
  MERA_B3_CASE(false, 1, false, 1)
#undef MERA_B3_CASE
  return hipErrorInvalidValue;
}

}  // namespace b3

hipError_t launch_contract_b3(const TcArgs& a, bool akc, bool va, bool bnc, bool vb, bool kal,
                              bool c_f64, hipStream_t s) {
  // the split kernel uses the same 128x128 tile (and tile order) as contract.hip
  return c_f64 ? b3::dispatch<double>(a, a.per_xcd * 8, akc, va, bnc, vb, kal, s)
               : b3::dispatch<float>(a, a.per_xcd * 8, akc, va, bnc, vb, kal, s);
}

}  // namespace mera
