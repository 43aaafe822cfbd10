// Split-bf16 ("3xBF16") contraction kernel for gfx950.
//
// Every FP32 value x is represented by two bf16 numbers,
//   hi = bf16_rne(x),  lo = bf16_rne(x - hi),
// and the tile product is formed on BF16 MFMA (v_mfma_f32_16x16x32_bf16) as
//   hi_a*hi_b + hi_a*lo_b + lo_a*hi_b      (lo*lo, of relative size 2^-16, is dropped)
// with FP32 accumulation (Henry, Tang and Heinecke, "Leveraging the bfloat16
// artificial intelligence datatype for higher-precision computations",
// ARITH 2019).  Operands and FP32 results are kept in HBM as split tensors
// (hi and lo halves of 8 consecutive elements in two 16-byte halves of a
// 32-byte group; see split_hi in tc_common.h), so the split is done once, by
// the producer of a tensor; the loaders here read hi and lo halves and place
// them in the hi and lo slots of the LDS tile.  The addressing (separable leg
// offsets, XCD-aware tile order) is the same as in the FP64/FP32 kernel of
// contract.hip.
#include <hip/hip_runtime.h>

#include <cstring>

#include "engine.h"
#include "tc_common.h"

namespace mera {

namespace b3 {

typedef float f4_t __attribute__((ext_vector_type(4)));
typedef __bf16 bf8_t __attribute__((ext_vector_type(8)));
typedef uint32_t u4_t __attribute__((ext_vector_type(4)));
typedef uint32_t u2_t __attribute__((ext_vector_type(2)));

typedef uint16_t h4_t __attribute__((ext_vector_type(4)));

// hi and lo halves of element i of the split tensor at base (V = 1), or of
// elements i .. i + 3 (V = 4, i a multiple of 4: one 8-byte load each)
template <int V>
__device__ __forceinline__ void load_halves(const uint16_t* __restrict__ base, int64_t i, uint16_t* hi,
                                            uint16_t* lo) {
  const uint16_t* q = base + split_hi(i);
  if constexpr (V == 4) {
    const h4_t h = *reinterpret_cast<const h4_t*>(q);
    const h4_t l = *reinterpret_cast<const h4_t*>(q + 8);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      hi[v] = h[v];
      lo[v] = l[v];
    }
  } else {
    hi[0] = q[0];
    lo[0] = q[8];
  }
}

constexpr int kBM = 128;
constexpr int kBN = 128;
constexpr int kBK = 32;

// LDS tile of one operand: kBM rows of 128 bytes, i.e. eight 16-byte slots,
// logical slots 0..3 = hi of k 0-7, 8-15, 16-23, 24-31 and 4..7 = lo of the
// same.  Logical slot s of row r sits at physical slot s ^ swz(r).  gfx950's
// LDS serves a 16-byte-per-lane access without conflicts when each half-wave
// (32 lanes) touches 32 distinct 16-byte slots modulo 512 bytes; with
// swz(r) = rotate-left of the 3 bits ((r >> 2) & 7) that holds for the MFMA
// fragment reads (16 rows x 2 k-slots per half-wave), for the row loader's
// writes (32 consecutive rows at one slot) and for TileLoad's 8-byte writes
// (4 rows x 128 bytes).
constexpr int kRowBytes = 128;
constexpr int kTileBytes = kBM * kRowBytes;

__device__ __forceinline__ int swz(int r) { return (((r >> 2) & 3) << 1) | ((r >> 4) & 1); }
// byte offset of logical slot s of row r
__device__ __forceinline__ int slot_off(int r, int s) { return r * kRowBytes + ((s ^ swz(r)) << 4); }

// Operand loaders for the split kernel.  KC operands (contiguous along k)
// take TileLoad's geometry and offsets (V consecutive k of one row per
// thread) and read the hi and lo halves of those elements; operands
// contiguous along their rows (m for A, n for B) are read 16 k per thread at
// one row, so that every global load of a wave covers 64 consecutive rows and
// every LDS write is a 16-byte slot.
template <bool KC, int V, bool KAL, bool KSecond>
struct B3Load;

template <int V, bool KAL, bool KSecond>
struct B3Load<true, V, KAL, KSecond> {
  using TL = TileLoad<float, 128, kBK, true, V, KAL, KSecond>;  // geometry and offsets only
  TL t;
  uint16_t h[TL::NP][V], l[TL::NP][V];
  __device__ __forceinline__ void init(const Group& grow, const Group& gk, uint32_t row0,
                                       uint32_t nrows) {
    t.init(grow, gk, row0, nrows);
  }
  __device__ __forceinline__ void load_at(const float* __restrict__ base, int64_t kb) {
    const uint16_t* b16 = reinterpret_cast<const uint16_t*>(base);
#pragma unroll
    for (int i = 0; i < TL::NP; ++i) load_halves<V>(b16, t.roff[i] + kb + t.kd[0], h[i], l[i]);
  }
  __device__ __forceinline__ void load(const float* __restrict__ base, const Group& gk, uint32_t k0,
                                       uint32_t kend) {
    if constexpr (KAL) {
      load_at(base, goff<KSecond>(gk, k0));
    } else {
      const uint16_t* b16 = reinterpret_cast<const uint16_t*>(base);
      const uint32_t k = k0 + t.vec;
      const bool kok = k < kend;
      const int64_t ko = kok ? goff<KSecond>(gk, k) : 0;
#pragma unroll
      for (int i = 0; i < TL::NP; ++i) {
        if (kok && t.rok[i]) {
          load_halves<V>(b16, t.roff[i] + ko, h[i], l[i]);
        } else {
#pragma unroll
          for (int v = 0; v < V; ++v) h[i][v] = l[i][v] = 0;
        }
      }
    }
  }
  __device__ __forceinline__ void store(char* T) {
    const int s = t.vec >> 3;       // k-slot of this thread's k
    const int b = (t.vec & 7) * 2;  // byte offset inside the slot
    // passes step by LPP rows; with LPP a multiple of 32 the swizzle (bits
    // 2..4 of the row) is the same in every pass
    const int oh = slot_off(t.line, s) + b, ol = slot_off(t.line, 4 + s) + b;
#pragma unroll
    for (int i = 0; i < TL::NP; ++i) {
      const int r = t.line + i * TL::LPP;
      if constexpr (V == 4) {
        const int o = TL::LPP % 32 == 0 ? i * TL::LPP * kRowBytes : 0;
        const int ph = TL::LPP % 32 == 0 ? oh + o : slot_off(r, s) + b;
        const int pl = TL::LPP % 32 == 0 ? ol + o : slot_off(r, 4 + s) + b;
        *reinterpret_cast<h4_t*>(T + ph) = h4_t{h[i][0], h[i][1], h[i][2], h[i][3]};
        *reinterpret_cast<h4_t*>(T + pl) = h4_t{l[i][0], l[i][1], l[i][2], l[i][3]};
      } else {
#pragma unroll
        for (int v = 0; v < V; ++v) {
          *reinterpret_cast<uint16_t*>(T + slot_off(r, s) + b + 2 * v) = h[i][v];
          *reinterpret_cast<uint16_t*>(T + slot_off(r, 4 + s) + b + 2 * v) = l[i][v];
        }
      }
    }
  }
};

template <int V, bool KAL, bool KSecond>
struct B3Load<false, V, KAL, KSecond> {
  static_assert(kThreads == 2 * 128 && kBK == 32, "row loader geometry");
  int row, kg;
  int64_t roff, ks;
  uint16_t h[16], l[16];
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
    const uint16_t* b16 = reinterpret_cast<const uint16_t*>(base);
    const int64_t q = roff + kb + (int64_t)(kg * 16) * ks;
#pragma unroll
    for (int e = 0; e < 16; ++e) load_halves<1>(b16, q + (int64_t)e * ks, &h[e], &l[e]);
  }
  __device__ __forceinline__ void load(const float* __restrict__ base, const Group& gk, uint32_t k0,
                                       uint32_t kend) {
    const uint16_t* b16 = reinterpret_cast<const uint16_t*>(base);
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const uint32_t k = k0 + kg * 16 + e;
      if (k < kend) {
        load_halves<1>(b16, roff + goff<KSecond>(gk, k), &h[e], &l[e]);
      } else {
        h[e] = l[e] = 0;
      }
    }
  }
  __device__ __forceinline__ void store(char* T) {
    u4_t h0, h1, l0, l1;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      h0[e] = (uint32_t)h[2 * e] | ((uint32_t)h[2 * e + 1] << 16);
      l0[e] = (uint32_t)l[2 * e] | ((uint32_t)l[2 * e + 1] << 16);
      h1[e] = (uint32_t)h[8 + 2 * e] | ((uint32_t)h[8 + 2 * e + 1] << 16);
      l1[e] = (uint32_t)l[8 + 2 * e] | ((uint32_t)l[8 + 2 * e + 1] << 16);
    }
    *reinterpret_cast<u4_t*>(T + slot_off(row, 2 * kg)) = h0;
    *reinterpret_cast<u4_t*>(T + slot_off(row, 2 * kg + 1)) = h1;
    *reinterpret_cast<u4_t*>(T + slot_off(row, 4 + 2 * kg)) = l0;
    *reinterpret_cast<u4_t*>(T + slot_off(row, 5 + 2 * kg)) = l1;
  }
};

template <typename TC, bool A_KC, int VA, bool B_NC, int VB, bool KAL>
__global__ __launch_bounds__(kThreads) void tc_b3_kernel(TcArgs p) {
  static_assert(kBM == kBN, "one tile geometry for both operands");
  __shared__ __attribute__((aligned(16))) char smem[2 * kTileBytes];
  char* As = smem;
  char* Bs = smem + kTileBytes;

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

  f4_t acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = f4_t{0.f, 0.f, 0.f, 0.f};

  const int nk = (int)((kend - kbeg + kBK - 1) / kBK);
  const int lr = lane & 15;
  // Fragment rows are wm + 16 i + lr (wn + 16 j + lr): their swizzle is
  // ((lr >> 2) & 3) << 1 with bit 0 = parity of the block, so the byte
  // offsets are a per-lane base, the block's 2 KB step and one of four slot
  // offsets (hi / lo, even / odd block).
  const int x0 = ((lane >> 4) ^ (((lr >> 2) & 3) << 1)) << 4;  // hi slot, even block
  const int xo[4] = {x0, x0 ^ 16, x0 ^ 64, x0 ^ 80};          // hi even/odd, lo even/odd
  const int abase = (wm + lr) * kRowBytes, bbase = (wn + lr) * kRowBytes;
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
  for (int kt = 0; kt < nk; ++kt) {
    la.store(As);
    lb.store(Bs);
    __syncthreads();
    if (kt + 1 < nk) fetch(kt + 1);
    bf8_t ah[4], al[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      ah[i] = *reinterpret_cast<const bf8_t*>(As + abase + xo[i & 1] + i * 16 * kRowBytes);
      al[i] = *reinterpret_cast<const bf8_t*>(As + abase + xo[2 + (i & 1)] + i * 16 * kRowBytes);
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const bf8_t bh = *reinterpret_cast<const bf8_t*>(Bs + bbase + xo[j & 1] + j * 16 * kRowBytes);
      const bf8_t bl = *reinterpret_cast<const bf8_t*>(Bs + bbase + xo[2 + (j & 1)] + j * 16 * kRowBytes);
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
