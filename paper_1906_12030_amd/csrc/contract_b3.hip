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

template <int V>
__device__ __forceinline__ void load_f(const float* p, float* out) {
  if constexpr (V == 4) {
    f4_t v = *reinterpret_cast<const f4_t*>(p);
    out[0] = v.x;
    out[1] = v.y;
    out[2] = v.z;
    out[3] = v.w;
  } else {
    out[0] = *p;
  }
}

__device__ __forceinline__ void split(float x, __bf16& hi, __bf16& lo) {
  hi = (__bf16)x;
  lo = (__bf16)(x - (float)hi);
}

constexpr int kThreads = 256;
constexpr int kBM = 128;
constexpr int kBN = 128;
constexpr int kBK = 32;
constexpr int kPadK = 8;  // bf16 elements of padding per LDS row (keeps 16-lane b128 reads conflict-free)

template <typename TC, bool A_KC, int VA, bool B_NC, int VB>
__global__ __launch_bounds__(kThreads) void tc_b3_kernel(TcArgs p) {
  __shared__ __attribute__((aligned(16))) __bf16 Ah[kBM][kBK + kPadK];
  __shared__ __attribute__((aligned(16))) __bf16 Al[kBM][kBK + kPadK];
  __shared__ __attribute__((aligned(16))) __bf16 Bh[kBN][kBK + kPadK];
  __shared__ __attribute__((aligned(16))) __bf16 Bl[kBN][kBK + kPadK];

  int tm, tn;
  if (!tile_of_block(p, tm, tn)) return;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = (wave >> 1) * 64;
  const int wn = (wave & 1) * 64;
  const uint32_t m0 = (uint32_t)tm * kBM;
  const uint32_t n0 = (uint32_t)tn * kBN;
  const float* __restrict__ A = static_cast<const float*>(p.a);
  const float* __restrict__ B = static_cast<const float*>(p.b);

  constexpr int A_TPR = A_KC ? kBK / VA : kBM / VA;
  constexpr int A_RPP = kThreads / A_TPR;
  constexpr int A_NP = A_KC ? kBM / A_RPP : kBK / A_RPP;
  constexpr int B_TPR = B_NC ? kBN / VB : kBK / VB;
  constexpr int B_RPP = kThreads / B_TPR;
  constexpr int B_NP = B_NC ? kBK / B_RPP : kBN / B_RPP;

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

  float ra[A_NP][VA];
  float rb[B_NP][VB];

  auto load_tiles = [&](uint32_t k0) {
    if (A_KC) {
      const uint32_t k = k0 + a_vec;
      const bool kok = k < (uint32_t)p.K;
      const int64_t ko = kok ? goff<false>(p.gk, k) : 0;
#pragma unroll
      for (int i = 0; i < A_NP; ++i) {
        if (kok && a_ok[i]) {
          load_f<VA>(A + a_off[i] + ko, ra[i]);
        } else {
#pragma unroll
          for (int v = 0; v < VA; ++v) ra[i][v] = 0.f;
        }
      }
    } else {
#pragma unroll
      for (int i = 0; i < A_NP; ++i) {
        const uint32_t k = k0 + a_line + i * A_RPP;
        if (k < (uint32_t)p.K && a_ok[0]) {
          load_f<VA>(A + a_off[0] + goff<false>(p.gk, k), ra[i]);
        } else {
#pragma unroll
          for (int v = 0; v < VA; ++v) ra[i][v] = 0.f;
        }
      }
    }
    if (B_NC) {
#pragma unroll
      for (int i = 0; i < B_NP; ++i) {
        const uint32_t k = k0 + b_line + i * B_RPP;
        if (k < (uint32_t)p.K && b_ok[0]) {
          load_f<VB>(B + b_off[0] + goff<true>(p.gk, k), rb[i]);
        } else {
#pragma unroll
          for (int v = 0; v < VB; ++v) rb[i][v] = 0.f;
        }
      }
    } else {
      const uint32_t k = k0 + b_vec;
      const bool kok = k < (uint32_t)p.K;
      const int64_t ko = kok ? goff<true>(p.gk, k) : 0;
#pragma unroll
      for (int i = 0; i < B_NP; ++i) {
        if (kok && b_ok[i]) {
          load_f<VB>(B + b_off[i] + ko, rb[i]);
        } else {
#pragma unroll
          for (int v = 0; v < VB; ++v) rb[i][v] = 0.f;
        }
      }
    }
  };

  auto store_tiles = [&]() {
#pragma unroll
    for (int i = 0; i < A_NP; ++i)
#pragma unroll
      for (int v = 0; v < VA; ++v) {
        __bf16 h, l;
        split(ra[i][v], h, l);
        const int row = A_KC ? a_line + i * A_RPP : a_vec + v;
        const int col = A_KC ? a_vec + v : a_line + i * A_RPP;
        Ah[row][col] = h;
        Al[row][col] = l;
      }
#pragma unroll
    for (int i = 0; i < B_NP; ++i)
#pragma unroll
      for (int v = 0; v < VB; ++v) {
        __bf16 h, l;
        split(rb[i][v], h, l);
        const int row = B_NC ? b_vec + v : b_line + i * B_RPP;
        const int col = B_NC ? b_line + i * B_RPP : b_vec + v;
        Bh[row][col] = h;
        Bl[row][col] = l;
      }
  };

  f4_t acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = f4_t{0.f, 0.f, 0.f, 0.f};

  const int nk = (p.K + kBK - 1) / kBK;
  const int lr = lane & 15;
  const int lk = (lane >> 4) * 8;
  load_tiles(0);
  for (int kt = 0; kt < nk; ++kt) {
    store_tiles();
    __syncthreads();
    if (kt + 1 < nk) load_tiles((uint32_t)(kt + 1) * kBK);
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
      const uint32_t m = m0 + wm + i * 16 + 4 * (lane >> 4) + r;
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

template <typename TC, bool AKC, int VA, bool BNC, int VB>
hipError_t launch_one(const TcArgs& a, int blocks, hipStream_t s) {
  hipLaunchKernelGGL((tc_b3_kernel<TC, AKC, VA, BNC, VB>), dim3(blocks), dim3(kThreads), 0, s, a);
  return hipGetLastError();
}

template <typename TC>
hipError_t dispatch(const TcArgs& a, int blocks, bool akc, bool va, bool bnc, bool vb,
                    hipStream_t s) {
  if (akc) {
    if (bnc) {
      if (va) return vb ? launch_one<TC, true, 4, true, 4>(a, blocks, s) : launch_one<TC, true, 4, true, 1>(a, blocks, s);
      return vb ? launch_one<TC, true, 1, true, 4>(a, blocks, s) : launch_one<TC, true, 1, true, 1>(a, blocks, s);
    }
    if (va) return vb ? launch_one<TC, true, 4, false, 4>(a, blocks, s) : launch_one<TC, true, 4, false, 1>(a, blocks, s);
    return vb ? launch_one<TC, true, 1, false, 4>(a, blocks, s) : launch_one<TC, true, 1, false, 1>(a, blocks, s);
  }
  if (bnc) {
    if (va) return vb ? launch_one<TC, false, 4, true, 4>(a, blocks, s) : launch_one<TC, false, 4, true, 1>(a, blocks, s);
    return vb ? launch_one<TC, false, 1, true, 4>(a, blocks, s) : launch_one<TC, false, 1, true, 1>(a, blocks, s);
  }
  if (va) return vb ? launch_one<TC, false, 4, false, 4>(a, blocks, s) : launch_one<TC, false, 4, false, 1>(a, blocks, s);
  return vb ? launch_one<TC, false, 1, false, 4>(a, blocks, s) : launch_one<TC, false, 1, false, 1>(a, blocks, s);
}

}  // namespace b3

hipError_t launch_contract_b3(const TcArgs& a, bool akc, bool va, bool bnc, bool vb, bool c_f64,
                              hipStream_t s) {
  // the split kernel uses the same 128x128 tile (and tile order) as contract.hip
  TcArgs args = a;
  return c_f64 ? b3::dispatch<double>(args, args.per_xcd * 8, akc, va, bnc, vb, s)
               : b3::dispatch<float>(args, args.per_xcd * 8, akc, va, bnc, vb, s);
}

}  // namespace mera
