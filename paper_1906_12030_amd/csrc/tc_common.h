// Descriptor of one contraction launch and the device helpers shared by the
// FP64/FP32 and split-bf16 kernels (internal).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace mera {

constexpr int kMaxDims = 6;

// One index group (the m, n or k legs of a contraction) after merging legs
// that are contiguous in both operands that carry it.
struct Group {
  int32_t nd;
  int32_t size[kMaxDims];  // outer ... inner
  int64_t sx[kMaxDims];    // strides in the first operand of the group
  int64_t sy[kMaxDims];    // strides in the second operand of the group
};

struct TcArgs {
  const void* a;
  const void* b;
  void* c;
  double* part;  // split-k partial sums, dense [splits][M][N] (used when splits > 1)
  int32_t M, N, K;
  Group gm;  // x = A, y = C
  Group gn;  // x = B, y = C
  Group gk;  // x = A, y = B
  double alpha, beta;
  int32_t tiles_m, tiles_n, per_xcd, group_m;
  int32_t splits, kchunk;  // k range of split s: [s*kchunk, min(K, (s+1)*kchunk))
  int32_t cvec;            // 64-wide output column spans are contiguous (vector stores)
  int32_t csplit;          // FP32 C is a split tensor (see split_hi)
  // Large-tile kernel only: 0 = C's innermost leg is an n leg (stores along
  // n); 1 = it is the innermost m leg, with unit stride, a multiple of 4 long
  // and every other C stride a multiple of 4 (four consecutive rows form one
  // aligned vector); 2 = it is an m leg otherwise (element stores along m).
  int32_t cm;
  // Large-tile kernel, split C stored along n: 1 when every 8-aligned group of 8
  // consecutive output columns is one planar group of C (innermost n leg with
  // unit stride and an extent that is a multiple of 8, every other C stride a
  // multiple of 8), so that a lane can store the 16-byte hi or lo half of a group.
  int32_t cgroup8;
  // Large-tile kernel and split-k reduction: row m of this launch is row
  // m_base + m of the contraction (a launch over the last rows only).
  int32_t m_base;
  // 128 x 128 kernels: every 2-aligned pair of consecutive output columns is
  // adjacent in C (innermost n leg with unit stride and an even extent, every
  // other C stride even, C 16-byte aligned): one 16-byte store per two doubles.
  int32_t cvec2;
};

// Split tensors.  The split-bf16 path keeps every FP32 value x as two bf16
// numbers, hi = bf16_rne(x) and lo = bf16_rne(x - hi), in 4 bytes per element,
// grouped by 8 consecutive elements: the 32-byte group i / 8 holds the hi halves
// of its 8 elements (bytes 0..15, element i % 8 at halfword i % 8), then their lo
// halves (bytes 16..31).  A 16-byte read of either half of a group is one bf16x8
// MFMA operand, so the split of each value is done once, by the kernel that
// produces the tensor, and the loaders need no regrouping.  A split tensor of n
// elements occupies 32 * ceil(n / 8) bytes and starts 32-byte aligned.
__device__ __forceinline__ int64_t split_hi(int64_t i) { return ((i >> 3) << 4) | (i & 7); }
__device__ __forceinline__ uint16_t bf16_bits(float x) { return __builtin_bit_cast(uint16_t, (__bf16)x); }
__device__ __forceinline__ float bf16_value(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }
// element i of the split tensor at base: store x / load hi + lo
__device__ __forceinline__ void split_store(void* base, int64_t i, float x) {
  uint16_t* b = static_cast<uint16_t*>(base) + split_hi(i);
  const uint16_t h = bf16_bits(x);
  b[0] = h;
  b[8] = bf16_bits(x - bf16_value(h));
}
__device__ __forceinline__ float split_load(const void* base, int64_t i) {
  const uint16_t* b = static_cast<const uint16_t*>(base) + split_hi(i);
  return bf16_value(b[0]) + bf16_value(b[8]);
}
// elements i .. i + 3 (i a multiple of 4, so they share a group): two 8-byte stores
__device__ __forceinline__ void split_store4(void* base, int64_t i, const float (&x)[4]) {
  typedef uint16_t h4_t __attribute__((ext_vector_type(4)));
  h4_t h, l;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    h[e] = bf16_bits(x[e]);
    l[e] = bf16_bits(x[e] - bf16_value(h[e]));
  }
  uint16_t* b = static_cast<uint16_t*>(base) + split_hi(i);
  *reinterpret_cast<h4_t*>(b) = h;
  *reinterpret_cast<h4_t*>(b + 8) = l;
}

// Offset of linear group index idx in operand x (Second = false) or y.
template <bool Second>
__device__ __forceinline__ int64_t goff(const Group& g, uint32_t idx) {
  int64_t off = 0;
#pragma unroll
  for (int d = kMaxDims - 1; d >= 0; --d) {
    if (d < g.nd) {
      const uint32_t sz = (uint32_t)g.size[d];
      const uint32_t q = idx / sz;
      const uint32_t r = idx - q * sz;
      off += (int64_t)r * (Second ? g.sy[d] : g.sx[d]);
      idx = q;
    }
  }
  return off;
}

// Tile of a logical tile index: XCD x owns the contiguous range of logical
// tiles [x * per_xcd, (x + 1) * per_xcd), walked in groups of group_m tile rows
// (column-major inside a group) so that concurrently running workgroups of one
// XCD share A and B panels in its L2.
__device__ __forceinline__ void tile_at(const TcArgs& p, int logical, int& tm, int& tn, int& split) {
  const int total = p.tiles_m * p.tiles_n;
  split = logical / total;
  logical -= split * total;
  const int gsz_full = p.group_m * p.tiles_n;
  const int group = logical / gsz_full;
  const int first_m = group * p.group_m;
  const int gsize = min(p.tiles_m - first_m, p.group_m);
  const int in_group = logical - group * gsz_full;
  tm = first_m + in_group % gsize;
  tn = in_group / gsize;
}

// Tile of this workgroup.  Hardware dispatches consecutive workgroups round
// robin over the 8 XCDs, so workgroup b runs on XCD b % 8 and takes logical
// tile (b % 8) * per_xcd + b / 8.
__device__ __forceinline__ bool tile_of_block(const TcArgs& p, int& tm, int& tn, int& split) {
  const int bid = blockIdx.x;
  const int logical = (bid & 7) * p.per_xcd + (bid >> 3);
  if (logical >= p.tiles_m * p.tiles_n * p.splits) return false;
  tile_at(p, logical, tm, tn, split);
  return true;
}

hipError_t launch_contract_b3(const TcArgs& a, bool akc, bool va, bool bnc, bool vb, bool kal,
                              bool c_f64, hipStream_t s);
// Large-tile split-bf16 kernel (both operands contiguous along k, k-aligned):
// whether an M x N output suits it (and its column tile), and the launch.
bool contract_b3x_fits(int64_t M, int64_t N, int64_t K, int& bn);
hipError_t launch_contract_b3x(const TcArgs& a, int bn, bool c_f64, hipStream_t s);
// Workgroup slots of the large-tile kernel on the current device (one per CU).
int b3x_slots();

}  // namespace mera

namespace mera {

constexpr int kThreads = 256;

template <typename T, int V>
__device__ __forceinline__ void load_vec(const T* p, T* out) {
  if constexpr (V == 1) {
    out[0] = *p;
  } else {
    typedef T vt __attribute__((ext_vector_type(V)));
    const vt v = *reinterpret_cast<const vt*>(p);
#pragma unroll
    for (int i = 0; i < V; ++i) out[i] = v[i];
  }
}

// Registers-side loader of one operand tile: ROWS rows (m for A, n for B) by
// BK k-columns.  KC: the operand is contiguous along k (each thread loads V
// consecutive k of one row); otherwise contiguous along the rows (V
// consecutive rows at one k).  KSecond selects the operand's k strides in the
// k group (A: first, B: second).  KAL: the innermost k leg's extent is a
// multiple of BK, so a whole k-tile lies in one run of that leg and its
// offsets are a uniform base plus a per-thread constant; otherwise every
// k offset is decomposed leg by leg (and masked against K).
template <typename T, int ROWS, int BK, bool KC, int V, bool KAL, bool KSecond>
struct TileLoad {
  static constexpr int TPL = KC ? BK / V : ROWS / V;  // threads per line
  static constexpr int LPP = kThreads / TPL;          // lines per pass
  static constexpr int NP = KC ? ROWS / LPP : BK / LPP;
  static_assert(NP >= 1 && LPP * TPL == kThreads, "tile geometry");
  static constexpr int NR = KC ? NP : 1;  // row offsets held per thread
  static constexpr int NK = KC ? 1 : NP;  // k lines per thread

  int line, vec;
  int64_t roff[NR];
  bool rok[NR];
  int64_t kd[NK];  // KAL: offset of this thread's k (or k lines) from the k-tile base
  T r[NP][V];

  __device__ __forceinline__ void init(const Group& grow, const Group& gk, uint32_t row0,
                                       uint32_t nrows) {
    const int tid = threadIdx.x;
    line = tid / TPL;
    vec = (tid % TPL) * V;
#pragma unroll
    for (int i = 0; i < NR; ++i) {
      const uint32_t rr = KC ? row0 + line + i * LPP : row0 + vec;
      rok[i] = rr < nrows;
      // rows past the end read a valid element instead (their products only
      // reach output rows that are never stored)
      roff[i] = rok[i] ? goff<false>(grow, rr) : 0;
    }
    const int64_t si = KSecond ? gk.sy[gk.nd - 1] : gk.sx[gk.nd - 1];
#pragma unroll
    for (int i = 0; i < NK; ++i) kd[i] = KC ? (int64_t)vec * si : (int64_t)(line + i * LPP) * si;
  }

  // k-aligned tile whose k offset (uniform) is kb: no masking at all
  __device__ __forceinline__ void load_at(const T* __restrict__ base, int64_t kb) {
    load_at(base, kb, r);
  }
  __device__ __forceinline__ void load_at(const T* __restrict__ base, int64_t kb, T (&d)[NP][V]) {
#pragma unroll
    for (int i = 0; i < NP; ++i) load_vec<T, V>(base + roff[KC ? i : 0] + kb + kd[KC ? 0 : i], d[i]);
  }

  __device__ __forceinline__ void load(const T* __restrict__ base, const Group& gk, uint32_t k0,
                                       uint32_t K) {
    load(base, gk, k0, K, r);
  }
  // into a caller-held register tile d (several tiles in flight)
  __device__ __forceinline__ void load(const T* __restrict__ base, const Group& gk, uint32_t k0,
                                       uint32_t K, T (&d)[NP][V]) {
    if constexpr (KAL) {
      const int64_t kb = goff<KSecond>(gk, k0);
      load_at(base, kb, d);
    } else {
      if constexpr (KC) {
        const uint32_t k = k0 + vec;
        const bool kok = k < K;
        const int64_t ko = kok ? goff<KSecond>(gk, k) : 0;
#pragma unroll
        for (int i = 0; i < NP; ++i) {
          if (kok && rok[i]) {
            load_vec<T, V>(base + roff[i] + ko, d[i]);
          } else {
#pragma unroll
            for (int v = 0; v < V; ++v) d[i][v] = T(0);
          }
        }
      } else {
#pragma unroll
        for (int i = 0; i < NP; ++i) {
          const uint32_t k = k0 + line + i * LPP;
          if (k < K && rok[0]) {
            load_vec<T, V>(base + roff[0] + goff<KSecond>(gk, k), d[i]);
          } else {
#pragma unroll
            for (int v = 0; v < V; ++v) d[i][v] = T(0);
          }
        }
      }
    }
  }
};

// Uniform walk over k-tiles of a k group whose innermost leg's extent is a
// multiple of the tile: keeps the leg digits of the tile start and its offsets
// in both operands, advancing by carries instead of divisions.  The group is
// copied at init, innermost leg first, into registers indexed only by
// compile-time constants, so a step issues no memory loads; it is one add and
// one compare unless the innermost leg wraps.
template <int BK>
struct KWalk {
  int32_t dig[kMaxDims];       // digits, innermost leg first
  int32_t sz[kMaxDims];        // extents, innermost first
  int64_t ca[kMaxDims], cb[kMaxDims];  // offset change when leg j wraps into leg j+1
  int64_t sa, sb;              // offset change of one k-tile step
  int32_t nd;
  int64_t oa, ob;
  __device__ __forceinline__ void init(const Group& g, uint32_t k0) {
    nd = g.nd;
    oa = 0;
    ob = 0;
#pragma unroll
    for (int j = 0; j < kMaxDims; ++j) {
      dig[j] = 0;
      sz[j] = 1;
      ca[j] = 0;
      cb[j] = 0;
      if (j < g.nd) {
        const int d = g.nd - 1 - j;
        sz[j] = g.size[d];
        const uint32_t q = k0 / (uint32_t)sz[j];
        dig[j] = (int32_t)(k0 - q * (uint32_t)sz[j]);
        oa += (int64_t)dig[j] * g.sx[d];
        ob += (int64_t)dig[j] * g.sy[d];
        k0 = q;
        if (d > 0) {
          ca[j] = g.sx[d - 1] - (int64_t)g.size[d] * g.sx[d];
          cb[j] = g.sy[d - 1] - (int64_t)g.size[d] * g.sy[d];
        }
      }
    }
    sa = (int64_t)BK * g.sx[g.nd - 1];
    sb = (int64_t)BK * g.sy[g.nd - 1];
  }
  __device__ __forceinline__ void next() {
    dig[0] += BK;
    oa += sa;
    ob += sb;
    // carries toward the outer legs (rare: once per extent / BK steps)
#pragma unroll
    for (int j = 0; j < kMaxDims - 1; ++j) {
      if (j + 1 >= nd || dig[j] < sz[j]) break;
      dig[j] -= sz[j];
      dig[j + 1] += 1;
      oa += ca[j];
      ob += cb[j];
    }
  }
};

// Output offsets of the tile's rows and columns in LDS (-1 = outside the
// matrix).  Split-k launches write dense partial sums instead.
template <int TM, int TN>
__device__ __forceinline__ void stage_c_offsets(const TcArgs& p, uint32_t m0, uint32_t n0, int split,
                                                int64_t* rows, int64_t* cols) {
  const int t = threadIdx.x;
  for (int i = t; i < TM + TN; i += kThreads) {
    if (i < TM) {
      const uint32_t m = m0 + i;
      int64_t o = -1;
      if (m < (uint32_t)p.M)
        o = p.splits > 1 ? ((int64_t)split * p.M + m) * p.N : goff<true>(p.gm, m);
      rows[i] = o;
    } else {
      const uint32_t n = n0 + (i - TM);
      int64_t o = -1;
      if (n < (uint32_t)p.N) o = p.splits > 1 ? (int64_t)n : goff<true>(p.gn, n);
      cols[i - TM] = o;
    }
  }
}

// Element `off` of C as a number, and y stored there (a split tensor when
// p.csplit).
template <typename TC>
__device__ __forceinline__ double load_c(const TcArgs& p, const TC* C, int64_t off) {
  if constexpr (sizeof(TC) == 4) {
    if (p.csplit) return (double)split_load(C, off);
  }
  return (double)C[off];
}
template <typename TC>
__device__ __forceinline__ void store_c(const TcArgs& p, TC* C, int64_t off, double y) {
  if constexpr (sizeof(TC) == 4) {
    if (p.csplit) {
      split_store(C, off, (float)y);
      return;
    }
  }
  C[off] = (TC)y;
}
// Four consecutive elements off .. off + 3 of C (off a multiple of 4, 16-byte
// aligned): y = alpha * x + beta * C, one vector store (two for double C, two
// 8-byte stores for a split C).
template <typename TC, typename X>
__device__ __forceinline__ void store_c4(const TcArgs& p, TC* C, int64_t off, const X& x, double alpha,
                                         double beta) {
  if constexpr (sizeof(TC) == 4) {
    if (p.csplit && alpha == 1.0 && beta == 0.0) {  // plain store: no rescaling in double
      const float f[4] = {(float)x[0], (float)x[1], (float)x[2], (float)x[3]};
      split_store4(C, off, f);
      return;
    }
  }
  double y[4];
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    y[e] = alpha * (double)x[e];
    if (beta != 0.0) y[e] += beta * load_c(p, C, off + e);
  }
  if constexpr (sizeof(TC) == 4) {
    if (p.csplit) {
      const float f[4] = {(float)y[0], (float)y[1], (float)y[2], (float)y[3]};
      split_store4(C, off, f);
      return;
    }
    typedef float f4v __attribute__((ext_vector_type(4)));
    *reinterpret_cast<f4v*>(C + off) = f4v{(float)y[0], (float)y[1], (float)y[2], (float)y[3]};
  } else {
    typedef double d2v __attribute__((ext_vector_type(2)));
    *reinterpret_cast<d2v*>(C + off) = d2v{y[0], y[1]};
    *reinterpret_cast<d2v*>(C + off + 2) = d2v{y[2], y[3]};
  }
}

// Epilogue shared by the MFMA kernels.  Each wave owns a 64x64 block of the
// 128x128 tile held as 4x4 MFMA 16x16 accumulators; row-group by row-group
// (16 rows) the wave parks its accumulators in LDS and re-reads them so that
// each lane stores 16 contiguous bytes and 16 lanes cover one 64-wide row
// span.  ROWF(lane, r) is the row of accumulator register r within a 16x16
// block.  LDS needs 2 KB of offset tables plus 4 x 16 x (64+pad) accumulators.
template <typename AT, typename TC, typename ACC, typename ROWF>
__device__ __forceinline__ void write_tile(const TcArgs& p, ACC (&acc)[4][4], uint32_t m0,
                                           uint32_t n0, int split, char* lds, ROWF rowf) {
  constexpr int VA = 16 / sizeof(AT);  // accumulator elements per 16-byte read
  constexpr int PADE = VA;
  constexpr int LD = 64 + PADE;
  int64_t* rows = reinterpret_cast<int64_t*>(lds);
  int64_t* cols = rows + 128;
  AT* stage = reinterpret_cast<AT*>(lds + 2048);
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = (wave >> 1) * 64;
  const int wn = (wave & 1) * 64;
  AT* st = stage + wave * 16 * LD;
  stage_c_offsets<128, 128>(p, m0, n0, split, rows, cols);
  TC* __restrict__ C = p.splits > 1 ? reinterpret_cast<TC*>(p.part) : static_cast<TC*>(p.c);
  const double alpha = p.splits > 1 ? 1.0 : p.alpha;
  const double beta = p.splits > 1 ? 0.0 : p.beta;
  const bool vec = p.cvec != 0;
  if constexpr (VA == 2) {
    static_assert(sizeof(TC) == 8, "double accumulators store to a double C");
    if (p.splits == 1 && alpha == 1.0 && beta == 0.0 && (vec || p.cvec2) && m0 + 128 <= (uint32_t)p.M &&
        n0 + 128 <= (uint32_t)p.N) {
      // Whole tile inside C, plain store: lane l writes columns 2 (l % 32) and
      // 2 (l % 32) + 1 of rows 2 it + l / 32 of each 16-row group, one 16-byte
      // store per pair, with no rescaling and no per-element offset lookups.
      const int col = (lane & 31) * 2;
      __syncthreads();  // offsets staged
      const int64_t co = cols[wn + col];
      typedef AT vt __attribute__((ext_vector_type(2)));
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        if (i > 0) __syncthreads();  // previous row group consumed
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
          for (int r = 0; r < 4; ++r) st[rowf(lane, r) * LD + j * 16 + (lane & 15)] = (AT)acc[i][j][r];
        __syncthreads();
#pragma unroll
        for (int it = 0; it < 8; ++it) {
          const int row = 2 * it + (lane >> 5);
          const int64_t ro = rows[wm + i * 16 + row];
          const vt x = *reinterpret_cast<const vt*>(&st[row * LD + col]);
          *reinterpret_cast<vt*>(C + ro + co) = x;
        }
      }
      return;
    }
  }
  // unrolled: acc must stay in registers (a runtime index would demote it to scratch)
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    __syncthreads();  // offsets staged / previous row group consumed
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) st[rowf(lane, r) * LD + j * 16 + (lane & 15)] = (AT)acc[i][j][r];
    __syncthreads();
    constexpr int PER_ROW = 64 / VA;          // 16-byte vectors per 64-wide row
    constexpr int ITER = 16 * PER_ROW / 64;   // vectors per lane
#pragma unroll
    for (int it = 0; it < ITER; ++it) {
      const int idx = it * 64 + lane;
      const int row = idx / PER_ROW;
      const int col = (idx % PER_ROW) * VA;
      const int64_t ro = rows[wm + i * 16 + row];
      if (ro < 0) continue;
      AT v[VA];
      typedef AT vt __attribute__((ext_vector_type(VA)));
      const vt x = *reinterpret_cast<const vt*>(&st[row * LD + col]);
#pragma unroll
      for (int e = 0; e < VA; ++e) v[e] = x[e];
      const int64_t co = cols[wn + col];
      if (vec && co >= 0) {
        if constexpr (VA == 4) {
          store_c4(p, C, ro + co, v, alpha, beta);
        } else {  // two doubles from double accumulators: one 16-byte store
          double y[VA];
#pragma unroll
          for (int e = 0; e < VA; ++e) {
            y[e] = alpha * (double)v[e];
            if (beta != 0.0) y[e] += beta * load_c(p, C, ro + co + e);
          }
          typedef TC ot __attribute__((ext_vector_type(VA)));
          ot o;
#pragma unroll
          for (int e = 0; e < VA; ++e) o[e] = (TC)y[e];
          *reinterpret_cast<ot*>(C + ro + co) = o;
        }
      } else {
#pragma unroll
        for (int e = 0; e < VA; ++e) {
          const int64_t ce = cols[wn + col + e];
          if (ce < 0) continue;
          double y = alpha * (double)v[e];
          if (beta != 0.0) y += beta * load_c(p, C, ro + ce);
          store_c(p, C, ro + ce, y);
        }
      }
    }
  }
}

}  // namespace mera
