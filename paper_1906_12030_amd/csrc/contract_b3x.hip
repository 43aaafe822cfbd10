// Large-tile split-bf16 contraction kernel for gfx950 (operands contiguous
// along k).
//
// Same arithmetic as contract_b3.hip (split tensors, three BF16 MFMA
// products per multiply-add, FP32 accumulation), organised for the long
// chi^9 contractions whose k-tiles both operands store contiguously:
//   * 256 x BN output tile, 512 threads = 8 waves on v_mfma_f32_16x16x32_bf16:
//     BN = 192 or 256 in a 2 (m) x 4 (n) wave grid (each wave 128 x BN/4,
//     its B fragments held for the k-tile and its A fragments streamed
//     through a ring of four), BN = 288 in a 4 x 2 grid (each wave 64 x 144,
//     A fragments held, B fragments streamed; 21 % fewer LDS bytes per flop
//     than 256 x 192); twice the tile edge of the 128 x 128 kernel halves the
//     bytes that have to come through L2 per flop;
//   * the order of fragment reads, loads and MFMAs after each k-tile's barrier
//     is fixed with scheduling groups: only the fragments of A blocks 0, 1 and
//     B blocks 0, 1 are read before the first MFMA (all eight waves read
//     them at once after the barrier), the other fragments are read in groups
//     right after a wait, each with 11 or 23 MFMAs of cover before the next
//     wait (the LDS-DMA loads in the loop make the compiler wait for all
//     outstanding LDS reads at every wait, so the reads must be issued early
//     rather than counted);
//   * operand k-tiles (32 split elements, 128 bytes, per row) go straight
//     from global memory into LDS with global_load_lds_dwordx4, in a two-stage ring
//     with one barrier per k-tile: the loads of tile kt+1 fly while the
//     MFMAs of tile kt run, and no registers are spent on staging;
//   * LDS rows are 128 bytes (eight 16-byte slots: the hi, then the lo halves
//     of k 0-7, then of k 8-15, ...); slot s of
//     row r is stored at s ^ swz(r), swz(r) = (r & 7) ^ ((r >> 3) & 1), so
//     that in every fragment read (lane l: row l % 16, slot 2 (l / 16) + h)
//     each group of 8 consecutive lanes hits 8 distinct 16-byte slots modulo
//     128 bytes, each group of 16 lanes 16 distinct slots modulo 256 bytes and
//     each group of 32 lanes 32 distinct slots modulo 512 bytes: no bank
//     conflict whichever of these lane groups the LDS serves per cycle (the
//     LDS bank-conflict counter showed 2-way conflicts with the previous
//     swizzle, which only met the last condition);
//   * each lane reads its 8 consecutive k of a row as two 16-byte slots:
//     in a split tensor these are the hi halves and the lo halves of the
//     8 elements (see split_hi in tc_common.h), i.e. the two bf16x8 MFMA
//     operands themselves, so no regrouping instruction sits between the
//     LDS read and the MFMA.
#include <hip/hip_runtime.h>

#include <atomic>

#include "engine.h"
#include "tc_common.h"

namespace mera {

namespace b3x {

typedef float f4_t __attribute__((ext_vector_type(4)));
typedef __bf16 bf8_t __attribute__((ext_vector_type(8)));
typedef uint32_t u4_t __attribute__((ext_vector_type(4)));
typedef float f2_t __attribute__((ext_vector_type(2)));
typedef __bf16 bf2_t __attribute__((ext_vector_type(2)));

constexpr int kThreadsX = 512;
constexpr int kBM = 256;
constexpr int kBK = 32;
constexpr int kRowBytes = kBK * 4;  // one row of a k-tile: 32 split elements

// slot swizzle: the row's low three bits, bit 0 flipped by row bit 3
__device__ __forceinline__ int swz(int r) { return (r & 7) ^ ((r >> 3) & 1); }


// Workgroup barrier without the memory fence of __syncthreads(): that fence
// would wait for every LDS-DMA load of the wave (vmcnt(0)), including the
// ones of the next k-tile; the loop orders LDS itself (wait_vmcnt before the
// barrier that publishes a stage, MFMA operands consumed before the barrier
// that frees it).  The empty asm keeps the compiler from moving memory
// accesses across the barrier.
__device__ __forceinline__ void barrier_nofence() {
  __asm__ volatile("" ::: "memory");
  __builtin_amdgcn_s_barrier();
  __asm__ volatile("" ::: "memory");
}

// Wait until at most n vector-memory operations of this wave are in flight
// (s_waitcnt with the expcnt and lgkmcnt fields at their maxima).
template <int N>
__device__ __forceinline__ void wait_vmcnt() {
  static_assert(N >= 0 && N < 64, "vmcnt range");
  __builtin_amdgcn_s_waitcnt((N & 15) | (7 << 4) | (15 << 8) | ((N >> 4) << 14));
}

template <int BN>
struct Geo {
  static constexpr int kWGN = BN > 256 ? 2 : 4;  // waves along n
  static constexpr int kWGM = 8 / kWGN;          // waves along m
  static constexpr int kWM = kBM / kWGM;         // rows of a wave
  static constexpr int kWMB = kWM / 16;          // 16-row blocks of a wave
  static constexpr int kWN = BN / kWGN;          // columns of a wave
  static constexpr int kWNB = kWN / 16;          // 16-column blocks of a wave
  static constexpr int kATile = kBM * kRowBytes;
  static constexpr int kBTile = BN * kRowBytes;
  static constexpr int kStage = kATile + kBTile;
  static constexpr int kAChunks = kBM / 8, kBChunks = BN / 8;  // 1 KB (8-row) DMA chunks
  static constexpr int kAIns = (kAChunks + 7) / 8;  // per wave
  static constexpr int kBIns = (kBChunks + 7) / 8;
  static_assert(kWN % 16 == 0 && BN % 8 == 0, "tile width");
};

// LDS bytes of the kernel: two stages, reused by the epilogue, and a junk
// kilobyte for the DMA instructions that have no chunk of a tile to load.
template <int BN>
constexpr int lds_bytes() {
  return 2 * Geo<BN>::kStage + (Geo<BN>::kBChunks % 8 == 0 ? 0 : 1024);
}

// sched_group_barrier masks: MFMA, VMEM read, LDS read
constexpr int kSgMfma = 0x008, kSgVmem = 0x020, kSgDsRead = 0x100;

// Scheduling groups of the streamed blocks J, J+1 (of NB, PER MFMAs each): the
// first MFMA of block J (before it, the wait for the fragments of J and J+1),
// the fragment reads of blocks J+2 and J+3, then the other MFMAs of J and J+1,
// which give those reads time to land before the next pair's wait.
template <int J, int NB, int PER>
__device__ __forceinline__ void pin_pairs() {
  if constexpr (J < NB) {
    constexpr int ahead = J + 3 < NB ? 2 : J + 2 < NB ? 1 : 0;
    __builtin_amdgcn_sched_group_barrier(kSgMfma, 1, 0);
    if constexpr (ahead > 0) __builtin_amdgcn_sched_group_barrier(kSgDsRead, 2 * ahead, 0);
    __builtin_amdgcn_sched_group_barrier(kSgMfma, PER * (J + 1 < NB ? 2 : 1) - 1, 0);
    pin_pairs<J + 2, NB, PER>();
  }
}

// Epilogue: when C is contiguous along n, each wave parks one 16-row group of
// its accumulators in LDS and re-reads it so that every lane stores 16
// contiguous bytes along n; when C is contiguous along m (TcArgs::cm), the
// accumulators already hold four consecutive rows per lane and are stored
// directly.
template <typename TC, int BN>
__device__ __forceinline__ void write_tile_x(const TcArgs& p, f4_t (&acc)[Geo<BN>::kWMB][Geo<BN>::kWNB],
                                             uint32_t m0, uint32_t n0, int split, char* lds,
                                             int wm, int wn) {
  using G = Geo<BN>;
  constexpr int LD = BN + 4;  // floats per staged row (pad keeps 16-byte alignment)
  int64_t* rows = reinterpret_cast<int64_t*>(lds);
  int64_t* cols = rows + kBM;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  // one 16-row x BN staging block per row of waves (the waves sharing wm)
  float* st = reinterpret_cast<float*>(lds + (kBM + BN) * 8) + (wave / G::kWGN) * 16 * LD;
  for (int i = tid; i < kBM + BN; i += kThreadsX) {
    if (i < kBM) {
      const uint32_t m = m0 + i;
      int64_t o = -1;
      if (m < (uint32_t)p.M)
        o = p.splits > 1 ? ((int64_t)split * p.M + m) * p.N : goff<true>(p.gm, (uint32_t)p.m_base + m);
      rows[i] = o;
    } else {
      const uint32_t n = n0 + (i - kBM);
      int64_t o = -1;
      if (n < (uint32_t)p.N) o = p.splits > 1 ? (int64_t)n : goff<true>(p.gn, n);
      cols[i - kBM] = o;
    }
  }
  TC* __restrict__ C = p.splits > 1 ? reinterpret_cast<TC*>(p.part) : static_cast<TC*>(p.c);
  const double alpha = p.splits > 1 ? 1.0 : p.alpha;
  const double beta = p.splits > 1 ? 0.0 : p.beta;
  if (p.cm != 0 && p.splits == 1) {
    // C contiguous along m: lane (lr, kq) holds rows 4 kq .. 4 kq + 3 of each
    // 16 x 16 block, column lr, i.e. four consecutive C elements; a wave's
    // store covers 16 columns x 16 rows.  No staging needed.
    __syncthreads();  // offsets staged
    const bool mvec = p.cm == 1;
#pragma unroll
    for (int i = 0; i < G::kWMB; ++i) {
      const int r0 = wm + i * 16 + 4 * (lane >> 4);
      if (rows[r0] < 0) continue;  // rows past M come last
#pragma unroll
      for (int j = 0; j < G::kWNB; ++j) {
        const int64_t co = cols[wn + j * 16 + (lane & 15)];
        if (co < 0) continue;
        if (mvec) {  // rows r0 .. r0 + 3 are all inside M (M % 4 == 0) and adjacent in C
          store_c4(p, C, rows[r0] + co, acc[i][j], alpha, beta);
        } else {
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int64_t re = rows[r0 + e];
            if (re < 0) continue;
            double y = alpha * (double)acc[i][j][e];
            if (beta != 0.0) y += beta * load_c(p, C, re + co);
            store_c(p, C, re + co, y);
          }
        }
      }
    }
    return;
  }
  if (p.cgroup8 && p.splits == 1 && alpha == 1.0 && beta == 0.0 && m0 + kBM <= (uint32_t)p.M &&
      n0 + BN <= (uint32_t)p.N) {
    // Whole tile inside C, plain split store along n.  The two lanes of a pair
    // (2g, 2g+1) share one 8-column group of a tile row: each converts four of
    // its values (the first or the last four) to hi and lo bf16 halves, the
    // pair swaps the halves the other lane stores (DPP), and lane 2g writes the
    // group's 16-byte hi half, lane 2g+1 its lo half, so one store
    // instruction of a wave covers 64 consecutive group halves of C.
    constexpr int HALVES = BN / 4;       // group halves per tile row
    constexpr int ROWS8 = 16 / G::kWGN;  // rows of each 16-row group written by a wave
    constexpr int IT8 = ROWS8 * HALVES / 64;
    static_assert(ROWS8 * HALVES % 64 == 0 && HALVES % 2 == 0, "epilogue geometry");
    const int wr8 = (wave % G::kWGN) * ROWS8;
    const bool lo = (lane & 1) != 0;
    __syncthreads();  // offsets staged
    int rr[IT8], cc[IT8];
    int64_t cb[IT8];
#pragma unroll
    for (int it = 0; it < IT8; ++it) {
      const int idx = it * 64 + lane;  // a pair never straddles a tile row (HALVES is even)
      rr[it] = wr8 + idx / HALVES;
      cc[it] = 8 * ((idx % HALVES) >> 1);
      cb[it] = cols[cc[it]];
    }
    // two bf16 (round to nearest even) packed in a word, and the value of each half
    auto pack = [](float a, float b) {
      return __builtin_bit_cast(uint32_t, __builtin_convertvector(f2_t{a, b}, bf2_t));
    };
    auto low_of = [](uint32_t w) { return __uint_as_float(w << 16); };
    auto high_of = [](uint32_t w) { return __uint_as_float(w & 0xffff0000u); };
    // the value of lane l ^ 1 (quad_perm 1, 0, 3, 2)
    auto swap_pair = [](uint32_t v) {
      return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0xB1, 0xF, 0xF, true);
    };
    char* __restrict__ Cb = static_cast<char*>(p.c);
#pragma unroll
    for (int i = 0; i < G::kWMB; ++i) {
      if (i > 0) __syncthreads();  // previous row group consumed
#pragma unroll
      for (int j = 0; j < G::kWNB; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          st[(4 * (lane >> 4) + r) * LD + wn + j * 16 + (lane & 15)] = acc[i][j][r];
      __syncthreads();
#pragma unroll
      for (int it = 0; it < IT8; ++it) {
        const f4_t x = *reinterpret_cast<const f4_t*>(st + rr[it] * LD + cc[it] + (lo ? 4 : 0));
        const int64_t ro = rows[wm + i * 16 + rr[it]];
        const uint32_t h0 = pack(x[0], x[1]), h1 = pack(x[2], x[3]);
        const uint32_t l0 = pack(x[0] - low_of(h0), x[1] - high_of(h0));
        const uint32_t l1 = pack(x[2] - low_of(h1), x[3] - high_of(h1));
        // lane 2g sends its lo words and keeps its hi words; lane 2g+1 the reverse
        const uint32_t r0 = swap_pair(lo ? h0 : l0), r1 = swap_pair(lo ? h1 : l1);
        const u4_t w = lo ? u4_t{r0, r1, l0, l1} : u4_t{h0, h1, r0, r1};
        // the group starts at element ro + cb (a multiple of 8): byte 4 (ro + cb)
        *reinterpret_cast<u4_t*>(Cb + 4 * (ro + cb[it]) + (lo ? 16 : 0)) = w;
      }
    }
    return;
  }
  const bool vec = p.cvec != 0;
  // The waves of a row of waves park their 16 x kWN blocks side by side, then
  // each writes 16 / kWGN whole rows of the tile (BN contiguous columns): a
  // store instruction covers up to 1 KB of one output row.
  constexpr int PER_ROW = BN / 4;                 // 16-byte vectors per tile row
  constexpr int ROWS = 16 / G::kWGN;              // rows written by each wave
  constexpr int ITER = ROWS * PER_ROW / 64;       // vectors per lane
  static_assert(ROWS * PER_ROW % 64 == 0, "epilogue geometry");
  const int wr = (wave % G::kWGN) * ROWS;         // this wave's first row in the group
#pragma unroll
  for (int i = 0; i < G::kWMB; ++i) {
    __syncthreads();  // offsets staged / previous row group consumed
#pragma unroll
    for (int j = 0; j < G::kWNB; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r)
        st[(4 * (lane >> 4) + r) * LD + wn + j * 16 + (lane & 15)] = acc[i][j][r];
    __syncthreads();
#pragma unroll
    for (int it = 0; it < ITER; ++it) {
      const int idx = it * 64 + lane;
      const int row = wr + idx / PER_ROW;
      const int col = (idx % PER_ROW) * 4;
      const int64_t ro = rows[wm + i * 16 + row];
      if (ro < 0) continue;
      const f4_t x = *reinterpret_cast<const f4_t*>(&st[row * LD + col]);
      const int64_t co = cols[col];
      if (vec && co >= 0) {
        store_c4(p, C, ro + co, x, alpha, beta);
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int64_t ce = cols[col + e];
          if (ce < 0) continue;
          double y = alpha * (double)x[e];
          if (beta != 0.0) y += beta * load_c(p, C, ro + ce);
          store_c(p, C, ro + ce, y);
        }
      }
    }
  }
}

template <typename TC, int BN>
__global__ __launch_bounds__(kThreadsX) void tc_b3x_kernel(TcArgs p) {
  using G = Geo<BN>;
  __shared__ __attribute__((aligned(1024))) char smem[lds_bytes<BN>()];

  int tm, tn, split;
  if (!tile_of_block(p, tm, tn, split)) return;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = (wave / G::kWGN) * G::kWM;
  const int wn = (wave % G::kWGN) * G::kWN;
  const uint32_t m0 = (uint32_t)tm * kBM;
  const uint32_t n0 = (uint32_t)tn * BN;
  const uint32_t kbeg = (uint32_t)split * (uint32_t)p.kchunk;
  const uint32_t kend = min((uint32_t)p.K, kbeg + (uint32_t)p.kchunk);
  const int nk = (int)((kend - kbeg) / kBK);  // k-aligned: whole tiles only
  const char* __restrict__ A = static_cast<const char*>(p.a);
  const char* __restrict__ B = static_cast<const char*>(p.b);

  // DMA sources: chunk c (8 rows) of a tile is loaded by wave c % 8 as its
  // instruction c / 8; lane l fills physical slot l % 8 of row 8c + l / 8,
  // i.e. logical slot s = (l % 8) ^ swz(row): bytes 16 s .. 16 s + 15 of the
  // row's 128-byte k-tile, the hi (s even) or lo (s odd) halves of elements
  // k = 8 (s / 2) .. 8 (s / 2) + 7.
  int64_t asrc[G::kAIns], bsrc[G::kBIns];
  {
    const int rl = lane >> 3, ph = lane & 7;
#pragma unroll
    for (int q = 0; q < G::kAIns; ++q) {
      const int r = (q * 8 + wave) * 8 + rl;
      const uint32_t rr = m0 + r;
      const int64_t ro = rr < (uint32_t)p.M ? goff<false>(p.gm, (uint32_t)p.m_base + rr) : 0;
      asrc[q] = 4 * (ro + 4 * (ph ^ swz(r)));
    }
#pragma unroll
    for (int q = 0; q < G::kBIns; ++q) {
      const int r = (q * 8 + wave) * 8 + rl;
      const uint32_t rr = n0 + r;
      const int64_t ro = (r < BN && rr < (uint32_t)p.N) ? goff<false>(p.gn, rr) : 0;
      bsrc[q] = 4 * (ro + 4 * (ph ^ swz(r)));
    }
  }
  KWalk<kBK> kw;
  kw.init(p.gk, kbeg);
  // B chunks past the tile (BN = 288: 36 chunks, the fifth instruction of waves
  // 4-7) are loaded into a junk kilobyte behind the stages, so that every wave
  // issues the same instructions and the loop body stays one basic block.
  auto issue = [&](int stage, int64_t ka, int64_t kb) {
    char* sa = smem + stage * G::kStage;
    char* sb = sa + G::kATile;
#pragma unroll
    for (int q = 0; q < G::kAIns; ++q)
      __builtin_amdgcn_global_load_lds(reinterpret_cast<const void*>(A + asrc[q] + ka),
                                       sa + (q * 8 + wave) * 1024, 16, 0, 0);
#pragma unroll
    for (int q = 0; q < G::kBIns; ++q) {
      const int c = q * 8 + wave;
      char* dst = (G::kBChunks % 8 == 0 || c < G::kBChunks) ? sb + c * 1024 : smem + 2 * G::kStage;
      __builtin_amdgcn_global_load_lds(reinterpret_cast<const void*>(B + bsrc[q] + kb), dst, 16, 0, 0);
    }
  };

  f4_t acc[G::kWMB][G::kWNB];
#pragma unroll
  for (int i = 0; i < G::kWMB; ++i)
#pragma unroll
    for (int j = 0; j < G::kWNB; ++j) acc[i][j] = f4_t{0.f, 0.f, 0.f, 0.f};

  // fragment offsets: rows wm + 16 i + lr (wn + 16 j + lr), slots 2 kq (hi) and
  // 2 kq + 1 (lo) of k = 8 kq .. 8 kq + 7
  const int lr = lane & 15, kq = lane >> 4, sw = swz(lr);
  const int x0 = ((2 * kq) ^ sw) << 4, x1 = ((2 * kq + 1) ^ sw) << 4;
  const int abase = (wm + lr) * kRowBytes, bbase = (wn + lr) * kRowBytes;

  // One barrier per k-tile: after a wave's own loads of tile kt have landed it
  // waits at the barrier, which then also proves that every wave has finished
  // tile kt-1, so the loads of tile kt+1 may overwrite that stage while the
  // MFMAs of tile kt run.  The k offsets of tile kt+1 are computed before the
  // barrier, and the last tile reloads its own (in-bounds) k range into the
  // free stage, so everything after the barrier is branch-free; the order of
  // the fragment reads, the loads and the MFMAs there is fixed by scheduling
  // groups: the fragments of A blocks 0, 1 and B blocks 0, 1, the loads of
  // tile kt+1, their MFMAs (the reads of the remaining held fragments and of
  // the next two streamed blocks after the first of them), then pairs of
  // streamed blocks, each pair's first MFMA followed by the reads of the next
  // pair (pin_pairs).
  issue(0, 4 * kw.oa, 4 * kw.ob);
  for (int kt = 0; kt < nk; ++kt) {
    if (kt + 1 < nk) kw.next();
    const int64_t ka = 4 * kw.oa, kb = 4 * kw.ob;
    wait_vmcnt<0>();
    barrier_nofence();
    const char* sa = smem + (kt & 1) * G::kStage;
    const char* sb = sa + G::kATile;
    // a lane's two slots of a 16-row block: the hi and the lo halves of its 8
    // elements, i.e. the two bf16x8 MFMA operands
    auto rd = [&](const char* base, int row16, u4_t (&r)[2]) {
      r[0] = *reinterpret_cast<const u4_t*>(base + row16 * 16 * kRowBytes + x0);
      r[1] = *reinterpret_cast<const u4_t*>(base + row16 * 16 * kRowBytes + x1);
    };
    // MFMAs of A blocks [i0, i1) x B blocks [j0, j1), the three products in
    // turn (consecutive MFMAs into one accumulator are (i1 - i0)(j1 - j0)
    // apart); a and b map a block to its fragment slots
    auto mfmas = [&](int i0, int i1, int j0, int j1, auto&& a, auto&& b) {
#pragma unroll
      for (int q = 0; q < 3; ++q)
#pragma unroll
        for (int i = i0; i < i1; ++i)
#pragma unroll
          for (int j = j0; j < j1; ++j) {
            const u4_t(&fa)[2] = a(i);
            const u4_t(&fb)[2] = b(j);
            // products lo x hi, hi x lo, hi x hi
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                __builtin_bit_cast(bf8_t, fa[q == 0 ? 1 : 0]), __builtin_bit_cast(bf8_t, fb[q == 1 ? 1 : 0]),
                acc[i][j], 0, 0, 0);
          }
    };
    if constexpr (G::kWMB == 8) {
      // 2 x 4 (or 2 x 3) waves: B fragments held for the k-tile, A fragments
      // streamed through a ring of four.  First A blocks 0, 1 against B blocks
      // 0, 1 (8 fragment reads before the first MFMA), then against the other
      // B blocks, then pairs of A blocks against all of them.
      constexpr int NB = G::kWNB;
      u4_t ra[4][2], rb[NB][2];
      auto fa = [&](int i) -> const u4_t(&)[2] { return ra[i % 4]; };
      auto fb = [&](int j) -> const u4_t(&)[2] { return rb[j]; };
      rd(sa + abase, 0, ra[0]);
      rd(sa + abase, 1, ra[1]);
      rd(sb + bbase, 0, rb[0]);
      rd(sb + bbase, 1, rb[1]);
      issue((kt + 1) & 1, ka, kb);
      mfmas(0, 2, 0, 2, fa, fb);
#pragma unroll
      for (int j = 2; j < NB; ++j) rd(sb + bbase, j, rb[j]);
      rd(sa + abase, 2, ra[2]);
      rd(sa + abase, 3, ra[3]);
      mfmas(0, 2, 2, NB, fa, fb);
#pragma unroll
      for (int i = 2; i < 8; i += 2) {
        if (i + 2 < 8) {
          rd(sa + abase, i + 2, ra[(i + 2) % 4]);
          rd(sa + abase, i + 3, ra[(i + 3) % 4]);
        }
        mfmas(i, i + 2, 0, NB, fa, fb);
      }
      __builtin_amdgcn_sched_group_barrier(kSgDsRead, 8, 0);
      __builtin_amdgcn_sched_group_barrier(kSgVmem, G::kAIns + G::kBIns, 0);
      __builtin_amdgcn_sched_group_barrier(kSgMfma, 1, 0);
      __builtin_amdgcn_sched_group_barrier(kSgDsRead, 2 * (NB - 2) + 4, 0);
      __builtin_amdgcn_sched_group_barrier(kSgMfma, 11, 0);
      __builtin_amdgcn_sched_group_barrier(kSgMfma, 6 * (NB - 2), 0);
      pin_pairs<2, 8, 3 * NB>();
    } else {
      // 4 x 2 waves: A fragments held for the k-tile, B fragments streamed
      // through a ring of four.  First A blocks 0, 1 against B blocks 0, 1
      // (8 fragment reads before the first MFMA), then A blocks 2, 3 against
      // them, then all A blocks against pairs of B blocks.
      constexpr int NB = G::kWNB;
      constexpr int MB = G::kWMB;
      static_assert(MB == 4, "4 x 2 wave grid");
      u4_t ra[MB][2], rb[4][2];
      auto fa = [&](int i) -> const u4_t(&)[2] { return ra[i]; };
      auto fb = [&](int j) -> const u4_t(&)[2] { return rb[j % 4]; };
      rd(sa + abase, 0, ra[0]);
      rd(sa + abase, 1, ra[1]);
      rd(sb + bbase, 0, rb[0]);
      rd(sb + bbase, 1, rb[1]);
      issue((kt + 1) & 1, ka, kb);
      mfmas(0, 2, 0, 2, fa, fb);
      rd(sa + abase, 2, ra[2]);
      rd(sa + abase, 3, ra[3]);
      rd(sb + bbase, 2, rb[2]);
      rd(sb + bbase, 3, rb[3]);
      mfmas(2, 4, 0, 2, fa, fb);
#pragma unroll
      for (int j = 2; j < NB; j += 2) {
        if (j + 2 < NB) rd(sb + bbase, j + 2, rb[(j + 2) % 4]);
        if (j + 3 < NB) rd(sb + bbase, j + 3, rb[(j + 3) % 4]);
        mfmas(0, MB, j, j + 2 < NB ? j + 2 : NB, fa, fb);
      }
      __builtin_amdgcn_sched_group_barrier(kSgDsRead, 8, 0);
      __builtin_amdgcn_sched_group_barrier(kSgVmem, G::kAIns + G::kBIns, 0);
      __builtin_amdgcn_sched_group_barrier(kSgMfma, 1, 0);
      __builtin_amdgcn_sched_group_barrier(kSgDsRead, 8, 0);
      __builtin_amdgcn_sched_group_barrier(kSgMfma, 11, 0);
      __builtin_amdgcn_sched_group_barrier(kSgMfma, 12, 0);
      pin_pairs<2, NB, 3 * MB>();
    }
  }
  wait_vmcnt<0>();    // the last tile's reload has landed
  barrier_nofence();  // the epilogue reuses the stages

  write_tile_x<TC, BN>(p, acc, m0, n0, split, smem, wm, wn);
}

}  // namespace b3x

bool contract_b3x_fits(int64_t M, int64_t N, int64_t K, int& bn) {
  // 256-row tiles; the column tile that wastes the least of N (ties: 256)
  if (M < 256 || N < 192) return false;
  const int64_t w288 = (N + 287) / 288 * 288 - N;
  const int64_t w256 = (N + 255) / 256 * 256 - N;
  const int64_t w192 = (N + 191) / 192 * 192 - N;
  bn = w192 < w256 ? 192 : 256;
  // 256 x 288 (4 x 2 waves of 64 x 144) reads 21 % fewer LDS bytes per flop than
  // 256 x 192 and is faster for long k ranges; for short ones (a few k-tiles
  // per output tile) its larger epilogue costs more than it saves
  if (K >= 2048 && w288 <= (bn == 192 ? w192 : w256)) bn = 288;
  return true;
}

namespace {

// Compute units of the current device, looked up once per device (256 when the
// query fails, e.g. without a device).
int device_cus() {
  static std::atomic<int> cache[64];
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  int v = cache[dev].load(std::memory_order_relaxed);
  if (v == 0) {
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 8)
      cus = 256;
    v = cus;
    cache[dev].store(v, std::memory_order_relaxed);
  }
  return v;
}

}  // namespace

int b3x_slots() { return device_cus(); }

hipError_t launch_contract_b3x(const TcArgs& a, int bn, bool c_f64, hipStream_t s) {
  const int blocks = a.per_xcd * 8;
  if (bn == 256) {
    if (c_f64)
      hipLaunchKernelGGL((b3x::tc_b3x_kernel<double, 256>), dim3(blocks), dim3(b3x::kThreadsX), 0, s, a);
    else
      hipLaunchKernelGGL((b3x::tc_b3x_kernel<float, 256>), dim3(blocks), dim3(b3x::kThreadsX), 0, s, a);
  } else if (bn == 288) {
    if (c_f64)
      hipLaunchKernelGGL((b3x::tc_b3x_kernel<double, 288>), dim3(blocks), dim3(b3x::kThreadsX), 0, s, a);
    else
      hipLaunchKernelGGL((b3x::tc_b3x_kernel<float, 288>), dim3(blocks), dim3(b3x::kThreadsX), 0, s, a);
  } else if (bn == 192) {
    if (c_f64)
      hipLaunchKernelGGL((b3x::tc_b3x_kernel<double, 192>), dim3(blocks), dim3(b3x::kThreadsX), 0, s, a);
    else
      hipLaunchKernelGGL((b3x::tc_b3x_kernel<float, 192>), dim3(blocks), dim3(b3x::kThreadsX), 0, s, a);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace mera

