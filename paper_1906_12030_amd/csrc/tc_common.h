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
  int32_t M, N, K;
  Group gm;  // x = A, y = C
  Group gn;  // x = B, y = C
  Group gk;  // x = A, y = B
  double alpha, beta;
  int32_t tiles_m, tiles_n, per_xcd, group_m;
};

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

// Tile of this workgroup.  Hardware dispatches consecutive workgroups round
// robin over the 8 XCDs, so workgroup b runs on XCD b % 8; remap so that each
// XCD owns a contiguous range of logical tiles, then walk that range in groups
// of group_m tile rows (column-major inside a group) so that concurrently
// running workgroups of one XCD share A and B panels in its L2.
__device__ __forceinline__ bool tile_of_block(const TcArgs& p, int& tm, int& tn) {
  const int bid = blockIdx.x;
  const int xcd = bid & 7;
  const int idx = bid >> 3;
  const int logical = xcd * p.per_xcd + idx;
  const int total = p.tiles_m * p.tiles_n;
  if (logical >= total) return false;
  const int gsz_full = p.group_m * p.tiles_n;
  const int group = logical / gsz_full;
  const int first_m = group * p.group_m;
  const int gsize = min(p.tiles_m - first_m, p.group_m);
  const int in_group = logical - group * gsz_full;
  tm = first_m + in_group % gsize;
  tn = in_group / gsize;
  return true;
}

hipError_t launch_contract_b3(const TcArgs& a, bool akc, bool va, bool bnc, bool vb, bool c_f64,
                              hipStream_t s);

}  // namespace mera
