// Tile orders shared by the contraction kernels (FP64 HERK, the FP32 and
// BF16x3 Gram kernels and their split-K reductions): every kernel that
// decodes a tile id must use the same order, so it is defined once here.
#pragma once

#include <hip/hip_runtime.h>

namespace ssrpa {

// Spread consecutive block ids over the 8 XCDs so that neighbouring tiles
// (which share operand panels) run on the same XCD and share its L2.
__device__ __forceinline__ int xcd_remap(int b, int total) {
  const int per = total / 8;
  if (b >= per * 8) return b;
  return (b & 7) * per + (b >> 3);
}

// Logical index of this block when the whole grid (x fastest, then y, z;
// gridDim.x = nx) is spread over the XCDs in contiguous runs: the blocks
// of one XCD then cover a contiguous range of (z, y, x).  Split-K kernels
// with y = split (and z = frequency) give each XCD few K ranges, so the
// rows its blocks stage are fetched into its L2 about once.
__device__ __forceinline__ int xcd_linear(int nx) {
  const int l = blockIdx.x + nx * (blockIdx.y + (int)gridDim.y * blockIdx.z);
  return xcd_remap(l, nx * (int)gridDim.y * (int)gridDim.z);
}

// Sub-tiles of one wave that the result needs: bit n i + j (i, j < n) is
// set when the 16 x 16 sub-tile at rows r0 + 16 i, columns c0 + 16 j holds
// an element of the lower triangle (row >= column) of an ncol x ncol
// matrix.  The others (above the diagonal of a diagonal tile, or in the
// padding past ncol) are dropped by the reductions, so their products are
// skipped.  The mask is made wave-uniform.
template <int n>
__device__ __forceinline__ unsigned live_subtiles(int r0, int c0, int ncol) {
  unsigned m = 0;
#pragma unroll
  for (int i = 0; i < n; ++i)
#pragma unroll
    for (int j = 0; j < n; ++j) {
      const int r = r0 + 16 * i, c = c0 + 16 * j;
      if (r < ncol && c < ncol && r + 15 >= c) m |= 1u << (n * i + j);
    }
  return __builtin_amdgcn_readfirstlane(m);
}

// Lower-triangle tile t -> (I, J) in blocks of kSB x kSB tiles: blocks in
// lower-triangle order, tiles row by row inside a block.  Consecutive tile
// ids (which the XCD remap keeps on one XCD) then share few operand panels,
// so they hit in that XCD's L2.  T = tiles per side.
constexpr int kSB = 8;
__device__ __forceinline__ int2 tri_tile_blocked(int t, int T) {
  const int nb = (T + kSB - 1) / kSB;
  int acc = 0;
  for (int bI = 0; bI < nb; ++bI) {
    const int rI = min(kSB, T - bI * kSB);
    for (int bJ = 0; bJ <= bI; ++bJ) {
      const int cJ = min(kSB, T - bJ * kSB);
      const int cnt = bJ < bI ? rI * cJ : rI * (rI + 1) / 2;
      if (t < acc + cnt) {
        const int l = t - acc;
        int i, j;
        if (bJ < bI) {
          i = l / cJ;
          j = l - i * cJ;
        } else {
          i = (int)((sqrt(8.0 * l + 1.0) - 1.0) * 0.5);
          while (i * (i + 1) / 2 > l) --i;
          while ((i + 1) * (i + 2) / 2 <= l) ++i;
          j = l - i * (i + 1) / 2;
        }
        return make_int2(bI * kSB + i, bJ * kSB + j);
      }
      acc += cnt;
    }
  }
  return make_int2(0, 0);  // not reached for t < T (T + 1) / 2
}

}  // namespace ssrpa
