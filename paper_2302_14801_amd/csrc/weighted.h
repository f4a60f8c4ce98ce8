// weighted.h -- the neighbourhood-weighted splat of Sec. 4.2.4 in exact
// integer form, shared by the in-core weighted pass and the chunked build's
// levels above the chunk roots.
//
// Positions are on the half-cell lattice of the 2^21 quantization grid (units
// of half a finest cell): a point at 2q + 1, a voxel of a node at level L + 1
// at the centre of its cell of level L + 8.  A sample reaches the cell of its
// parent's grid (level L) that contains it and, per axis, the neighbour on
// the side of its offset, with w = 65536 - floor(65536 * distance in cells)
// where positive.
#pragma once
#include "common.h"

namespace lod {

constexpr uint32_t kWeightOne = 65536;

// floor(sqrt(x)) for x < 2^40: the single-precision square root of x
// (rounded to 24 bits) is within 2^-4 of sqrt(x) there, so its truncation is
// within one of the answer; the integer checks settle the last step.
__device__ __forceinline__ uint64_t isqrt_u64(uint64_t x) {
  uint64_t r = (uint64_t)__fsqrt_rn((float)x);
  for (int i = 0; i < 2 && r * r > x; ++i) --r;
  for (int i = 0; i < 2 && (r + 1) * (r + 1) <= x; ++i) ++r;
  return r;
}

// Calls f(code, w) for every cell of node A's grid (level L, origin G = A's
// coordinates * 128 per axis) that a sample at pos2 reaches with weight w > 0:
// the cell containing it and, per axis, the neighbour on the side of its
// offset (the 2x2x2 cells whose centres surround it), inside A only.
template <class F>
__device__ __forceinline__ void wtargets(uint32_t L, const uint32_t G[3], const uint64_t pos2[3], F&& f) {
  const uint32_t cs = 15 - L;  // log2 of A's cell size in pos2 units
  int64_t cand[3][2];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const int64_t k = (int64_t)(pos2[a] >> cs);
    const int64_t fo = (int64_t)pos2[a] - (k << cs);
    cand[a][0] = k;
    cand[a][1] = fo < ((int64_t)1 << (cs - 1)) ? k - 1 : k + 1;
  }
#pragma unroll
  for (int m = 0; m < 8; ++m) {
    int64_t c[3];
    uint32_t loc[3];
    bool inside = true;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      c[a] = cand[a][(m >> a) & 1];
      const int64_t l = c[a] - ((int64_t)G[a] << 7);
      inside &= l >= 0 && l <= 127;
      loc[a] = (uint32_t)l;
    }
    if (!inside) continue;
    uint64_t d2 = 0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const int64_t d = (int64_t)pos2[a] - ((2 * c[a] + 1) << (cs - 1));
      d2 += (uint64_t)(d * d);
    }
    const uint64_t r = isqrt_u64(d2 << (2 * L + 2));  // floor(65536 * distance)
    if (r >= kWeightOne) continue;
    f(morton7(loc[0], loc[1], loc[2]), kWeightOne - r);
  }
}

}  // namespace lod
