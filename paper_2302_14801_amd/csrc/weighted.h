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

// wtargets() in 32-bit arithmetic (the same cells and weights).  pos2 < 2^22.
// Per axis, the sample's own cell has offset d0 from its centre (|d0| <= half
// a cell) and the neighbour on the side of the offset lies one cell minus
// |d0| away; a candidate is kept when its squared distance is below one
// squared cell, 2^(2 cs) <= 2^30, so each axis term fits in 30 bits, the sum in
// 32, and 65536^2 * distance^2 = d2 * 4^(L+1) < 2^32.  The square root of that
// is taken in single precision (within 2^-7 of the exact root, which is below
// 65536) and corrected to the integer floor.
template <class F>
__device__ __forceinline__ void wtargets32(uint32_t L, const uint32_t G[3], const uint32_t pos2[3], F&& f) {
  const uint32_t cs = 15 - L;  // log2 of A's cell size in pos2 units
  const uint32_t one = 1u << cs, half = one >> 1;
  const uint32_t lim = 1u << (2 * cs);
  int32_t loc0[3], loc1[3];
  uint32_t dd0[3], dd1[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const uint32_t k = pos2[a] >> cs, fo = pos2[a] & (one - 1u);
    const int32_t d0 = (int32_t)fo - (int32_t)half;
    const uint32_t e = one - (uint32_t)(d0 < 0 ? -d0 : d0);
    const int32_t base = (int32_t)(G[a] << 7);
    loc0[a] = (int32_t)k - base;
    loc1[a] = (int32_t)k + (fo < half ? -1 : 1) - base;
    dd0[a] = (uint32_t)(d0 * d0);
    dd1[a] = e * e;
  }
  // one copy of the loop body (f is inlined once): each axis picks its term
#pragma unroll 1
  for (uint32_t m = 0; m < 8; ++m) {
    const bool b0 = m & 1u, b1 = m & 2u, b2 = m & 4u;
    const uint32_t d2 = (b0 ? dd1[0] : dd0[0]) + (b1 ? dd1[1] : dd0[1]) + (b2 ? dd1[2] : dd0[2]);
    if (d2 >= lim) continue;
    const int32_t lx = b0 ? loc1[0] : loc0[0], ly = b1 ? loc1[1] : loc0[1], lz = b2 ? loc1[2] : loc0[2];
    if ((uint32_t)lx > 127u || (uint32_t)ly > 127u || (uint32_t)lz > 127u) continue;
    const uint32_t x = d2 << (2 * L + 2);
    uint32_t r = (uint32_t)__fsqrt_rn((float)x);
    if ((uint64_t)r * r > x) --r;
    else if ((uint64_t)(r + 1) * (r + 1) <= x) ++r;
    f(morton7((uint32_t)lx, (uint32_t)ly, (uint32_t)lz), kWeightOne - r);
  }
}

// floor(s / ws) for quotients below 256 and s < 2^53 (sums of weighted 8-bit
// colours): the double quotient is within one of it, and one integer check
// settles it.
__device__ __forceinline__ uint32_t wdiv(uint64_t s, uint64_t ws) {
  uint32_t q = (uint32_t)((double)s / (double)ws);
  if ((uint64_t)q * ws > s) --q;
  else if ((uint64_t)(q + 1) * ws <= s) ++q;
  return q;
}

}  // namespace lod
