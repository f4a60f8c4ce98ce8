// k_weighted.hip -- neighbourhood-weighted average (Sec. 4.2.4).
//
// Every sample of an inner node A (a point of a leaf child, or a voxel of an
// inner child) adds w * RGB and w to the 2x2x2 cells of A's 128^3 grid whose
// centres surround it, w = 1 - distance to the cell centre in cells, clamped
// at 0; only the cell containing a sample is occupied, and an occupied cell's
// colour is floor(sum(w * c) / sum(w)), A = 255.  Cells outside A receive
// nothing (samples of other nodes are not considered).
//
// Exact reading (shared with the oracle by definition, not by code):
//   * positions on the half-cell lattice of the 2^21 quantization grid, in
//     units of half a finest cell: a point at 2q + 1 (the centre of its
//     quantization cell), a child voxel at the centre of its cell (level
//     L + 8 for a node at level L);
//   * w = 65536 - floor(65536 * d), d from an exact integer square root;
//   * integer sums, truncating division.
// Sums are order-free, so global 64-bit atomics give the same result in any
// order.
//
// The occupied cells, their order and their positions in the voxel lists are
// those of the cell average (the same occupancy rule), so this pass runs after
// the average build and rewrites the colours, level by level from the deepest
// inner level up: a node's samples include its inner children's weighted
// voxels.  Before a level is sampled, each of its inner nodes gets an
// occupancy bitmap of its 2^21 cells in Morton order plus, per 64-bit word,
// the list index of the word's first voxel: the position of an occupied cell
// is that index plus the set bits below it (the lists are sorted by cell).
//
// A child's samples are taken per aligned 16^3 or 32^3 block of the parent's
// grid (a contiguous range of the child's points or sorted voxels): a
// workgroup sums the block's splats per target cell in LDS, by the cell's rank
// among the block's occupied cells (a small hash takes the cells around the
// block).
// Cells one cell or more inside the block get all their samples from it and
// take their colour there; the other cells add their sums to global 64-bit
// sums, and a last pass gives them their colour.
#include "common.h"
#include "launch.h"
#include "scan.h"
#include "weighted.h"

namespace lod {

constexpr int kWSplit = 16;  // workgroups per node in the bitmap and colour passes
constexpr uint32_t kWWords = 1u << 15;  // 64-bit words of a node's 2^21-cell bitmap

// The kernels of one level run over that level's nodes only: `ln` lists the
// nodes of the level (of all trees of the call).  Its inner nodes get the
// bitmap slots 0, 1, ... (in any order): a tree has at most n / (T + 1)
// inner nodes on one level, each holding more than T points.
__global__ void __launch_bounds__(256) k_wslots(Nodes nodes, const uint32_t* __restrict__ ln, uint32_t cnt,
                                                uint32_t* wslot, uint32_t* slot_ctr) {
  const uint32_t i = blockIdx.x * 256 + threadIdx.x;
  if (i >= cnt) return;
  const uint32_t n = ln[i];
  if (!nodes.is_leaf[n]) wslot[n] = atomicAdd(slot_ctr, 1u);
}

// The bitmap words of the inner nodes in ln (set = true) or their reset
// (set = false).  A wave takes 64 consecutive voxels of a node's list (sorted
// by cell, so a word's voxels are consecutive): a segmented OR over the lanes
// of each word gives its bits, added with one atomic OR per (wave, word); the
// first voxel of every word writes the word's list index, or, when
// resetting, zeroes the word.  The bitmaps are zero before setting.  When
// setting, the node's list is also cut at its 64 aligned 32^3 blocks of cells
// (contiguous code ranges): bseg[64 n + b] = [first, end) of block b,
// relative to the node's first voxel (zero for empty blocks).
__global__ void __launch_bounds__(256) k_wbits(Nodes nodes, const uint32_t* __restrict__ ln,
                                               const TreeInfo* __restrict__ trees, const uint64_t* __restrict__ vox,
                                               const uint32_t* __restrict__ wslot, unsigned long long* bits,
                                               uint32_t* wpre, uint2* bseg, bool set) {
  const uint32_t n = ln[blockIdx.x];
  if (nodes.is_leaf[n]) return;
  const uint64_t base = trees[nodes.tree[n]].vbase + nodes.offset[n];
  const uint32_t cnt = nodes.count[n];
  const uint64_t sb = (uint64_t)wslot[n] * kWWords;
  const uint32_t lane = threadIdx.x & 63u;
  constexpr uint32_t kNone = 0xffffffffu;  // no voxel (its word and block match no real one)
  // wave-uniform loop: every lane takes part in the shuffles
  for (uint32_t w0 = blockIdx.y * 256 + (threadIdx.x & ~63u); w0 < cnt; w0 += kWSplit * 256) {
    const uint32_t i = w0 + lane;
    const bool valid = i < cnt;
    const uint32_t code = valid ? voxel_code(vox[base + i]) : kNone, word = code >> 6;
    uint32_t prev = __shfl_up(code, 1, 64);
    if (lane == 0) prev = i > 0 ? voxel_code(vox[base + i - 1]) : kNone;
    uint32_t next = __shfl_down(code, 1, 64);
    if (lane == 63) next = i + 1 < cnt ? voxel_code(vox[base + i + 1]) : kNone;
    const bool first = valid && (prev >> 6) != word;
    if (!set) {
      if (first) bits[sb + word] = 0ull;
      continue;
    }
    if (valid) {
      const uint32_t b = code >> 15;
      if ((prev >> 15) != b) bseg[64ull * n + b].x = i;
      if ((next >> 15) != b) bseg[64ull * n + b].y = i + 1;
    }
    if (first) wpre[sb + word] = i;
    // segmented inclusive OR over the lanes of each word
    uint32_t lo = valid && (code & 63u) < 32u ? 1u << (code & 31u) : 0u;
    uint32_t hi = valid && (code & 63u) >= 32u ? 1u << (code & 31u) : 0u;
#pragma unroll
    for (uint32_t d = 1; d < 64; d <<= 1) {
      const uint32_t l2 = __shfl_up(lo, d, 64), h2 = __shfl_up(hi, d, 64), w2 = __shfl_up(word, d, 64);
      if (lane >= d && w2 == word) {
        lo |= l2;
        hi |= h2;
      }
    }
    if (valid && ((next >> 6) != word || lane == 63))
      atomicOr(bits + sb + word, ((unsigned long long)hi << 32) | lo);
  }
}

// Voxel index of cell `code` of the node whose bitmap starts at sb and whose
// list starts at vbase, or ~0 when the cell is not occupied.
__device__ __forceinline__ uint32_t wfind(const unsigned long long* __restrict__ bits, const uint32_t* __restrict__ wpre,
                                          uint64_t sb, uint64_t vbase, uint32_t code) {
  const unsigned long long word = bits[sb + (code >> 6)];
  const uint32_t b = code & 63u;
  if (!((word >> b) & 1ull)) return 0xffffffffu;
  return (uint32_t)(vbase + wpre[sb + (code >> 6)] + (uint32_t)__popcll(word & ((1ull << b) - 1ull)));
}

constexpr int kWProbe = 32;  // LDS hash probes before a splat goes to the global sums

__device__ __forceinline__ void wadd_global(unsigned long long* acc, uint32_t vi, uint64_t w, uint64_t R, uint64_t Gc,
                                            uint64_t B) {
  unsigned long long* a4 = acc + 4ull * vi;
  atomicAdd(a4 + 0, (unsigned long long)(w * R));
  atomicAdd(a4 + 1, (unsigned long long)(w * Gc));
  atomicAdd(a4 + 2, (unsigned long long)(w * B));
  atomicAdd(a4 + 3, (unsigned long long)w);
}

// The samples of the children at level L + 1 (points of leaves, voxels of
// inner nodes) into their parents (level L), one workgroup per child and
// aligned block of the parent's cells inside the child's octant.  Blocks are
// 16^3 cells (LB = 4, 64 per child: a leaf's micro-bucket, its points two
// levels down, or an inner child's 32^3 block of its own cells) or 32^3 cells
// (LB = 5, 8 per child: a leaf's work item, or an octant of an inner child's
// own cells); either is a contiguous range of the child's points or sorted
// voxels.  The deepest levels, with many sparse blocks, take 32^3 blocks (fewer
// border cells, less set-up per sample); the upper levels, with few dense
// blocks, take 16^3.  A block's cells are a contiguous range of 8^LB cell
// codes.  Its bitmap words are read into LDS once: a target cell inside the
// block that is occupied has a rank among the block's occupied cells, and its
// sums are kept in LDS at that rank (cells without samples of their own are
// not voxels and get nothing); the cells around the block are summed in a
// small LDS hash.  A cell at least one cell inside the block gets samples from
// this block only (weights vanish beyond one cell, and the block lies inside
// one child's octant), so its colour is final here and is written directly;
// cells on the block's border and the cells around it take the sums through
// global atomics and get their colour in k_wfinal (as do cells around the
// block that a full hash cannot take).  A block with more occupied cells than
// the LDS holds is summed in windows of ranks, one pass over its samples per
// window (32^3), or sends its own cells' sums to the global atomics (16^3).
constexpr uint32_t kWLThreads = 512;
template <int LB>
struct WBlk;
template <>
struct WBlk<4> {
  static constexpr uint32_t kWords = 64;      // 64-bit occupancy words of a block
  static constexpr uint32_t kPer = 64;        // blocks per child
  static constexpr uint32_t kRankCap = 1536;  // occupied cells of a block summed in LDS (at a time)
  static constexpr uint32_t kOutSlots = 512;  // hash slots of the cells around the block
  static constexpr bool kWindows = false;
};
template <>
struct WBlk<5> {
  static constexpr uint32_t kWords = 512;
  static constexpr uint32_t kPer = 8;
  static constexpr uint32_t kRankCap = 1792;
  static constexpr uint32_t kOutSlots = 256;
  static constexpr bool kWindows = true;
};
template <int LB>
struct WBlockLocal {
  using P = WBlk<LB>;
  unsigned long long sum[4][P::kRankCap];    // w * R, w * G, w * B, w of the block's cells, by rank
  unsigned long long osum[4][P::kOutSlots];  // the same for the cells around the block
  uint32_t okey[P::kOutSlots];               // cell code + 1 (0 = empty)
  unsigned long long bbits[P::kWords];       // the block's occupancy words
  uint16_t brank[P::kWords];                 // rank in the block of each word's first cell
  uint32_t sh[kWLThreads / 64 + 1];
  uint32_t first_word;                       // the block's first occupied word
};
// Samples of a (child, block) pair; cnt = 0 for an empty block.
template <int LB>
__device__ __forceinline__ void wblock_range(const Nodes& nodes, const ItemDesc* __restrict__ desc,
                                             const uint2* __restrict__ bseg, const TreeInfo* __restrict__ trees,
                                             uint32_t n, uint32_t sub, bool leaf, uint64_t& first, uint32_t& cnt) {
  if (leaf) {
    if (LB == 4) {
      // work item sub / 8 of the leaf (a child cell), micro-bucket sub % 8
      const ItemDesc& d = desc[8 * n + (sub >> 3)];
      cnt = d.P ? d.mc[sub & 7u] : 0u;
      uint32_t o = d.I0;
      for (uint32_t k = 0; k < (sub & 7u); ++k) o += d.mc[k];
      first = o;
    } else {
      const ItemDesc& d = desc[8 * n + sub];
      cnt = d.P;
      first = d.I0;
    }
  } else {
    uint32_t lo = 0, hi = 0;
    if (LB == 4) {
      const uint2 sg = bseg[64ull * n + sub];
      lo = sg.x;
      hi = sg.y;
    } else {
      // the octant: its 8 blocks of the child's list, contiguous (the list is sorted)
      lo = 0xffffffffu;
      for (uint32_t q = 0; q < 8; ++q) {
        const uint2 sg = bseg[64ull * n + 8 * sub + q];
        if (sg.y > sg.x) {
          lo = min(lo, sg.x);
          hi = max(hi, sg.y);
        }
      }
      if (hi == 0) lo = 0;
    }
    cnt = hi - lo;
    first = trees[nodes.tree[n]].vbase + nodes.offset[n] + lo;
  }
}

// The non-empty (child, block) pairs of a level: list[0 .. *count) holds
// kPer * (position in ln) + block, in any order.
template <int LB>
__global__ void __launch_bounds__(256) k_wblocks(Nodes nodes, const uint32_t* __restrict__ ln, uint32_t nch,
                                                 const ItemDesc* __restrict__ desc, const uint2* __restrict__ bseg,
                                                 const TreeInfo* __restrict__ trees, uint32_t* list, uint32_t* count) {
  constexpr uint32_t kPer = WBlk<LB>::kPer;
  const uint32_t idx = blockIdx.x * 256 + threadIdx.x;
  if (idx >= kPer * nch) return;
  const uint32_t n = ln[idx / kPer];
  uint64_t first;
  uint32_t cnt;
  wblock_range<LB>(nodes, desc, bseg, trees, n, idx % kPer, nodes.is_leaf[n] != 0, first, cnt);
  if (cnt) list[atomicAdd(count, 1u)] = idx;
}

template <int LB>
__global__ void __launch_bounds__(kWLThreads) k_wsplat_block(Nodes nodes, const uint32_t* __restrict__ ln,
                                                             const uint32_t* __restrict__ blocks,
                                                             const uint32_t* __restrict__ nblocks, uint32_t L,
                                                             const ItemDesc* __restrict__ desc,
                                                             const uint2* __restrict__ bseg,
                                                             const TreeInfo* __restrict__ trees, const Cube* cube,
                                                             const uint4* __restrict__ Y, uint64_t* vox,
                                                             const uint32_t* __restrict__ wslot,
                                                             const unsigned long long* __restrict__ bits,
                                                             const uint32_t* __restrict__ wpre,
                                                             unsigned long long* acc) {
  using P = WBlk<LB>;
  constexpr uint32_t kTpw = kWLThreads / P::kWords;  // threads per word in the flush (8 or 1)
  constexpr uint32_t kBpt = 64 / kTpw;               // cells per thread in the flush
  __shared__ WBlockLocal<LB> lt;
  // the grid covers every (child, block) pair of the level; the list holds
  // the non-empty ones
  if (blockIdx.x >= *nblocks) return;
  const uint32_t idx = blocks[blockIdx.x];
  const uint32_t n = ln[idx / P::kPer], sub = idx % P::kPer, t = threadIdx.x;
  const bool leaf = nodes.is_leaf[n] != 0;
  uint64_t first;
  uint32_t cnt;
  wblock_range<LB>(nodes, desc, bseg, trees, n, sub, leaf, first, cnt);
  if (cnt == 0) return;
  const uint32_t A = nodes.parent[n];
  const uint64_t ka = nodes.key[A], kn = nodes.key[n];
  const uint32_t G[3] = {compact21(ka), compact21(ka >> 1), compact21(ka >> 2)};
  const uint32_t C[3] = {compact21(kn), compact21(kn >> 1), compact21(kn >> 2)};
  const uint64_t sb = (uint64_t)wslot[A] * kWWords, vbase = trees[nodes.tree[A]].vbase + nodes.offset[A];
  const CubeD cd = load_cube(cube + nodes.tree[n]);
  // the block's cells in A's grid: codes blk * 8^LB + [0, 8^LB), blk = the
  // child's octant, then the block's place inside it
  const uint32_t blk = (uint32_t)(kn & 7u) * P::kPer + sub;
  // a sample: a point record, or a voxel word in .x / .y
  auto load = [&](uint32_t i) -> uint4 {
    if (leaf) return Y[first + i];
    const uint64_t v = vox[first + i];
    return make_uint4((uint32_t)v, (uint32_t)(v >> 32), 0u, 0u);
  };
  uint4 nxt = make_uint4(0, 0, 0, 0);
  if (t < cnt) nxt = load(t);
  // the block's bitmap words and the rank of each word's first cell
  const uint64_t wbase = sb + (uint64_t)blk * P::kWords;
  const unsigned long long wd = t < P::kWords ? bits[wbase + t] : 0ull;
  uint32_t nocc;
  const uint32_t ex = block_excl_scan<kWLThreads>((uint32_t)__popcll(wd), lt.sh, &nocc);
  if (t < P::kWords) {
    lt.bbits[t] = wd;
    lt.brank[t] = (uint16_t)ex;
  }
  if (t == 0) lt.first_word = P::kWords;
  for (uint32_t i = t; i < P::kOutSlots; i += kWLThreads) {
    lt.okey[i] = 0;
    lt.osum[0][i] = lt.osum[1][i] = lt.osum[2][i] = lt.osum[3][i] = 0;
  }
  __syncthreads();
  if (wd) atomicMin(&lt.first_word, t);
  __syncthreads();
  // list index (from A's first voxel) of the block's first cell
  const uint32_t lbase = nocc ? wpre[wbase + lt.first_word] : 0u;
  // the block's own cells are summed in LDS (in windows of ranks), or, for a
  // 16^3 block with more occupied cells than the LDS holds, globally
  const bool local = P::kWindows || nocc <= P::kRankCap;
  const uint32_t wend = local ? nocc : 1u;
  for (uint32_t w0 = 0; w0 < wend; w0 += P::kRankCap) {  // uniform
    const uint32_t wn = local ? min(P::kRankCap, nocc - w0) : 0u;
    for (uint32_t i = t; i < wn; i += kWLThreads) lt.sum[0][i] = lt.sum[1][i] = lt.sum[2][i] = lt.sum[3][i] = 0;
    __syncthreads();
    const bool around = w0 == 0;  // the cells around the block are summed in the first pass
    for (uint32_t i = t; i < cnt; i += kWLThreads) {
      uint4 v;
      if (around) {  // the next sample is loaded while this one is splat
        v = nxt;
        if (i + kWLThreads < cnt) nxt = load(i + kWLThreads);
      } else {
        v = load(i);
      }
      uint32_t pos2[3];
      uint32_t rgba;
      if (leaf) {
        // a point at the centre of its 2^21-grid cell
        pos2[0] = 2u * quantize(__uint_as_float(v.x), cd.lo[0], cd.scale) + 1u;
        pos2[1] = 2u * quantize(__uint_as_float(v.y), cd.lo[1], cd.scale) + 1u;
        pos2[2] = 2u * quantize(__uint_as_float(v.z), cd.lo[2], cd.scale) + 1u;
        rgba = v.w;
      } else {
        // a child voxel at the centre of its cell (level L + 8)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          const uint32_t j = (C[a] << 7) + ((v.x >> (8 * a)) & 0xffu);
          pos2[a] = (2u * j + 1u) << (13 - L);
        }
        rgba = v.y;
      }
      const uint32_t R = rgba & 0xffu, Gc = (rgba >> 8) & 0xffu, B = (rgba >> 16) & 0xffu;
      wtargets32(L, G, pos2, [&](uint32_t code, uint32_t w) {
        if ((code >> (3 * LB)) == blk) {
          // a cell of the block without samples of its own is not a voxel
          const uint32_t wi = (code >> 6) & (P::kWords - 1u), b = code & 63u;
          const unsigned long long cw = lt.bbits[wi];
          if (!((cw >> b) & 1ull)) return;
          const uint32_t rank = lt.brank[wi] + (uint32_t)__popcll(cw & ((1ull << b) - 1ull));
          if (!local) {
            wadd_global(acc, (uint32_t)(vbase + lbase + rank), w, R, Gc, B);
            return;
          }
          const uint32_t r = rank - w0;
          if (r >= wn) return;  // another window's cell
          atomicAdd(&lt.sum[0][r], (unsigned long long)(w * R));
          atomicAdd(&lt.sum[1][r], (unsigned long long)(w * Gc));
          atomicAdd(&lt.sum[2][r], (unsigned long long)(w * B));
          atomicAdd(&lt.sum[3][r], (unsigned long long)w);
          return;
        }
        if (!around) return;
        uint32_t slot = (code * 0x9E3779B1u) % P::kOutSlots;
#pragma unroll 1
        for (int probe = 0; probe < kWProbe; ++probe) {
          const uint32_t prev = atomicCAS(&lt.okey[slot], 0u, code + 1);
          if (prev == 0u || prev == code + 1) {
            atomicAdd(&lt.osum[0][slot], (unsigned long long)(w * R));
            atomicAdd(&lt.osum[1][slot], (unsigned long long)(w * Gc));
            atomicAdd(&lt.osum[2][slot], (unsigned long long)(w * B));
            atomicAdd(&lt.osum[3][slot], (unsigned long long)w);
            return;
          }
          slot = (slot + 1) % P::kOutSlots;
        }
        // table full around this code: straight to the global sums
        const uint32_t vi = wfind(bits, wpre, sb, vbase, code);
        if (vi != 0xffffffffu) wadd_global(acc, vi, w, R, Gc, B);
      });
    }
    __syncthreads();
    // the window's cells of the block: kTpw threads per word, kBpt cells each
    if (local) {
      const uint32_t wi = t / kTpw, sh = kBpt * (t % kTpw);
      const unsigned long long cw = lt.bbits[wi];
      const unsigned long long mask = kBpt == 64 ? ~0ull : ((1ull << kBpt) - 1ull);
      const uint32_t r0 = lt.brank[wi] + (uint32_t)__popcll(cw & ((1ull << sh) - 1ull));
      uint32_t k = 0;
      for (unsigned long long m = (cw >> sh) & mask; m; m &= m - 1, ++k) {
        const uint32_t r = r0 + k - w0;
        if (r >= wn) continue;
        const uint32_t b = sh + (uint32_t)(__ffsll(m) - 1);
        const uint32_t cl = (wi << 6) | b;  // the cell's Morton index in the block
        // inside by one cell on every axis: the axis's LB bits of the index
        // are neither all zero nor all one
        constexpr uint32_t mx = LB == 4 ? 0x249u : 0x1249u;
        const uint32_t ix = cl & mx, iy = cl & (mx << 1), iz = cl & (mx << 2);
        const bool interior = ix != 0u && ix != mx && iy != 0u && iy != (mx << 1) && iz != 0u && iz != (mx << 2);
        const unsigned long long s0 = lt.sum[0][r], s1 = lt.sum[1][r], s2 = lt.sum[2][r], ws = lt.sum[3][r];
        const uint32_t vi = (uint32_t)(vbase + lbase) + r0 + k;
        if (interior) {
          // every occupied cell holds a sample of its own: ws > 0
          const uint32_t rgba = wdiv(s0, ws) | (wdiv(s1, ws) << 8) | (wdiv(s2, ws) << 16) | (255u << 24);
          vox[vi] = make_voxel32((blk << (3 * LB)) | cl, rgba);
        } else {
          unsigned long long* a4 = acc + 4ull * vi;
          atomicAdd(a4 + 0, s0);
          atomicAdd(a4 + 1, s1);
          atomicAdd(a4 + 2, s2);
          atomicAdd(a4 + 3, ws);
        }
      }
    }
    // the cells around the block: their voxel index from the node's bitmap
    if (around)
      for (uint32_t k = t; k < P::kOutSlots; k += kWLThreads) {
        const uint32_t key = lt.okey[k];
        if (key == 0u) continue;
        const uint32_t vi = wfind(bits, wpre, sb, vbase, key - 1u);
        if (vi == 0xffffffffu) continue;  // not an occupied cell
        unsigned long long* a4 = acc + 4ull * vi;
        atomicAdd(a4 + 0, lt.osum[0][k]);
        atomicAdd(a4 + 1, lt.osum[1][k]);
        atomicAdd(a4 + 2, lt.osum[2][k]);
        atomicAdd(a4 + 3, lt.osum[3][k]);
      }
    __syncthreads();  // before the next window clears the sums
  }
}

// Colours of the voxels of the inner nodes in ln from their sums (kWSplit
// workgroups per node); cells without sums were written by k_wsplat_leaf.
__global__ void __launch_bounds__(256) k_wfinal(Nodes nodes, const uint32_t* __restrict__ ln,
                                                const TreeInfo* __restrict__ trees, uint64_t* vox,
                                                const unsigned long long* __restrict__ acc) {
  const uint32_t n = ln[blockIdx.x];
  if (nodes.is_leaf[n]) return;
  const uint64_t base = trees[nodes.tree[n]].vbase + nodes.offset[n];
  const uint32_t cnt = nodes.count[n];
  for (uint32_t i = blockIdx.y * 256 + threadIdx.x; i < cnt; i += kWSplit * 256) {
    const unsigned long long* a4 = acc + 4ull * (base + i);
    const uint64_t ws = a4[3];
    if (ws == 0) continue;  // colour already final
    const uint32_t rgba = wdiv(a4[0], ws) | (wdiv(a4[1], ws) << 8) | (wdiv(a4[2], ws) << 16) | (255u << 24);
    vox[base + i] = (vox[base + i] & 0xffffffffull) | ((uint64_t)rgba << 32);
  }
}

hipError_t launch_weighted(const Nodes& nodes, const uint32_t* lnodes, const uint64_t* loff, uint32_t deepest,
                           const TreeInfo* trees, const Cube* cube, const void* desc, const void* Y, uint64_t* vox,
                           uint32_t* wslot, unsigned long long* bits, uint32_t* wpre, uint2* bseg,
                           unsigned long long* acc, uint32_t* blocks, uint32_t* nblocks, uint32_t* slot_ctr,
                           hipStream_t s) {
  for (int L = (int)deepest - 1; L >= 0; --L) {
    const uint32_t l = (uint32_t)L;
    const uint32_t* pa = lnodes + loff[l];       // the parents' level
    const uint32_t* ch = lnodes + loff[l + 1];   // the children's level
    const uint32_t na = (uint32_t)(loff[l + 1] - loff[l]), nch = (uint32_t)(loff[l + 2] - loff[l + 1]);
    if (!na || !nch) continue;
    hipError_t e = hipMemsetAsync(slot_ctr, 0, sizeof(uint32_t), s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_wslots, dim3((na + 255) / 256), dim3(256), 0, s, nodes, pa, na, wslot, slot_ctr);
    hipLaunchKernelGGL(k_wbits, dim3(na, kWSplit), dim3(256), 0, s, nodes, pa, trees, (const uint64_t*)vox,
                       (const uint32_t*)wslot, bits, wpre, bseg, true);
    // the non-empty blocks only (most micro-buckets of a surface are empty);
    // 32^3 blocks for the two deepest parent levels, 16^3 above them
    const bool big = l + 2 >= deepest;
    if ((e = hipMemsetAsync(nblocks, 0, sizeof(uint32_t), s)) != hipSuccess) return e;
    const uint32_t per = big ? WBlk<5>::kPer : WBlk<4>::kPer;
    if (big)
      hipLaunchKernelGGL(k_wblocks<5>, dim3((per * nch + 255) / 256), dim3(256), 0, s, nodes, ch, nch,
                         (const ItemDesc*)desc, (const uint2*)bseg, trees, blocks, nblocks);
    else
      hipLaunchKernelGGL(k_wblocks<4>, dim3((per * nch + 255) / 256), dim3(256), 0, s, nodes, ch, nch,
                         (const ItemDesc*)desc, (const uint2*)bseg, trees, blocks, nblocks);
    // one workgroup per possible block (those beyond the count end at once):
    // the count stays on the device and the levels run without a host wait
    if (big)
      hipLaunchKernelGGL(k_wsplat_block<5>, dim3(per * nch), dim3(kWLThreads), 0, s, nodes, ch,
                         (const uint32_t*)blocks, (const uint32_t*)nblocks, l, (const ItemDesc*)desc,
                         (const uint2*)bseg, trees, cube, (const uint4*)Y, vox, (const uint32_t*)wslot,
                         (const unsigned long long*)bits, (const uint32_t*)wpre, acc);
    else
      hipLaunchKernelGGL(k_wsplat_block<4>, dim3(per * nch), dim3(kWLThreads), 0, s, nodes, ch,
                         (const uint32_t*)blocks, (const uint32_t*)nblocks, l, (const ItemDesc*)desc,
                         (const uint2*)bseg, trees, cube, (const uint4*)Y, vox, (const uint32_t*)wslot,
                         (const unsigned long long*)bits, (const uint32_t*)wpre, acc);
    hipLaunchKernelGGL(k_wfinal, dim3(na, kWSplit), dim3(256), 0, s, nodes, pa, trees, vox,
                       (const unsigned long long*)acc);
    // the bitmaps are cleared word by word (from the unchanged cell lists) for
    // the next level's nodes
    hipLaunchKernelGGL(k_wbits, dim3(na, kWSplit), dim3(256), 0, s, nodes, pa, trees, (const uint64_t*)vox,
                       (const uint32_t*)wslot, bits, wpre, bseg, false);
  }
  return hipGetLastError();
}

uint64_t weighted_bitmap_words() { return kWWords; }

}  // namespace lod
