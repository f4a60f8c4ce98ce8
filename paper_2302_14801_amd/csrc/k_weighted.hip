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
// A child's samples are taken per aligned 16^3 block of the parent's grid
// (a leaf's micro-bucket of points, or a 32^3 block of an inner child's own
// cells, which is a contiguous range of its sorted voxel list): a workgroup
// sums the block's splats per target cell in LDS, by the cell's rank among
// the block's occupied cells (a small hash takes the cells around the block).
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
// aligned 16^3 block of the parent's cells inside the child's octant (64 per
// child): a leaf's micro-bucket (its points two levels down), or an inner
// child's 32^3 block of its own cells (a contiguous range of its voxel list).
// A block's cells are a contiguous range of 4096 cell codes.  The block's 64
// bitmap words are read into LDS once: a target cell inside the block that is
// occupied has a rank among the block's occupied cells, and its sums are kept
// in LDS at that rank (cells without samples of their own are not voxels and
// get nothing); cells around the block are summed in a small LDS hash.  A
// cell at least one cell inside the block gets samples from this block only
// (weights vanish beyond one cell, and the block lies inside one child's
// octant), so its colour is final here and is written directly; cells on the
// block's border and the cells around it take the sums through global
// atomics and get their colour in k_wfinal.  A block with more occupied cells
// than the LDS holds sends its own cells' sums through the atomics as well,
// and so does a full hash for the cells around it.
constexpr uint32_t kWRankCap = 1536;  // occupied cells of a block summed in LDS
constexpr uint32_t kWOutSlots = 512;  // hash slots of the cells around the block
constexpr uint32_t kWLThreads = 512;
struct WBlockLocal {
  unsigned long long sum[4][kWRankCap];    // w * R, w * G, w * B, w of the block's cells, by rank
  unsigned long long osum[4][kWOutSlots];  // the same for the cells around the block
  uint32_t okey[kWOutSlots];               // cell code + 1 (0 = empty)
  unsigned long long bbits[64];            // the block's occupancy words
  uint32_t bpre[64];                       // list index (from the node's first voxel) of each word's first cell
  uint32_t brank[64];                      // rank in the block of each word's first cell
  uint32_t nocc;                           // occupied cells of the block
};
// Samples of a (child, block) pair: the leaf micro-bucket's point range or
// the inner child's voxel range; cnt = 0 for an empty block.
__device__ __forceinline__ void wblock_range(const Nodes& nodes, const ItemDesc* __restrict__ desc,
                                             const uint2* __restrict__ bseg, const TreeInfo* __restrict__ trees,
                                             uint32_t n, uint32_t sub, bool leaf, uint64_t& first, uint32_t& cnt) {
  if (leaf) {
    // work item sub / 8 of the leaf (a child cell), micro-bucket sub % 8
    const ItemDesc& d = desc[8 * n + (sub >> 3)];
    cnt = d.P ? d.mc[sub & 7u] : 0u;
    uint32_t o = d.I0;
    for (uint32_t k = 0; k < (sub & 7u); ++k) o += d.mc[k];
    first = o;
  } else {
    const uint2 sg = bseg[64ull * n + sub];
    cnt = sg.y - sg.x;
    first = trees[nodes.tree[n]].vbase + nodes.offset[n] + sg.x;
  }
}

// The non-empty (child, block) pairs of a level: list[0 .. *count) holds
// 64 * (position in ln) + block, in any order.
__global__ void __launch_bounds__(256) k_wblocks(Nodes nodes, const uint32_t* __restrict__ ln, uint32_t nch,
                                                 const ItemDesc* __restrict__ desc, const uint2* __restrict__ bseg,
                                                 const TreeInfo* __restrict__ trees, uint32_t* list, uint32_t* count) {
  const uint32_t idx = blockIdx.x * 256 + threadIdx.x;
  if (idx >= 64 * nch) return;
  const uint32_t n = ln[idx >> 6];
  uint64_t first;
  uint32_t cnt;
  wblock_range(nodes, desc, bseg, trees, n, idx & 63u, nodes.is_leaf[n] != 0, first, cnt);
  if (cnt) list[atomicAdd(count, 1u)] = idx;
}

__global__ void __launch_bounds__(kWLThreads) k_wsplat_block(Nodes nodes, const uint32_t* __restrict__ ln,
                                                             const uint32_t* __restrict__ blocks, uint32_t L,
                                                             const ItemDesc* __restrict__ desc,
                                                             const uint2* __restrict__ bseg,
                                                             const TreeInfo* __restrict__ trees, const Cube* cube,
                                                             const uint4* __restrict__ Y, uint64_t* vox,
                                                             const uint32_t* __restrict__ wslot,
                                                             const unsigned long long* __restrict__ bits,
                                                             const uint32_t* __restrict__ wpre,
                                                             unsigned long long* acc) {
  __shared__ WBlockLocal lt;
  const uint32_t idx = blocks[blockIdx.x];
  const uint32_t n = ln[idx >> 6], sub = idx & 63u, t = threadIdx.x;
  const bool leaf = nodes.is_leaf[n] != 0;
  uint64_t first;
  uint32_t cnt;
  wblock_range(nodes, desc, bseg, trees, n, sub, leaf, first, cnt);
  if (cnt == 0) return;
  const uint32_t A = nodes.parent[n];
  const uint64_t ka = nodes.key[A], kn = nodes.key[n];
  const uint32_t G[3] = {compact21(ka), compact21(ka >> 1), compact21(ka >> 2)};
  const uint32_t C[3] = {compact21(kn), compact21(kn >> 1), compact21(kn >> 2)};
  const uint64_t sb = (uint64_t)wslot[A] * kWWords, vbase = trees[nodes.tree[A]].vbase + nodes.offset[A];
  const CubeD cd = load_cube(cube + nodes.tree[n]);
  // the block's cells in A's grid: codes blk * 4096 + [0, 4096), blk = the
  // child's octant, then the octants of the two levels below it (for a leaf,
  // the work item's and the micro-bucket's)
  const uint32_t blk = ((uint32_t)(kn & 7u) << 6) | sub;
  // a sample: a point record, or a voxel word in .x / .y
  auto load = [&](uint32_t i) -> uint4 {
    if (leaf) return Y[first + i];
    const uint64_t v = vox[first + i];
    return make_uint4((uint32_t)v, (uint32_t)(v >> 32), 0u, 0u);
  };
  uint4 nxt = make_uint4(0, 0, 0, 0);
  if (t < cnt) nxt = load(t);
  if (t < 64) {
    // the block's bitmap words, the list index of each word's first cell and
    // its rank in the block
    const uint64_t w0 = sb + ((uint64_t)blk << 6);
    const unsigned long long wd = bits[w0 + t];
    const uint32_t pc = (uint32_t)__popcll(wd);
    const uint32_t inc = wave_incl_scan(pc);
    const unsigned long long nz = __ballot(wd != 0ull);
    const uint32_t start = nz ? wpre[w0 + (uint32_t)(__ffsll((unsigned long long)nz) - 1)] : 0u;
    lt.bbits[t] = wd;
    lt.bpre[t] = start + inc - pc;
    lt.brank[t] = inc - pc;
    if (t == 63) lt.nocc = inc;
  }
  for (uint32_t i = t; i < kWOutSlots; i += kWLThreads) {
    lt.okey[i] = 0;
    lt.osum[0][i] = lt.osum[1][i] = lt.osum[2][i] = lt.osum[3][i] = 0;
  }
  __syncthreads();
  const uint32_t nocc = lt.nocc;
  const bool local = nocc <= kWRankCap;  // the block's own cells are summed in LDS
  if (local)
    for (uint32_t i = t; i < nocc; i += kWLThreads) lt.sum[0][i] = lt.sum[1][i] = lt.sum[2][i] = lt.sum[3][i] = 0;
  __syncthreads();
  for (uint32_t i = t; i < cnt; i += kWLThreads) {
    // the next sample is loaded while this one is splat
    const uint4 v = nxt;
    if (i + kWLThreads < cnt) nxt = load(i + kWLThreads);
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
      if ((code >> 12) == blk) {
        // a cell of the block without samples of its own is not a voxel
        const uint32_t wi = (code >> 6) & 63u, b = code & 63u;
        const unsigned long long wd = lt.bbits[wi];
        if (!((wd >> b) & 1ull)) return;
        const uint32_t below = (uint32_t)__popcll(wd & ((1ull << b) - 1ull));
        if (local) {
          const uint32_t r = lt.brank[wi] + below;
          atomicAdd(&lt.sum[0][r], (unsigned long long)(w * R));
          atomicAdd(&lt.sum[1][r], (unsigned long long)(w * Gc));
          atomicAdd(&lt.sum[2][r], (unsigned long long)(w * B));
          atomicAdd(&lt.sum[3][r], (unsigned long long)w);
        } else {
          wadd_global(acc, (uint32_t)(vbase + lt.bpre[wi] + below), w, R, Gc, B);
        }
        return;
      }
      uint32_t slot = (code * 0x9E3779B1u) >> 23;  // 9 bits
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
        slot = (slot + 1) & (kWOutSlots - 1);
      }
      // table full around this code: straight to the global sums
      const uint32_t vi = wfind(bits, wpre, sb, vbase, code);
      if (vi != 0xffffffffu) wadd_global(acc, vi, w, R, Gc, B);
    });
  }
  __syncthreads();
  // the block's own cells: 8 threads per bitmap word, 8 cells each
  if (local) {
    const uint32_t wi = t >> 3, sh = 8 * (t & 7u);
    const unsigned long long wd = lt.bbits[wi];
    uint32_t m = (uint32_t)(wd >> sh) & 0xffu;
    const uint32_t r = lt.brank[wi] + (uint32_t)__popcll(wd & ((1ull << sh) - 1ull));
    const uint32_t vi0 = (uint32_t)(vbase + lt.bpre[wi]) + (r - lt.brank[wi]);
    for (uint32_t k = 0; m; m &= m - 1, ++k) {
      const uint32_t b = sh + (uint32_t)(__ffs(m) - 1);
      const uint32_t c = (blk << 12) | (wi << 6) | b;
      // inside by one cell on every axis: the axis's 4 bits of the block's
      // 12-bit Morton index are neither all zero nor all one
      const uint32_t c12 = c & 4095u, ix = c12 & 0x249u, iy = c12 & 0x492u, iz = c12 & 0x924u;
      const bool interior = ix != 0u && ix != 0x249u && iy != 0u && iy != 0x492u && iz != 0u && iz != 0x924u;
      const unsigned long long s0 = lt.sum[0][r + k], s1 = lt.sum[1][r + k], s2 = lt.sum[2][r + k],
                               ws = lt.sum[3][r + k];
      const uint32_t vi = vi0 + k;
      if (interior) {
        // every occupied cell holds a sample of its own: ws > 0
        const uint32_t rgba = wdiv(s0, ws) | (wdiv(s1, ws) << 8) | (wdiv(s2, ws) << 16) | (255u << 24);
        vox[vi] = make_voxel32(c, rgba);
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
  for (uint32_t k = t; k < kWOutSlots; k += kWLThreads) {
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
                           unsigned long long* acc, uint32_t* blocks, uint32_t* nblocks, uint32_t* h_nblocks,
                           uint32_t* slot_ctr, hipStream_t s) {
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
    // the non-empty blocks only (most micro-buckets of a surface are empty)
    if ((e = hipMemsetAsync(nblocks, 0, sizeof(uint32_t), s)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_wblocks, dim3((64 * nch + 255) / 256), dim3(256), 0, s, nodes, ch, nch, (const ItemDesc*)desc,
                       (const uint2*)bseg, trees, blocks, nblocks);
    if ((e = hipMemcpyAsync(h_nblocks, nblocks, sizeof(uint32_t), hipMemcpyDeviceToHost, s)) != hipSuccess) return e;
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
    const uint32_t nblk = std::min<uint32_t>(*h_nblocks, 64 * nch);
    if (nblk)
      hipLaunchKernelGGL(k_wsplat_block, dim3(nblk), dim3(kWLThreads), 0, s, nodes, ch, (const uint32_t*)blocks,
                         l, (const ItemDesc*)desc, (const uint2*)bseg, trees, cube, (const uint4*)Y, vox,
                         (const uint32_t*)wslot, (const unsigned long long*)bits, (const uint32_t*)wpre, acc);
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
