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
// A child's samples (its points in leaf order, or its voxels in Morton order)
// are taken in chunks of consecutive samples, which cover a compact region of
// the parent's grid: a workgroup first sums a chunk's splats per target cell
// in an LDS hash table, then adds each cell's sums to the global ones, so the
// global table and the global atomics see one update per (chunk, cell) instead
// of one per (sample, cell).  A splat that finds the LDS table full goes to the
// global sums directly (the sums are the same either way).
#include "common.h"
#include "launch.h"
#include "scan.h"

namespace lod {

constexpr int kWSplit = 16;  // workgroups per child node in the splat
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

constexpr uint32_t kWWords = 1u << 15;  // 64-bit words of a node's 2^21-cell bitmap

// A slot (bitmap) for every inner node at level L.
__global__ void __launch_bounds__(256) k_wslots(Nodes nodes, uint32_t num_nodes, uint32_t L, uint32_t* wslot,
                                                uint32_t* slot_ctr) {
  const uint32_t n = blockIdx.x * 256 + threadIdx.x;
  if (n >= num_nodes || nodes.is_leaf[n] || nodes.level[n] != L) return;
  wslot[n] = atomicAdd(slot_ctr + L, 1u);
}

// The bitmap words of the inner nodes at level L (set = true) or their reset
// (set = false): the first voxel of every 64-cell word writes the whole word
// (the word's voxels follow it in the list) and, when setting, its own index.
__global__ void __launch_bounds__(256) k_wbits(Nodes nodes, uint32_t num_nodes, uint32_t L,
                                               const TreeInfo* __restrict__ trees, const uint64_t* __restrict__ vox,
                                               const uint32_t* __restrict__ wslot, unsigned long long* bits,
                                               uint32_t* wpre, bool set) {
  const uint32_t n = blockIdx.x;
  if (n >= num_nodes || nodes.is_leaf[n] || nodes.level[n] != L) return;
  const uint64_t base = trees[nodes.tree[n]].vbase + nodes.offset[n];
  const uint32_t cnt = nodes.count[n];
  const uint64_t sb = (uint64_t)wslot[n] * kWWords;
  for (uint32_t i = blockIdx.y * 256 + threadIdx.x; i < cnt; i += kWSplit * 256) {
    const uint32_t word = voxel_code(vox[base + i]) >> 6;
    if (i > 0 && (voxel_code(vox[base + i - 1]) >> 6) == word) continue;
    if (!set) {
      bits[sb + word] = 0ull;
      continue;
    }
    unsigned long long b = 0;
    for (uint32_t j = i; j < cnt && j < i + 64; ++j) {
      const uint32_t c = voxel_code(vox[base + j]);
      if ((c >> 6) != word) break;
      b |= 1ull << (c & 63u);
    }
    bits[sb + word] = b;
    wpre[sb + word] = i;
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

constexpr int kWChunk = 256;       // samples per chunk (one per thread)
constexpr uint32_t kWSlots = 1024;  // LDS hash slots per workgroup
constexpr int kWProbe = 32;         // LDS probes before a splat goes global

// A chunk puts at most one splat of each sample on a cell, so a cell's chunk
// sums stay below 256 * 65536 * 255 < 2^32 (colour) and 2^24 (weight): two
// 32-bit sums share each 64-bit LDS word.
struct WLocal {
  uint32_t key[kWSlots];  // cell code + 1 (0 = empty)
  unsigned long long rg[kWSlots], bw[kWSlots];  // R | G << 32, B | w << 32
};
static_assert(kWChunk <= 256, "packed chunk sums need at most 256 samples per chunk");

__device__ __forceinline__ void wadd_global(unsigned long long* acc, uint32_t vi, uint64_t w, uint64_t R, uint64_t Gc,
                                            uint64_t B) {
  unsigned long long* a4 = acc + 4ull * vi;
  atomicAdd(a4 + 0, (unsigned long long)(w * R));
  atomicAdd(a4 + 1, (unsigned long long)(w * Gc));
  atomicAdd(a4 + 2, (unsigned long long)(w * B));
  atomicAdd(a4 + 3, (unsigned long long)w);
}

// Splat one sample of node A (level L, grid origin G = A's coordinates * 128,
// per axis) at pos2 with colour rgba into the workgroup's LDS table.
__device__ __forceinline__ void wsplat(uint32_t L, const uint32_t G[3], const uint64_t pos2[3], uint32_t rgba, WLocal& lt,
                                       const unsigned long long* __restrict__ bits, const uint32_t* __restrict__ wpre,
                                       uint64_t sb, uint64_t vbase, unsigned long long* acc) {
  const uint32_t cs = 15 - L;  // log2 of A's cell size in pos2 units
  int64_t cand[3][2];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const int64_t k = (int64_t)(pos2[a] >> cs);
    const int64_t f = (int64_t)pos2[a] - (k << cs);
    cand[a][0] = k;
    cand[a][1] = f < ((int64_t)1 << (cs - 1)) ? k - 1 : k + 1;
  }
  const uint64_t R = rgba & 0xffu, Gc = (rgba >> 8) & 0xffu, B = (rgba >> 16) & 0xffu;
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
    const uint64_t w = kWeightOne - r;
    const uint32_t code = morton7(loc[0], loc[1], loc[2]);
    uint32_t slot = (code * 0x9E3779B1u) >> 22;  // 10 bits
    bool done = false;
    for (int probe = 0; probe < kWProbe; ++probe) {
      const uint32_t prev = atomicCAS(&lt.key[slot], 0u, code + 1);
      if (prev == 0u || prev == code + 1) {
        atomicAdd(&lt.rg[slot], (unsigned long long)((w * R) | ((w * Gc) << 32)));
        atomicAdd(&lt.bw[slot], (unsigned long long)((w * B) | (w << 32)));
        done = true;
        break;
      }
      slot = (slot + 1) & (kWSlots - 1);
    }
    if (!done) {  // the LDS table is full around this code: straight to the global sums
      const uint32_t vi = wfind(bits, wpre, sb, vbase, code);
      if (vi != 0xffffffffu) wadd_global(acc, vi, w, R, Gc, B);
    }
  }
}

// Samples of the nodes at level L + 1 into their parents (level L): the
// workgroups (n, y) of node n take its chunks y, y + kWSplit, ...
__global__ void __launch_bounds__(256) k_wsplat(Nodes nodes, uint32_t num_nodes, uint32_t L,
                                                const TreeInfo* __restrict__ trees, const Cube* cube,
                                                const uint4* __restrict__ Y, const uint64_t* __restrict__ vox,
                                                const uint32_t* __restrict__ wslot,
                                                const unsigned long long* __restrict__ bits,
                                                const uint32_t* __restrict__ wpre, unsigned long long* acc) {
  __shared__ WLocal lt;
  const uint32_t n = blockIdx.x, t = threadIdx.x;
  if (n >= num_nodes || nodes.level[n] != L + 1) return;
  const uint32_t cnt = nodes.count[n];
  if (blockIdx.y * kWChunk >= cnt) return;
  const uint32_t A = nodes.parent[n];
  const uint64_t ka = nodes.key[A];
  const uint32_t G[3] = {compact21(ka), compact21(ka >> 1), compact21(ka >> 2)};
  const uint64_t sb = (uint64_t)wslot[A] * kWWords, vbase = trees[nodes.tree[A]].vbase + nodes.offset[A];
  const bool leaf = nodes.is_leaf[n] != 0;
  const CubeD cd = load_cube(cube + nodes.tree[n]);
  const uint64_t kn = nodes.key[n];
  const uint32_t C[3] = {compact21(kn), compact21(kn >> 1), compact21(kn >> 2)};
  const uint64_t first = leaf ? nodes.offset[n] : trees[nodes.tree[n]].vbase + nodes.offset[n];
  for (uint32_t i = t; i < kWSlots; i += 256) {
    lt.key[i] = 0;
    lt.rg[i] = lt.bw[i] = 0;
  }
  __syncthreads();
  for (uint32_t c0 = blockIdx.y * kWChunk; c0 < cnt; c0 += kWSplit * kWChunk) {
    const uint32_t i = c0 + t;
    if (i < cnt) {
      uint64_t pos2[3];
      uint32_t rgba;
      if (leaf) {
        // a point at the centre of its 2^21-grid cell
        const uint4 v = Y[first + i];
        pos2[0] = 2ull * quantize(__uint_as_float(v.x), cd.lo[0], cd.scale) + 1;
        pos2[1] = 2ull * quantize(__uint_as_float(v.y), cd.lo[1], cd.scale) + 1;
        pos2[2] = 2ull * quantize(__uint_as_float(v.z), cd.lo[2], cd.scale) + 1;
        rgba = v.w;
      } else {
        // a child voxel at the centre of its cell (level L + 8)
        const uint64_t v = vox[first + i];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          const uint64_t j = ((uint64_t)C[a] << 7) + ((v >> (8 * a)) & 0xffu);
          pos2[a] = (2 * j + 1) << (13 - L);
        }
        rgba = (uint32_t)(v >> 32);
      }
      wsplat(L, G, pos2, rgba, lt, bits, wpre, sb, vbase, acc);
    }
    __syncthreads();
    // each touched cell once to the global sums (if it is occupied), then
    // the slot is cleared for the next chunk
    for (uint32_t k = t; k < kWSlots; k += 256) {
      const uint32_t key = lt.key[k];
      if (key == 0u) continue;
      const uint32_t vi = wfind(bits, wpre, sb, vbase, key - 1);
      if (vi != 0xffffffffu) {
        unsigned long long* a4 = acc + 4ull * vi;
        const unsigned long long rg = lt.rg[k], bw = lt.bw[k];
        atomicAdd(a4 + 0, rg & 0xffffffffull);
        atomicAdd(a4 + 1, rg >> 32);
        atomicAdd(a4 + 2, bw & 0xffffffffull);
        atomicAdd(a4 + 3, bw >> 32);
      }
      lt.key[k] = 0;
      lt.rg[k] = lt.bw[k] = 0;
    }
    __syncthreads();
  }
}

// Leaf points sorted by their depth-1 cell (the parent's grid) inside each
// micro-bucket, so that a chunk of consecutive points covers few cells.  The
// order of points inside a leaf is free; the voxel lists are already built.
// One workgroup per work item; micro-buckets of more than kWSortMax points
// keep their order (the sums do not depend on it).
constexpr uint32_t kWSortMax = 2048;
__global__ void __launch_bounds__(256) k_wsort(const ItemDesc* __restrict__ desc, const Cube* cube, uint4* Y,
                                               uint32_t* Yid) {
  __shared__ uint4 sp[kWSortMax];
  __shared__ uint32_t sid[kWSortMax];
  __shared__ uint16_t scell[kWSortMax];
  __shared__ uint32_t hist[4096];
  __shared__ uint32_t sh[256 / 64 + 1];
  const ItemDesc& d = desc[blockIdx.x];
  const uint32_t P = d.P, t = threadIdx.x;
  if (P == 0) return;
  const CubeD cd = load_cube(cube + d.tree);
  const uint32_t sub_bit = 15u - d.lvl;  // bit level of the depth-1 cells (level lvl + 6)
  uint32_t off = d.I0;
  for (uint32_t jm = 0; jm < 8; ++jm) {
    const uint32_t cnt = d.mc[jm];
    const uint32_t o = off;
    off += cnt;
    if (cnt < 2 || cnt > kWSortMax) continue;  // uniform
    for (uint32_t i = t; i < 4096; i += 256) hist[i] = 0;
    __syncthreads();
    for (uint32_t i = t; i < cnt; i += 256) {
      const uint4 v = Y[o + i];
      sp[i] = v;
      if (Yid) sid[i] = Yid[o + i];
      const uint32_t c = point_cell(__uint_as_float(v.x), __uint_as_float(v.y), __uint_as_float(v.z), cd, sub_bit, 4);
      scell[i] = (uint16_t)c;
      atomicAdd(&hist[c], 1u);
    }
    __syncthreads();
    // exclusive scan of the 4096 counts (16 per thread)
    uint32_t loc[16], run = 0;
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      loc[k] = hist[16 * t + k];
      run += loc[k];
    }
    uint32_t tot;
    uint32_t ex = block_excl_scan<256>(run, sh, &tot);
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      hist[16 * t + k] = ex;
      ex += loc[k];
    }
    __syncthreads();
    for (uint32_t i = t; i < cnt; i += 256) {
      const uint32_t pos = atomicAdd(&hist[scell[i]], 1u);
      Y[o + pos] = sp[i];
      if (Yid) Yid[o + pos] = sid[i];
    }
    __syncthreads();
  }
}

void launch_weighted_sort(uint32_t num_nodes, const void* desc, const Cube* cube, void* Y, uint32_t* Yid, hipStream_t s) {
  if (!num_nodes) return;
  hipLaunchKernelGGL(k_wsort, dim3(8 * num_nodes), dim3(256), 0, s, (const ItemDesc*)desc, cube, (uint4*)Y, Yid);
}

// Colours of the voxels of the inner nodes at level L from their sums
// (kWSplit workgroups per node).
__global__ void __launch_bounds__(256) k_wfinal(Nodes nodes, uint32_t num_nodes, uint32_t L,
                                                const TreeInfo* __restrict__ trees, uint64_t* vox,
                                                const unsigned long long* __restrict__ acc) {
  const uint32_t n = blockIdx.x;
  if (n >= num_nodes || nodes.is_leaf[n] || nodes.level[n] != L) return;
  const uint64_t base = trees[nodes.tree[n]].vbase + nodes.offset[n];
  const uint32_t cnt = nodes.count[n];
  for (uint32_t i = blockIdx.y * 256 + threadIdx.x; i < cnt; i += kWSplit * 256) {
    const unsigned long long* a4 = acc + 4ull * (base + i);
    const uint64_t ws = a4[3];
    if (ws == 0) continue;  // unreachable: a cell's own sample weighs more than 0.13
    const uint32_t rgba = (uint32_t)(a4[0] / ws) | ((uint32_t)(a4[1] / ws) << 8) | ((uint32_t)(a4[2] / ws) << 16) |
                          (255u << 24);
    vox[base + i] = (vox[base + i] & 0xffffffffull) | ((uint64_t)rgba << 32);
  }
}

void launch_weighted(const Nodes& nodes, uint32_t num_nodes, uint32_t deepest, const TreeInfo* trees, const Cube* cube,
                     const void* Y, uint64_t* vox, uint32_t* wslot, uint32_t* slot_ctr, unsigned long long* bits,
                     uint32_t* wpre, unsigned long long* acc, hipStream_t s) {
  if (!num_nodes || deepest == 0) return;
  for (int L = (int)deepest - 1; L >= 0; --L) {
    const uint32_t l = (uint32_t)L;
    hipLaunchKernelGGL(k_wslots, dim3((num_nodes + 255) / 256), dim3(256), 0, s, nodes, num_nodes, l, wslot, slot_ctr);
    hipLaunchKernelGGL(k_wbits, dim3(num_nodes, kWSplit), dim3(256), 0, s, nodes, num_nodes, l, trees,
                       (const uint64_t*)vox, (const uint32_t*)wslot, bits, wpre, true);
    hipLaunchKernelGGL(k_wsplat, dim3(num_nodes, kWSplit), dim3(256), 0, s, nodes, num_nodes, l, trees, cube,
                       (const uint4*)Y, (const uint64_t*)vox, (const uint32_t*)wslot, (const unsigned long long*)bits,
                       (const uint32_t*)wpre, acc);
    hipLaunchKernelGGL(k_wfinal, dim3(num_nodes, kWSplit), dim3(256), 0, s, nodes, num_nodes, l, trees, vox,
                       (const unsigned long long*)acc);
    // the bitmaps are cleared word by word (from the unchanged cell lists) for
    // the next level's nodes
    hipLaunchKernelGGL(k_wbits, dim3(num_nodes, kWSplit), dim3(256), 0, s, nodes, num_nodes, l, trees,
                       (const uint64_t*)vox, (const uint32_t*)wslot, bits, wpre, false);
  }
}

uint64_t weighted_bitmap_words() { return kWWords; }

}  // namespace lod
