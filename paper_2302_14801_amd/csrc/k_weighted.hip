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
// voxels.  A hash table over all inner voxels, keyed by (node, cell), finds
// the position of a target cell.
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

__device__ __forceinline__ uint64_t whash_slot(uint64_t key, uint64_t mask) {
  return ((key * 0x9E3779B97F4A7C15ull) >> 24) & mask;
}
__device__ __forceinline__ uint64_t whash_key(uint32_t node, uint32_t code) {
  return (((uint64_t)node << 21) | code) + 1;  // 0 marks an empty slot
}

// floor(sqrt(x)) for x < 2^52: a correctly rounded double square root is
// within one of it; the integer checks settle the last step.
__device__ __forceinline__ uint64_t isqrt_u64(uint64_t x) {
  uint64_t r = (uint64_t)__dsqrt_rn((double)x);
  for (int i = 0; i < 2 && r * r > x; ++i) --r;
  for (int i = 0; i < 2 && (r + 1) * (r + 1) <= x; ++i) ++r;
  return r;
}

// kWSplit workgroups per inner node: insert (node, cell) -> voxel index for
// each of its voxels (linear probing; the table holds at least twice the
// voxels).
__global__ void __launch_bounds__(256) k_whash_insert(Nodes nodes, uint32_t num_nodes, const TreeInfo* __restrict__ trees,
                                                      const uint64_t* __restrict__ vox, unsigned long long* hkeys,
                                                      uint32_t* hvals, uint64_t mask) {
  const uint32_t n = blockIdx.x;
  if (n >= num_nodes || nodes.is_leaf[n]) return;
  const uint64_t base = trees[nodes.tree[n]].vbase + nodes.offset[n];
  const uint32_t cnt = nodes.count[n];
  for (uint32_t i = blockIdx.y * 256 + threadIdx.x; i < cnt; i += kWSplit * 256) {
    const uint64_t v = vox[base + i];
    const uint64_t key = whash_key(n, morton7((uint32_t)v & 0xffu, (uint32_t)(v >> 8) & 0xffu, (uint32_t)(v >> 16) & 0xffu));
    uint64_t s = whash_slot(key, mask);
    for (uint64_t probe = 0; probe <= mask; ++probe) {
      const unsigned long long prev = atomicCAS(&hkeys[s], 0ull, (unsigned long long)key);
      if (prev == 0ull || prev == key) {
        hvals[s] = (uint32_t)(base + i);
        break;
      }
      s = (s + 1) & mask;
    }
  }
}

__device__ __forceinline__ uint32_t whash_find(const unsigned long long* __restrict__ hkeys,
                                               const uint32_t* __restrict__ hvals, uint64_t mask, uint64_t key) {
  uint64_t s = whash_slot(key, mask);
  for (uint64_t probe = 0; probe <= mask; ++probe) {
    const uint64_t k = hkeys[s];
    if (k == key) return hvals[s];
    if (k == 0) break;
    s = (s + 1) & mask;
  }
  return 0xffffffffu;
}

constexpr int kWChunk = 256;       // samples per chunk (one per thread)
constexpr uint32_t kWSlots = 1024;  // LDS hash slots per workgroup
constexpr int kWProbe = 32;         // LDS probes before a splat goes global

struct WLocal {
  uint32_t key[kWSlots];  // cell code + 1 (0 = empty)
  unsigned long long sum[kWSlots][4];
};

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
__device__ __forceinline__ void wsplat(uint32_t A, uint32_t L, const uint32_t G[3], const uint64_t pos2[3], uint32_t rgba,
                                       WLocal& lt, const unsigned long long* __restrict__ hkeys,
                                       const uint32_t* __restrict__ hvals, uint64_t mask, unsigned long long* acc) {
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
        atomicAdd(&lt.sum[slot][0], (unsigned long long)(w * R));
        atomicAdd(&lt.sum[slot][1], (unsigned long long)(w * Gc));
        atomicAdd(&lt.sum[slot][2], (unsigned long long)(w * B));
        atomicAdd(&lt.sum[slot][3], (unsigned long long)w);
        done = true;
        break;
      }
      slot = (slot + 1) & (kWSlots - 1);
    }
    if (!done) {  // the LDS table is full around this code: straight to the global sums
      const uint32_t vi = whash_find(hkeys, hvals, mask, whash_key(A, code));
      if (vi != 0xffffffffu) wadd_global(acc, vi, w, R, Gc, B);
    }
  }
}

// Samples of the nodes at level L + 1 into their parents (level L): the
// workgroups (n, y) of node n take its chunks y, y + kWSplit, ...
__global__ void __launch_bounds__(256) k_wsplat(Nodes nodes, uint32_t num_nodes, uint32_t L,
                                                const TreeInfo* __restrict__ trees, const Cube* cube,
                                                const uint4* __restrict__ Y, const uint64_t* __restrict__ vox,
                                                const unsigned long long* __restrict__ hkeys,
                                                const uint32_t* __restrict__ hvals, uint64_t mask,
                                                unsigned long long* acc) {
  __shared__ WLocal lt;
  const uint32_t n = blockIdx.x, t = threadIdx.x;
  if (n >= num_nodes || nodes.level[n] != L + 1) return;
  const uint32_t cnt = nodes.count[n];
  if (blockIdx.y * kWChunk >= cnt) return;
  const uint32_t A = nodes.parent[n];
  const uint64_t ka = nodes.key[A];
  const uint32_t G[3] = {compact21(ka), compact21(ka >> 1), compact21(ka >> 2)};
  const bool leaf = nodes.is_leaf[n] != 0;
  const CubeD cd = load_cube(cube + nodes.tree[n]);
  const uint64_t kn = nodes.key[n];
  const uint32_t C[3] = {compact21(kn), compact21(kn >> 1), compact21(kn >> 2)};
  const uint64_t first = leaf ? nodes.offset[n] : trees[nodes.tree[n]].vbase + nodes.offset[n];
  for (uint32_t i = t; i < kWSlots; i += 256) {
    lt.key[i] = 0;
    lt.sum[i][0] = lt.sum[i][1] = lt.sum[i][2] = lt.sum[i][3] = 0;
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
      wsplat(A, L, G, pos2, rgba, lt, hkeys, hvals, mask, acc);
    }
    __syncthreads();
    // each touched cell once to the global sums (if it is occupied), then
    // the slot is cleared for the next chunk
    for (uint32_t k = t; k < kWSlots; k += 256) {
      const uint32_t key = lt.key[k];
      if (key == 0u) continue;
      const uint32_t vi = whash_find(hkeys, hvals, mask, whash_key(A, key - 1));
      if (vi != 0xffffffffu) {
        unsigned long long* a4 = acc + 4ull * vi;
        atomicAdd(a4 + 0, lt.sum[k][0]);
        atomicAdd(a4 + 1, lt.sum[k][1]);
        atomicAdd(a4 + 2, lt.sum[k][2]);
        atomicAdd(a4 + 3, lt.sum[k][3]);
      }
      lt.key[k] = 0;
      lt.sum[k][0] = lt.sum[k][1] = lt.sum[k][2] = lt.sum[k][3] = 0;
    }
    __syncthreads();
  }
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
                     const void* Y, uint64_t* vox, unsigned long long* hkeys, uint32_t* hvals, uint64_t hmask,
                     unsigned long long* acc, hipStream_t s) {
  if (!num_nodes || deepest == 0) return;
  hipLaunchKernelGGL(k_whash_insert, dim3(num_nodes, kWSplit), dim3(256), 0, s, nodes, num_nodes, trees, (const uint64_t*)vox,
                     hkeys, hvals, hmask);
  for (int L = (int)deepest - 1; L >= 0; --L) {
    hipLaunchKernelGGL(k_wsplat, dim3(num_nodes, kWSplit), dim3(256), 0, s, nodes, num_nodes, (uint32_t)L, trees, cube,
                       (const uint4*)Y, (const uint64_t*)vox, (const unsigned long long*)hkeys, (const uint32_t*)hvals,
                       hmask, acc);
    hipLaunchKernelGGL(k_wfinal, dim3(num_nodes, kWSplit), dim3(256), 0, s, nodes, num_nodes, (uint32_t)L, trees, vox,
                       (const unsigned long long*)acc);
  }
}

}  // namespace lod
