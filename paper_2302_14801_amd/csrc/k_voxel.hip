// k_voxel.hip -- bottom-up voxel sampling of inner nodes (Sec. 4.2).
//
// Every inner node at level L gets the occupied cells of its 128^3 grid (cells
// at level L + 7), and each child fills one 64^3 octant of that grid (Fig. 1
// caption).  A child's samples are its points (leaf child) or its voxels
// (inner child).  Sampling strategies: cell-wise average (Sec. 4.2.3) and the
// two pick strategies (Sec. 4.2.1, 4.2.2) made independent of arrival order.
//
// The gfx950 design differs from the paper's one-workgroup-per-node loop over
// a 128^3 grid in global memory:
//   * leaf children: the leaf's points are sorted by the cell two levels below
//     the leaf ("micro-bucket"), so each micro-bucket maps to at most 4096
//     cells of the parent's grid and is accumulated in a directly indexed LDS
//     array with 64-bit LDS atomics (packed R|G|n sums), then emitted in Morton
//     order from an LDS occupancy bitmask.  All leaves of all levels run in
//     one launch because they only depend on their own points.
//   * inner children: a child's voxel list is in Morton order, so the child
//     voxels that fold into one parent cell (2x2x2 -> 1) are consecutive; the
//     parent voxel is a reduction over a run of at most 8 entries.  This runs
//     level by level, deepest first.
// Voxel lists therefore come out in Morton order of (x, y, z), and the output
// is fully deterministic.
#include "common.h"
#include "launch.h"
#include "scan.h"

namespace lod {

constexpr int kLeafWG = 256;
constexpr uint32_t kSubCells = 4096;  // 2 levels of micro-bucket -> 4 levels of voxel cells = 12 bits
constexpr uint32_t kPackedMax = 65535;  // largest micro-bucket the packed 24/24/16-bit sums can hold

// Parent voxels from the points of every leaf (level >= 1).  One workgroup per
// node; non-leaves exit.  Voxels go to temp[offset .. offset + k) of the leaf
// (k <= points of the leaf), the count to nodes.aux.
template <int MODE>  // 0 average, 1 first, 2 random
__global__ void __launch_bounds__(kLeafWG) k_leaf_voxels(Nodes nodes, uint32_t num_nodes,
                                                         const GridDesc* __restrict__ grids,
                                                         const uint32_t* __restrict__ pool,
                                                         const uint4* __restrict__ pts, const uint32_t* __restrict__ ids,
                                                         const Cube* cube, uint64_t* __restrict__ temp,
                                                         uint32_t* __restrict__ temp_ids, uint32_t seed) {
  __shared__ uint64_t acc[kSubCells];    // average: R | G << 24 | n << 48 ; pick: best order key
  __shared__ uint32_t accb[kSubCells];   // average: sum of B ; pick: winner rgba
  __shared__ uint32_t accid[MODE ? kSubCells : 1];
  __shared__ uint64_t occ[kSubCells / 64];
  __shared__ uint32_t sh[kLeafWG / 64 + 1];
  const uint32_t n = blockIdx.x;
  if (n >= num_nodes || !nodes.is_leaf[n] || nodes.level[n] == 0) return;
  const uint32_t lvl = nodes.level[n];
  const int32_t gi = nodes.grid[n] >= 0 ? nodes.grid[n] : nodes.cover[n];
  const GridDesc G = grids[gi];
  const uint32_t rm = lvl + 2 - G.base_level;  // micro-bucket level relative to the grid
  const uint64_t leaf_rel = nodes.key[n] - (G.base_key << (3 * (lvl - G.base_level)));
  const uint32_t* mcnt = pool + G.pyr + pyr_level_offset(rm);
  const uint32_t* goff = pool + G.off;
  const uint32_t sub_shift = 3u * (15u - lvl);  // key >> sub_shift = voxel cell at level lvl + 6
  const uint32_t top9 = (uint32_t)(nodes.key[n] & 7u) << 18;
  const uint64_t init = MODE == 1 ? ~0ull : 0ull;
  const CubeD cd = load_cube(cube);
  const uint64_t out0 = nodes.offset[n];
  for (uint32_t i = threadIdx.x; i < kSubCells; i += kLeafWG) {
    acc[i] = init;
    accb[i] = 0;
  }
  if (threadIdx.x < kSubCells / 64) occ[threadIdx.x] = 0;
  __syncthreads();
  uint32_t vbase = 0;
  for (uint32_t jm = 0; jm < 64; ++jm) {
    const uint64_t idx = (leaf_rel << 6) | jm;
    const uint32_t cnt = mcnt[idx];
    if (cnt == 0) continue;
    const uint32_t off = goff[idx << (3 * (G.e - rm))];
    const uint32_t code_hi = top9 | (jm << 12);
    if (MODE == 0 && cnt > kPackedMax) {
      // Wide path for very large micro-buckets (only at the depth limit): one
      // window of 512 cells per pass with 64-bit sums in the same LDS.
      uint64_t* wr = acc;            // 512 x R
      uint64_t* wg = acc + 512;      // 512 x G
      uint64_t* wb = acc + 1024;     // 512 x B
      uint64_t* wn = acc + 1536;     // 512 x n
      for (uint32_t w0 = 0; w0 < kSubCells; w0 += 512) {
        for (uint32_t i = threadIdx.x; i < 2048; i += kLeafWG) acc[i] = 0;
        __syncthreads();
        for (uint32_t i = threadIdx.x; i < cnt; i += kLeafWG) {
          const uint4 v = pts[off + i];
          const uint64_t key = point_key(__uint_as_float(v.x), __uint_as_float(v.y), __uint_as_float(v.z), cd);
          const uint32_t sub = (uint32_t)(key >> sub_shift) & (kSubCells - 1);
          if (sub >= w0 && sub < w0 + 512) {
            const uint32_t s = sub - w0;
            atomicAdd((unsigned long long*)&wr[s], (unsigned long long)(v.w & 0xff));
            atomicAdd((unsigned long long*)&wg[s], (unsigned long long)((v.w >> 8) & 0xff));
            atomicAdd((unsigned long long*)&wb[s], (unsigned long long)((v.w >> 16) & 0xff));
            atomicAdd((unsigned long long*)&wn[s], 1ull);
          }
        }
        __syncthreads();
        // emit in cell order
        for (uint32_t s0 = 0; s0 < 512; s0 += kLeafWG) {
          const uint32_t s = s0 + threadIdx.x;
          const uint64_t c = wn[s];
          uint32_t tot;
          const uint32_t pos = block_excl_scan<kLeafWG>(c ? 1u : 0u, sh, &tot);
          if (c) {
            const uint32_t rgba = (uint32_t)(wr[s] / c) | ((uint32_t)(wg[s] / c) << 8) | ((uint32_t)(wb[s] / c) << 16) |
                                  (255u << 24);
            temp[out0 + vbase + pos] = make_voxel(code_hi | (w0 + s), rgba);
          }
          vbase += tot;
        }
        __syncthreads();
      }
      for (uint32_t i = threadIdx.x; i < kSubCells; i += kLeafWG) { acc[i] = init; accb[i] = 0; }
      __syncthreads();
      continue;
    }
    // accumulate
    for (uint32_t i = threadIdx.x; i < cnt; i += kLeafWG) {
      const uint4 v = pts[off + i];
      const uint64_t key = point_key(__uint_as_float(v.x), __uint_as_float(v.y), __uint_as_float(v.z), cd);
      const uint32_t sub = (uint32_t)(key >> sub_shift) & (kSubCells - 1);
      if (MODE == 0) {
        const uint64_t packed = (uint64_t)(v.w & 0xff) | ((uint64_t)((v.w >> 8) & 0xff) << 24) | (1ull << 48);
        atomicAdd((unsigned long long*)&acc[sub], (unsigned long long)packed);
        atomicAdd(&accb[sub], (v.w >> 16) & 0xffu);
      } else {
        const uint64_t k = pick_order(ids[off + i], seed, MODE == 2);
        if (MODE == 1) atomicMin((unsigned long long*)&acc[sub], (unsigned long long)k);
        else atomicMax((unsigned long long*)&acc[sub], (unsigned long long)k);
      }
      atomicOr((unsigned long long*)&occ[sub >> 6], 1ull << (sub & 63));
    }
    __syncthreads();
    if (MODE != 0) {
      // the winner of every cell deposits its colour and id
      for (uint32_t i = threadIdx.x; i < cnt; i += kLeafWG) {
        const uint32_t id = ids[off + i];
        const uint4 v = pts[off + i];
        const uint64_t key = point_key(__uint_as_float(v.x), __uint_as_float(v.y), __uint_as_float(v.z), cd);
        const uint32_t sub = (uint32_t)(key >> sub_shift) & (kSubCells - 1);
        if (acc[sub] == pick_order(id, seed, MODE == 2)) {
          accb[sub] = v.w;
          accid[sub] = id;
        }
      }
      __syncthreads();
    }
    // emit: each thread owns 16 consecutive cells (a quarter of a bitmask word)
    const uint32_t word = threadIdx.x >> 2, q = (threadIdx.x & 3u) * 16u;
    const uint32_t bits = (uint32_t)((occ[word] >> q) & 0xffffu);
    uint32_t tot;
    uint32_t pos = block_excl_scan<kLeafWG>((uint32_t)__popc(bits), sh, &tot);
    for (uint32_t m = bits; m; m &= m - 1) {
      const uint32_t s = word * 64 + q + (uint32_t)__ffs(m) - 1;
      uint32_t rgba;
      if (MODE == 0) {
        const uint64_t a = acc[s];
        const uint32_t c = (uint32_t)(a >> 48);
        rgba = (uint32_t)((a & 0xffffffu) / c) | ((uint32_t)(((a >> 24) & 0xffffffu) / c) << 8) |
               ((accb[s] / c) << 16) | (255u << 24);
      } else {
        rgba = accb[s];
        temp_ids[out0 + vbase + pos] = accid[s];
      }
      temp[out0 + vbase + pos] = make_voxel(code_hi | s, rgba);
      acc[s] = init;
      accb[s] = 0;
      ++pos;
    }
    vbase += tot;
    __syncthreads();
    if (threadIdx.x < kSubCells / 64) occ[threadIdx.x] = 0;
    __syncthreads();
  }
  if (threadIdx.x == 0) nodes.aux[n] = vbase;
}

// Capacity for all voxel lists: per level, at most min(2^21, points) per node
// and at most (voxels from leaf children) + (bound of the level below).  One
// workgroup.
constexpr int kBoundWG = 1024;
__global__ void __launch_bounds__(kBoundWG) k_voxel_bound(Nodes nodes, TreeState* st) {
  __shared__ uint64_t sh[2][kBoundWG / 64];
  uint32_t deepest = 0;
  for (uint32_t L = 0; L < 22; ++L)
    if (st->level_end[L] > st->level_begin[L]) deepest = L;
  uint64_t below = 0, total = 0;
  for (int L = (int)deepest; L >= 0; --L) {
    uint64_t by_points = 0, from_leaves = 0;
    for (uint32_t j = st->level_begin[L] + threadIdx.x; j < st->level_end[L]; j += kBoundWG)
      if (!nodes.is_leaf[j]) by_points += min((uint64_t)nodes.npoints[j], (uint64_t)1 << 21);
    for (uint32_t j = st->level_begin[L + 1] + threadIdx.x; j < st->level_end[L + 1]; j += kBoundWG)
      if (nodes.is_leaf[j]) from_leaves += nodes.aux[j];
    by_points = wave_sum(by_points);
    from_leaves = wave_sum(from_leaves);
    if (lane_id() == 0) {
      sh[0][threadIdx.x / 64] = by_points;
      sh[1][threadIdx.x / 64] = from_leaves;
    }
    __syncthreads();
    uint64_t a = 0, b = 0;
    for (int w = 0; w < kBoundWG / 64; ++w) { a += sh[0][w]; b += sh[1][w]; }
    __syncthreads();
    const uint64_t bl = min(a, b + below);
    total += bl;
    below = bl;
  }
  if (threadIdx.x == 0) {
    st->voxel_bound = total;
    st->voxel_total = 0;
  }
}

// Number of parent voxels an inner node contributes: runs of equal (code >> 3)
// in its Morton-ordered list.  One workgroup per node of the level.
constexpr int kRunWG = 256;
__global__ void __launch_bounds__(kRunWG) k_runs(Nodes nodes, uint32_t begin, uint32_t end,
                                                 const uint64_t* __restrict__ vox) {
  __shared__ uint32_t sh[kRunWG / 64];
  const uint32_t j = begin + blockIdx.x;
  if (j >= end || nodes.is_leaf[j]) return;
  const uint64_t o = nodes.offset[j];
  const uint32_t cnt = nodes.count[j];
  uint32_t runs = 0;
  for (uint32_t i = threadIdx.x; i < cnt; i += kRunWG) {
    const uint32_t c = voxel_code(vox[o + i]) >> 3;
    runs += (i == 0 || (voxel_code(vox[o + i - 1]) >> 3) != c) ? 1u : 0u;
  }
  runs = wave_sum(runs);
  if (lane_id() == 0) sh[threadIdx.x / 64] = runs;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t t = 0;
    for (int w = 0; w < kRunWG / 64; ++w) t += sh[w];
    nodes.aux[j] = t;
  }
}

// Voxel offsets of the inner nodes of one level (one workgroup): the node's
// list is its children's contributions in octant order; nodes follow each
// other in key order after everything already written.
constexpr int kOffWG = 1024;
__global__ void __launch_bounds__(kOffWG) k_level_offsets(Nodes nodes, uint32_t begin, uint32_t end, TreeState* st) {
  __shared__ uint64_t sh[kOffWG / 64 + 1];
  uint64_t base = st->voxel_total;
  for (uint32_t c0 = begin; c0 < end; c0 += kOffWG) {
    const uint32_t j = c0 + threadIdx.x;
    uint64_t total = 0;
    if (j < end && !nodes.is_leaf[j]) {
      const uint32_t fc = nodes.first_child[j];
      const uint32_t nc = (uint32_t)__popc(nodes.child_mask[j]);
      for (uint32_t k = 0; k < nc; ++k) {
        nodes.jobofs[fc + k] = (uint32_t)total;
        total += nodes.aux[fc + k];
      }
    }
    uint64_t tot;
    const uint64_t ex = block_excl_scan<kOffWG>(total, sh, &tot);
    if (j < end && !nodes.is_leaf[j]) {
      nodes.offset[j] = base + ex;
      nodes.count[j] = (uint32_t)total;
    }
    base += tot;
  }
  if (threadIdx.x == 0) st->voxel_total = base;
}

// Write the voxels of the level-L parents: one workgroup per node of level
// L + 1 (every such node is a child of an inner node).  Leaf children copy
// their staged voxels; inner children reduce runs of their own voxels.
constexpr int kWriteWG = 256;
template <int MODE>
__global__ void __launch_bounds__(kWriteWG) k_write(Nodes nodes, uint32_t begin, uint32_t end,
                                                    const uint64_t* __restrict__ temp, const uint32_t* __restrict__ temp_ids,
                                                    uint64_t* __restrict__ vox, uint32_t* __restrict__ vids, uint32_t seed) {
  __shared__ uint32_t sh[kWriteWG / 64 + 1];
  const uint32_t j = begin + blockIdx.x;
  if (j >= end) return;
  const uint32_t p = nodes.parent[j];
  const uint64_t dst = nodes.offset[p] + nodes.jobofs[j];
  if (nodes.is_leaf[j]) {
    const uint64_t src = nodes.offset[j];
    const uint32_t cnt = nodes.aux[j];
    for (uint32_t i = threadIdx.x; i < cnt; i += kWriteWG) {
      vox[dst + i] = temp[src + i];
      if (MODE) vids[dst + i] = temp_ids[src + i];
    }
    return;
  }
  const uint64_t o = nodes.offset[j];
  const uint32_t cnt = nodes.count[j];
  const uint32_t oct = (uint32_t)(nodes.key[j] & 7u) << 18;
  uint32_t base = 0;
  for (uint32_t i0 = 0; i0 < cnt; i0 += kWriteWG) {
    const uint32_t i = i0 + threadIdx.x;
    uint32_t c = 0, start = 0;
    if (i < cnt) {
      c = voxel_code(vox[o + i]) >> 3;
      start = (i == 0 || (voxel_code(vox[o + i - 1]) >> 3) != c) ? 1u : 0u;
    }
    uint32_t tot;
    const uint32_t r = block_excl_scan<kWriteWG>(start, sh, &tot);
    if (start) {
      uint32_t sr = 0, sg = 0, sb = 0, nn = 0;
      uint64_t best = MODE == 1 ? ~0ull : 0ull;
      uint32_t brgba = 0, bid = 0;
      for (uint32_t k = i; k < cnt && k < i + 8; ++k) {
        const uint64_t v = vox[o + k];
        if ((voxel_code(v) >> 3) != c) break;
        const uint32_t rgba = (uint32_t)(v >> 32);
        if (MODE == 0) {
          sr += rgba & 0xffu;
          sg += (rgba >> 8) & 0xffu;
          sb += (rgba >> 16) & 0xffu;
          ++nn;
        } else {
          const uint32_t id = vids[o + k];
          const uint64_t key = pick_order(id, seed, MODE == 2);
          if (MODE == 1 ? key < best : key > best) {
            best = key;
            brgba = rgba;
            bid = id;
          }
        }
      }
      uint32_t rgba;
      if (MODE == 0) rgba = (sr / nn) | ((sg / nn) << 8) | ((sb / nn) << 16) | (255u << 24);
      else rgba = brgba;
      vox[dst + base + r] = make_voxel(oct | c, rgba);
      if (MODE) vids[dst + base + r] = bid;
    }
    base += tot;
  }
}

void launch_leaf_voxels(uint32_t mode, const Nodes& nodes, uint32_t num_nodes, const GridDesc* grids,
                        const uint32_t* pool, const void* pts, const uint32_t* ids, const Cube* cube, uint64_t* temp,
                        uint32_t* temp_ids, uint32_t seed, hipStream_t s) {
  if (!num_nodes) return;
  if (mode == 0)
    hipLaunchKernelGGL(k_leaf_voxels<0>, dim3(num_nodes), dim3(kLeafWG), 0, s, nodes, num_nodes, grids, pool,
                       (const uint4*)pts, ids, cube, temp, temp_ids, seed);
  else if (mode == 1)
    hipLaunchKernelGGL(k_leaf_voxels<1>, dim3(num_nodes), dim3(kLeafWG), 0, s, nodes, num_nodes, grids, pool,
                       (const uint4*)pts, ids, cube, temp, temp_ids, seed);
  else
    hipLaunchKernelGGL(k_leaf_voxels<2>, dim3(num_nodes), dim3(kLeafWG), 0, s, nodes, num_nodes, grids, pool,
                       (const uint4*)pts, ids, cube, temp, temp_ids, seed);
}

void launch_voxel_bound(const Nodes& nodes, TreeState* st, hipStream_t s) {
  hipLaunchKernelGGL(k_voxel_bound, dim3(1), dim3(kBoundWG), 0, s, nodes, st);
}

void launch_level(uint32_t mode, const Nodes& nodes, uint32_t pbegin, uint32_t pend, uint32_t cbegin, uint32_t cend,
                  const uint64_t* temp, const uint32_t* temp_ids, uint64_t* vox, uint32_t* vids, TreeState* st,
                  uint32_t seed, hipStream_t s) {
  if (cend <= cbegin) return;
  hipLaunchKernelGGL(k_runs, dim3(cend - cbegin), dim3(kRunWG), 0, s, nodes, cbegin, cend, (const uint64_t*)vox);
  hipLaunchKernelGGL(k_level_offsets, dim3(1), dim3(kOffWG), 0, s, nodes, pbegin, pend, st);
  if (mode == 0)
    hipLaunchKernelGGL(k_write<0>, dim3(cend - cbegin), dim3(kWriteWG), 0, s, nodes, cbegin, cend, temp, temp_ids, vox,
                       vids, seed);
  else if (mode == 1)
    hipLaunchKernelGGL(k_write<1>, dim3(cend - cbegin), dim3(kWriteWG), 0, s, nodes, cbegin, cend, temp, temp_ids, vox,
                       vids, seed);
  else
    hipLaunchKernelGGL(k_write<2>, dim3(cend - cbegin), dim3(kWriteWG), 0, s, nodes, cbegin, cend, temp, temp_ids, vox,
                       vids, seed);
}

}  // namespace lod
