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

#include <algorithm>

namespace lod {

constexpr int kLeafWG = 256;
constexpr uint32_t kSubCells = 4096;  // 2 levels of micro-bucket -> 4 levels of voxel cells = 12 bits
constexpr uint32_t kPackedMax = 65535;  // largest micro-bucket the packed 24/24/16-bit sums can hold
constexpr int kLeafPF = 4;              // points in flight per thread

// Wide accumulation for one micro-bucket whose cells may hold more samples
// than the packed 16-bit fields allow: windows of 512 cells with 64-bit sums
// of R, G, B and the count, re-reading the micro-bucket's points per window.
__device__ void leaf_wide_average(uint64_t* acc /* 2048 words of LDS */, uint32_t* sh, const uint4* __restrict__ pts,
                                  uint32_t off, uint32_t cnt, uint32_t sub_shift, const CubeD& cd, uint32_t code_hi,
                                  uint64_t* __restrict__ temp, uint64_t out, uint32_t& vbase) {
  uint64_t* wr = acc;
  uint64_t* wg = acc + 512;
  uint64_t* wb = acc + 1024;
  uint64_t* wn = acc + 1536;
  for (uint32_t w0 = 0; w0 < kSubCells; w0 += 512) {
    for (uint32_t i = threadIdx.x; i < 2048; i += kLeafWG) acc[i] = 0;
    lds_barrier();
    for (uint32_t i = threadIdx.x; i < cnt; i += kLeafWG) {
      const uint4 v = pts[off + i];
      const uint64_t key = point_key(__uint_as_float(v.x), __uint_as_float(v.y), __uint_as_float(v.z), cd);
      const uint32_t sub = (uint32_t)(key >> sub_shift) & (kSubCells - 1);
      if (sub >= w0 && sub < w0 + 512) {
        const uint32_t q = sub - w0;
        atomicAdd((unsigned long long*)&wr[q], (unsigned long long)(v.w & 0xff));
        atomicAdd((unsigned long long*)&wg[q], (unsigned long long)((v.w >> 8) & 0xff));
        atomicAdd((unsigned long long*)&wb[q], (unsigned long long)((v.w >> 16) & 0xff));
        atomicAdd((unsigned long long*)&wn[q], 1ull);
      }
    }
    lds_barrier();
    for (uint32_t s0 = 0; s0 < 512; s0 += kLeafWG) {
      const uint32_t q = s0 + threadIdx.x;
      const uint64_t c = wn[q];
      uint32_t tot;
      const uint32_t pos = block_excl_scan<kLeafWG>(c ? 1u : 0u, sh, &tot);
      if (c) {
        const uint32_t rgba = (uint32_t)(wr[q] / c) | ((uint32_t)(wg[q] / c) << 8) | ((uint32_t)(wb[q] / c) << 16) |
                              (255u << 24);
        temp[out + vbase + pos] = make_voxel(code_hi | (w0 + q), rgba);
      }
      vbase += tot;
    }
    lds_barrier();
  }
}

// Parent voxels from the points of every leaf (level >= 1).  One workgroup per
// node; non-leaves exit.  Voxels go to temp[offset .. offset + k) of the leaf
// (k <= points of the leaf), the count to nodes.aux.
//
// One 64-bit LDS atomic per point:
//   average: acc[cell] += R | G << 16 | B << 32 | 1 << 48.  The 16-bit fields
//            are exact while a cell holds at most 257 samples (255 * 257 <
//            2^16); a micro-bucket with a fuller cell is redone by the wide
//            path above.
//   pick:    acc[cell] = min/max of the sample's order key; a second pass over
//            the micro-bucket lets the winner deposit its colour and id.
// Occupied cells are those whose accumulator left its initial value; the
// emission walks the 4096 cells in order (16 per thread), which lists the
// voxels in Morton order.
//
// A work item is one leaf and one of its 8 child cells (8 micro-buckets), so
// that large leaves spread over 8 workgroups.  Its voxels go to temp starting
// at the first point of that child cell (never more voxels than points); the
// count and start are recorded per (leaf, child cell) in gcount / gstart.
template <int MODE>  // 0 average, 1 first, 2 random
__global__ void __launch_bounds__(kLeafWG) k_leaf_voxels(Nodes nodes, uint32_t num_nodes,
                                                         const GridDesc* __restrict__ grids,
                                                         const uint32_t* __restrict__ pool,
                                                         const uint4* __restrict__ pts, const uint32_t* __restrict__ ids,
                                                         const Cube* cube, uint64_t* __restrict__ temp,
                                                         uint32_t* __restrict__ temp_ids, uint32_t* __restrict__ gcount,
                                                         uint32_t* __restrict__ gstart, uint32_t seed) {
  __shared__ uint64_t acc[kSubCells];
  __shared__ uint32_t wcount[64];
  __shared__ uint32_t wover[4];
  __shared__ uint32_t wrgba[MODE ? kSubCells : 1];
  __shared__ uint32_t wid[MODE ? kSubCells : 1];
  __shared__ uint32_t sh[kLeafWG / 64 + 1];
  const uint32_t n = blockIdx.x >> 3, grp = blockIdx.x & 7u;
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
  const uint64_t out0 = goff[((leaf_rel << 6) | (grp << 3)) << (3 * (G.e - rm))];
  bool any = false;
  for (uint32_t jm = grp * 8; jm < grp * 8 + 8; ++jm) any |= mcnt[(leaf_rel << 6) | jm] != 0;
  if (!any) {
    if (threadIdx.x == 0) {
      gcount[blockIdx.x] = 0;
      gstart[blockIdx.x] = (uint32_t)out0;
    }
    return;
  }
  for (uint32_t i = threadIdx.x; i < kSubCells; i += kLeafWG) acc[i] = init;
  lds_barrier();
  uint32_t vbase = 0;
  for (uint32_t jm = grp * 8; jm < grp * 8 + 8; ++jm) {
    const uint64_t idx = (leaf_rel << 6) | jm;
    const uint32_t cnt = mcnt[idx];
    if (cnt == 0) continue;
    const uint32_t off = goff[idx << (3 * (G.e - rm))];
    const uint32_t code_hi = top9 | (jm << 12);
    if (MODE == 0 && cnt > kPackedMax) {
      leaf_wide_average(acc, sh, pts, off, cnt, sub_shift, cd, code_hi, temp, out0, vbase);
      for (uint32_t i = threadIdx.x; i < kSubCells; i += kLeafWG) acc[i] = init;
      lds_barrier();
      continue;
    }
    // accumulate: every thread first issues all loads of a batch, then hashes
    for (uint32_t b0 = 0; b0 < cnt; b0 += kLeafWG * kLeafPF) {
      uint4 v[kLeafPF];
      uint32_t idv[kLeafPF];
#pragma unroll
      for (int k = 0; k < kLeafPF; ++k) {
        const uint32_t i = b0 + k * kLeafWG + threadIdx.x;
        if (i < cnt) {
          v[k] = pts[off + i];
          if (MODE) idv[k] = ids[off + i];
        }
      }
#pragma unroll
      for (int k = 0; k < kLeafPF; ++k) {
        const uint32_t i = b0 + k * kLeafWG + threadIdx.x;
        if (i >= cnt) continue;
        const uint64_t key = point_key(__uint_as_float(v[k].x), __uint_as_float(v[k].y), __uint_as_float(v[k].z), cd);
        const uint32_t sub = (uint32_t)(key >> sub_shift) & (kSubCells - 1);
        if (MODE == 0) {
          const uint64_t packed = (uint64_t)(v[k].w & 0xff) | ((uint64_t)((v[k].w >> 8) & 0xff) << 16) |
                                  ((uint64_t)((v[k].w >> 16) & 0xff) << 32) | (1ull << 48);
          atomicAdd((unsigned long long*)&acc[sub], (unsigned long long)packed);
        } else {
          const uint64_t ok = pick_order(idv[k], seed, MODE == 2);
          if (MODE == 1) atomicMin((unsigned long long*)&acc[sub], (unsigned long long)ok);
          else atomicMax((unsigned long long*)&acc[sub], (unsigned long long)ok);
        }
      }
    }
    lds_barrier();
    if (MODE != 0) {
      // the winner of every cell deposits its colour and id
      for (uint32_t i = threadIdx.x; i < cnt; i += kLeafWG) {
        const uint32_t id = ids[off + i];
        const uint4 v = pts[off + i];
        const uint64_t key = point_key(__uint_as_float(v.x), __uint_as_float(v.y), __uint_as_float(v.z), cd);
        const uint32_t sub = (uint32_t)(key >> sub_shift) & (kSubCells - 1);
        if (acc[sub] == pick_order(id, seed, MODE == 2)) {
          wrgba[sub] = v.w;
          wid[sub] = id;
        }
      }
      lds_barrier();
    }
    // emit.  Lane l of wave w owns cells 256k + 64w + l (k = 0..15); the
    // wave's ballot over cells 256k + 64w .. +63 is occupancy word 4k + w, so
    // word order is cell (Morton) order.  One exchange of the 64 word counts
    // gives every word its prefix, and each lane writes its own occupied
    // cells at prefix(word) + occupied lanes below it.
    {
      const uint32_t w = threadIdx.x / 64, l = lane_id();
      uint64_t bal[16];
      uint32_t over = 0;
#pragma unroll
      for (uint32_t k = 0; k < 16; ++k) {
        const uint64_t a = acc[256 * k + 64 * w + l];
        if (MODE == 0) over |= (a >> 48) > 257 ? 1u : 0u;
        bal[k] = __ballot(a != init);
      }
      const bool any_over = MODE == 0 && __ballot(over != 0) != 0;
      if (l == 0) {
#pragma unroll
        for (uint32_t k = 0; k < 16; ++k) wcount[4 * k + w] = (uint32_t)__popcll(bal[k]);
        wover[w] = any_over ? 1u : 0u;
      }
      lds_barrier();
      const bool redo = MODE == 0 && (wover[0] | wover[1] | wover[2] | wover[3]);
      const uint32_t mine = wcount[l];
      const uint32_t incl = wave_incl_scan(mine);
      const uint32_t total = __shfl(incl, 63, 64);
      const uint32_t excl = incl - mine;
      if (!redo) {
        const uint64_t below = (l == 0) ? 0ull : (~0ull >> (64 - l));
        // word prefixes, read with every lane active (a shuffle from a lane
        // masked off by a branch is undefined)
#pragma unroll
        for (uint32_t k = 0; k < 16; ++k) {
          const uint32_t pre = (uint32_t)__shfl(excl, (int)(4 * k + w), 64);
          if ((bal[k] >> l) & 1ull) {
            const uint32_t pos = pre + (uint32_t)__popcll(bal[k] & below);
            const uint32_t s = 256 * k + 64 * w + l;
            const uint64_t a = acc[s];
            uint32_t rgba;
            if (MODE == 0) {
              // floor(sum / n): sums < 2^16 and n <= 257 are exact in float and
              // the correctly rounded quotient (< 256) stays at least 1/n away
              // from the next integer when it is not one, so truncation is exact
              const float c = (float)(uint32_t)(a >> 48);
              rgba = (uint32_t)__fdiv_rn((float)(uint32_t)(a & 0xffffu), c) |
                     ((uint32_t)__fdiv_rn((float)(uint32_t)((a >> 16) & 0xffffu), c) << 8) |
                     ((uint32_t)__fdiv_rn((float)(uint32_t)((a >> 32) & 0xffffu), c) << 16) | (255u << 24);
            } else {
              rgba = wrgba[s];
              temp_ids[out0 + vbase + pos] = wid[s];
            }
            temp[out0 + vbase + pos] = make_voxel(code_hi | s, rgba);
            acc[s] = init;
          }
        }
        vbase += total;
        lds_barrier();
      } else {
        // a cell overflowed the packed fields: clear and redo this micro-bucket exactly
        lds_barrier();
        for (uint32_t i = threadIdx.x; i < kSubCells; i += kLeafWG) acc[i] = init;
        lds_barrier();
        leaf_wide_average(acc, sh, pts, off, cnt, sub_shift, cd, code_hi, temp, out0, vbase);
        for (uint32_t i = threadIdx.x; i < kSubCells; i += kLeafWG) acc[i] = init;
        lds_barrier();
      }
    }
  }
  if (threadIdx.x == 0) {
    gcount[blockIdx.x] = vbase;
    gstart[blockIdx.x] = (uint32_t)out0;
  }
}

// Voxel count of every leaf: the sum over its 8 child-cell work items.
__global__ void k_leaf_sums(Nodes nodes, uint32_t num_nodes, const uint32_t* __restrict__ gcount) {
  const uint32_t n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= num_nodes || !nodes.is_leaf[n]) return;
  uint32_t s = 0;
  if (nodes.level[n] != 0)
    for (uint32_t g = 0; g < 8; ++g) s += gcount[8 * n + g];
  nodes.aux[n] = s;
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
    st->inner_total = 0;
  }
}

// ------------------------------------------------------------ inner levels
//
// The voxels of all inner nodes of one level are contiguous and each node's
// list is in Morton order.  A parent cell collects the child voxels whose
// codes agree above the lowest 3 bits (2x2x2 -> 1), i.e. a run of at most 8
// consecutive entries of one node.  Whoever writes a voxel also writes its
// owner node and a one-byte flag telling whether it starts such a run (first
// voxel of a child's contribution, or a change of code >> 3); an exclusive
// prefix sum over the flags of a level numbers the runs, and every run is
// reduced by the thread at its start.

constexpr uint32_t kTile = 4096;
constexpr int kTileWG = 256;
constexpr uint32_t kTilePT = kTile / kTileWG;  // 16 flags per thread, read as 4 words

__device__ __forceinline__ uint32_t flags4(const uint8_t* __restrict__ f, uint64_t i, uint64_t V) {
  // 4 consecutive flags starting at i, one byte each; zero past V (byte loads:
  // a level's flags need not start on a word boundary)
  uint32_t w = 0;
#pragma unroll
  for (uint32_t k = 0; k < 4; ++k)
    if (i + k < V) w |= (uint32_t)f[i + k] << (8 * k);
  return w;
}

// (1) run starts per tile of the level's voxels
__global__ void __launch_bounds__(kTileWG) k_run_tiles(const TreeState* st, uint32_t lvl,
                                                       const uint8_t* __restrict__ vflag, uint32_t* __restrict__ tilesum) {
  __shared__ uint32_t sh[kTileWG / 64];
  const uint64_t vb = st->level_vbegin[lvl], V = st->level_vcount[lvl];
  const uint8_t* f = vflag + vb;
  const uint32_t ntiles = (uint32_t)((V + kTile - 1) / kTile);
  for (uint32_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    uint32_t c = 0;
    for (uint32_t k = 0; k < kTilePT / 4; ++k) {
      const uint64_t j = (uint64_t)t * kTile + 4ull * (k * kTileWG + threadIdx.x);
      if (j < V) c += (uint32_t)__popc(flags4(f, j, V) & 0x01010101u);
    }
    c = wave_sum(c);
    if (lane_id() == 0) sh[threadIdx.x / 64] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
      uint32_t s = 0;
      for (int w = 0; w < kTileWG / 64; ++w) s += sh[w];
      tilesum[t] = s;
    }
    __syncthreads();
  }
}

// (2) exclusive scan of the tile counts (one workgroup); tilesum[ntiles] = total
constexpr int kScanWG = 1024;
__global__ void __launch_bounds__(kScanWG) k_tile_scan(const TreeState* st, uint32_t lvl, uint32_t* tilesum) {
  __shared__ uint32_t sh[kScanWG / 64 + 1];
  const uint64_t V = st->level_vcount[lvl];
  const uint32_t ntiles = (uint32_t)((V + kTile - 1) / kTile);
  uint32_t base = 0;
  for (uint32_t t0 = 0; t0 < ntiles; t0 += kScanWG) {
    const uint32_t t = t0 + threadIdx.x;
    const uint32_t v = t < ntiles ? tilesum[t] : 0u;
    uint32_t tot;
    const uint32_t ex = block_excl_scan<kScanWG>(v, sh, &tot);
    if (t < ntiles) tilesum[t] = base + ex;
    base += tot;
  }
  if (threadIdx.x == 0) tilesum[ntiles] = base;
}

// (3) global run index of every voxel of the level (runidx[V] = number of runs)
__global__ void __launch_bounds__(kTileWG) k_run_index(const TreeState* st, uint32_t lvl,
                                                       const uint8_t* __restrict__ vflag,
                                                       const uint32_t* __restrict__ tilesum, uint32_t* __restrict__ runidx,
                                                       uint32_t* __restrict__ runpos) {
  __shared__ uint32_t sh[kTileWG / 64 + 1];
  const uint64_t vb = st->level_vbegin[lvl], V = st->level_vcount[lvl];
  const uint8_t* f = vflag + vb;
  const uint32_t ntiles = (uint32_t)((V + kTile - 1) / kTile);
  for (uint32_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const uint64_t j0 = (uint64_t)t * kTile + (uint64_t)threadIdx.x * kTilePT;  // contiguous per thread
    uint32_t w[kTilePT / 4];
    uint32_t local = 0;
#pragma unroll
    for (uint32_t k = 0; k < kTilePT / 4; ++k) {
      w[k] = j0 + 4 * k < V ? flags4(f, j0 + 4 * k, V) : 0u;
      local += (uint32_t)__popc(w[k] & 0x01010101u);
    }
    uint32_t tot;
    uint32_t ex = block_excl_scan<kTileWG>(local, sh, &tot) + tilesum[t];
#pragma unroll
    for (uint32_t k = 0; k < kTilePT; ++k) {
      const uint64_t j = j0 + k;
      const uint32_t f = (w[k / 4] >> (8 * (k & 3))) & 1u;
      if (j < V) {
        runidx[j] = ex;
        if (f) runpos[ex] = (uint32_t)j;
      }
      ex += f;
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) runidx[V] = tilesum[ntiles];
}

// (4) voxel offsets of the level's inner nodes (one workgroup): a node's list
// is its children's contributions in octant order, nodes follow in key order.
constexpr int kOffWG = 1024;
__global__ void __launch_bounds__(kOffWG) k_level_offsets(Nodes nodes, uint32_t lvl, uint32_t begin, uint32_t end,
                                                          TreeState* st, const uint32_t* __restrict__ runidx) {
  __shared__ uint64_t sh[kOffWG / 64 + 1];
  const uint64_t level_base = st->voxel_total;
  const uint64_t cvb = st->level_vbegin[lvl + 1];
  uint64_t base = level_base;
  for (uint32_t c0 = begin; c0 < end; c0 += kOffWG) {
    const uint32_t j = c0 + threadIdx.x;
    const bool inner = j < end && !nodes.is_leaf[j];
    uint64_t total = 0;
    if (inner) {
      const uint32_t fc = nodes.first_child[j];
      const uint32_t nc = (uint32_t)__popc(nodes.child_mask[j]);
      for (uint32_t k = 0; k < nc; ++k) {
        const uint32_t c = fc + k;
        nodes.jobofs[c] = (uint32_t)total;
        if (nodes.is_leaf[c]) {
          total += nodes.aux[c];
        } else {
          const uint64_t r0 = nodes.offset[c] - cvb;
          total += runidx[r0 + nodes.count[c]] - runidx[r0];
        }
      }
    }
    uint64_t tot;
    const uint64_t ex = block_excl_scan<kOffWG>(total, sh, &tot);
    if (inner) {
      const uint64_t off = base + ex;
      nodes.offset[j] = off;
      nodes.count[j] = (uint32_t)total;
      const uint32_t fc = nodes.first_child[j];
      const uint32_t nc = (uint32_t)__popc(nodes.child_mask[j]);
      for (uint32_t k = 0; k < nc; ++k) {
        const uint32_t c = fc + k;
        if (!nodes.is_leaf[c]) {
          nodes.dstbase[c] = off + nodes.jobofs[c];
          nodes.firstrun[c] = runidx[nodes.offset[c] - cvb];
        }
      }
    }
    base += tot;
  }
  if (threadIdx.x == 0) {
    st->level_vbegin[lvl] = level_base;
    st->level_vcount[lvl] = base - level_base;
    st->voxel_total = base;
  }
}

// (5) reduce every run of the child level into its parent's list: one
// thread per run (the run starts were listed densely by k_run_index)
template <int MODE>
__global__ void __launch_bounds__(kTileWG) k_write_runs(Nodes nodes, const TreeState* st, uint32_t clvl,
                                                        const uint32_t* __restrict__ runidx,
                                                        const uint32_t* __restrict__ runpos, uint64_t* vox,
                                                        uint32_t* vids, uint8_t* vflag, uint32_t* vowner,
                                                        uint32_t seed) {
  const uint64_t vb = st->level_vbegin[clvl], V = st->level_vcount[clvl];
  if (V == 0) return;
  const uint32_t R = runidx[V];
  const uint32_t stride = gridDim.x * kTileWG;
  for (uint32_t r = blockIdx.x * kTileWG + threadIdx.x; r < R; r += stride) {
    const uint64_t j = runpos[r];
    const uint64_t jend = r + 1 < R ? runpos[r + 1] : V;
    const uint64_t i = vb + j;
    const uint32_t c = vowner[i];
    const uint32_t rank = r - nodes.firstrun[c];
    const uint64_t dst = nodes.dstbase[c] + rank;
    const uint64_t v0 = vox[i];
    const uint32_t code = voxel_code(v0) >> 3;
    const uint32_t oct = (uint32_t)(nodes.key[c] & 7u) << 18;
    uint32_t sr = 0, sg = 0, sb = 0, nn = 0, brgba = 0, bid = 0;
    uint64_t best = MODE == 1 ? ~0ull : 0ull;
    for (uint64_t k = i; k < vb + jend; ++k) {
      const uint64_t v = k == i ? v0 : vox[k];
      const uint32_t rgba = (uint32_t)(v >> 32);
      if (MODE == 0) {
        sr += rgba & 0xffu;
        sg += (rgba >> 8) & 0xffu;
        sb += (rgba >> 16) & 0xffu;
        ++nn;
      } else {
        const uint32_t id = vids[k];
        const uint64_t key = pick_order(id, seed, MODE == 2);
        if (MODE == 1 ? key < best : key > best) {
          best = key;
          brgba = rgba;
          bid = id;
        }
      }
    }
    const uint32_t rgba =
        MODE == 0 ? ((sr / nn) | ((sg / nn) << 8) | ((sb / nn) << 16) | (255u << 24)) : brgba;
    vox[dst] = make_voxel(oct | code, rgba);
    if (MODE) vids[dst] = bid;
    vowner[dst] = nodes.parent[c];
    // the new voxel starts a run of the next level up if it opens this child's
    // contribution or if its code >> 3 differs from the previous run's
    vflag[dst] = (rank == 0 || (code >> 3) != ((voxel_code(vox[i - 1]) >> 3) >> 3)) ? 1 : 0;
  }
}

// (6) leaf children: copy their staged voxels (8 segments, one per child
// cell) into the parent's list.  A segment's first voxel always starts a run
// of the next level up: different child cells differ in the code bits above
// the lowest 3.
template <int MODE>
__global__ void __launch_bounds__(kTileWG) k_copy_leaf_voxels(Nodes nodes, uint32_t begin, uint32_t end,
                                                              const uint32_t* __restrict__ gcount,
                                                              const uint32_t* __restrict__ gstart,
                                                              const uint64_t* __restrict__ temp,
                                                              const uint32_t* __restrict__ temp_ids,
                                                              uint64_t* __restrict__ vox, uint32_t* __restrict__ vids,
                                                              uint8_t* __restrict__ vflag, uint32_t* __restrict__ vowner) {
  const uint32_t c = begin + blockIdx.x;
  if (c >= end || !nodes.is_leaf[c]) return;
  const uint32_t p = nodes.parent[c];
  uint64_t dst = nodes.offset[p] + nodes.jobofs[c];
  for (uint32_t g = 0; g < 8; ++g) {
    const uint32_t cnt = gcount[8 * c + g];
    const uint64_t src = gstart[8 * c + g];
    for (uint32_t i = threadIdx.x; i < cnt; i += kTileWG) {
      const uint64_t v = temp[src + i];
      vox[dst + i] = v;
      if (MODE) vids[dst + i] = temp_ids[src + i];
      vowner[dst + i] = p;
      vflag[dst + i] = (i == 0 || (voxel_code(v) >> 3) != (voxel_code(temp[src + i - 1]) >> 3)) ? 1 : 0;
    }
    dst += cnt;
  }
}

__global__ void k_fill_u64(uint64_t* p, uint64_t n) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = 0;
}

void launch_leaf_voxels(uint32_t mode, const Nodes& nodes, uint32_t num_nodes, const GridDesc* grids,
                        const uint32_t* pool, const void* pts, const uint32_t* ids, const Cube* cube, uint64_t* temp,
                        uint32_t* temp_ids, uint32_t* gcount, uint32_t* gstart, uint32_t seed, hipStream_t s) {
  if (!num_nodes) return;
  const dim3 grid(num_nodes * 8);
  if (mode == 0)
    hipLaunchKernelGGL(k_leaf_voxels<0>, grid, dim3(kLeafWG), 0, s, nodes, num_nodes, grids, pool, (const uint4*)pts,
                       ids, cube, temp, temp_ids, gcount, gstart, seed);
  else if (mode == 1)
    hipLaunchKernelGGL(k_leaf_voxels<1>, grid, dim3(kLeafWG), 0, s, nodes, num_nodes, grids, pool, (const uint4*)pts,
                       ids, cube, temp, temp_ids, gcount, gstart, seed);
  else
    hipLaunchKernelGGL(k_leaf_voxels<2>, grid, dim3(kLeafWG), 0, s, nodes, num_nodes, grids, pool, (const uint4*)pts,
                       ids, cube, temp, temp_ids, gcount, gstart, seed);
  hipLaunchKernelGGL(k_leaf_sums, dim3((num_nodes + 255) / 256), dim3(256), 0, s, nodes, num_nodes, gcount);
}

void launch_voxel_bound(const Nodes& nodes, TreeState* st, hipStream_t s) {
  hipLaunchKernelGGL(k_voxel_bound, dim3(1), dim3(kBoundWG), 0, s, nodes, st);
}

void launch_fill_zero(uint64_t* p, uint64_t n, hipStream_t s) {
  if (!n) return;
  uint64_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_fill_u64, dim3((uint32_t)blocks), dim3(256), 0, s, p, n);
}

void launch_level(uint32_t mode, const Nodes& nodes, uint32_t L, uint32_t pbegin, uint32_t pend, uint32_t cbegin,
                  uint32_t cend, uint64_t vcap, const uint64_t* temp, const uint32_t* temp_ids, uint64_t* vox,
                  uint32_t* vids, TreeState* st, uint32_t* tilesum, uint32_t* runidx, uint32_t* runpos,
                  uint8_t* vflag, uint32_t* vowner, const uint32_t* gcount, const uint32_t* gstart, uint32_t seed,
                  hipStream_t s) {
  const uint64_t tiles = (vcap + kTile - 1) / kTile;
  const uint32_t grid = (uint32_t)std::min<uint64_t>(std::max<uint64_t>(tiles, 1), 2048);
  const uint32_t cl = L + 1;
  hipLaunchKernelGGL(k_run_tiles, dim3(grid), dim3(kTileWG), 0, s, st, cl, vflag, tilesum);
  hipLaunchKernelGGL(k_tile_scan, dim3(1), dim3(kScanWG), 0, s, st, cl, tilesum);
  hipLaunchKernelGGL(k_run_index, dim3(grid), dim3(kTileWG), 0, s, st, cl, vflag, tilesum, runidx, runpos);
  hipLaunchKernelGGL(k_level_offsets, dim3(1), dim3(kOffWG), 0, s, nodes, L, pbegin, pend, st, runidx);
  const uint32_t wgrid = (uint32_t)std::min<uint64_t>(std::max<uint64_t>((vcap / 4 + kTileWG - 1) / kTileWG, 1), 4096);
  const uint32_t nc = cend - cbegin;
#define LOD_LEVEL(M)                                                                                               \
  hipLaunchKernelGGL(k_write_runs<M>, dim3(wgrid), dim3(kTileWG), 0, s, nodes, st, cl, runidx, runpos, vox, vids,  \
                     vflag, vowner, seed);                                                                                \
  if (nc)                                                                                                          \
    hipLaunchKernelGGL(k_copy_leaf_voxels<M>, dim3(nc), dim3(kTileWG), 0, s, nodes, cbegin, cend, gcount, gstart,     \
                       temp, temp_ids, vox, vids, vflag, vowner);
  if (mode == 0) {
    LOD_LEVEL(0)
  } else if (mode == 1) {
    LOD_LEVEL(1)
  } else {
    LOD_LEVEL(2)
  }
#undef LOD_LEVEL
}

}  // namespace lod
