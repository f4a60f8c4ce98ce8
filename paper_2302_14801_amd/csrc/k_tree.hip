// k_tree.hip -- octree nodes from the counting grids (Sec. 4.1.2 merging and
// Sec. 4.1.3 creating target pointers).
//
// The paper merges 2x2x2 groups bottom-up while their sum stays within T and
// no member is unmergeable.  Because a cell's count is the sum of its
// children's, that procedure yields exactly the nodes of the top-down rule
// used here: a node is inner iff it holds more than T points and lies above
// the depth limit, otherwise it is a leaf.  Nodes are enumerated level by
// level so that they come out in ascending (level, key) order with the
// children of a node consecutive.  Counts come from the grid pyramids; a node
// whose children lie below the deepest level of its grid is queued for
// refinement (the "extended counting grid" of Sec. 4.1.5) and enumeration
// resumes after it has been partitioned.
#include <algorithm>

#include "common.h"
#include "launch.h"
#include "scan.h"

namespace lod {

// The root of every tree (one thread per cloud): node slot node_begin of the
// tree's region, counted by root grid c.
__global__ void k_tree_init(uint32_t leaf_cap, uint32_t max_level, const GridDesc* grids, const uint32_t* pool,
                            Nodes nodes, TreeState* sts, const uint32_t* node_begin, const uint32_t* node_end,
                            uint32_t nclouds) {
  const uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nclouds) return;
  TreeState* st = sts + c;
  const GridDesc g = grids[c];
  const uint32_t n = pool[g.pyr];  // level 0 of the root grid: all points of the cloud
  const uint32_t r = node_begin[c];
  memset(st, 0, sizeof(TreeState));
  nodes.level[r] = 0;
  nodes.key[r] = 0;
  nodes.npoints[r] = n;
  const bool inner = n > leaf_cap && max_level > 0;
  nodes.is_leaf[r] = inner ? 0 : 1;
  nodes.child_mask[r] = 0;
  nodes.first_child[r] = 0;
  nodes.offset[r] = g.seg_start;
  nodes.count[r] = inner ? 0 : n;
  nodes.cover[r] = (int32_t)c;
  nodes.grid[r] = (int32_t)c;
  nodes.parent[r] = 0xffffffffu;
  nodes.tree[r] = c;
  st->num_nodes = r + 1;
  st->node_begin = r;
  st->node_end = node_end[c];
  st->next_level = 0;
  st->level_begin[0] = r;
  st->level_end[0] = r + 1;
  st->status = 0;
}

constexpr int kTreeWG = 1024;

// Enumerate levels until done or until inner nodes need refinement (one
// workgroup per tree; finished trees return at once).  Nodes to refine are
// appended to the build-wide lists.
__global__ void __launch_bounds__(kTreeWG) k_tree_build(uint32_t leaf_cap, uint32_t max_level,
                                                        const GridDesc* __restrict__ grids,
                                                        const uint32_t* __restrict__ pool, Nodes nodes, TreeState* sts,
                                                        uint32_t* refine, uint32_t* leaf_refine, BuildState* bs) {
  __shared__ uint32_t sh[kTreeWG / 64 + 1];
  __shared__ uint32_t s_need, s_inner;
  const uint32_t tree = blockIdx.x;
  TreeState* st = sts + tree;
  if (st->status == 1 || build_stopped(bs)) return;
  uint32_t L = st->next_level;
  uint32_t num = st->num_nodes;
  const uint32_t max_nodes = st->node_end;
  for (;;) {
    if (L >= max_level) {
      if (threadIdx.x == 0) { st->status = 1; st->next_level = L; }
      break;
    }
    const uint32_t b = st->level_begin[L], e = st->level_end[L];
    if (threadIdx.x == 0) { s_need = 0; s_inner = 0; }
    __syncthreads();
    const uint32_t first_new = num;
    for (uint32_t c0 = b; c0 < e; c0 += kTreeWG / 8) {
      const uint32_t j = c0 + threadIdx.x / 8;
      const uint32_t o = threadIdx.x & 7u;
      uint32_t cnt = 0, idx = 0, r = 0;
      int32_t cov = -1;
      uint64_t ck = 0;
      GridDesc G;
      if (j < e && !nodes.is_leaf[j]) {
        cov = nodes.grid[j] >= 0 ? nodes.grid[j] : nodes.cover[j];
        G = grids[cov];
        ck = (nodes.key[j] << 3) | o;
        r = L + 1 - G.base_level;
        idx = (uint32_t)(ck - (G.base_key << (3 * r)));
        cnt = pool[G.pyr + pyr_level_offset(r) + idx];
      }
      const uint32_t exists = cnt > 0 ? 1u : 0u;
      uint32_t tot;
      const uint32_t pos = block_excl_scan<kTreeWG>(exists, sh, &tot);
      const uint64_t bal = __ballot(exists);
      const uint32_t grp = (uint32_t)((bal >> (lane_id() & ~7u)) & 0xffu);
      if (exists) {
        const uint32_t n = num + pos;
        if (n < max_nodes) {
          const uint32_t lvl = L + 1;
          const bool inner = cnt > leaf_cap && lvl < max_level;
          const uint32_t D = G.base_level + G.e;
          int32_t gchild = -1;
          if (r == G.e) gchild = ((const int32_t*)(pool + G.child))[idx];
          nodes.level[n] = (uint8_t)lvl;
          nodes.key[n] = ck;
          nodes.npoints[n] = cnt;
          nodes.is_leaf[n] = inner ? 0 : 1;
          nodes.child_mask[n] = 0;
          nodes.first_child[n] = 0;
          nodes.offset[n] = pool[G.off + ((uint64_t)idx << (3 * (G.e - r)))];
          nodes.count[n] = inner ? 0 : cnt;
          nodes.cover[n] = cov;
          nodes.grid[n] = gchild;
          nodes.parent[n] = j;
          nodes.tree[n] = tree;
          if (inner) {
            atomicOr(&s_inner, 1u);
            if (r == G.e && gchild < 0) {
              atomicOr(&s_need, 1u);
              refine[atomicAdd(&bs->nref, 1u)] = n;
            }
          } else {
            const uint32_t sd = gchild >= 0 ? grids[gchild].base_level + grids[gchild].e : D;
            if (sd < lvl + 2) leaf_refine[atomicAdd(&bs->nlref, 1u)] = n;
          }
        }
        // the lowest existing octant of each parent records its children
        if ((grp & ((1u << o) - 1u)) == 0) {
          nodes.first_child[j] = n;
          nodes.child_mask[j] = (uint8_t)grp;
        }
      }
      num += tot;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      st->level_begin[L + 1] = first_new;
      st->level_end[L + 1] = num;
      if (num > max_nodes) {
        st->overflow = 1;
        atomicOr(&bs->overflow, 1u);
      }
    }
    L += 1;
    const bool need = s_need != 0;
    const bool any_inner = s_inner != 0;
    __syncthreads();
    if (num > max_nodes) {
      if (threadIdx.x == 0) { st->status = 1; st->next_level = L; }
      break;
    }
    if (need) {
      if (threadIdx.x == 0) { st->status = 2; st->next_level = L; }
      break;
    }
    if (!any_inner) {
      if (threadIdx.x == 0) { st->status = 1; st->next_level = L; }
      break;
    }
  }
  if (threadIdx.x == 0) st->num_nodes = min(num, max_nodes);
}

// Segments (and grid descriptors) for the nodes of `list` (*nlist_ptr of
// them), which need a deeper partition: each gets an extended grid of E
// levels below the node (Sec. 4.1.5).  The grids are numbered from
// bs->num_grids on and stored from pool word bs->used_words on
// (k_refine_commit advances both afterwards).  If they do not fit in
// grid_cap descriptors and word_cap words, nothing is refined and the build
// is flagged (kOverGrids); need_grids / need_words record what was asked.
__global__ void k_refine_segments(Nodes nodes, const uint32_t* list, const uint32_t* nlist_ptr, uint32_t E,
                                  BuildState* bs, uint32_t grid_cap, uint64_t word_cap, GridDesc* grids, Segment* segs,
                                  uint32_t* nseg_ptr) {
  const uint32_t nl = build_stopped(bs) ? 0u : *nlist_ptr;
  const uint32_t first_grid = bs->num_grids;
  const uint64_t slot_base = bs->used_words;
  const uint64_t gw = grid_words(E);
  const bool fits = (uint64_t)first_grid + nl <= grid_cap && slot_base + (uint64_t)nl * gw <= word_cap;
  const uint32_t r0 = blockIdx.x * blockDim.x + threadIdx.x;
  if (r0 == 0) {
    *nseg_ptr = fits ? nl : 0u;
    if (nl) {
      atomicAdd(&bs->need_grids, nl);
      atomicAdd((unsigned long long*)&bs->need_words, (unsigned long long)((uint64_t)nl * gw));
    }
    if (!fits) atomicOr(&bs->overflow, (uint32_t)kOverGrids);
  }
  if (!fits) return;
  for (uint32_t r = r0; r < nl; r += gridDim.x * blockDim.x) {
    const uint32_t n = list[r];
    const uint32_t gi = first_grid + r;
    Segment sg;
    sg.start = (uint32_t)nodes.offset[n];
    sg.count = nodes.npoints[n];
    sg.grid = gi;
    sg.level = nodes.level[n];
    sg.chunk_begin = 0;
    sg.chunk_count = 0;
    sg.key = nodes.key[n];
    sg.group_begin = 0;
    sg.group_count = 0;
    sg.cloud = nodes.tree[n];
    sg.pad = 0;
    segs[r] = sg;
    GridDesc d;
    d.base_level = sg.level;
    d.e = E;
    d.base_key = sg.key;
    d.pyr = slot_base + (uint64_t)r * gw;
    d.off = d.pyr + pyr_level_offset(E + 1);
    d.child = d.off + ((uint64_t)1 << (3 * E));
    d.seg_start = sg.start;
    d.seg_count = sg.count;
    grids[gi] = d;
    nodes.grid[n] = (int32_t)gi;
  }
}

// The refined grids are in use: advance the grid and pool counters.
__global__ void k_refine_commit(BuildState* bs, const uint32_t* nseg_ptr, uint32_t E) {
  const uint32_t n = *nseg_ptr;
  bs->num_grids += n;
  bs->used_words += (uint64_t)n * grid_words(E);
}

// Where every tree's nodes go in the compact node table (one workgroup): a
// tree's nodes move from its region of slots to [node_base, node_base +
// num_nodes), node_base the prefix sum of the node counts; with a single
// tree the region already starts at slot 0 and nothing moves.  Also the
// level ranges (compact numbering), the deepest level, the first point of
// the tree's cloud, and the total in bs->total_nodes.
constexpr int kInfoWG = 1024;
__global__ void __launch_bounds__(kInfoWG) k_tree_info(const TreeState* __restrict__ sts, const CloudInfo* __restrict__ clouds,
                                                       uint32_t ntrees, TreeInfo* trees, BuildState* bs) {
  __shared__ uint32_t sh[kInfoWG / 64 + 1];
  uint32_t base = 0;
  for (uint32_t c0 = 0; c0 < ntrees; c0 += kInfoWG) {
    const uint32_t c = c0 + threadIdx.x;
    uint32_t n = 0;
    if (c < ntrees) n = sts[c].num_nodes - sts[c].node_begin;
    uint32_t tot;
    const uint32_t ex = block_excl_scan<kInfoWG>(n, sh, &tot);
    if (c < ntrees) {
      const TreeState& ts = sts[c];
      TreeInfo ti;
      ti.node_base = ntrees == 1 ? ts.node_begin : base + ex;
      ti.num_nodes = n;
      ti.point_base = clouds[c].start;
      ti.deepest = 0;
      const uint32_t shift = ti.node_base - ts.node_begin;
      for (int L = 0; L < 23; ++L) {
        if (ts.level_end[L] > ts.level_begin[L]) {
          ti.level_begin[L] = ts.level_begin[L] + shift;
          ti.level_end[L] = ts.level_end[L] + shift;
          ti.deepest = (uint32_t)L;
        } else {
          ti.level_begin[L] = ti.level_end[L] = 0;
        }
      }
      ti.vbase = 0;
      ti.vtotal = 0;
      trees[c] = ti;
    }
    base += tot;
  }
  if (threadIdx.x == 0) bs->total_nodes = base;
}

// Tree of compact node i: the last tree whose first node is <= i.
__device__ __forceinline__ uint32_t node_tree(const TreeInfo* __restrict__ trees, uint32_t ntrees, uint32_t i) {
  uint32_t lo = 0, hi = ntrees;
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) / 2;
    if (trees[mid].node_base <= i) lo = mid;
    else hi = mid;
  }
  return lo;
}

// Move every tree's nodes from its capacity region to its compact range
// [node_base, node_base + num_nodes), shifting node references.
__global__ void k_compact_nodes(Nodes src, Nodes dst, const TreeInfo* __restrict__ trees,
                                const uint32_t* __restrict__ cap_begin, uint32_t ntrees, const BuildState* bs) {
  if (build_stopped(bs)) return;
  const uint32_t total = bs->total_nodes;
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < total; i += gridDim.x * blockDim.x) {
  const uint32_t c = node_tree(trees, ntrees, i);
  const uint32_t nb = trees[c].node_base;
  const uint32_t j = cap_begin[c] + (i - nb);
  const uint32_t shift = nb - cap_begin[c];  // modular: references move by the same amount
  const bool leaf = src.is_leaf[j] != 0;
  dst.level[i] = src.level[j];
  dst.is_leaf[i] = src.is_leaf[j];
  dst.child_mask[i] = src.child_mask[j];
  dst.key[i] = src.key[j];
  dst.npoints[i] = src.npoints[j];
  dst.count[i] = src.count[j];
  dst.first_child[i] = leaf ? 0u : src.first_child[j] + shift;
  dst.offset[i] = src.offset[j];
  dst.cover[i] = src.cover[j];
  dst.grid[i] = src.grid[j];
  const uint32_t par = src.parent[j];
  dst.parent[i] = par == 0xffffffffu ? par : par + shift;
  dst.tree[i] = src.tree[j];
  }
}

// Output node table: per-tree node indices and per-tree point / voxel offsets.
__global__ void k_finalize_nodes(Nodes nodes, const TreeInfo* __restrict__ trees, const BuildState* bs,
                                 uint8_t* o_level, uint8_t* o_leaf, uint8_t* o_mask, uint64_t* o_key,
                                 uint32_t* o_npts, uint32_t* o_count, uint32_t* o_first, uint64_t* o_off) {
  if (build_stopped(bs)) return;
  const uint32_t total = bs->total_nodes;
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < total; i += gridDim.x * blockDim.x) {
  const TreeInfo& ti = trees[nodes.tree[i]];
  const bool leaf = nodes.is_leaf[i] != 0;
  o_level[i] = nodes.level[i];
  o_leaf[i] = nodes.is_leaf[i];
  o_mask[i] = nodes.child_mask[i];
  o_key[i] = nodes.key[i];
  o_npts[i] = nodes.npoints[i];
  o_count[i] = nodes.count[i];
  o_first[i] = leaf ? 0u : nodes.first_child[i] - ti.node_base;
  o_off[i] = leaf ? nodes.offset[i] - ti.point_base : nodes.offset[i];
  }
}

static uint32_t node_blocks(uint32_t max_nodes) {
  return std::max<uint32_t>(1, std::min<uint32_t>((max_nodes + 255) / 256, 4096));
}

void launch_compact_nodes(const Nodes& src, const Nodes& dst, const TreeInfo* trees, const uint32_t* cap_begin,
                          uint32_t ntrees, uint32_t max_nodes, const BuildState* bs, hipStream_t s) {
  hipLaunchKernelGGL(k_compact_nodes, dim3(node_blocks(max_nodes)), dim3(256), 0, s, src, dst, trees, cap_begin,
                     ntrees, bs);
}

void launch_finalize_nodes(const Nodes& nodes, const TreeInfo* trees, uint32_t max_nodes, const BuildState* bs,
                           uint8_t* o_level, uint8_t* o_leaf, uint8_t* o_mask, uint64_t* o_key, uint32_t* o_npts,
                           uint32_t* o_count, uint32_t* o_first, uint64_t* o_off, hipStream_t s) {
  hipLaunchKernelGGL(k_finalize_nodes, dim3(node_blocks(max_nodes)), dim3(256), 0, s, nodes, trees, bs, o_level,
                     o_leaf, o_mask, o_key, o_npts, o_count, o_first, o_off);
}

void launch_tree_init(uint32_t leaf_cap, uint32_t max_level, const GridDesc* grids, const uint32_t* pool,
                      const Nodes& nodes, TreeState* sts, const uint32_t* node_begin, const uint32_t* node_end,
                      uint32_t nclouds, hipStream_t s) {
  hipLaunchKernelGGL(k_tree_init, dim3((nclouds + 255) / 256), dim3(256), 0, s, leaf_cap, max_level, grids, pool, nodes,
                     sts, node_begin, node_end, nclouds);
}

void launch_tree_build(uint32_t leaf_cap, uint32_t max_level, const GridDesc* grids, const uint32_t* pool,
                       const Nodes& nodes, TreeState* sts, uint32_t nclouds, uint32_t* refine, uint32_t* leaf_refine,
                       BuildState* bs, hipStream_t s) {
  hipLaunchKernelGGL(k_tree_build, dim3(nclouds), dim3(kTreeWG), 0, s, leaf_cap, max_level, grids, pool, nodes, sts,
                     refine, leaf_refine, bs);
}

void launch_refine_segments(const Nodes& nodes, const uint32_t* list, const uint32_t* nlist, uint32_t max_list,
                            uint32_t E, BuildState* bs, uint32_t grid_cap, uint64_t word_cap, GridDesc* grids,
                            Segment* segs, uint32_t* nseg, hipStream_t s) {
  const uint32_t blocks = std::max<uint32_t>(1, std::min<uint32_t>((max_list + 255) / 256, 1024));
  hipLaunchKernelGGL(k_refine_segments, dim3(blocks), dim3(256), 0, s, nodes, list, nlist, E, bs, grid_cap, word_cap,
                     grids, segs, nseg);
}

void launch_refine_commit(BuildState* bs, const uint32_t* nseg, uint32_t E, hipStream_t s) {
  hipLaunchKernelGGL(k_refine_commit, dim3(1), dim3(1), 0, s, bs, nseg, E);
}

void launch_tree_info(const TreeState* sts, const CloudInfo* clouds, uint32_t ntrees, TreeInfo* trees, BuildState* bs,
                      hipStream_t s) {
  hipLaunchKernelGGL(k_tree_info, dim3(1), dim3(kInfoWG), 0, s, sts, clouds, ntrees, trees, bs);
}

}  // namespace lod
