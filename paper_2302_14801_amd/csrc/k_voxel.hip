// k_voxel.hip -- bottom-up voxel sampling of inner nodes (Sec. 4.2).
//
// Every inner node A at level L gets the occupied cells of its 128^3 grid
// (cells at level L + 7, Fig. 1).  Sampling is hierarchical: the samples of a
// cell of A are the points of a leaf child, or the voxels of an inner child
// (Sec. 4.2.1-4.2.3), so a cell of A holds one sample per occupied sub-cell
// of the level below.  Two consequences shape the gfx950 design:
//
//   * Inside the region of a leaf at level l, the cells of every ancestor at
//     depth k = 1..6 above it (levels l + 7 - k, all finer than the leaf)
//     depend on the leaf's own points only.  One kernel therefore computes,
//     for every leaf, its contributions to all of those ancestors at once,
//     level after level in LDS and registers, instead of one pass per level.
//   * A node N exactly 7 levels below A is a single cell of A's grid; its
//     "self voxel" reduces the self voxels of N's children (for a leaf, the
//     voxels of its 8 child cells).
// The voxel list of A is thus a sequence, in Morton order, of pieces: the
// depth-(l - L) list of each leaf below A with l <= L + 6, and the self voxel
// of each node at level L + 7 below A.  In a depth-first order of the tree,
// A's pieces are the qualifying nodes of A's subtree range, already in Morton
// order, so their offsets are block-wide prefix sums over that range.  Voxel
// lists come out sorted by cell, and the output is fully deterministic.
//
// Stages (each launched once per build, whatever the depth of the tree):
//   k_item_desc      descriptor and coarse-list space of every (leaf, child
//                    cell) work item; in the average modes also the list of
//                    items for the sparse kernel
//   k_leaf_sparse    average modes: the depth 1..6 lists of the items that fit
//                    its LDS (occupancy mask, ranks, one accumulator per
//                    occupied cell)
//   k_leaf_voxels    the depth 1..6 lists of every item (average modes: of the
//                    items the sparse kernel leaves)
//   k_piece_sizes    piece sizes of every node; self voxels of deep leaves
//   k_vox_tree       subtree sizes, depth-first order, inner self voxels
//   k_piece_count    voxel count of every inner node
//   k_voxel_offsets  voxel offset of every inner node (node order)
//   k_piece_offsets  output position of every piece; writes the self voxels
//   k_gather         copies every item's lists to their output positions
#include "common.h"
#include "launch.h"
#include "scan.h"

#include <algorithm>

namespace lod {

constexpr int kLeafWG = 256;
constexpr uint32_t kSubCells = 4096;    // cells of a micro-bucket at depth 1 (4 levels = 12 bits)
constexpr uint32_t kPackedMax = 65535;  // largest micro-bucket the packed 16-bit fields can hold
constexpr uint32_t kLeafSlots = 8;      // points per thread per pass
constexpr uint32_t kLeafPass = kLeafWG * kLeafSlots;
constexpr uint32_t kNoCell = 0xffffffffu;
constexpr uint64_t kMaxOneItemBlocks = 1ull << 22;  // workgroups of the one-item leaf launch (2^30 threads)
constexpr uint32_t kCodeMask = (1u << 21) - 1;
constexpr uint32_t kListCap = 3072;  // occupied depth-1 cells of a micro-bucket the shared list holds
// the sparse leaf kernel of the average modes (k_leaf_sparse)
constexpr int kSpWG = 512;                          // 8 waves
constexpr uint32_t kSpSlots = 16;                   // points per thread
constexpr uint32_t kSpMaxPts = kSpWG * kSpSlots;    // 8192
constexpr uint32_t kSpWords = 32768 / 32;           // occupancy words of an item
// occupied cells of all depths an item may have (LDS: 10 B each, 14 B in mode 3)
__host__ __device__ constexpr uint32_t sp_cap(int mode) { return mode == 3 ? 4096u : 6144u; }
constexpr uint32_t kSpNone = 0xffffu;               // no point in a slot

// Cells of one work item (a leaf's child cell) in the grid of the ancestor
// k = 1..6 levels above the leaf: 8^(6-k).
__host__ __device__ __forceinline__ uint32_t item_cells(uint32_t k) { return 1u << (3 * (6 - k)); }
// Start of the depth-k list (k = 2..6) in an item's block of coarse lists;
// k = 7 gives the size of the block.  p = points of the item (no list is
// longer than the item's points or cells).
__host__ __device__ __forceinline__ uint32_t coarse_base(uint32_t k, uint32_t p) {
  uint32_t b = 0;
  for (uint32_t j = 2; j < k; ++j) b += p < item_cells(j) ? p : item_cells(j);
  return b;
}
// Code of a cell in the grid of the ancestor k levels above a leaf (a cell at
// level l + 7 - k): the leaf's key extended by 3*(7-k) bits of position inside
// the leaf, cut to the grid's 21 bits.
__device__ __forceinline__ uint32_t anc_code(uint64_t leaf_key, uint32_t k, uint32_t rel) {
  return (uint32_t)(((leaf_key << (3 * (7 - k))) | rel) & kCodeMask);
}

// floor(sum / n) for 1 <= n <= 257 and sum <= 255 n (the mean of 8-bit
// values), from r = rcp(n) (relative error at most 2^-23): the computed
// sum * r + 2^-10 lies within 2^-14 of sum / n + 2^-10 (each rounding is below
// 2^-17 for values under 256).  The true quotient is either an integer q,
// which gives a value in (q, q + 2^-9), or at least 1/n >= 1/257 below the next
// integer, which 2^-10 + 2^-14 does not reach; truncation is exact either way.
// (n < 2^23 is converted through the mantissa: the compiler otherwise widens
// a count taken from the top bits of a 64-bit word into a 64-bit conversion)
__device__ __forceinline__ float rcp_count(uint32_t n) {
  return __builtin_amdgcn_rcpf(__uint_as_float(0x4b000000u | n) - 8388608.0f);
}
__device__ __forceinline__ uint32_t floor_div(uint32_t sum, float r) {
  return (uint32_t)__fadd_rn(__fmul_rn((float)sum, r), 0x1p-10f);
}
__device__ __forceinline__ uint32_t mean_rgba(uint32_t sr, uint32_t sg, uint32_t sb, uint32_t n) {
  const float r = rcp_count(n);
  return floor_div(sr, r) | (floor_div(sg, r) << 8) | (floor_div(sb, r) << 16) | (255u << 24);
}

// Modes of the voxel stage: 0 average, 1 first, 2 random (the sampling
// strategies), 3 average that also keeps the smallest sample id of every cell
// (the accepted sample of a full-precision lower level).
__host__ __device__ constexpr bool avg_mode(int m) { return m == 0 || m == 3; }

// Samples of one cell: channel sums and count (average modes; mode 3 also the
// smallest id, 2^32 - 1 while empty), or the pick so far (pick modes; n > 0
// marks it valid).
template <int MODE>
struct Smp {
  uint32_t r, g, b, n;
  uint64_t ok;  // order key of the pick; its low 32 bits are the id
  uint32_t col;
};
template <int MODE>
__device__ __forceinline__ Smp<MODE> smp_empty() {
  Smp<MODE> s;
  s.r = s.g = s.b = s.n = 0;
  s.ok = MODE == 3 ? 0xffffffffull : 0ull;
  s.col = 0;
  return s;
}
template <int MODE>
__device__ __forceinline__ bool pick_better(uint64_t a, uint64_t b) {
  return MODE == 1 ? a < b : a > b;
}
// one voxel (colour, id) as a sample
template <int MODE>
__device__ __forceinline__ void smp_add(Smp<MODE>& s, uint32_t rgba, uint32_t id, uint32_t seed) {
  if (avg_mode(MODE)) {
    s.r += rgba & 0xffu;
    s.g += (rgba >> 8) & 0xffu;
    s.b += (rgba >> 16) & 0xffu;
    if (MODE == 3) s.ok = min(s.ok, (uint64_t)id);
  } else {
    const uint64_t k = pick_order(id, seed, MODE == 2);
    if (s.n == 0 || pick_better<MODE>(k, s.ok)) {
      s.ok = k;
      s.col = rgba;
    }
  }
  s.n += 1;
}
template <int MODE>
__device__ __forceinline__ void smp_merge(Smp<MODE>& a, const Smp<MODE>& b) {
  if (avg_mode(MODE)) {
    a.r += b.r;
    a.g += b.g;
    a.b += b.b;
    if (MODE == 3) a.ok = min(a.ok, b.ok);
  } else if (b.n && (a.n == 0 || pick_better<MODE>(b.ok, a.ok))) {
    a.ok = b.ok;
    a.col = b.col;
  }
  a.n += b.n;
}
// merge with the samples of lane ^ m (every lane of the wave executes this)
// (average: sums of at most 8 voxels, so two 16-bit fields share a word)
template <int MODE>
__device__ __forceinline__ void smp_xor(Smp<MODE>& s, int m) {
  if (avg_mode(MODE)) {
    const uint32_t rg = (uint32_t)__shfl_xor((int)(s.r | (s.g << 16)), m, 64);
    const uint32_t bn = (uint32_t)__shfl_xor((int)(s.b | (s.n << 16)), m, 64);
    s.r += rg & 0xffffu;
    s.g += rg >> 16;
    s.b += bn & 0xffffu;
    s.n += bn >> 16;
    if (MODE == 3) s.ok = min(s.ok, (uint64_t)(uint32_t)__shfl_xor((int)(uint32_t)s.ok, m, 64));
  } else {
    Smp<MODE> o = smp_empty<MODE>();
    o.n = __shfl_xor(s.n, m, 64);
    o.ok = __shfl_xor(s.ok, m, 64);
    o.col = __shfl_xor(s.col, m, 64);
    smp_merge<MODE>(s, o);
  }
}
// Lane exchanges without the LDS crossbar: DPP (quad permutations, rotations
// within a row of 16 lanes) and, across the two rows of a half-wave, a
// swizzle.  Used for all-lane reductions, where the order of the merges does
// not matter (sums are exact, picks are min/max).
template <int CTRL>
__device__ __forceinline__ uint32_t dpp_get(uint32_t x) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, CTRL, 0xf, 0xf, false);
}
constexpr int kQuadXor1 = 0xB1;   // quad_perm [1,0,3,2]
constexpr int kQuadXor2 = 0x4E;   // quad_perm [2,3,0,1]
constexpr int kRowRor1 = 0x121;   // row_ror:n = 0x120 + n
constexpr int kRowRor2 = 0x122;
constexpr int kRowRor4 = 0x124;
constexpr int kRowRor8 = 0x128;
constexpr int kRowShr1 = 0x111;   // row_shr:n = 0x110 + n
constexpr int kRowShr2 = 0x112;
constexpr int kRowShr4 = 0x114;
constexpr int kRowShr8 = 0x118;
constexpr int kSwap16 = 0x10000 | 0x401F;  // ds_swizzle: lane ^ 16 within 32 lanes
template <int CTRL>
__device__ __forceinline__ uint32_t lane_get(uint32_t x) {
  if constexpr (CTRL >= 0x10000) return (uint32_t)__builtin_amdgcn_ds_swizzle((int)x, CTRL & 0xffff);
  else return dpp_get<CTRL>(x);
}
// merge with the samples of the lane selected by CTRL (every lane executes this)
template <int MODE, int CTRL>
__device__ __forceinline__ void smp_lane(Smp<MODE>& s) {
  if (avg_mode(MODE)) {
    const uint32_t rg = lane_get<CTRL>(s.r | (s.g << 16));
    const uint32_t bn = lane_get<CTRL>(s.b | (s.n << 16));
    s.r += rg & 0xffffu;
    s.g += rg >> 16;
    s.b += bn & 0xffffu;
    s.n += bn >> 16;
    if (MODE == 3) s.ok = min(s.ok, (uint64_t)lane_get<CTRL>((uint32_t)s.ok));
  } else {
    Smp<MODE> o = smp_empty<MODE>();
    o.n = lane_get<CTRL>(s.n);
    o.ok = (uint64_t)lane_get<CTRL>((uint32_t)s.ok) | ((uint64_t)lane_get<CTRL>((uint32_t)(s.ok >> 32)) << 32);
    o.col = lane_get<CTRL>(s.col);
    smp_merge<MODE>(s, o);
  }
}
// Inclusive prefix sum over the wave (row scans by shifts, then the row
// totals carried by broadcasts of lanes 15 and 31).
__device__ __forceinline__ uint32_t wave_incl_scan_dpp(uint32_t x) {
  x += dpp_get<kRowShr1>(x);
  x += dpp_get<kRowShr2>(x);
  x += dpp_get<kRowShr4>(x);
  x += dpp_get<kRowShr8>(x);
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x142, 0xa, 0xf, false);  // row_bcast:15 -> rows 1, 3
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x143, 0xc, 0xf, false);  // row_bcast:31 -> rows 2, 3
  return x;
}
// Sum over each row of 16 lanes, in every lane of the row.
__device__ __forceinline__ uint32_t row_sum_dpp(uint32_t x) {
  x += dpp_get<kRowRor8>(x);
  x += dpp_get<kRowRor4>(x);
  x += dpp_get<kRowRor2>(x);
  x += dpp_get<kRowRor1>(x);
  return x;
}

// the cell's voxel colour: floor of the mean per channel with A = 255
// (sums of at most 8 voxels here), or the pick's colour
template <int MODE>
__device__ __forceinline__ uint32_t smp_rgba(const Smp<MODE>& s) {
  if (avg_mode(MODE)) return mean_rgba(s.r, s.g, s.b, s.n);
  return s.col;
}

// Coordinates of a depth-1 cell inside its micro-bucket from its 12-bit
// Morton index: x | y << 8 | z << 16, 4 bits each.
__device__ __forceinline__ uint32_t cell_xyz(uint32_t sc) {
  auto c4 = [](uint32_t v) { return (v & 1u) | ((v >> 2) & 2u) | ((v >> 4) & 4u) | ((v >> 6) & 8u); };
  return c4(sc) | (c4(sc >> 1) << 8) | (c4(sc >> 2) << 16);
}

// Exclusive prefix over the wave of counts below 2^BITS: one ballot per bit.
template <int BITS>
__device__ __forceinline__ uint32_t wave_prefix_small(uint32_t c) {
  const uint64_t below = (1ull << lane_id()) - 1;
  uint32_t r = 0;
#pragma unroll
  for (int b = 0; b < BITS; ++b) r += (uint32_t)__popcll(__ballot((c >> b) & 1u) & below) << b;
  return r;
}

// Point range of work item (leaf n, child cell grp) and what is needed to
// find its micro-buckets (cells two levels below the leaf) in the leaf's grid.
struct Item {
  GridDesc G;
  uint32_t rm;    // micro-bucket level relative to the grid
  uint64_t mb0;   // index of the item's first micro-bucket at that level
  uint32_t fine;  // 3 * (G.e - rm): micro-bucket index -> finest-cell index
  uint32_t I0, I1;
};
__device__ __forceinline__ Item item_of(const Nodes& nodes, uint32_t n, uint32_t grp, const GridDesc* __restrict__ grids,
                                        const uint32_t* __restrict__ pool) {
  Item it;
  const uint32_t lvl = nodes.level[n];
  const int32_t gi = nodes.grid[n] >= 0 ? nodes.grid[n] : nodes.cover[n];
  it.G = grids[gi];
  it.rm = lvl + 2 - it.G.base_level;
  const uint64_t leaf_rel = nodes.key[n] - (it.G.base_key << (3 * (lvl - it.G.base_level)));
  it.mb0 = (leaf_rel << 6) | ((uint64_t)grp << 3);
  it.fine = 3 * (it.G.e - it.rm);
  it.I0 = pool[it.G.off + (it.mb0 << it.fine)];
  it.I1 = it.I0 + pool[it.G.pyr + pyr_level_offset(it.rm - 1) + (it.mb0 >> 3)];  // points of the child cell
  return it;
}

// ------------------------------------------------------------ item descriptors
//
// One thread per item.  Coarse-list blocks are handed out by a wave-wide
// prefix sum and one atomic add per wave on bs->coarse_used.  With `sparse`
// (the average modes) the item is also routed: an empty item gets its list
// lengths (all zero) here, an item of at most kSpMaxPts points goes on the
// sparse kernel's list, a larger one on the general kernel's (`redo`); both
// lists are filled with one atomic add per wave.
__device__ __forceinline__ void wave_append(bool take, uint32_t value, uint32_t* ctr, uint32_t* list) {
  const uint64_t m = __ballot(take);
  if (!m) return;
  const uint32_t leader = (uint32_t)__ffsll((unsigned long long)m) - 1;
  uint32_t base = 0;
  if (lane_id() == leader) base = atomicAdd(ctr, (uint32_t)__popcll(m));
  base = __shfl(base, leader, 64);
  if (take) list[base + (uint32_t)__popcll(m & ((1ull << lane_id()) - 1))] = value;
}
__global__ void __launch_bounds__(256) k_item_desc(Nodes nodes, const GridDesc* __restrict__ grids,
                                                   const uint32_t* __restrict__ pool, BuildState* bs,
                                                   ItemDesc* __restrict__ desc, uint64_t t2cap, bool sparse,
                                                   uint32_t* __restrict__ icnt, uint32_t* __restrict__ slist,
                                                   uint32_t* __restrict__ redo) {
  if (build_stopped(bs)) return;
  const uint32_t nitems = 8u * bs->total_nodes;
  for (uint32_t i0 = blockIdx.x * 256; i0 < nitems; i0 += gridDim.x * 256) {  // uniform per workgroup
  const uint32_t i = i0 + threadIdx.x;
  const bool valid = i < nitems;
  ItemDesc d;
  d.I0 = d.P = d.lvl = d.tree = 0;
  d.lkey = 0;
  for (uint32_t j = 0; j < 8; ++j) d.mc[j] = 0;
  if (valid) {
    const uint32_t n = i >> 3;
    if (nodes.is_leaf[n] && nodes.level[n] != 0) {
      const Item it = item_of(nodes, n, i & 7u, grids, pool);
      d.I0 = it.I0;
      d.P = it.I1 - it.I0;
      d.lvl = nodes.level[n];
      d.tree = nodes.tree[n];
      d.lkey = nodes.key[n];
      const uint32_t* mcnt = pool + it.G.pyr + pyr_level_offset(it.rm);
      for (uint32_t j = 0; j < 8; ++j) d.mc[j] = mcnt[it.mb0 | j];
    }
  }
  const uint64_t sz = coarse_base(7, d.P);
  const uint64_t incl = wave_incl_scan(sz);
  const uint64_t total = __shfl(incl, 63, 64);
  uint64_t base = 0;
  if (lane_id() == 63 && total) {
    base = atomicAdd((unsigned long long*)&bs->coarse_used, (unsigned long long)total);
    // the pool is an estimate: past it the build stops and is repeated
    if (base + total > t2cap) atomicOr(&bs->overflow, (uint32_t)kOverCoarse);
  }
  base = __shfl(base, 63, 64);
  d.t2 = base + incl - sz;
  if (valid) {
    const uint4* src = (const uint4*)&d;
    uint4* dst = (uint4*)(desc + i);
    for (int k = 0; k < 4; ++k) dst[k] = src[k];
  }
  if (sparse) {
    if (valid && d.P == 0)
      for (int k = 0; k < 6; ++k) icnt[6ull * i + k] = 0;
    wave_append(valid && d.P != 0 && d.P <= kSpMaxPts, i, &bs->sparse_items, slist);
    wave_append(valid && d.P > kSpMaxPts, i, &bs->redo_items, redo);
  }
  }
}

// ------------------------------------------------------------ leaf kernel
//
// A work item is one leaf and one of its 8 child cells (8 micro-buckets), so
// that large leaves spread over 8 workgroups.  Its points are contiguous and
// sorted by micro-bucket.  They are read in passes of kLeafPass points, every
// thread issuing all of its loads of a pass at once, and each point is kept
// in registers as (15-bit cell within the child cell, colour, id).  The
// micro-buckets are then reduced one after the other into a directly indexed
// LDS array of the 4096 depth-1 cells (parent's grid) of one micro-bucket,
// with one 64-bit LDS atomic per point:
//   average: acc[cell] += R | G << 16 | B << 32 | 1 << 48.  The 16-bit fields
//            are exact while a cell holds at most 257 samples (255 * 257 <
//            2^16); overflowing fields only carry upward, so a cell with
//            more samples shows a count above 257 (see below).
//   pick:    acc[cell] = min/max of the sample's order key, whose low 32 bits
//            are the point id; the winner then replaces it by its colour and
//            id (ids are unique, so no other point can match afterwards).
//   mode 3:  as average, plus a 32-bit LDS atomic min of the id per cell.
// Every sample also sets its cell's bit in an occupancy bitmask of the 4096
// depth-1 cells (two masks alternate between micro-buckets, so one is
// cleared while the other fills).  After the barrier every wave reads the
// whole mask and counts the occupied cells of each depth (a depth-2 cell is
// a nonzero byte, a depth-3 cell a nonzero pair of words, a depth-4 cell
// eight of those) in the earlier waves' quarters and in total (DPP row sums),
// and its own lanes' counts before them (a DPP wave scan), so that all list
// positions follow without any counting during the accumulation.  The
// emission (thread t owns depth-1 cells 16t .. 16t+15, i.e. depth-2 cells 2t
// and 2t+1) writes the depth-1 voxels and reduces them upward through
// registers and DPP lane exchanges: depth 2 in the thread, depth 3 over 4
// lanes, depth 4 over 32 lanes.  Depth 5 (the micro-bucket) and 6 (the item)
// are reduced at the end.  An average cell seen with more than 257
// samples sends its micro-bucket to a second, exact round.
// Depth-1 lists go to T1 at the item's first point (never more voxels than
// points), the coarse lists to the item's block in T2.  icnt receives the 6
// list lengths and iself the depth-6 voxel (colour, id) of every item.
// Workgroup b takes work item item0 + b; with LOOP also item0 + b + gridDim.x,
// ... (a loop over items keeps more registers live: the one-item form is the
// fast one, launched over the expected number of items, and the looping form
// takes whatever items lie beyond it).  With `list`, the indices are positions
// in that list of items (bs->redo_items of them) instead of items.
template <int MODE, bool LOOP>  // MODE: 0 average, 1 first, 2 random, 3 average with smallest ids
__global__ void __launch_bounds__(kLeafWG, MODE == 0 ? 4 : 1) k_leaf_voxels(const ItemDesc* __restrict__ desc,
                                                                          const uint4* __restrict__ pts,
                                                                          const uint32_t* __restrict__ ids,
                                                                          const Cube* cube, uint64_t* __restrict__ T1,
                                                                          uint32_t* __restrict__ T1id,
                                                                          uint64_t* __restrict__ T2,
                                                                          uint32_t* __restrict__ T2id,
                                                                          uint32_t* __restrict__ icnt,
                                                                          uint64_t* __restrict__ iself, uint32_t seed,
                                                                          const BuildState* bs, uint32_t item0,
                                                                          const uint32_t* __restrict__ list) {
  __shared__ uint64_t acc[kSubCells];
  __shared__ uint32_t bm1[2][kSubCells / 32];  // depth-1 occupancy, alternating between micro-buckets
  __shared__ uint32_t over[8];                 // a cell of the micro-bucket passed 257 samples
  __shared__ uint32_t k4m[8];                  // occupied depth-4 cells of each micro-bucket
  __shared__ uint64_t k4ok[8][8];              // depth-4 voxels of each micro-bucket: pick key and colour
  __shared__ uint32_t k4col[8][8];
  __shared__ uint32_t minid[MODE == 3 ? kSubCells : 1];  // mode 3: smallest id of every depth-1 cell
  __shared__ uint16_t clist[avg_mode(MODE) ? kListCap : 1];  // occupied depth-1 cells in Morton order
  const uint32_t t = threadIdx.x, w = t >> 6, l = lane_id();
  if (build_stopped(bs)) return;
  // all work items, or (list) the ones the sparse kernel handed over
  const uint32_t nitems = list ? bs->redo_items : 8u * bs->total_nodes;
  for (uint32_t li = item0 + blockIdx.x; li < nitems; li += gridDim.x) {
  const uint32_t item = list ? list[li] : li;
  if (LOOP) __syncthreads();  // the previous item's reads of LDS are done
  const ItemDesc& sd = desc[item];  // uniform: scalar loads
  const uint32_t P = sd.P;
  if (P == 0) {  // an empty child cell, or not a leaf item (uniform)
    if (t < 6) icnt[6 * item + t] = 0;
    if (LOOP) continue;
    return;
  }
  const uint64_t init = MODE == 1 ? ~0ull : 0ull;
  for (uint32_t i = t; i < kSubCells; i += kLeafWG) acc[i] = init;
  if (MODE == 3)
    for (uint32_t i = t; i < kSubCells; i += kLeafWG) minid[i] = ~0u;
  if (t < kSubCells / 32) {
    bm1[0][t] = 0;
    bm1[1][t] = 0;
  }
  if (t < 8) {
    k4m[t] = 0;
    over[t] = 0;
  }
  const CubeD cd = load_cube(cube + sd.tree);
  __syncthreads();
  const uint32_t I0 = sd.I0, I1 = I0 + P, lvl = sd.lvl, grp = item & 7u;
  const uint64_t lkey = sd.lkey, t2b = sd.t2;
  const uint32_t sub_bit = 15u - lvl;  // bit level of the depth-1 cells (level lvl + 6)
  const uint32_t cb3 = coarse_base(3, P), cb4 = coarse_base(4, P), cb5 = coarse_base(5, P), cb6 = coarse_base(6, P);
  const uint64_t below = (1ull << l) - 1;  // lanes under this one
  // Voxel coordinates.  A depth-1 cell has global coordinates (X, Y, Z) at
  // level lvl + 6; the ancestor k levels up holds it in its cell with
  // coordinates (X, Y, Z) >> (k - 1), taken mod 128.  X = the leaf's
  // coordinates << 6 | micro-bucket << 4 | the thread's part | the cell's
  // part (thread t owns cells 16t .. 16t+15: Morton bits 4..11 of the cell
  // index are t, bits 0..3 the cell within the thread).
  const uint32_t X0 = compact21(lkey), Y0 = compact21(lkey >> 1), Z0 = compact21(lkey >> 2);
  const uint32_t xt = (((t >> 2) & 1u) << 2) | (((t >> 5) & 1u) << 3);
  const uint32_t yt = ((t & 1u) << 1) | (((t >> 3) & 1u) << 2) | (((t >> 6) & 1u) << 3);
  const uint32_t zt = (((t >> 1) & 1u) << 1) | (((t >> 4) & 1u) << 2) | (((t >> 7) & 1u) << 3);
  auto vox_at = [](uint32_t sh, uint32_t X, uint32_t Y, uint32_t Z, uint32_t rgba) -> uint64_t {
    return (uint64_t)(((X >> sh) & 127u) | (((Y >> sh) & 127u) << 8) | (((Z >> sh) & 127u) << 16)) |
           ((uint64_t)rgba << 32);
  };
  uint32_t base1 = 0, base2 = 0, base3 = 0, base4 = 0;  // list lengths so far
  uint32_t nproc = 0;                                   // micro-buckets emitted so far (bitmask alternation)
  for (uint32_t P0 = I0; P0 < I1; P0 += kLeafPass) {
    const uint32_t P1 = min(P0 + kLeafPass, I1);
    uint32_t cell[kLeafSlots], col[kLeafSlots], pid[kLeafSlots];
    {
      uint4 v[kLeafSlots];
#pragma unroll
      for (uint32_t k = 0; k < kLeafSlots; ++k) {
        const uint32_t i = P0 + k * kLeafWG + t;
        if (i < P1) {
          v[k] = pts[i];
          if (MODE) pid[k] = ids[i];
        }
      }
#pragma unroll
      for (uint32_t k = 0; k < kLeafSlots; ++k) {
        const uint32_t i = P0 + k * kLeafWG + t;
        cell[k] = kNoCell;
        if (i < P1) {
          cell[k] = point_cell(__uint_as_float(v[k].x), __uint_as_float(v[k].y), __uint_as_float(v[k].z), cd, sub_bit, 5);
          col[k] = v[k].w;
        }
      }
    }
    uint32_t next = I0;  // first point of the next micro-bucket
    for (uint32_t jm = 0; jm < 8; ++jm) {
      const uint32_t cnt = sd.mc[jm];
      const uint32_t off = next;
      next += cnt;
      if (cnt == 0) continue;
      if (off >= P1 || off + cnt <= P0) continue;  // no points in this pass
      const bool wide = avg_mode(MODE) && cnt > kPackedMax;
      uint32_t* occ = bm1[nproc & 1];
      if (!wide) {
        // every sample: one LDS reduction on its cell and one occupancy bit
        // (no returned values, so nothing waits)
#pragma unroll
        for (uint32_t k = 0; k < kLeafSlots; ++k) {
          // slots whose points all lie outside the micro-bucket (a uniform test:
          // the points are sorted by micro-bucket)
          const uint32_t pk = P0 + k * kLeafWG;
          if (pk >= off + cnt || pk + kLeafWG <= off) continue;
          // keep the per-slot work inside the loop over micro-buckets (hoisted
          // out of it, it would hold several registers per slot)
          asm volatile("" : "+v"(cell[k]), "+v"(col[k]));
          if ((cell[k] >> 12) != jm) continue;
          const uint32_t sc = cell[k] & (kSubCells - 1);
          if (avg_mode(MODE)) {
            const uint64_t packed = (uint64_t)(col[k] & 0xff) | ((uint64_t)((col[k] >> 8) & 0xff) << 16) |
                                    ((uint64_t)((col[k] >> 16) & 0xff) << 32) | (1ull << 48);
            atomicAdd((unsigned long long*)&acc[sc], (unsigned long long)packed);
            if (MODE == 3) atomicMin(&minid[sc], pid[k]);
          } else {
            const uint64_t ok = pick_order(pid[k], seed, MODE == 2);
            if (MODE == 1) atomicMin((unsigned long long*)&acc[sc], (unsigned long long)ok);
            else atomicMax((unsigned long long*)&acc[sc], (unsigned long long)ok);
          }
          atomicOr(&occ[sc >> 5], 1u << (sc & 31));
        }
      }
      if (off + cnt > P1) break;  // continues in the next pass
      lds_barrier();
      if (!avg_mode(MODE)) {
        // the winner of every cell deposits its colour beside its id
        if (off >= P0) {
#pragma unroll
          for (uint32_t k = 0; k < kLeafSlots; ++k) {
            if ((cell[k] >> 12) != jm) continue;
            const uint32_t sc = cell[k] & (kSubCells - 1);
            if (acc[sc] == pick_order(pid[k], seed, MODE == 2)) acc[sc] = ((uint64_t)col[k] << 32) | pid[k];
          }
        } else {
          // the micro-bucket began in an earlier pass: read its points again
          for (uint32_t i = off + t; i < off + cnt; i += kLeafWG) {
            const uint32_t id = ids[i];
            const uint4 v = pts[i];
            const uint32_t sc = point_cell(__uint_as_float(v.x), __uint_as_float(v.y), __uint_as_float(v.z), cd, sub_bit, 4);
            if (acc[sc] == pick_order(id, seed, MODE == 2)) acc[sc] = ((uint64_t)v.w << 32) | id;
          }
        }
        lds_barrier();
      }
      // coordinates of the micro-bucket's first depth-1 cell at level lvl + 6,
      // and of the thread's first one
      const uint32_t Xm = (X0 << 6) | (((jm & 1u) | ((grp & 1u) << 1)) << 4);
      const uint32_t Ym = (Y0 << 6) | ((((jm >> 1) & 1u) | (((grp >> 1) & 1u) << 1)) << 4);
      const uint32_t Zm = (Z0 << 6) | ((((jm >> 2) & 1u) | (((grp >> 2) & 1u) << 1)) << 4);
      const uint32_t Xb = Xm | xt, Yb = Ym | yt, Zb = Zm | zt;
      // Emission at depths 1..4, run once, or twice when an average cell
      // overflowed the packed sums (second round: exact colours of the wide
      // accumulation).  The occupancy bits are exact in both rounds, so the
      // second round rewrites the same positions.
      bool redo = wide;
      uint32_t tot1 = 0, tot2 = 0, tot3 = 0, tot4 = 0;
      for (int round = wide ? 1 : 0; round < 2; ++round) {
        if (round == 1) {
          if (!redo) break;
          // exact 64-bit sums over windows of 512 cells, re-reading the points;
          // the floored colours are kept in the upper half of acc
          uint64_t* wr = acc;
          uint64_t* wg = acc + 512;
          uint64_t* wb = acc + 1024;
          uint64_t* wn = acc + 1536;
          uint32_t* colw = (uint32_t*)(acc + 2048);
          for (uint32_t w0 = 0; w0 < kSubCells; w0 += 512) {
            for (uint32_t i = t; i < 2048; i += kLeafWG) acc[i] = 0;
            lds_barrier();
            for (uint32_t i = t; i < cnt; i += kLeafWG) {
              const uint4 v = pts[off + i];
              const uint32_t sc = point_cell(__uint_as_float(v.x), __uint_as_float(v.y), __uint_as_float(v.z), cd, sub_bit, 4);
              if (w0 == 0) {
                atomicOr(&occ[sc >> 5], 1u << (sc & 31));
                if (MODE == 3) atomicMin(&minid[sc], ids[off + i]);
              }
              if (sc >= w0 && sc < w0 + 512) {
                const uint32_t q = sc - w0;
                atomicAdd((unsigned long long*)&wr[q], (unsigned long long)(v.w & 0xff));
                atomicAdd((unsigned long long*)&wg[q], (unsigned long long)((v.w >> 8) & 0xff));
                atomicAdd((unsigned long long*)&wb[q], (unsigned long long)((v.w >> 16) & 0xff));
                atomicAdd((unsigned long long*)&wn[q], 1ull);
              }
            }
            lds_barrier();
            for (uint32_t q = t; q < 512; q += kLeafWG) {
              const uint64_t c = wn[q];
              if (c) {
                // sums below 2^40 and counts below 2^32 are exact in double; the
                // quotient (<= 255) is at least 2^-32 from the next integer when
                // it is not one, far above the rounding error: floor is exact
                const double dc = (double)c;
                colw[w0 + q] = (uint32_t)((double)wr[q] / dc) | ((uint32_t)((double)wg[q] / dc) << 8) |
                               ((uint32_t)((double)wb[q] / dc) << 16) | (255u << 24);
              }
            }
            lds_barrier();
          }
        }
        // positions: every wave reads the whole depth-1 bitmask (lane l: words
        // 2l, 2l+1; row r of the wave reads quarter r, the cells of wave r)
        // and sums its occupied cells of depths 1..3 per row (packed 13, 10
        // and 7-bit fields: at most 4096, 512 and 64 cells), which gives the
        // list lengths of the earlier waves' quarters and of the micro-bucket
        const uint32_t wa = occ[2 * l], wb2 = occ[2 * l + 1];
        auto nzb = [](uint32_t x) {  // nonzero bytes: occupied depth-2 cells of a word
          uint32_t y = x | (x >> 4);
          y |= y >> 2;
          y |= y >> 1;
          return (uint32_t)__popc(y & 0x01010101u);
        };
        const uint32_t rs = row_sum_dpp(((uint32_t)__popc(wa) + (uint32_t)__popc(wb2)) | ((nzb(wa) + nzb(wb2)) << 13) |
                                        (((wa | wb2) != 0u ? 1u : 0u) << 23));
        const uint32_t q0 = (uint32_t)__builtin_amdgcn_readlane((int)rs, 0);
        const uint32_t q1 = (uint32_t)__builtin_amdgcn_readlane((int)rs, 16);
        const uint32_t q2 = (uint32_t)__builtin_amdgcn_readlane((int)rs, 32);
        const uint32_t q3 = (uint32_t)__builtin_amdgcn_readlane((int)rs, 48);
        const uint32_t qa = q0 + q1 + q2 + q3;
        const uint32_t qc = (w > 0 ? q0 : 0u) + (w > 1 ? q1 : 0u) + (w > 2 ? q2 : 0u);
        tot1 = qa & 0x1fffu;
        tot2 = (qa >> 13) & 0x3ffu;
        tot3 = qa >> 23;
        const uint32_t cross1 = qc & 0x1fffu, cross2 = (qc >> 13) & 0x3ffu, cross3 = qc >> 23;
        const uint64_t b3 = __ballot((wa | wb2) != 0u);  // bit l: depth-3 cell l occupied
        uint32_t m4 = 0;  // occupied depth-4 cells (a depth-4 cell is 8 depth-3 cells)
#pragma unroll
        for (int q = 0; q < 8; ++q) m4 |= ((b3 >> (8 * q)) & 0xffu) ? (1u << q) : 0u;
        const uint32_t cross4 = (uint32_t)__popc(m4 & ((1u << (2 * w)) - 1u));
        tot4 = (uint32_t)__popc(m4);
        // depth 1: cells 16t .. 16t + 15 (the half word t & 1 of word t >> 1);
        // in-wave positions of the depth-1 and depth-2 voxels by one scan of
        // (depth-1 cells | depth-2 cells << 11)
        const uint32_t word = occ[t >> 1];
        uint32_t m = (t & 1) ? (word >> 16) : (word & 0xffffu);
        const uint32_t own = (uint32_t)__popc(m) | ((((m & 0xffu) != 0u ? 1u : 0u) + ((m >> 8) != 0u ? 1u : 0u)) << 11);
        const uint32_t exs = wave_incl_scan_dpp(own) - own;
        uint32_t pos = base1 + cross1 + (exs & 0x7ffu);
        Smp<MODE> h0 = smp_empty<MODE>(), h1 = smp_empty<MODE>();
        const uint32_t* colw = (const uint32_t*)(acc + 2048);
        bool ovf = false;
        if (avg_mode(MODE) && round == 0 && tot1 <= kListCap) {
          // Average modes: the occupied cells go into a list in Morton order
          // (a cell's index there is its rank), which all threads then share,
          // whatever the cells' spread over the threads.
          for (uint32_t mm = m, lp = cross1 + (exs & 0x7ffu); mm; mm &= mm - 1)
            clist[lp++] = (uint16_t)(16 * t + (uint32_t)__ffs(mm) - 1);
          lds_barrier();
          // depth 1: the voxels, each one's colour put back into acc as one
          // sample of its depth-2 cell
          const uint64_t vox1 = vox_at(0, Xm, Ym, Zm, 0);
          for (uint32_t i = t; i < tot1; i += kLeafWG) {
            const uint32_t sc = clist[i];
            const uint64_t a = acc[sc];
            const uint32_t c = (uint32_t)(a >> 48);
            ovf |= c > 257;  // the packed sums are exact up to 257 samples
            const uint32_t rgba =
                mean_rgba((uint32_t)(a & 0xffffu), (uint32_t)((a >> 16) & 0xffffu), (uint32_t)((a >> 32) & 0xffffu), c);
            if (MODE == 3) T1id[I0 + base1 + i] = minid[sc];
            T1[I0 + base1 + i] = vox1 | cell_xyz(sc) | ((uint64_t)rgba << 32);
            acc[sc] = (uint64_t)(rgba & 0xffu) | ((uint64_t)((rgba >> 8) & 0xffu) << 16) |
                      ((uint64_t)((rgba >> 16) & 0xffu) << 32) | (1ull << 48);
          }
          lds_barrier();
          // depth-2 cells 2t and 2t + 1 of the thread: sums of their depth-1
          // voxels (at most 8 of 8-bit values per field); acc and the smallest
          // ids return to their empty state
#pragma unroll
          for (uint32_t e = 0; e < 2; ++e) {
            if (((m >> (8 * e)) & 0xffu) == 0) continue;
            uint64_t* q = acc + 16 * t + 8 * e;
            uint64_t sum = 0;
#pragma unroll 2
            for (uint32_t k = 0; k < 8; ++k) {
              sum += q[k];
              q[k] = 0;
            }
            Smp<MODE>& h = e ? h1 : h0;
            h.r = (uint32_t)(sum & 0xffffu);
            h.g = (uint32_t)((sum >> 16) & 0xffffu);
            h.b = (uint32_t)((sum >> 32) & 0xffffu);
            h.n = (uint32_t)(sum >> 48);
            if (MODE == 3) {
              uint32_t* mi = minid + 16 * t + 8 * e;
              uint32_t mn = ~0u;
#pragma unroll
              for (uint32_t k = 0; k < 8; ++k) {
                mn = min(mn, mi[k]);
                mi[k] = ~0u;
              }
              h.ok = mn;
            }
          }
          m = 0;
        }
        while (m) {
          const uint32_t b = (uint32_t)(__ffs(m) - 1);
          m &= m - 1;
          const uint32_t sc = 16 * t + b;
          uint32_t rgba, id = 0;
          if (avg_mode(MODE)) {
            if (round == 1) {
              rgba = colw[sc];
            } else {
              const uint64_t a = acc[sc];
              acc[sc] = init;
              const uint32_t c = (uint32_t)(a >> 48);
              // the 16-bit fields are exact up to 257 samples; a larger
              // observed count (carries only add to it) sends the
              // micro-bucket to the exact round
              ovf |= c > 257;
              rgba = mean_rgba((uint32_t)(a & 0xffffu), (uint32_t)((a >> 16) & 0xffffu),
                               (uint32_t)((a >> 32) & 0xffffu), c);
            }
            if (MODE == 3) {
              id = minid[sc];
              minid[sc] = ~0u;
              T1id[I0 + pos] = id;
            }
          } else {
            const uint64_t a = acc[sc];
            acc[sc] = init;
            rgba = (uint32_t)(a >> 32);
            id = (uint32_t)a;
            T1id[I0 + pos] = id;
          }
          T1[I0 + pos] = vox_at(0, Xb | (b & 1u) | ((b >> 2) & 2u), Yb | ((b >> 1) & 1u), Zb | ((b >> 2) & 1u), rgba);
          ++pos;
          if (b < 8) smp_add<MODE>(h0, rgba, id, seed);
          else smp_add<MODE>(h1, rgba, id, seed);
        }
        if (avg_mode(MODE) && ovf) over[jm] = 1;
        // depth 2: cells 2t, 2t + 1
        pos = base2 + cross2 + (exs >> 11);
        Smp<MODE> g3 = smp_empty<MODE>();
#pragma unroll
        for (uint32_t e = 0; e < 2; ++e) {
          const Smp<MODE>& h = e ? h1 : h0;
          if (h.n) {
            const uint32_t rgba = smp_rgba<MODE>(h), id = (uint32_t)h.ok;
            T2[t2b + pos] = vox_at(1, Xb | (e << 1), Yb, Zb, rgba);
            if (MODE) T2id[t2b + pos] = id;
            ++pos;
            smp_add<MODE>(g3, rgba, id, seed);
          }
        }
        // depth 3: cell t / 4, over lanes 4q .. 4q + 3
        smp_lane<MODE, kQuadXor1>(g3);
        smp_lane<MODE, kQuadXor2>(g3);
        const bool lead3 = (l & 3) == 0;
        pos = base3 + cross3 + (uint32_t)__popcll(__ballot(lead3 && g3.n) & below);
        Smp<MODE> g4 = smp_empty<MODE>();
        if (g3.n) {
          const uint32_t rgba = smp_rgba<MODE>(g3), id = (uint32_t)g3.ok;
          if (lead3) {
            T2[t2b + cb3 + pos] = vox_at(2, Xb, Yb, Zb, rgba);
            if (MODE) T2id[t2b + cb3 + pos] = id;
          }
          smp_add<MODE>(g4, rgba, id, seed);
        }
        // depth 4: cell t / 32, over the 8 groups of 4 lanes of a half-wave (the
        // 4 lanes of a group hold the same depth-3 voxel; exchanges that keep
        // a lane's place in its group take each group once): the 4 groups of
        // a row by rotations by 4 and 8 lanes, then the two rows
        smp_lane<MODE, kRowRor4>(g4);
        smp_lane<MODE, kRowRor8>(g4);
        smp_lane<MODE, kSwap16>(g4);
        const bool lead4 = (l & 31) == 0;
        pos = base4 + cross4 + (uint32_t)__popcll(__ballot(lead4 && g4.n) & below);
        if (lead4 && g4.n) {
          const uint32_t rgba = smp_rgba<MODE>(g4), id = (uint32_t)g4.ok;
          T2[t2b + cb4 + pos] = vox_at(3, Xb, Yb, Zb, rgba);
          if (MODE) T2id[t2b + cb4 + pos] = id;
          k4col[jm][t >> 5] = rgba;
          k4ok[jm][t >> 5] = g4.ok;
        }
        if (t == 0) k4m[jm] = m4;
        // the other bitmask (the previous micro-bucket's, read by every wave
        // before the last barrier) is cleared for the next one
        if (t < kSubCells / 32) bm1[(nproc + 1) & 1][t] = 0;
        lds_barrier();
        if (avg_mode(MODE) && round == 0) redo = over[jm] != 0;
      }
      if (redo) {
        for (uint32_t i = t; i < kSubCells; i += kLeafWG) acc[i] = init;
        lds_barrier();
      }
      base1 += tot1;
      base2 += tot2;
      base3 += tot3;
      base4 += tot4;
      ++nproc;
    }
  }
  // ---- depth 5 (the micro-buckets) and 6 (the item), from the depth-4
  // voxels; lanes 0..7 of wave 0 take the 8 micro-buckets
  if (w == 0) {
    Smp<MODE> s5 = smp_empty<MODE>();
    if (t < 8) {
      const uint32_t m4 = k4m[t];
      for (uint32_t c = 0; c < 8; ++c)
        if ((m4 >> c) & 1u) smp_add<MODE>(s5, k4col[t][c], (uint32_t)k4ok[t][c], seed);
    }
    const uint32_t has = (t < 8 && s5.n) ? 1u : 0u;
    const uint32_t p5 = wave_prefix_small<1>(has);
    const uint32_t c5 = (uint32_t)__shfl(p5 + has, 7, 64);
    uint32_t rgba = 0, id = 0;
    if (has) {
      rgba = smp_rgba<MODE>(s5);
      id = (uint32_t)s5.ok;
      T2[t2b + cb5 + p5] = make_voxel(anc_code(lkey, 5, (grp << 3) | t), rgba);
      if (MODE) T2id[t2b + cb5 + p5] = id;
    }
    Smp<MODE> s6 = smp_empty<MODE>();
    if (has) smp_add<MODE>(s6, rgba, id, seed);
    smp_xor<MODE>(s6, 1);
    smp_xor<MODE>(s6, 2);
    smp_xor<MODE>(s6, 4);
    if (t == 0) {
      uint32_t c6 = 0;
      if (s6.n) {
        const uint32_t rgba = smp_rgba<MODE>(s6);
        T2[t2b + cb6] = make_voxel(anc_code(lkey, 6, grp), rgba);
        if (MODE) T2id[t2b + cb6] = (uint32_t)s6.ok;
        iself[item] = ((uint64_t)rgba << 32) | (uint32_t)s6.ok;
        c6 = 1;
      }
      uint32_t* ic = icnt + 6 * item;
      ic[0] = base1;
      ic[1] = base2;
      ic[2] = base3;
      ic[3] = base4;
      ic[4] = c5;
      ic[5] = c6;
    }
  }
  if (!LOOP) break;
  }
}

// ------------------------------------------------------------ sparse leaf kernel (average modes)
//
// The average modes' fast path.  A work item's 8 micro-buckets are taken at
// once: their 32768 depth-1 cells (5 levels below the leaf's child cell) form
// a 32768-bit occupancy mask in LDS, and one workgroup-wide scan of the mask
// ranks the occupied cells of every depth (a cell's rank is its position in
// its depth's list, which is in Morton order).  Each depth then has one
// accumulator and one cell code per occupied cell, packed one depth after the
// other in a pool: a sample adds its colour to its cell's accumulator with
// one 64-bit LDS atomic (16-bit fields, as in the general kernel), and each
// depth is emitted one occupied cell per thread, whose colour is in turn a
// sample of its parent.  The work is proportional to the points and the
// occupied cells; nothing is done per empty cell.
//   Phase A: load the points (at most kSpMaxPts, kept in registers as cell
//            code and colour) and set the occupancy bits.
//   Phase B: thread t owns mask words 2t, 2t + 1: depth-1 cells 64t..64t+63,
//            i.e. depth-2 cells 8t..8t+7 (its "byte mask") and depth-3 cell
//            t; depth-4 cell g is threads 8g..8g+7 and the depth-5 cell (a
//            micro-bucket) w is wave w.  A block scan of (depth-1 cells |
//            depth-2 cells << 16) per thread, ballots and the waves' totals
//            give the rank of each word's first depth-1 cell, of each thread's
//            first depth-2 cell, and of each depth-3, 4 and 5 cell.
//   Phase C: every sample into its depth-1 cell.
//   Depths 1 .. 5: one occupied cell per thread: mean colour, voxel, and the
//            colour into the parent's accumulator.  Depth 6 is the item.
// Mode 3 also keeps the smallest sample id of every pooled cell (an LDS atomic
// min per sample, and each emitted cell's id into its parent's).
// The kernel takes the items k_item_desc listed for it (at most kSpMaxPts
// points; larger ones go straight to the general kernel).  An item with more
// occupied cells than the pool holds, or a cell with more than 257 samples
// (beyond the exact range of the 16-bit sums), is listed in `redo` and left to
// the general kernel, which rewrites all of its outputs.  Lists, counts and the
// item's own voxel are those of k_leaf_voxels<MODE>.

// Voxel of a cell with 21-bit Morton code `code` in its ancestor's grid.
__device__ __forceinline__ uint64_t sp_voxel(uint32_t code, uint32_t rgba) { return make_voxel32(code, rgba); }
// An 8-bit colour as one sample in the packed form of the accumulators.
__device__ __forceinline__ uint64_t sp_sample(uint32_t rgba) {
  return (uint64_t)(rgba & 0xffu) | ((uint64_t)((rgba >> 8) & 0xffu) << 16) |
         ((uint64_t)((rgba >> 16) & 0xffu) << 32) | (1ull << 48);
}
__device__ __forceinline__ uint32_t sp_mean(uint64_t a) {
  return mean_rgba((uint32_t)(a & 0xffffu), (uint32_t)((a >> 16) & 0xffffu), (uint32_t)((a >> 32) & 0xffffu),
                   (uint32_t)(a >> 48));
}

template <int MODE>  // 0 average, 3 average with the smallest sample id of every cell
__global__ void __launch_bounds__(kSpWG, 4) k_leaf_sparse(const ItemDesc* __restrict__ desc,
                                                       const uint4* __restrict__ pts, const uint32_t* __restrict__ ids,
                                                       const Cube* cube, uint64_t* __restrict__ T1,
                                                       uint32_t* __restrict__ T1id, uint64_t* __restrict__ T2,
                                                       uint32_t* __restrict__ T2id, uint32_t* __restrict__ icnt,
                                                       uint64_t* __restrict__ iself, BuildState* bs,
                                                       const uint32_t* __restrict__ list, uint32_t* __restrict__ redo) {
  static_assert(MODE == 0 || MODE == 3, "the sparse kernel takes the average modes");
  __shared__ uint32_t mask[kSpWords];
  __shared__ uint16_t wpre[kSpWords];  // rank of the first occupied depth-1 cell of each word
  constexpr uint32_t kCap = sp_cap(MODE);
  __shared__ uint64_t acc[kCap];     // accumulators of depths 1 .. 6, one after the other
  __shared__ uint16_t code[kCap];    // cell codes (index within the item at that depth)
  __shared__ uint32_t minid[MODE == 3 ? kCap : 1];  // mode 3: smallest sample id of every cell
  __shared__ uint16_t pre2[kSpWG];     // rank of each thread's first depth-2 cell
  __shared__ uint16_t rk3[kSpWG];      // rank of each depth-3 cell
  __shared__ uint8_t bm2[kSpWG];       // each thread's depth-2 cells
  __shared__ uint8_t rk4[64], rk5[8];  // ranks of the depth-4 and depth-5 cells
  __shared__ uint32_t wtot[8], wocc[8];
  __shared__ uint32_t flag, nxt;
  const uint32_t t0 = threadIdx.x;
  if (build_stopped(bs)) return;
  // Resident workgroups take list positions from a counter.  While an item's
  // voxels are emitted, the first kSpWG * 8 points of the next one are
  // already on their way into registers.
  const uint32_t nlist = bs->sparse_items;
  if (t0 == 0) nxt = atomicAdd(&bs->sparse_next, 1u);
  __syncthreads();
  const uint32_t li0 = nxt;
  if (li0 >= nlist) return;
  uint32_t item = list[li0];
  uint4 pv[8];  // the current item's first points
  {
    const ItemDesc& sn = desc[item];
#pragma unroll
    for (uint32_t k = 0; k < 8; ++k) {
      uint4 x = make_uint4(0u, 0u, 0u, 0u);  // every lane assigns: the old values die here
      if (k * kSpWG + t0 < sn.P) x = pts[sn.I0 + k * kSpWG + t0];
      pv[k] = x;
    }
  }
  for (;;) {
  // values derived from the thread index are recomputed in every iteration
  // (hoisted out of the loop they would hold registers throughout)
  uint32_t t = t0;
  asm volatile("" : "+v"(t));
  const uint32_t w = t >> 6, l = t & 63u;
  const ItemDesc& sd = desc[item];  // uniform: scalar loads
  const uint32_t P = sd.P;
  const CubeD cd = load_cube(cube + sd.tree);
  const uint32_t I0 = sd.I0, lvl = sd.lvl, grp = item & 7u;
  const uint32_t lk = (uint32_t)sd.lkey;
  const uint64_t t2b = sd.t2;
  const uint32_t sub_bit = 15u - lvl;  // bit level of the depth-1 cells (level lvl + 6)
  __syncthreads();  // the previous item's reads of LDS (and of nxt) are done
  mask[t] = 0;
  mask[t + kSpWG] = 0;
  if (t == 0) {
    flag = 0;
    nxt = atomicAdd(&bs->sparse_next, 1u);
  }
  __syncthreads();
  const uint32_t li = nxt;
  const bool more = li < nlist;

  // ---- phase A: cells, colours, occupancy
  uint32_t col[kSpSlots], cc[kSpSlots / 2];
#pragma unroll
  for (uint32_t h = 0; h < 2; ++h) {
    const uint32_t b0 = h * 8 * kSpWG;
    if (b0 >= P) {  // uniform
#pragma unroll
      for (uint32_t k = 0; k < 4; ++k) cc[4 * h + k] = kSpNone | (kSpNone << 16);
      continue;
    }
    uint4 v1[8];  // the points after the first 8 * kSpWG
    if (h) {
#pragma unroll
      for (uint32_t k = 0; k < 8; ++k)
        if (b0 + k * kSpWG + t < P) v1[k] = pts[I0 + b0 + k * kSpWG + t];
    }
#pragma unroll
    for (uint32_t k = 0; k < 8; ++k) {
      const uint32_t i = b0 + k * kSpWG + t;
      uint32_t c = kSpNone;
      if (i < P) {
        const uint4 v = h ? v1[k] : pv[k];
        const uint32_t qx = (quantize_in_cube(__uint_as_float(v.x), cd.lo[0], cd.scale) >> sub_bit) & 31u;
        const uint32_t qy = (quantize_in_cube(__uint_as_float(v.y), cd.lo[1], cd.scale) >> sub_bit) & 31u;
        const uint32_t qz = (quantize_in_cube(__uint_as_float(v.z), cd.lo[2], cd.scale) >> sub_bit) & 31u;
        c = spread10(qx) | (spread10(qy) << 1) | (spread10(qz) << 2);
        atomicOr(&mask[c >> 5], 1u << (c & 31u));
        col[8 * h + k] = v.w;
      }
      if (k & 1) cc[4 * h + k / 2] |= c << 16;
      else cc[4 * h + k / 2] = c;
    }
  }
  __syncthreads();

  // ---- phase B: ranks
  const uint32_t m0 = mask[2 * t], m1 = mask[2 * t + 1];
  auto nzb = [](uint32_t x) {  // nonzero bytes of a word, as 4 bits
    uint32_t y = x | (x >> 4);
    y |= y >> 2;
    y |= y >> 1;
    y &= 0x01010101u;
    return (y | (y >> 7) | (y >> 14) | (y >> 21)) & 15u;
  };
  const uint32_t b2 = nzb(m0) | (nzb(m1) << 4);  // occupied depth-2 cells 8t + b
  const uint32_t a = (uint32_t)(__popc(m0) + __popc(m1)) | ((uint32_t)__popc(b2) << 16);
  const uint32_t inc = wave_incl_scan_dpp(a);
  const uint64_t b3 = __ballot(b2 != 0u);  // bit l: depth-3 cell 64w + l occupied
  uint32_t m4 = 0;                         // occupied depth-4 cells (groups of 8 lanes) of the wave
#pragma unroll
  for (int q = 0; q < 8; ++q) m4 |= ((b3 >> (8 * q)) & 0xffu) ? (1u << q) : 0u;
  if (l == 63) {
    wtot[w] = inc;
    wocc[w] = (uint32_t)__popcll(b3) | ((uint32_t)__popc(m4) << 10) | ((inc != 0u ? 1u : 0u) << 20);
  }
  __syncthreads();
  uint32_t xa = 0, xo = 0, ta = 0, to = 0;
#pragma unroll
  for (uint32_t v = 0; v < 8; ++v) {
    const uint32_t A = wtot[v], O = wocc[v];
    if (v < w) {
      xa += A;
      xo += O;
    }
    ta += A;
    to += O;
  }
  const uint32_t exa = inc - a;
  const uint32_t ex1 = (xa & 0xffffu) + (exa & 0xffffu), ex2 = (xa >> 16) + (exa >> 16);
  const uint32_t tot1 = ta & 0xffffu, tot2 = ta >> 16;
  const uint32_t tot3 = to & 0x3ffu, tot4 = (to >> 10) & 0x7fu, tot5 = (to >> 20) & 0xfu;
  // pool offsets of depths 2 .. 6
  const uint32_t o2 = tot1, o3p = o2 + tot2, o4 = o3p + tot3, o5 = o4 + tot4, o6 = o5 + tot5;
  const bool fits = o6 + 1 <= kCap;  // uniform
  if (fits) {
    wpre[2 * t] = (uint16_t)ex1;
    wpre[2 * t + 1] = (uint16_t)(ex1 + (uint32_t)__popc(m0));
    pre2[t] = (uint16_t)ex2;
    bm2[t] = (uint8_t)b2;
    const uint64_t below = (1ull << l) - 1;
    rk3[t] = (uint16_t)((xo & 0x3ffu) + (uint32_t)__popcll(b3 & below));
    if ((l & 7u) == 0)
      rk4[t >> 3] = (uint8_t)(((xo >> 10) & 0x7fu) + (uint32_t)__popc(m4 & ((1u << (l >> 3)) - 1u)));
    if (l == 0) rk5[w] = (uint8_t)((xo >> 20) & 0xfu);
    for (uint32_t r = t; r <= o6; r += kSpWG) {
      acc[r] = 0;
      if (MODE == 3) minid[r] = ~0u;
    }
  }
  __syncthreads();

  // ---- phase C: samples into their depth-1 cells
  if (fits) {
#pragma unroll
    for (uint32_t h = 0; h < 2; ++h) {
      uint32_t pid[MODE == 3 ? 8 : 1];  // mode 3: the points' ids, 8 slots at a time
      if (MODE == 3) {
#pragma unroll
        for (uint32_t k = 0; k < 8; ++k)
          if ((8 * h + k) * kSpWG + t < P) pid[MODE == 3 ? k : 0] = ids[I0 + (8 * h + k) * kSpWG + t];
      }
#pragma unroll
      for (uint32_t k = 0; k < 8; ++k) {
        const uint32_t kk = 8 * h + k;
        const uint32_t c = (cc[kk / 2] >> (16 * (kk & 1))) & 0xffffu;
        if (c != kSpNone) {
          const uint32_t r = wpre[c >> 5] + (uint32_t)__popc(mask[c >> 5] & ((1u << (c & 31u)) - 1u));
          atomicAdd((unsigned long long*)&acc[r], (unsigned long long)sp_sample(col[kk]));
          if (MODE == 3) atomicMin(&minid[r], pid[MODE == 3 ? k : 0]);
          code[r] = (uint16_t)c;
        }
      }
    }
  }
  // the next item's first points
  uint32_t nitem = 0;
  if (more) {
    nitem = list[li];
    const ItemDesc& sn = desc[nitem];
#pragma unroll
    for (uint32_t k = 0; k < 8; ++k) {
      uint4 x = make_uint4(0u, 0u, 0u, 0u);
      if (k * kSpWG + t < sn.P) x = pts[sn.I0 + k * kSpWG + t];
      pv[k] = x;
    }
  }
  __syncthreads();

  // ---- depth 1: voxels, and their colours into the depth-2 cells
  if (fits) {
    const uint32_t hi = ((lk & 7u) << 18) | (grp << 15);
    bool ovf = false;
    for (uint32_t r = t; r < tot1; r += kSpWG) {
      const uint64_t s = acc[r];
      const uint32_t c = code[r];
      ovf |= (uint32_t)(s >> 48) > 257u;  // the packed sums are exact up to 257 samples
      const uint32_t rgba = sp_mean(s);
      T1[(uint64_t)I0 + r] = sp_voxel(hi | c, rgba);
      const uint32_t d = c >> 3, u = c >> 6;  // depth-2 cell, its owner thread
      const uint32_t r2 = o2 + pre2[u] + (uint32_t)__popc(bm2[u] & ((1u << (d & 7u)) - 1u));
      atomicAdd((unsigned long long*)&acc[r2], (unsigned long long)sp_sample(rgba));
      if (MODE == 3) {
        const uint32_t id = minid[r];
        T1id[(uint64_t)I0 + r] = id;
        atomicMin(&minid[r2], id);
      }
      code[r2] = (uint16_t)d;
    }
    if (ovf) flag = 1;
  }
  __syncthreads();
  if (fits && !flag) {  // uniform
    // ---- depths 2 .. 5: the same one level up (depth 2 -> 3 -> 4 -> 5 -> 6)
    const uint32_t cb[5] = {0u, coarse_base(3, P), coarse_base(4, P), coarse_base(5, P), coarse_base(6, P)};
    const uint32_t off[6] = {o2, o3p, o4, o5, o6, o6 + 1};
    const uint32_t tot[4] = {tot2, tot3, tot4, tot5};
#pragma unroll
    for (uint32_t k = 0; k < 4; ++k) {  // depth k + 2
      const uint32_t dep = k + 2;
      const uint32_t hi = ((lk & ((1u << (3 * dep)) - 1u)) << (21 - 3 * dep)) | (grp << (18 - 3 * dep));
      for (uint32_t r = t; r < tot[k]; r += kSpWG) {
        const uint64_t s = acc[off[k] + r];
        const uint32_t c = code[off[k] + r];
        const uint32_t rgba = sp_mean(s);
        T2[t2b + cb[k] + r] = sp_voxel(hi | c, rgba);
        uint32_t rp;  // the parent's rank
        if (k == 0) rp = rk3[c >> 3];
        else if (k == 1) rp = rk4[c >> 3];
        else if (k == 2) rp = rk5[c >> 3];
        else rp = 0;
        atomicAdd((unsigned long long*)&acc[off[k + 1] + rp], (unsigned long long)sp_sample(rgba));
        if (MODE == 3) {
          const uint32_t id = minid[off[k] + r];
          T2id[t2b + cb[k] + r] = id;
          atomicMin(&minid[off[k + 1] + rp], id);
        }
        if (k < 3) code[off[k + 1] + rp] = (uint16_t)(c >> 3);
      }
      __syncthreads();
    }
    // ---- depth 6: the item
    if (t == 0) {
      const uint32_t rgba = sp_mean(acc[o6]);
      T2[t2b + cb[4]] = sp_voxel(((lk & 262143u) << 3) | grp, rgba);
      const uint32_t id6 = MODE == 3 ? minid[o6] : 0u;
      if (MODE == 3) T2id[t2b + cb[4]] = id6;
      iself[item] = ((uint64_t)rgba << 32) | id6;
      uint32_t* ic = icnt + 6 * item;
      ic[0] = tot1;
      ic[1] = tot2;
      ic[2] = tot3;
      ic[3] = tot4;
      ic[4] = tot5;
      ic[5] = 1;
    }
  } else if (t == 0) {
    redo[atomicAdd(&bs->redo_items, 1u)] = item;
  }
  if (!more) break;
  item = nitem;
  }
}

// ------------------------------------------------------------ tree pass
//
// Piece sizes of every node (one thread per node):
//   psize[8N + d], d = 1..6: length of leaf N's depth-d list (0 if N is inner
//   or has no ancestor d levels up); psize[8N + 7] = 1 for every node at level
//   >= 7 (its self voxel in the ancestor 7 levels up).
// Leaves at level >= 7 also get their self voxel from their items' voxels.
template <int MODE>
__global__ void __launch_bounds__(256) k_piece_sizes(Nodes nodes, VoxTree vt, const BuildState* bs,
                                                     const uint32_t* __restrict__ icnt,
                                                     const uint64_t* __restrict__ iself, uint32_t seed) {
  if (build_stopped(bs)) return;
  const uint32_t num_nodes = bs->total_nodes;
  for (uint32_t j = blockIdx.x * 256 + threadIdx.x; j < num_nodes; j += gridDim.x * 256) {
  const uint32_t L = nodes.level[j];
  const bool leaf = nodes.is_leaf[j] != 0;
  uint32_t ps[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  uint32_t c6[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  if (leaf && L >= 1) {
    const uint4* q = (const uint4*)(icnt + 48ull * j);  // 8 items x 6 lengths
#pragma unroll
    for (uint32_t k = 0; k < 12; ++k) {
      const uint4 u = q[k];
      const uint32_t e[4] = {u.x, u.y, u.z, u.w};
#pragma unroll
      for (uint32_t h = 0; h < 4; ++h) {
        const uint32_t f = 4 * k + h, d = f % 6 + 1;
        ps[d] += e[h];
        if (d == 6) c6[f / 6] = e[h];
      }
    }
    for (uint32_t d = 1; d <= 6; ++d)
      if (d > L) ps[d] = 0;
  }
  ps[7] = L >= 7 ? 1u : 0u;
  uint4* o = (uint4*)(vt.psize + 8ull * j);
  o[0] = make_uint4(ps[0], ps[1], ps[2], ps[3]);
  o[1] = make_uint4(ps[4], ps[5], ps[6], ps[7]);
  if (leaf && L >= 7) {
    Smp<MODE> sm = smp_empty<MODE>();
#pragma unroll
    for (uint32_t g = 0; g < 8; ++g)
      if (c6[g]) {
        const uint64_t v = iself[8ull * j + g];
        smp_add<MODE>(sm, (uint32_t)(v >> 32), (uint32_t)v, seed);
      }
    vt.selfc[j] = smp_rgba<MODE>(sm);
    vt.selfid[j] = (uint32_t)sm.ok;
  }
  }
}

// One workgroup per tree: subtree sizes (bottom-up), depth-first positions
// (top-down: a node, then its children's subtrees in octant order; a tree's
// positions are its own node range), and the self voxels of the inner nodes
// at level >= 7 (bottom-up).
constexpr int kVTWG = 1024;
template <int MODE>
__global__ void __launch_bounds__(kVTWG) k_vox_tree(Nodes nodes, VoxTree vt, const TreeInfo* __restrict__ trees,
                                                    uint32_t seed, const BuildState* bs) {
  if (build_stopped(bs)) return;
  const TreeInfo& ti = trees[blockIdx.x];
  const int deepest = (int)ti.deepest;
  for (int L = deepest; L >= 0; --L) {
    for (uint32_t j = ti.level_begin[L] + threadIdx.x; j < ti.level_end[L]; j += kVTWG) {
      uint32_t s = 1;
      if (!nodes.is_leaf[j]) {
        const uint32_t fc = nodes.first_child[j], nc = (uint32_t)__popc(nodes.child_mask[j]);
        for (uint32_t k = 0; k < nc; ++k) s += vt.sz[fc + k];
      }
      vt.sz[j] = s;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    vt.dfs[ti.node_base] = ti.node_base;
    vt.dfs_node[ti.node_base] = ti.node_base;
  }
  __syncthreads();
  for (int L = 0; L <= deepest; ++L) {
    for (uint32_t j = ti.level_begin[L] + threadIdx.x; j < ti.level_end[L]; j += kVTWG) {
      if (nodes.is_leaf[j]) continue;
      uint32_t r = vt.dfs[j] + 1;
      const uint32_t fc = nodes.first_child[j], nc = (uint32_t)__popc(nodes.child_mask[j]);
      for (uint32_t k = 0; k < nc; ++k) {
        vt.dfs[fc + k] = r;
        vt.dfs_node[r] = fc + k;
        r += vt.sz[fc + k];
      }
    }
    __syncthreads();
  }
  for (int L = deepest; L >= 7; --L) {
    for (uint32_t j = ti.level_begin[L] + threadIdx.x; j < ti.level_end[L]; j += kVTWG) {
      if (nodes.is_leaf[j]) continue;
      Smp<MODE> s = smp_empty<MODE>();
      const uint32_t fc = nodes.first_child[j], nc = (uint32_t)__popc(nodes.child_mask[j]);
      for (uint32_t k = 0; k < nc; ++k) smp_add<MODE>(s, vt.selfc[fc + k], vt.selfid[fc + k], seed);
      vt.selfc[j] = smp_rgba<MODE>(s);
      vt.selfid[j] = (uint32_t)s.ok;
    }
    __syncthreads();
  }
}

constexpr int kPrefWG = 1024;

// ------------------------------------------------------------ offsets
//
// The pieces of inner node A are the nodes N of A's depth-first range with
// d = level(N) - level(A) <= 7 and psize[8N + d] > 0, in that order.
constexpr int kPieceWG = 256;
__device__ __forceinline__ uint32_t piece_size(const Nodes& nodes, const VoxTree& vt, uint32_t i, uint32_t e,
                                               uint32_t L, uint32_t& N, uint32_t& d) {
  if (i >= e) return 0;
  N = vt.dfs_node[i];
  d = nodes.level[N] - L;
  return d <= 7 ? vt.psize[8ull * N + d] : 0u;
}

__global__ void __launch_bounds__(kPieceWG) k_piece_count(Nodes nodes, VoxTree vt, const BuildState* bs) {
  __shared__ uint32_t sh[kPieceWG / 64];
  if (build_stopped(bs)) return;
  const uint32_t num_nodes = bs->total_nodes;
  for (uint32_t a = blockIdx.x; a < num_nodes; a += gridDim.x) {
  if (nodes.is_leaf[a]) continue;  // uniform
  const uint32_t L = nodes.level[a], b = vt.dfs[a] + 1, e = vt.dfs[a] + vt.sz[a];
  uint32_t s = 0;
  for (uint32_t i = b + threadIdx.x; i < e; i += kPieceWG) {
    uint32_t N, d;
    s += piece_size(nodes, vt, i, e, L, N, d);
  }
  s = wave_sum(s);
  if (lane_id() == 0) sh[threadIdx.x / 64] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t tot = 0;
    for (int q = 0; q < kPieceWG / 64; ++q) tot += sh[q];
    nodes.count[a] = tot;
  }
  __syncthreads();
  }
}

// Voxel offsets of the inner nodes of a tree in node order, counted from the
// tree's first voxel (one workgroup per tree); the total goes to vtotal.
__global__ void __launch_bounds__(kPrefWG) k_voxel_offsets(Nodes nodes, TreeInfo* trees, const BuildState* bs) {
  __shared__ uint64_t sh[kPrefWG / 64 + 1];
  if (build_stopped(bs)) return;
  TreeInfo& ti = trees[blockIdx.x];
  const uint32_t b = ti.node_base, e = ti.node_base + ti.num_nodes;
  uint64_t base = 0;
  for (uint32_t j0 = b; j0 < e; j0 += kPrefWG) {
    const uint32_t j = j0 + threadIdx.x;
    const bool inner = j < e && !nodes.is_leaf[j];
    uint64_t tot;
    const uint64_t ex = block_excl_scan<kPrefWG>(inner ? (uint64_t)nodes.count[j] : (uint64_t)0, sh, &tot);
    if (inner) nodes.offset[j] = base + ex;
    base += tot;
  }
  if (threadIdx.x == 0) ti.vtotal = base;
}

// First voxel of every tree in the build's voxel array (prefix sum of the
// trees' voxel counts, one workgroup) and the total; a total above the
// output's capacity flags the build (kOverVoxels), and nothing is written.
__global__ void __launch_bounds__(kPrefWG) k_voxel_bases(TreeInfo* trees, uint32_t ntrees, uint64_t vcap,
                                                         BuildState* bs) {
  __shared__ uint64_t sh[kPrefWG / 64 + 1];
  if (build_stopped(bs)) return;
  uint64_t base = 0;
  for (uint32_t c0 = 0; c0 < ntrees; c0 += kPrefWG) {
    const uint32_t c = c0 + threadIdx.x;
    uint64_t tot;
    const uint64_t ex = block_excl_scan<kPrefWG>(c < ntrees ? trees[c].vtotal : (uint64_t)0, sh, &tot);
    if (c < ntrees) trees[c].vbase = base + ex;
    base += tot;
  }
  if (threadIdx.x == 0) {
    bs->vtotal = base;
    if (base > vcap) atomicOr(&bs->overflow, (uint32_t)kOverVoxels);
  }
}

__device__ __forceinline__ bool voxels_refused(const BuildState* bs) {
  return (*(volatile const uint32_t*)&bs->overflow & (kOverStop | kOverVoxels)) != 0;
}

// Output position of every piece of inner node A; self voxels are written
// here directly.
template <int MODE>
__global__ void __launch_bounds__(kPieceWG) k_piece_offsets(Nodes nodes, VoxTree vt, const BuildState* bs,
                                                            const TreeInfo* __restrict__ trees,
                                                            uint64_t* __restrict__ vox, uint32_t* __restrict__ vids) {
  __shared__ uint32_t sh[kPieceWG / 64 + 1];
  if (voxels_refused(bs)) return;
  const uint32_t num_nodes = bs->total_nodes;
  for (uint32_t a = blockIdx.x; a < num_nodes; a += gridDim.x) {
  if (nodes.is_leaf[a]) continue;  // uniform
  const uint32_t L = nodes.level[a], b = vt.dfs[a] + 1, e = vt.dfs[a] + vt.sz[a];
  uint64_t run = trees[nodes.tree[a]].vbase + nodes.offset[a];
  for (uint32_t i0 = b; i0 < e; i0 += kPieceWG) {
    uint32_t N = 0, d = 0;
    const uint32_t s = piece_size(nodes, vt, i0 + threadIdx.x, e, L, N, d);
    uint32_t tot;
    const uint32_t ex = block_excl_scan<kPieceWG>(s, sh, &tot);
    if (s) {
      const uint64_t o = run + ex;
      vt.poff[8ull * N + d] = o;
      if (d == 7) {
        vox[o] = make_voxel((uint32_t)nodes.key[N] & kCodeMask, vt.selfc[N]);
        if (MODE) vids[o] = vt.selfid[N];
      }
    }
    run += tot;
  }
  }
}

// Copy every item's depth-1..6 lists to their output positions: the leaf's
// piece for that depth plus the lengths of the leaf's earlier items.  One
// workgroup per leaf: its 48 lists (6 depths x 8 items) are described once,
// then each wave copies every fourth list.
constexpr int kGatherWG = 256;
template <int MODE>
__global__ void __launch_bounds__(kGatherWG) k_gather(Nodes nodes, VoxTree vt, const BuildState* bs,
                                                      const uint32_t* __restrict__ icnt,
                                                      const ItemDesc* __restrict__ desc,
                                                      const uint64_t* __restrict__ T1, const uint32_t* __restrict__ T1id,
                                                      const uint64_t* __restrict__ T2, const uint32_t* __restrict__ T2id,
                                                      uint64_t* __restrict__ vox, uint32_t* __restrict__ vids) {
  __shared__ uint64_t sdst[48], ssrc[48];
  __shared__ uint32_t scnt[48], spre[49];
  const uint32_t t = threadIdx.x;
  if (voxels_refused(bs)) return;
  const uint32_t num_nodes = bs->total_nodes;
  for (uint32_t n = blockIdx.x; n < num_nodes; n += gridDim.x) {
  if (!nodes.is_leaf[n] || nodes.level[n] == 0) continue;  // uniform
  const uint32_t L = nodes.level[n];
  // list j: depth k = j / 8 + 1 of item g = j % 8
  const uint32_t k = t / 8 + 1, g = t % 8;
  if (t < 48) scnt[t] = k <= L ? icnt[6ull * (8 * n + g) + k - 1] : 0u;
  __syncthreads();
  if (t < 64) {
    // where each list goes and comes from, and its first element in the
    // leaf's lists taken one after the other
    const uint32_t c = t < 48 ? scnt[t] : 0u;
    uint64_t dst = 0, src = 0;
    if (c) {
      dst = vt.poff[8ull * n + k];
      for (uint32_t q = 0; q < g; ++q) dst += scnt[t - g + q];
      const ItemDesc& d = desc[8 * n + g];
      src = k == 1 ? (uint64_t)d.I0 : d.t2 + coarse_base(k, d.P);
    }
    const uint32_t inc = wave_incl_scan(c);
    if (t < 48) {
      sdst[t] = dst;
      ssrc[t] = src;
      spre[t] = inc - c;
    }
    if (t == 47) spre[48] = inc;
  }
  __syncthreads();
  // every thread copies elements t, t + kGatherWG, ... of the leaf's lists,
  // four at a time (its list index only moves forward)
  const uint32_t total = spre[48];
  uint32_t j = 0;
  for (uint32_t e0 = t; e0 < total; e0 += 4 * kGatherWG) {
    uint64_t a[4], dv[4];
    uint32_t iv[4];
#pragma unroll
    for (uint32_t q = 0; q < 4; ++q) {
      const uint32_t e = e0 + q * kGatherWG;
      if (e < total) {
        while (spre[j + 1] <= e) ++j;
        const uint32_t off = e - spre[j];
        const uint64_t src = ssrc[j] + off;
        dv[q] = sdst[j] + off;
        a[q] = j < 8 ? T1[src] : T2[src];
        if (MODE) iv[q] = j < 8 ? T1id[src] : T2id[src];
      }
    }
#pragma unroll
    for (uint32_t q = 0; q < 4; ++q) {
      if (e0 + q * kGatherWG < total) {
        vox[dv[q]] = a[q];
        if (MODE) vids[dv[q]] = iv[q];
      }
    }
  }
  __syncthreads();
  }
}

// ------------------------------------------------------------ full precision
//
// Full-precision samples of the lower levels (Sec. 7): the input coordinates
// of every voxel's accepted sample with the voxel's colour, one thread per
// voxel of the call.  The voxel's tree is the last one whose first voxel is
// not after it (trees without voxels share their first voxel with the next).
__global__ void __launch_bounds__(256) k_voxel_points(const uint64_t* __restrict__ vox, const uint32_t* __restrict__ vids,
                                                      const BuildState* bs, const TreeInfo* __restrict__ trees,
                                                      const CloudInfo* __restrict__ clouds, uint32_t ntrees,
                                                      const uint4* __restrict__ pts, uint4* __restrict__ out) {
  if (voxels_refused(bs)) return;
  const uint64_t vtotal = bs->vtotal;
  for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < vtotal; i += (uint64_t)gridDim.x * 256) {
  uint32_t lo = 0, hi = ntrees - 1;
  while (lo < hi) {
    const uint32_t mid = (lo + hi + 1) >> 1;
    if (trees[mid].vbase <= i) lo = mid;
    else hi = mid - 1;
  }
  const uint4 p = pts[(uint64_t)clouds[lo].start + vids[i]];
  out[i] = make_uint4(p.x, p.y, p.z, (uint32_t)(vox[i] >> 32));
  }
}

// ------------------------------------------------------------ launchers

uint64_t coarse_space_bound(uint64_t n, uint32_t num_nodes) {
  // a block holds at most min(5p, 4681) entries for an item of p points
  return std::min<uint64_t>(5 * n, (uint64_t)coarse_base(7, 0xffffffffu) * 8ull * num_nodes) + 1;
}

static uint32_t grid_blocks(uint64_t units, uint32_t per_block, uint32_t cap) {
  return (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>((units + per_block - 1) / per_block, cap));
}

void launch_item_desc(const Nodes& nodes, uint32_t max_nodes, const GridDesc* grids, const uint32_t* pool,
                      BuildState* bs, void* desc, uint64_t t2cap, bool sparse, uint32_t* icnt, uint32_t* slist,
                      uint32_t* redo, hipStream_t s) {
  hipLaunchKernelGGL(k_item_desc, dim3(grid_blocks(8ull * max_nodes, 256, 4096)), dim3(256), 0, s, nodes, grids, pool,
                     bs, (ItemDesc*)desc, t2cap, sparse, icnt, slist, redo);
}

// Workgroups of the sparse leaf kernel that fit on the device at once (two
// per compute unit at four waves per SIMD).
static uint32_t sparse_resident_blocks() {
  static int cached[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) dev = 0;
  if (!cached[dev]) {
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) cus = 256;
    cached[dev] = cus;
  }
  return 2u * (uint32_t)cached[dev];
}

#define LOD_MODE_SWITCH(mode, M, BODY) \
  switch (mode) {                      \
    case 0: {                          \
      constexpr int M = 0;             \
      BODY;                            \
    } break;                           \
    case 1: {                          \
      constexpr int M = 1;             \
      BODY;                            \
    } break;                           \
    case 2: {                          \
      constexpr int M = 2;             \
      BODY;                            \
    } break;                           \
    default: {                         \
      constexpr int M = 3;             \
      BODY;                            \
    } break;                           \
  }

void launch_leaf_voxels(uint32_t mode, uint32_t max_nodes, uint32_t expect_items, const void* desc, const void* pts,
                        const uint32_t* ids, const Cube* cube, uint64_t* T1, uint32_t* T1id, uint64_t* T2,
                        uint32_t* T2id, uint32_t* icnt, uint64_t* iself, uint32_t seed, BuildState* bs,
                        const uint32_t* slist, uint32_t* redo, hipStream_t s) {
  // one workgroup per expected item (the workgroups past the real count
  // return at once), then a resident grid that loops over any items beyond;
  // a launch holds fewer than 2^32 threads
  const uint64_t cap = 8ull * max_nodes;
  const uint32_t g1 =
      (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(std::min<uint64_t>(cap, expect_items), kMaxOneItemBlocks));
  const ItemDesc* d = (const ItemDesc*)desc;
  const uint4* p = (const uint4*)pts;
  if (mode == 0 || mode == 3) {
    // the sparse kernel over its list (resident workgroups), then the general
    // kernel over the items listed for it (one-item form for the first g1 / 16,
    // looping form for any more)
    const uint32_t gs = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(sparse_resident_blocks(), cap));
    const uint32_t g2 = std::max<uint32_t>(1, g1 / 16);
#define LOD_SPARSE(M)                                                                                                 \
  hipLaunchKernelGGL((k_leaf_sparse<M>), dim3(gs), dim3(kSpWG), 0, s, d, p, ids, cube, T1, T1id, T2, T2id, icnt,   \
                     iself, bs, slist, redo);                                                                         \
  hipLaunchKernelGGL((k_leaf_voxels<M, false>), dim3(g2), dim3(kLeafWG), 0, s, d, p, ids, cube, T1, T1id, T2, T2id, \
                     icnt, iself, seed, bs, 0u, (const uint32_t*)redo);                                               \
  hipLaunchKernelGGL((k_leaf_voxels<M, true>), dim3(256), dim3(kLeafWG), 0, s, d, p, ids, cube, T1, T1id, T2, T2id,  \
                     icnt, iself, seed, bs, g2, (const uint32_t*)redo);
    if (mode == 0) {
      LOD_SPARSE(0)
    } else {
      LOD_SPARSE(3)
    }
#undef LOD_SPARSE
    return;
  }
  LOD_MODE_SWITCH(mode, M, {
    hipLaunchKernelGGL((k_leaf_voxels<M, false>), dim3(g1), dim3(kLeafWG), 0, s, d, p, ids, cube, T1, T1id, T2, T2id,
                       icnt, iself, seed, bs, 0u, (const uint32_t*)nullptr);
    if (cap > g1)
      hipLaunchKernelGGL((k_leaf_voxels<M, true>), dim3(grid_blocks(cap - g1, 1, 1024)), dim3(kLeafWG), 0, s, d, p, ids,
                         cube, T1, T1id, T2, T2id, icnt, iself, seed, bs, g1, (const uint32_t*)nullptr);
  })
}

void launch_voxel_tree(uint32_t mode, const Nodes& nodes, const VoxTree& vt, uint32_t max_nodes, TreeInfo* trees,
                       uint32_t ntrees, uint64_t vcap, const uint32_t* icnt, const uint64_t* iself, uint32_t seed,
                       BuildState* bs, hipStream_t s) {
  LOD_MODE_SWITCH(mode, M, {
    hipLaunchKernelGGL(k_piece_sizes<M>, dim3(grid_blocks(max_nodes, 256, 4096)), dim3(256), 0, s, nodes, vt, bs,
                       icnt, iself, seed);
    hipLaunchKernelGGL(k_vox_tree<M>, dim3(ntrees), dim3(kVTWG), 0, s, nodes, vt, (const TreeInfo*)trees, seed, bs);
  })
  hipLaunchKernelGGL(k_piece_count, dim3(grid_blocks(max_nodes, 1, 4096)), dim3(kPieceWG), 0, s, nodes, vt, bs);
  hipLaunchKernelGGL(k_voxel_offsets, dim3(ntrees), dim3(kPrefWG), 0, s, nodes, trees, bs);
  hipLaunchKernelGGL(k_voxel_bases, dim3(1), dim3(kPrefWG), 0, s, trees, ntrees, vcap, bs);
}

void launch_voxel_gather(uint32_t mode, const Nodes& nodes, const VoxTree& vt, uint32_t max_nodes,
                         const TreeInfo* trees, const uint32_t* icnt, const void* desc, const uint64_t* T1,
                         const uint32_t* T1id, const uint64_t* T2, const uint32_t* T2id, uint64_t* vox, uint32_t* vids,
                         const BuildState* bs, hipStream_t s) {
  LOD_MODE_SWITCH(mode, M, {
    hipLaunchKernelGGL(k_piece_offsets<M>, dim3(grid_blocks(max_nodes, 1, 4096)), dim3(kPieceWG), 0, s, nodes, vt, bs,
                       trees, vox, vids);
    hipLaunchKernelGGL(k_gather<M>, dim3(grid_blocks(max_nodes, 1, 4096)), dim3(kGatherWG), 0, s, nodes, vt, bs, icnt,
                       (const ItemDesc*)desc, T1, T1id, T2, T2id, vox, vids);
  })
}
#undef LOD_MODE_SWITCH

void launch_voxel_points(const uint64_t* vox, const uint32_t* vids, uint64_t vcap, const BuildState* bs,
                         const TreeInfo* trees, const CloudInfo* clouds, uint32_t ntrees, const void* pts, void* out,
                         hipStream_t s) {
  if (!ntrees) return;
  hipLaunchKernelGGL(k_voxel_points, dim3(grid_blocks(vcap, 256, 8192)), dim3(256), 0, s, vox, vids, bs, trees, clouds,
                     ntrees, (const uint4*)pts, (uint4*)out);
}

}  // namespace lod
