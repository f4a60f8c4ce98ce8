// launch.h -- host-side launchers of the gfx950 kernels (internal to the library).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.h"

namespace lod {

// k_split.hip
// Bounding-box tiles of a cloud of `count` points.
uint32_t bbox_tiles(uint32_t count);
void launch_bbox(const void* pts, const CloudInfo* clouds, uint32_t nclouds, uint32_t ntiles, BBoxAcc* acc, Cube* cube,
                 hipStream_t st);
// The same in steps, for one cloud streamed in pieces: reset the accumulator,
// add a piece (clouds: one entry describing the piece), make the cube
// (clouds: one entry with the whole count).
void launch_bbox_reset(BBoxAcc* acc, hipStream_t st);
void launch_bbox_add(const void* pts, const CloudInfo* piece, uint32_t ntiles, BBoxAcc* acc, hipStream_t st);
void launch_bbox_cube(const BBoxAcc* acc, const CloudInfo* whole, Cube* cube, hipStream_t st);
void launch_init_roots(const CloudInfo* clouds, uint32_t nclouds, uint32_t E0, Segment* segs, uint32_t* nseg,
                       GridDesc* grids, hipStream_t st);
void launch_make_chunks(Segment* segs, const uint32_t* nseg, uint32_t max_segs, uint32_t chunk, Chunk* chunks,
                        uint32_t* nchunk, uint32_t max_chunks, ChunkGroup* groups, uint32_t* ngroup,
                        uint32_t max_groups, hipStream_t st);
// Counts of a partition: the cells of the points of every chunk, from the
// records, or (dig non-null) from the cells the previous insert stored
// beside them.
void launch_part_count(uint32_t E, const void* pts, const uint16_t* dig, const Cube* cube, const Segment* segs,
                       const Chunk* chunks, const uint32_t* nchunk, uint32_t max_chunks, uint32_t* hist,
                       hipStream_t st);
void launch_part_colscan(const Segment* segs, const uint32_t* nseg, uint32_t max_segs, const ChunkGroup* groups,
                         const uint32_t* ngroup, uint32_t max_groups, uint32_t E, uint32_t* hist, uint32_t* gsum,
                         const GridDesc* grids, uint32_t* pool, hipStream_t st);
void launch_grid_finish(const Segment* segs, const uint32_t* nseg, uint32_t max_segs, const GridDesc* grids,
                        uint32_t* pool, hipStream_t st);
// Points per insert round of the partition scatter (with or without ids).
uint32_t scatter_round(bool ids);
// Insert of a partition.  expect_chunks: how many chunks get a workgroup of
// their own (the rest, up to max_chunks, are taken by a looping grid; results
// never depend on it).  dig (one u16 per destination record, or null): each
// record's cell E levels below its cell of this partition, for the next
// partition's count.
void launch_part_scatter(uint32_t E, bool ids, const void* src, const uint32_t* src_ids, void* dst, uint32_t* dst_ids,
                         uint16_t* dig, const Cube* cube, const Segment* segs, const Chunk* chunks,
                         const uint32_t* nchunk, uint32_t max_chunks, uint32_t expect_chunks, const uint32_t* hist,
                         const GridDesc* grids, const uint32_t* pool, hipStream_t st);
void launch_copy_segments(const void* src, const uint32_t* src_ids, void* dst, uint32_t* dst_ids, const Segment* segs,
                          const uint32_t* nseg, uint32_t max_segs, hipStream_t st);
void launch_segments_from_grid(GridDesc* grids, uint32_t ngrids, uint32_t* pool, uint32_t E2, uint64_t slot_base,
                               uint32_t first_grid, Segment* segs, uint32_t* nseg, hipStream_t st);
// n words of v (a kernel: safe inside a captured graph, unlike a memset).
void launch_fill_u32(uint32_t* p, uint32_t v, uint64_t n, hipStream_t st);
// The build state at the start of a build: zero, with the grid and pool
// counters at the grids and words the two main partitions reserve.
void launch_build_init(BuildState* bs, uint32_t num_grids, uint64_t used_words, hipStream_t st);

// k_tree.hip
void launch_tree_init(uint32_t leaf_cap, uint32_t max_level, const GridDesc* grids, const uint32_t* pool,
                      const Nodes& nodes, TreeState* sts, const uint32_t* node_begin, const uint32_t* node_end,
                      uint32_t nclouds, hipStream_t s);
void launch_tree_build(uint32_t leaf_cap, uint32_t max_level, const GridDesc* grids, const uint32_t* pool,
                       const Nodes& nodes, TreeState* sts, uint32_t nclouds, uint32_t* refine, uint32_t* leaf_refine,
                       BuildState* bs, hipStream_t s);
// Node table work sized by the capacity max_nodes; the real node count is
// read from bs->total_nodes on the device.
void launch_compact_nodes(const Nodes& src, const Nodes& dst, const TreeInfo* trees, const uint32_t* cap_begin,
                          uint32_t ntrees, uint32_t max_nodes, const BuildState* bs, hipStream_t s);
void launch_finalize_nodes(const Nodes& nodes, const TreeInfo* trees, uint32_t max_nodes, const BuildState* bs,
                           uint8_t* o_level, uint8_t* o_leaf, uint8_t* o_mask, uint64_t* o_key, uint32_t* o_npts,
                           uint32_t* o_count, uint32_t* o_first, uint64_t* o_off, hipStream_t s);
// Segments and grids for the nodes of `list` (*nlist of them, at most
// max_list): grids numbered from bs->num_grids, storage from pool word
// bs->used_words; refused (kOverGrids) beyond grid_cap / word_cap.
void launch_refine_segments(const Nodes& nodes, const uint32_t* list, const uint32_t* nlist, uint32_t max_list,
                            uint32_t E, BuildState* bs, uint32_t grid_cap, uint64_t word_cap, GridDesc* grids,
                            Segment* segs, uint32_t* nseg, hipStream_t s);
void launch_refine_commit(BuildState* bs, const uint32_t* nseg, uint32_t E, hipStream_t s);
// TreeInfo of every tree from its enumeration state; bs->total_nodes.
void launch_tree_info(const TreeState* sts, const CloudInfo* clouds, uint32_t ntrees, TreeInfo* trees, BuildState* bs,
                      hipStream_t s);

// k_voxel.hip (launches sized by the node capacity; counts on the device)
// Work-item descriptors: 64 bytes per item, 8 items per node; coarse-list
// blocks handed out from a pool of t2cap entries (kOverCoarse beyond).
// sparse (the average modes): also the lengths of empty items, the sparse leaf
// kernel's list `slist` and the general kernel's `redo` (capacity 8 * max_nodes each)
void launch_item_desc(const Nodes& nodes, uint32_t max_nodes, const GridDesc* grids, const uint32_t* pool,
                      BuildState* bs, void* desc, uint64_t t2cap, bool sparse, uint32_t* icnt, uint32_t* slist,
                      uint32_t* redo, hipStream_t s);
// The leaf kernels over the 8 * total_nodes work items: expect_items sets how
// many get a workgroup of their own (results never depend on it).  In the
// average modes the sparse kernel takes the items of `slist` (from
// launch_item_desc) and lists those it cannot hold in `redo` for the general kernel.
void launch_leaf_voxels(uint32_t mode, uint32_t max_nodes, uint32_t expect_items, const void* desc, const void* pts,
                        const uint32_t* ids, const Cube* cube, uint64_t* T1, uint32_t* T1id, uint64_t* T2,
                        uint32_t* T2id, uint32_t* icnt, uint64_t* iself, uint32_t seed, BuildState* bs,
                        const uint32_t* slist, uint32_t* redo, hipStream_t s);
// Piece sizes, depth-first order, voxel counts and offsets of every tree;
// the trees' first voxels and bs->vtotal (kOverVoxels above vcap).
void launch_voxel_tree(uint32_t mode, const Nodes& nodes, const VoxTree& vt, uint32_t max_nodes, TreeInfo* trees,
                       uint32_t ntrees, uint64_t vcap, const uint32_t* icnt, const uint64_t* iself, uint32_t seed,
                       BuildState* bs, hipStream_t s);
void launch_voxel_gather(uint32_t mode, const Nodes& nodes, const VoxTree& vt, uint32_t max_nodes,
                         const TreeInfo* trees, const uint32_t* icnt, const void* desc, const uint64_t* T1,
                         const uint32_t* T1id, const uint64_t* T2, const uint32_t* T2id, uint64_t* vox, uint32_t* vids,
                         const BuildState* bs, hipStream_t s);
// Neighbourhood-weighted colours of all inner voxels (after the average
// build), level by level.  lnodes: the node indices of the call grouped by
// level, level L at [loff[L], loff[L + 1]) (loff: host array of deepest + 2
// entries).  Occupancy bitmaps of a level's inner nodes: one slot of
// weighted_bitmap_words() 64-bit words and as many u32 word prefixes per
// inner node of the level (at most the sum over trees of n / (T + 1)), zero
// on entry and on return; wslot: one u32 per node; slot_ctr: one u32; acc: 4
// zeroed u64 per voxel; bseg: 64 zeroed uint2 per node; blocks: 64 u32 per
// node and nblocks one u32 (device): the list of a level's non-empty blocks
// and its length.  Runs without host waits.  desc and Y: the leaf items and
// leaf-ordered points.
hipError_t launch_weighted(const Nodes& nodes, const uint32_t* lnodes, const uint64_t* loff, uint32_t deepest,
                           const TreeInfo* trees, const Cube* cube, const void* desc, const void* Y, uint64_t* vox,
                           uint32_t* wslot, unsigned long long* bits, uint32_t* wpre, uint2* bseg,
                           unsigned long long* acc, uint32_t* blocks, uint32_t* nblocks, uint32_t* slot_ctr,
                           hipStream_t s);
uint64_t weighted_bitmap_words();
// Full-precision records (input coordinates of the accepted sample, voxel
// colour) of the bs->vtotal voxels of a call (at most vcap).
void launch_voxel_points(const uint64_t* vox, const uint32_t* vids, uint64_t vcap, const BuildState* bs,
                         const TreeInfo* trees, const CloudInfo* clouds, uint32_t ntrees, const void* pts, void* out,
                         hipStream_t s);
// Size of the coarse-list blocks of all work items, bounded from the node
// count alone (for allocation before the item prefix is known).
uint64_t coarse_space_bound(uint64_t n, uint32_t num_nodes);

// k_merge.hip: the chunked build.
// Level-h cell (Morton code, h <= 7) of each of n points in the cube, and
// their histogram (8^h counters, added to).
void launch_cells(const void* pts, uint32_t n, const Cube* cube, uint32_t h, uint32_t* cell, uint32_t* hist,
                  hipStream_t s);
// A piece sorted by cell (nbins <= 2^21 cells, hist: its histogram): tiles
// (nbins / 4096 rounded up, at most 1024) and cursor (nbins) are scratch;
// out / out_ids receive the points and their ids id0 + index (out_ids may be
// NULL).
void launch_sort_by_cell(const void* pts, const uint32_t* cell, uint32_t n, uint32_t id0, const uint32_t* hist,
                         uint32_t nbins, uint32_t* tiles, uint32_t* cursor, void* out, uint32_t* out_ids,
                         hipStream_t s);
// A job of the levels above the chunk roots: one child (octant `oct`) of a
// node at `level`, whose samples are `count` voxels (kind 0, 8-byte words of
// the child's grid) or points (kind 1, 16-byte records) at `src`, with ids
// (pick modes) at `ids`.  Weighted mode: the parent's and the child's cell
// coordinates (G, C: key bits per axis) and the jobs of the parent's eight
// octants in the same launch (sib, -1 where the octant has no child).
struct TopJob {
  const void* src;
  const uint32_t* ids;
  uint32_t count;
  uint32_t kind;
  uint32_t oct;
  uint32_t level;
  uint32_t G[3], C[3];
  int32_t sib[8];
};
// A cell of a job's dense grid: the sample count n; R, G, B sums (average),
// or the best pick order (a) and the winner's colour | id << 32 (b), or the
// weighted sums of w * R, w * G, w * B and w (a, b, c, w); the smallest
// sample id (full precision in the average modes).
struct TopCell {
  unsigned long long a, b, c, w;
  uint32_t n, mid;
};
constexpr uint32_t kTopCells = 1u << 18;  // 64^3 parent cells under one child octant
constexpr uint32_t kTopSlice = 4096;      // cells per workgroup of the count and emit passes
constexpr uint32_t kTopSlices = kTopCells / kTopSlice;
// mode: 0 average, 1 first, 2 random, 3 weighted.
void launch_top_clear(TopCell* grids, uint32_t njobs, uint32_t mode, hipStream_t s);
// full: keep the smallest sample id per cell (average modes; ids required).
void launch_top_splat(const TopJob* jobs, uint32_t njobs, uint32_t max_count, const Cube* cube, uint32_t mode,
                      uint32_t seed, bool full, TopCell* grids, hipStream_t s);
// Occupied cells per slice: njobs * kTopSlices counters.
void launch_top_count(const TopCell* grids, uint32_t njobs, uint32_t* slice_cnt, hipStream_t s);
// Voxels of the occupied cells in Morton order from slice_off (one u64 per
// slice), and their ids (the pick winner's, or the smallest) if vid is set.
void launch_top_emit(const TopJob* jobs, uint32_t njobs, const TopCell* grids, const uint64_t* slice_off,
                     uint32_t mode, uint64_t* vox, uint32_t* vid, hipStream_t s);
// Copies of runs of 16-, 8- or 4-byte elements into one array.
struct CopyRun {
  const void* src;
  uint64_t dst;  // element index in the destination
  uint64_t len;  // elements
};
void launch_copy_runs(const CopyRun* runs, uint32_t nruns, uint32_t elem_bytes, void* dst, hipStream_t s);
// out[i] = {rec[i].x, .y, .z, colour of vox[i]} (16-byte records).
void launch_voxel_records(const void* rec, const uint64_t* vox, uint64_t n, void* out, hipStream_t s);
// out[i] = {pts[ids[i]].x, .y, .z, colour of vox[i]}; an id >= npts sets *bad.
void launch_voxel_records_by_id(const void* pts, uint32_t npts, const uint32_t* ids, const uint64_t* vox, uint64_t n,
                                void* out, uint32_t* bad, hipStream_t s);

}  // namespace lod
