// launch.h -- host-side launchers of the gfx950 kernels (internal to the library).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.h"

namespace lod {

// k_split.hip
void launch_bbox(const void* pts, uint64_t n, BBoxAcc* acc, Cube* cube, hipStream_t st);
void launch_init_root(uint32_t n, uint32_t E0, Segment* segs, uint32_t* nseg, GridDesc* grids, hipStream_t st);
void launch_make_chunks(Segment* segs, const uint32_t* nseg, uint32_t max_segs, uint32_t chunk, Chunk* chunks,
                        uint32_t* nchunk, uint32_t max_chunks, ChunkGroup* groups, uint32_t* ngroup,
                        uint32_t max_groups, hipStream_t st);
void launch_part_count(uint32_t E, const void* pts, const Cube* cube, const Segment* segs, const Chunk* chunks,
                       const uint32_t* nchunk, uint32_t max_chunks, uint32_t* hist, hipStream_t st);
void launch_part_colscan(const Segment* segs, const uint32_t* nseg, uint32_t max_segs, const ChunkGroup* groups,
                         const uint32_t* ngroup, uint32_t max_groups, uint32_t E, uint32_t* hist, uint32_t* gsum,
                         const GridDesc* grids, uint32_t* pool, hipStream_t st);
void launch_grid_finish(const Segment* segs, const uint32_t* nseg, uint32_t max_segs, const GridDesc* grids,
                        uint32_t* pool, hipStream_t st);
void launch_part_scatter(uint32_t E, bool ids, const void* src, const uint32_t* src_ids, void* dst, uint32_t* dst_ids,
                         const Cube* cube, const Segment* segs, const Chunk* chunks, const uint32_t* nchunk,
                         uint32_t max_chunks, const uint32_t* hist, const GridDesc* grids, const uint32_t* pool,
                         hipStream_t st);
void launch_copy_segments(const void* src, const uint32_t* src_ids, void* dst, uint32_t* dst_ids, const Segment* segs,
                          const uint32_t* nseg, uint32_t max_segs, hipStream_t st);
void launch_segments_from_grid(GridDesc* grids, uint32_t g0, uint32_t* pool, uint32_t E2, uint64_t slot_base,
                               uint32_t first_grid, Segment* segs, uint32_t* nseg, hipStream_t st);

// k_tree.hip
void launch_tree_init(uint32_t leaf_cap, uint32_t max_level, const GridDesc* grids, const uint32_t* pool,
                      const Nodes& nodes, TreeState* st, hipStream_t s);
void launch_tree_build(uint32_t leaf_cap, uint32_t max_level, const GridDesc* grids, const uint32_t* pool,
                       const Nodes& nodes, TreeState* st, uint32_t* refine, uint32_t* leaf_refine, uint32_t max_nodes,
                       hipStream_t s);
void launch_refine_segments(const Nodes& nodes, const uint32_t* list, const uint32_t* nlist, uint32_t max_list,
                            uint32_t E, uint32_t first_grid, uint64_t slot_base, GridDesc* grids, Segment* segs,
                            uint32_t* nseg, hipStream_t s);

// k_voxel.hip
void launch_leaf_voxels(uint32_t mode, const Nodes& nodes, uint32_t num_nodes, const GridDesc* grids,
                        const uint32_t* pool, const void* pts, const uint32_t* ids, const Cube* cube, uint64_t* temp,
                        uint32_t* temp_ids, uint32_t* gcount, uint32_t* gstart, uint32_t seed, hipStream_t s);
void launch_voxel_bound(const Nodes& nodes, TreeState* st, hipStream_t s);
void launch_fill_zero(uint64_t* p, uint64_t n, hipStream_t s);
void launch_level(uint32_t mode, const Nodes& nodes, uint32_t L, uint32_t pbegin, uint32_t pend, uint32_t cbegin,
                  uint32_t cend, uint64_t vcap, const uint64_t* temp, const uint32_t* temp_ids, uint64_t* vox,
                  uint32_t* vids, TreeState* st, uint32_t* tilesum, uint32_t* runidx, uint32_t* runpos,
                  uint8_t* vflag, uint32_t* vowner, const uint32_t* gcount, const uint32_t* gstart, uint32_t seed,
                  hipStream_t s);

}  // namespace lod
