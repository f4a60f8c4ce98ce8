/*
 * lod_oracle.h -- plain CPU oracle for the hybrid voxel-point octree
 * (arXiv 2302.14801, Sec. 3-4).  TEST INFRASTRUCTURE ONLY: loaded by the
 * tests, the smoke check and the CPU-baseline leg of the benchmark, never by
 * the GPU product path.  Shares no code with it.
 */
#ifndef LOD_ORACLE_H
#define LOD_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { LOD_ORACLE_OK = 0, LOD_ORACLE_ERR_INVALID = -1, LOD_ORACLE_ERR_NONFINITE = -2, LOD_ORACLE_ERR_OOM = -3 };
enum { LOD_ORACLE_AVERAGE = 0, LOD_ORACLE_FIRST = 1, LOD_ORACLE_RANDOM = 2, LOD_ORACLE_WEIGHTED = 3 };

/* 16-byte input record: position and colour (Sec. 7: points and voxels share
 * one struct with float coordinates). */
typedef struct {
  float x, y, z;
  uint8_t r, g, b, a;
} lod_oracle_point;

/* Result.  Nodes are in ascending (level, key) order; the children of a node
 * are consecutive, starting at first_child.  `count` is the number of points
 * of a leaf or the number of voxels of an inner node, `offset` indexes
 * point_ids (leaf) or voxels (inner).  `npoints` is the number of input points
 * under the node.  A voxel is 8 bytes: x, y, z (cell in the node's 128^3
 * grid), 0, r, g, b, a. */
typedef struct {
  float aabb_min[3], aabb_max[3];
  double side, scale;
  uint32_t num_nodes;
  uint8_t* level;
  uint8_t* is_leaf;
  uint8_t* child_mask;
  uint64_t* key;
  uint32_t* npoints;
  uint32_t* count;
  uint32_t* first_child;
  uint64_t* offset;
  uint64_t num_points;
  uint32_t* point_ids;
  uint64_t num_voxels;
  uint8_t* voxels;
  uint32_t* voxel_ids; /* pick modes only, else NULL */
} lod_oracle_tree;

int lod_oracle_build(const lod_oracle_point* pts, uint64_t n, uint32_t leaf_cap, uint32_t max_level,
                     int sampling, uint32_t seed, lod_oracle_tree* out);
void lod_oracle_free(lod_oracle_tree* t);

/* Same build with the cube supplied instead of computed: lo is the cube's
 * minimum corner, side its edge.  Every point must lie inside the cube. */
int lod_oracle_build_in_cube(const lod_oracle_point* pts, uint64_t n, uint32_t leaf_cap, uint32_t max_level,
                             int sampling, uint32_t seed, const float lo[3], double side, lod_oracle_tree* out);

/* Individual steps, exposed so tests can pin them one at a time. */
int lod_oracle_cube(const lod_oracle_point* pts, uint64_t n, float lo[3], float hi[3], double* side,
                    double* scale);
int lod_oracle_keys(const lod_oracle_point* pts, uint64_t n, uint64_t* keys);
int lod_oracle_keys_in_cube(const lod_oracle_point* pts, uint64_t n, const float lo[3], double side,
                            uint64_t* keys);
uint32_t lod_oracle_hash(uint32_t id, uint32_t seed);

#ifdef __cplusplus
}
#endif
#endif
