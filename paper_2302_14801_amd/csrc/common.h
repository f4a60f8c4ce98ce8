// common.h -- device helpers and shared structures of the gfx950 octree builder.
//
// Geometry (Sec. 4.1.1 "project into the counting grid", read as): the cube is
// anchored at the bounding-box minimum with side = largest extent (1 if all
// points coincide); a coordinate is quantized to 2^21 cells per axis as
// floor((double(p) - double(lo)) * (2^21 / side)), clamped to 2^21 - 1.  The
// 63-bit Morton key interleaves the three 21-bit cell indices (x lowest), so
// the cell of any octree level L is the key prefix key >> 3 (21 - L) and the
// grids of all levels nest exactly.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lod {

constexpr int kKeyLevels = 21;
constexpr int kGridLevels = 7;  // an inner node's voxel grid is 128^3 = 2^7 per axis (Sec. 3)
constexpr uint32_t kMaxQ = (1u << kKeyLevels) - 1u;

struct Cube {
  float lo[3];
  float hi[3];
  double side;
  double scale;      // 2^21 / side
  uint32_t nonfinite;  // any NaN/Inf coordinate seen
  uint32_t pad;
};

// Bounding box accumulator: order-preserving integer encodings of floats.
struct BBoxAcc {
  uint32_t lo[3];
  uint32_t hi[3];
  uint32_t nonfinite;
  uint32_t pad;
};

__host__ __device__ inline uint32_t float_order(float f) {
  uint32_t u = __builtin_bit_cast(uint32_t, f);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__host__ __device__ inline float order_float(uint32_t u) {
  uint32_t v = (u & 0x80000000u) ? (u & 0x7fffffffu) : ~u;
  return __builtin_bit_cast(float, v);
}

// One axis: round-to-nearest double subtraction then multiplication, no
// contraction (the build also passes -ffp-contract=off).
__device__ __forceinline__ uint32_t quantize(float p, double lo, double scale) {
  double v = __dmul_rn(__dsub_rn((double)p, lo), scale);
  v = floor(v);
  if (!(v >= 0.0)) v = 0.0;  // also maps NaN (rejected input) to an in-range cell
  if (v > (double)kMaxQ) v = (double)kMaxQ;
  return (uint32_t)v;
}

// quantize() for a coordinate of a point inside the cube (p >= lo, as for
// every point of a cloud in its own cube or in a cube given for all of it):
// the scaled value is then at least 0 and at most 2^21 up to rounding, so the
// truncating conversion is the floor and only the upper clamp can apply.
// (For a NaN coordinate the conversion gives 0, as quantize() does; such an
// input fails the build anyway.)
__device__ __forceinline__ uint32_t quantize_in_cube(float p, double lo, double scale) {
  const double v = __dmul_rn(__dsub_rn((double)p, lo), scale);
  return min((uint32_t)v, kMaxQ);
}

// Spread the low 21 bits of v so that bit i lands at bit 3i.
__host__ __device__ __forceinline__ uint64_t spread21(uint32_t v) {
  uint64_t x = v & 0x1fffffu;
  x = (x | x << 32) & 0x1f00000000ffffull;
  x = (x | x << 16) & 0x1f0000ff0000ffull;
  x = (x | x << 8) & 0x100f00f00f00f00full;
  x = (x | x << 4) & 0x10c30c30c30c30c3ull;
  x = (x | x << 2) & 0x1249249249249249ull;
  return x;
}
// Inverse of spread21 for the x slot (bits 0, 3, 6, ...).
__host__ __device__ __forceinline__ uint32_t compact21(uint64_t x) {
  x &= 0x1249249249249249ull;
  x = (x ^ (x >> 2)) & 0x10c30c30c30c30c3ull;
  x = (x ^ (x >> 4)) & 0x100f00f00f00f00full;
  x = (x ^ (x >> 8)) & 0x1f0000ff0000ffull;
  x = (x ^ (x >> 16)) & 0x1f00000000ffffull;
  x = (x ^ (x >> 32)) & 0x1fffffull;
  return (uint32_t)x;
}

struct CubeD {  // device-side copy in registers
  double lo[3];
  double scale;
};

__device__ __forceinline__ CubeD load_cube(const Cube* c) {
  CubeD d;
  d.lo[0] = (double)c->lo[0];
  d.lo[1] = (double)c->lo[1];
  d.lo[2] = (double)c->lo[2];
  d.scale = c->scale;
  return d;
}

__device__ __forceinline__ uint64_t point_key(float x, float y, float z, const CubeD& c) {
  uint32_t qx = quantize(x, c.lo[0], c.scale);
  uint32_t qy = quantize(y, c.lo[1], c.scale);
  uint32_t qz = quantize(z, c.lo[2], c.scale);
  return spread21(qx) | (spread21(qy) << 1) | (spread21(qz) << 2);
}

// Spread the low 10 bits of v so that bit i lands at bit 3i (32-bit).
__host__ __device__ __forceinline__ uint32_t spread10(uint32_t v) {
  uint32_t x = v & 0x3ffu;
  x = (x | x << 16) & 0x030000ffu;
  x = (x | x << 8) & 0x0300f00fu;
  x = (x | x << 4) & 0x030c30c3u;
  x = (x | x << 2) & 0x09249249u;
  return x;
}

// Bits 0, 3, 6, ... of x gathered into bits 0, 1, 2, ... (inverse of spread10).
__host__ __device__ __forceinline__ uint32_t compact10(uint32_t x) {
  x &= 0x09249249u;
  x = (x | (x >> 2)) & 0x030c30c3u;
  x = (x | (x >> 4)) & 0x0300f00fu;
  x = (x | (x >> 8)) & 0x030000ffu;
  x = (x | (x >> 16)) & 0x000003ffu;
  return x;
}

// The E <= 10 key levels below bit level p of the Morton key, i.e.
// (point_key >> 3p) & (8^E - 1), from the E bits of each axis at and above p
// (for a point inside the cube).
__device__ __forceinline__ uint32_t point_cell(float x, float y, float z, const CubeD& c, uint32_t p, uint32_t E) {
  const uint32_t m = (1u << E) - 1u;
  const uint32_t qx = (quantize_in_cube(x, c.lo[0], c.scale) >> p) & m;
  const uint32_t qy = (quantize_in_cube(y, c.lo[1], c.scale) >> p) & m;
  const uint32_t qz = (quantize_in_cube(z, c.lo[2], c.scale) >> p) & m;
  return spread10(qx) | (spread10(qy) << 1) | (spread10(qz) << 2);
}

// 7-bit-per-axis Morton code of a voxel cell and its inverse.
__host__ __device__ __forceinline__ uint32_t morton7(uint32_t x, uint32_t y, uint32_t z) {
  return (uint32_t)(spread21(x) | (spread21(y) << 1) | (spread21(z) << 2));
}

// Voxel as one 64-bit word: bytes x, y, z, 0, r, g, b, a (little endian).
__host__ __device__ __forceinline__ uint64_t make_voxel(uint32_t code21, uint32_t rgba) {
  uint32_t x = compact21(code21), y = compact21(code21 >> 1), z = compact21(code21 >> 2);
  return (uint64_t)(x | (y << 8) | (z << 16)) | ((uint64_t)rgba << 32);
}
// make_voxel() in 32-bit arithmetic.
__host__ __device__ __forceinline__ uint64_t make_voxel32(uint32_t code21, uint32_t rgba) {
  return (uint64_t)(compact10(code21) | (compact10(code21 >> 1) << 8) | (compact10(code21 >> 2) << 16)) |
         ((uint64_t)rgba << 32);
}
__host__ __device__ __forceinline__ uint32_t voxel_code(uint64_t v) {
  return morton7((uint32_t)(v & 0xff), (uint32_t)((v >> 8) & 0xff), (uint32_t)((v >> 16) & 0xff));
}

// SplitMix64 output function (Steele, Lea, Flood, OOPSLA 2014).
__host__ __device__ __forceinline__ uint64_t splitmix64(uint64_t x) {
  uint64_t z = x + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
// Ordering key of a sample for the pick strategies: FIRST keeps the minimum,
// RANDOM the maximum.
__host__ __device__ __forceinline__ uint64_t pick_order(uint32_t id, uint32_t seed, bool random) {
  if (!random) return (uint64_t)id;
  uint32_t h = (uint32_t)(splitmix64(((uint64_t)seed << 32) | id) >> 32);
  return ((uint64_t)h << 32) | id;
}

// ---------------------------------------------------------------- grids
//
// A grid holds dense point counts for the e levels below a base node
// (base_level, base_key), the "counting grid" / "extended counting grid" of
// Sec. 4.1.1 and 4.1.5.  Storage in one u32 pool:
//   pyr   levels 0..e of the count pyramid, level j at pyr + (8^j - 1) / 7
//   off   8^e absolute point offsets (first point of every finest cell)
//   child 8^e grid indices refining a finest cell (-1 = none)
struct GridDesc {
  uint32_t base_level;
  uint32_t e;
  uint64_t base_key;
  uint64_t pyr;
  uint64_t off;
  uint64_t child;
  uint32_t seg_start;
  uint32_t seg_count;
};

__host__ __device__ __forceinline__ uint64_t pyr_level_offset(uint32_t j) {
  return (((uint64_t)1 << (3 * j)) - 1) / 7;
}
__host__ __device__ __forceinline__ uint64_t grid_words(uint32_t e) {
  return pyr_level_offset(e + 1) + 2ull * ((uint64_t)1 << (3 * e));
}

// A contiguous range of points to be partitioned by the e key levels below
// `level` (one grid per segment).
struct Segment {
  uint32_t start;
  uint32_t count;
  uint32_t grid;
  uint32_t level;
  uint32_t chunk_begin;
  uint32_t chunk_count;
  uint64_t key;  // prefix at `level`
  uint32_t group_begin;
  uint32_t group_count;
  uint32_t cloud;  // input cloud whose cube quantises the segment's points
  uint32_t pad;
};

// One independent input cloud of a build (lod_build: one, lod_build_batch:
// one per non-empty chunk).  Its points stay in [start, start + count) of
// every point buffer of the build.
struct CloudInfo {
  uint32_t start;
  uint32_t count;
  uint32_t tile_base;  // first bounding-box tile of the cloud
  uint32_t pad;
};
struct Chunk {
  uint32_t seg;
  uint32_t start;
  uint32_t count;
  uint32_t pad;
};
// A run of at most kGroupChunks consecutive chunks of one segment (column scans).
constexpr uint32_t kGroupChunks = 32;
// Key levels a refinement sorts: 4 below an inner node at the deepest sorted
// level (enumeration continues there), 2 below a leaf whose points are not
// yet sorted two levels down (the voxel stage's micro-buckets).
constexpr uint32_t kRefineInnerE = 4;
constexpr uint32_t kRefineLeafE = 2;
struct ChunkGroup {
  uint32_t seg;
  uint32_t first;  // first chunk
  uint32_t count;  // chunks in the group
  uint32_t index;  // group index within its segment
};

// Node table (struct of arrays), nodes in ascending (level, key) order.
struct Nodes {
  uint8_t* level;
  uint8_t* is_leaf;
  uint8_t* child_mask;
  uint64_t* key;
  uint32_t* npoints;
  uint32_t* count;        // points (leaf) or voxels (inner)
  uint32_t* first_child;
  uint64_t* offset;       // into the points (leaf) or the voxels (inner)
  int32_t* cover;   // grid whose range contains the node
  int32_t* grid;    // grid based at the node (-1 = none)
  uint32_t* parent;
  uint32_t* tree;   // input cloud (tree) of the node
};

// A voxel-stage work item (one leaf and one of its 8 child cells): what the
// leaf kernel, the gather and the weighted pass need about it, gathered once
// per item so that a leaf workgroup waits for one load before its points.
struct ItemDesc {
  uint32_t I0, P;  // first point and points of the item (P = 0: nothing to do)
  uint32_t lvl, tree;
  uint64_t lkey;   // the leaf's key
  uint64_t t2;     // start of the item's block of coarse lists
  uint32_t mc[8];  // points of each micro-bucket (cells two levels below the leaf), in order
};
static_assert(sizeof(ItemDesc) == 64, "ItemDesc is read as four 16-byte words");

// Where a finished tree sits in the build's arrays (device copy per tree).
struct TreeInfo {
  uint32_t node_base;  // first node of the tree in the compact node table
  uint32_t num_nodes;
  uint32_t point_base;  // first point of the tree's cloud
  uint32_t deepest;     // deepest level with nodes
  uint32_t level_begin[23];  // nodes of level L: [level_begin[L], level_end[L]) (compact)
  uint32_t level_end[23];
  uint64_t vbase;   // first voxel of the tree in the build's voxel array
  uint64_t vtotal;  // voxels of the tree
};

// Per-node data of the voxel stage.
struct VoxTree {
  uint32_t* sz;        // nodes in the subtree (the node included)
  uint32_t* dfs;       // depth-first position
  uint32_t* dfs_node;  // node at a depth-first position
  uint32_t* psize;     // 8 per node: piece lengths by depth above the node (1..7)
  uint64_t* poff;      // 8 per node: output position of each piece
  uint32_t* selfc;     // self voxel (nodes at level >= 7): colour and id
  uint32_t* selfid;
};

// Tree-builder state shared between launches (device memory).
// One per tree while it is built; node indices are absolute slots of the
// tree's region [node_begin, node_end) of the build's node table.
struct TreeState {
  uint32_t num_nodes;      // next free node slot
  uint32_t next_level;     // level whose nodes have not been enumerated yet
  uint32_t status;         // 0 running, 1 done, 2 needs refinement of inner nodes
  uint32_t node_begin;
  uint32_t node_end;
  uint32_t overflow;       // node capacity exceeded
  uint32_t level_begin[23];
  uint32_t level_end[23];
};

// Build-wide state of a build (device memory), zeroed by a kernel at the
// start.  The whole build is enqueued without reading anything back: counts
// that size later work live here, launches are sized by capacities fixed
// beforehand, and a capacity that turns out too small sets a flag that makes
// every later kernel of the build return at once; the host reads this state
// once, after the last kernel, and builds again with the needed capacities.
enum : uint32_t {
  kOverNodes = 1,   // a tree exceeded its node region
  kOverGrids = 2,   // the refinement grids exceeded their pool
  kOverVoxels = 4,  // the voxels exceeded the output's capacity
  kOverCoarse = 8,  // the coarse voxel lists of the leaf items exceeded their pool
  kOverStop = kOverNodes | kOverGrids | kOverCoarse  // flags after which the tree is unusable
};
struct BuildState {
  uint32_t nref;         // inner nodes queued for refinement in this round
  uint32_t nlref;        // leaves queued for refinement (all rounds)
  uint32_t overflow;     // kOver* flags
  uint32_t total_nodes;  // nodes of all trees (compact numbering)
  uint64_t coarse_used;  // entries of the coarse-list buffer handed out
  uint32_t num_grids;    // grid descriptors in use
  uint32_t need_grids;   // grid descriptors the refinements asked for (in use + refused)
  uint64_t used_words;   // pool words in use
  uint64_t need_words;   // pool words the refinements asked for
  uint64_t vtotal;       // voxels of all trees
  uint32_t redo_items;    // leaf work items handed to the general leaf kernel
  uint32_t sparse_items;  // leaf work items listed for the sparse leaf kernel
  uint32_t sparse_next;   // the sparse leaf kernel's next list position
  uint32_t pad;
};

__device__ __forceinline__ bool build_stopped(const BuildState* bs) {
  return (*(volatile const uint32_t*)&bs->overflow & kOverStop) != 0;
}

}  // namespace lod
