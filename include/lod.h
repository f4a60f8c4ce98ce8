/*
 * lod.h -- C ABI of the MI355X (gfx950) builder for the hybrid voxel-point
 * layered-point-cloud octree of Schuetz, Kerbl, Klaus, Wimmer,
 * "GPU-Accelerated LOD Generation for Point Clouds" (arXiv 2302.14801).
 *
 * The octree (Sec. 3): leaves hold at most T original points, inner nodes hold
 * the occupied cells ("voxels") of a 128^3 grid inscribed in the node; every
 * child replaces one 64^3 octant of its parent's grid (Fig. 1 caption).
 *
 * Conventions shared by every entry point:
 *   - Every call returns an lod_status; nothing throws across the ABI.  On
 *     failure the output handle is set to NULL and nothing is leaked; the text
 *     of the last error of the calling thread is available from
 *     lod_last_error().
 *   - Pointers named d_* are device pointers (HIP, the current device);
 *     pointers named h_* are host pointers.  Inputs are borrowed: the library
 *     never frees or keeps them beyond the call (lod_submit: until lod_poll
 *     returns something other than LOD_PENDING).
 *   - `hip_stream` is a hipStream_t (NULL = the default stream).  The build
 *     runs on that stream: the whole build is enqueued with capacities fixed
 *     beforehand, the stream is synchronised once at the end, and the call
 *     returns once the tree is complete.  If a capacity estimated from the
 *     input sizes (refinement grids, coarse voxel lists, voxel output) turns
 *     out too small, the device flags it and the build is repeated with the
 *     capacities it reported (the result never depends on it).
 *   - Results never depend on tuning (block sizes, grid depths, chunking).
 */
#ifndef LOD_H
#define LOD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  LOD_OK = 0,
  LOD_PENDING = 1,              /* lod_poll: request not finished yet */
  LOD_ERR_INVALID = -1,         /* bad argument (NULL pointer, leaf_cap 0, max_level > 14, n >= 2^32, ...) */
  LOD_ERR_NONFINITE = -2,       /* an input coordinate is NaN or infinite */
  LOD_ERR_OOM = -3,             /* device or host allocation failed */
  LOD_ERR_CAPACITY = -4,        /* an internal pool stayed exhausted after re-planning */
  LOD_ERR_TOO_LARGE = -5,       /* request larger than the server's whole memory budget */
  LOD_ERR_UNKNOWN_TICKET = -6,  /* lod_poll: no such ticket */
  LOD_ERR_HIP = -7              /* a HIP runtime call failed */
} lod_status;

/* 16-byte point record: input records and the records stored in leaves
 * (Sec. 7: points and voxels share one struct with float coordinates). */
typedef struct {
  float x, y, z;
  uint8_t r, g, b, a;
} lod_point;

/* 8-byte voxel: cell (x, y, z) in 0..127 of the owning inner node's 128^3
 * grid (Sec. 4.2.1: coordinates quantized to the sampling grid), pad = 0,
 * colour r, g, b, a. */
typedef struct {
  uint8_t x, y, z, pad;
  uint8_t r, g, b, a;
} lod_voxel;

/* Sampling strategies (Sec. 4.2):
 *   LOD_AVERAGE      cell-wise average (Sec. 4.2.3): per cell floor(sum / n) of
 *                    R, G and B over the samples that fall in it, A = 255;
 *                    every sample (a child's point, or a child's voxel)
 *                    counts once.
 *   LOD_PICK_FIRST   first-come (Sec. 4.2.1) made order-independent: the
 *                    sample with the smallest input index wins.
 *   LOD_PICK_RANDOM  random (Sec. 4.2.2, Listing 1) made order-independent:
 *                    the sample with the largest (h(id, seed) << 32 | id)
 *                    wins, h = high 32 bits of the SplitMix64 output function
 *                    of (seed << 32 | id).
 *   LOD_WEIGHTED     neighbourhood-weighted average (Sec. 4.2.4): every
 *                    sample adds w * (R, G, B) and w to the 2x2x2 cells of
 *                    the node's grid around it, w = 1 - distance to the cell
 *                    centre in cells, clamped at 0; only a sample's own cell
 *                    is occupied (the same cells as LOD_AVERAGE); colour =
 *                    floor(sum(w * c) / sum(w)), A = 255.  Exact reading: a
 *                    point sits at the centre of its 2^21-grid cell, a child
 *                    voxel at the centre of its cell; w is 65536 -
 *                    floor(65536 * distance) from an exact integer square
 *                    root.  Slower than the other modes (a pass per level
 *                    after the average build); scratch of about 32 B per
 *                    voxel plus 384 KB per inner node of the widest
 *                    level (at most n / (T + 1)).
 * Pick modes copy the winner's R, G, B, A and record its input index. */
typedef enum { LOD_AVERAGE = 0, LOD_PICK_FIRST = 1, LOD_PICK_RANDOM = 2, LOD_WEIGHTED = 3 } lod_sampling;

enum {
  LOD_FLAG_POINT_IDS = 1, /* keep each leaf point's input index (implied by pick modes) */
  LOD_FLAG_TIMING = 2,    /* record HIP events around every stage (lod_tree_timings) */
  /* Full-precision samples in the lower levels of detail (Sec. 7): besides the
   * quantised voxel cells, every inner-node sample is also given as a 16-byte
   * record with the input coordinates of an accepted sample of its cell and
   * the voxel's colour (voxel_points).  Pick modes accept the picked sample;
   * the average modes accept the sample with the smallest input index in the cell
   * (the arg-min over all points of the subtree that fall in the cell) and
   * keep their (weighted) average colour.  voxel_ids then holds the accepted sample's
   * index in every mode. */
  LOD_FLAG_FULL_PRECISION = 4,
  /* lod_build_batch records the launches of a batch of several clouds into a
   * HIP graph and runs it as one graph launch (weighted sampling, and builds
   * with LOD_FLAG_TIMING, enqueue their launches one by one).  With this flag
   * the launches are enqueued one by one instead; the result is the same. */
  LOD_FLAG_NO_GRAPH = 8,
  /* lod_build_batch / lod_build with the tune_* fields 0: use the plan that
   * lod_tune_batch chooses for a workload of this class (tuning it on this
   * call's input the first time the class is seen in the process). */
  LOD_FLAG_AUTOTUNE = 16,
  /* lod_build_chunked: stream the cloud through host memory, keeping only
   * the pieces in flight and one batch of chunks on the device.  Without it
   * the cloud stays on the device while it is sorted and cut into chunks
   * whenever it fits in half of the free device memory (one host -> device
   * pass instead of four PCIe crossings).  The result is the same. */
  LOD_FLAG_LOW_MEMORY = 32
};

typedef struct {
  uint32_t leaf_cap;     /* T (Sec. 3): a node with more than T points is split; default 50000; >= 1 */
  uint32_t max_level;    /* depth limit (Sec. 4.1.5, 8 + 4 = 12 by default); 0..14; leaves at
                            this level may hold more than T points */
  uint32_t sampling;     /* lod_sampling */
  uint32_t seed;         /* LOD_PICK_RANDOM only */
  uint32_t flags;        /* LOD_FLAG_* */
  uint32_t tune_levels0; /* 0 = automatic; else levels sorted by the first partition pass (1..4) */
  uint32_t tune_levels1; /* 0 = automatic; else levels sorted by the second pass (1..4) */
  uint32_t tune_chunk;   /* 0 = automatic; else points per partition work item (rounded to
                            whole insert rounds, at least one).  The tune_* fields choose
                            how the work is cut, never what is computed. */
} lod_params;

typedef struct lod_tree lod_tree;
typedef struct lod_server lod_server;

/* Read-only view of a finished tree.  All array pointers are DEVICE pointers,
 * valid until lod_tree_free.  Nodes are in ascending (level, key) order and
 * the children of a node are consecutive from node_first_child.
 *   node_key      Morton prefix of the node (3 * level bits; x is the lowest
 *                 bit of each 3-bit group), the cell at `level` that the node
 *                 covers within the bounding cube
 *   node_npoints  input points below the node
 *   node_count    points of a leaf, voxels of an inner node
 *   node_offset   index of the first point (leaf) or voxel (inner node)
 * Points of a leaf are its input records (any order inside the leaf); voxels
 * of an inner node are listed in Morton order of (x, y, z). */
typedef struct {
  float aabb_min[3], aabb_max[3];
  double cube_side;            /* side of the bounding cube, anchored at aabb_min */
  uint32_t num_nodes;
  uint32_t reserved;
  uint64_t num_points;
  uint64_t num_voxels;
  const uint8_t* node_level;
  const uint8_t* node_is_leaf;
  const uint8_t* node_child_mask;
  const uint64_t* node_key;
  const uint32_t* node_npoints;
  const uint32_t* node_count;
  const uint32_t* node_first_child;
  const uint64_t* node_offset;
  const lod_point* points;
  const uint32_t* point_ids;   /* NULL unless ids were kept */
  const lod_voxel* voxels;
  const uint32_t* voxel_ids;      /* pick modes, or with LOD_FLAG_FULL_PRECISION; else NULL */
  const lod_point* voxel_points;  /* with LOD_FLAG_FULL_PRECISION, else NULL */
} lod_tree_view;

/* Default parameters (T = 50000, max_level = 12, AVERAGE). */
void lod_params_default(lod_params* p);

/* Build the octree of n points (Sec. 4.1 split into leaves, Sec. 4.2 voxel
 * sampling).  d_points: device array of n records, borrowed.  n == 0 gives an
 * empty tree (0 nodes).  Errors: LOD_ERR_INVALID (NULL out/params, n >=
 * 2^32, bad params), LOD_ERR_NONFINITE, LOD_ERR_OOM, LOD_ERR_HIP. */
lod_status lod_build(const lod_point* d_points, uint64_t n, const lod_params* p, void* hip_stream,
                     lod_tree** out);

/* Build num_chunks independent trees, chunk i being the records
 * [h_offsets[i], h_offsets[i+1]) of d_points, each with its own bounding box
 * (Sec. 7: chunks of a bottom-up out-of-core pipeline).  out: array of
 * num_chunks handles, filled on success.  Result i equals lod_build on chunk i. */
lod_status lod_build_batch(const lod_point* d_points, const uint64_t* h_offsets, uint32_t num_chunks,
                           const lod_params* p, void* hip_stream, lod_tree** out);

/* Plan autotuner.  A build's plan -- the tune_* fields: levels sorted by the
 * first and second partition pass (the resolution of the root and the
 * extended counting grids, Sec. 4.1.1 and 4.1.5) and points per partition
 * work item -- changes only how the work is cut, never the result.
 * lod_tune_batch times lod_build_batch on the first min(64, num_chunks)
 * chunks of d_points (device, borrowed; offsets as for lod_build_batch) with
 * 17 candidate plans, one warm-up and the median of two runs each, and
 * writes p with the fastest plan to *tuned.  The choice is cached for the
 * process per workload class (chunk count, median and total chunk size as
 * powers of two, sampling, ids and full-precision flags, T, max_level); a
 * cached class returns at once.  If p already sets a tune_* field, *tuned =
 * p.  info (may be NULL) receives whether the plan came from the cache, the
 * sample, the plan and the sample's times with it and with the automatic
 * plan.  Errors: those of lod_build_batch. */
typedef struct {
  uint32_t cached;
  uint32_t sample_chunks;
  uint32_t levels0, levels1, chunk; /* the chosen plan (0 = automatic) */
  float best_ms, default_ms;        /* sample build times: chosen plan, automatic plan */
} lod_tune_info;
lod_status lod_tune_batch(const lod_point* d_points, const uint64_t* h_offsets, uint32_t num_chunks,
                          const lod_params* p, void* hip_stream, lod_params* tuned, lod_tune_info* info);

/* Chunked (out-of-core) build (Sec. 7: a bottom-up out-of-core pipeline cuts
 * the input into chunks of about 10M points, builds each on the GPU and
 * combines them).  h_points: HOST array of n records (pageable or pinned),
 * borrowed; the result equals lod_build on the whole cloud (same nodes, node
 * order, leaf point sets, voxels and ids; ids are indices into h_points).
 * The cloud goes to the GPU in pieces of max(chunk_points, 2^20) records for
 * its bounding cube and is sorted by cell piece by piece; it is cut at the
 * shallowest level b (at most min(7, max_level - 1)) whose cells hold at
 * most chunk_points points, and every cell of level b with more than T points
 * is built as a chunk (chunks are batched up to chunk_points points) with the
 * common cube; the levels above b are then voxelized from the chunk roots'
 * voxels and the points of the leaves above them.  When the cloud fits in
 * half of the free device memory (40 B per point with ids) and
 * LOD_FLAG_LOW_MEMORY is not set, the pieces stay on the device: one host ->
 * device pass.  Otherwise they stream: uploaded once for the cube and once
 * more to be sorted, sent back sorted (20 B per point of pinned host memory)
 * and uploaded again batch by batch; device memory then holds the build
 * workspace of one batch.  Both also hold the chunk results and the output
 * tree (about twice the output).
 * With n <= chunk_points, or max_level < 2, this is
 * the in-core build of a device copy.  Every sampling mode and flag; with
 * LOD_FLAG_FULL_PRECISION the accepted samples' records are gathered from
 * h_points by index at the end.  Errors: LOD_ERR_INVALID
 * (NULL out/params, n >= 2^32,
 * chunk_points 0, bad params), LOD_ERR_NONFINITE, LOD_ERR_OOM, LOD_ERR_HIP. */
lod_status lod_build_chunked(const lod_point* h_points, uint64_t n, const lod_params* p, uint64_t chunk_points,
                             void* hip_stream, lod_tree** out);

/* Allocation-free build, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation).  The same build as lod_build (same nodes, points, voxels and
 * ids) for one cloud of n points, with
 *   - its device scratch in one static array of LOD_NOALLOC_SCRATCH_BYTES
 *     inside the library, held by each GPU the library runs on until the
 *     process ends (256 MiB: clouds of up to 2^22 - 1 points fit with the
 *     default T and depth limit; a cloud that does not fit gives
 *     LOD_ERR_TOO_LARGE before anything is launched);
 *   - its output in the caller's device buffer d_out (256-byte aligned) of
 *     *out_bytes bytes: the leaf points (n records), ids (pick modes,
 *     LOD_FLAG_POINT_IDS, full precision), the node tables and as many
 *     voxels as fit.  On success *out_bytes is set to the bytes used and
 *     *view to device pointers into d_out (valid while the caller keeps
 *     d_out; nothing to free).  With d_out NULL nothing is built and
 *     *out_bytes receives the size for n + 64 voxels (a tree has fewer
 *     voxels than points in typical scans).  If the voxels do not fit, the
 *     result is LOD_ERR_CAPACITY and *out_bytes the size they need;
 *   - no hipMalloc, hipFree, host-pinned or other allocating call, and no
 *     HIP events or graphs.  Timing and autotuning flags are ignored;
 *     LOD_WEIGHTED gives LOD_ERR_INVALID.
 * Every call on a GPU uses that GPU's one array (the build clears what it
 * needs); calls are serialised within the process, and calls that overlap on
 * one GPU from several processes race.  The call returns once the tree is
 * complete on hip_stream.  Errors: as lod_build, plus LOD_ERR_TOO_LARGE and
 * LOD_ERR_CAPACITY as above. */
#define LOD_NOALLOC_SCRATCH_BYTES (256ull << 20)
lod_status lod_build_noalloc(const lod_point* d_points, uint64_t n, const lod_params* p, void* hip_stream,
                             void* d_out, uint64_t* out_bytes, lod_tree_view* view);

/* Per-stage device times in milliseconds of the build that made the tree,
 * measured with HIP events on the build stream (only with LOD_FLAG_TIMING;
 * otherwise all zero).  Stages: bounding box; the first partition (count,
 * offsets, insert); the second partition (count, offsets, insert); node
 * enumeration including refinement partitions; leaf voxels; inner levels;
 * and the whole build from the first to the last kernel.  All zero for a tree
 * that lod_build_chunked made from several chunks. */
typedef struct {
  float bbox;
  float count0, offsets0, scatter0;
  float count1, offsets1, scatter1;
  float tree;
  float leaf_voxels;
  float levels;
  float total;
} lod_timings;
lod_status lod_tree_timings(const lod_tree* t, lod_timings* out);

/* Copy of the tree's header and device array pointers. */
lod_status lod_tree_view_get(const lod_tree* t, lod_tree_view* v);
void lod_tree_free(lod_tree* t);

/* Server: requests (host point arrays) are admitted while their device
 * footprint fits in hbm_budget_bytes next to the trees still resident, and
 * built concurrently (continuous batching).  lod_submit returns a ticket;
 * lod_poll returns LOD_PENDING until the tree is ready, then hands over the
 * tree (the caller frees it with lod_tree_free, which also releases its share
 * of the budget).  A request that could never fit gives LOD_ERR_TOO_LARGE. */
lod_status lod_server_create(uint64_t hbm_budget_bytes, uint32_t max_inflight, const lod_params* p,
                             lod_server** out);
lod_status lod_submit(lod_server* s, const lod_point* h_points, uint64_t n, uint64_t* ticket);
lod_status lod_poll(lod_server* s, uint64_t ticket, lod_tree** out);
void lod_server_destroy(lod_server* s);

const char* lod_status_str(lod_status s);
const char* lod_last_error(void); /* thread-local text of the last failure */

#ifdef __cplusplus
}
#endif
#endif
