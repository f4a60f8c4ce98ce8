/*
 * lod_oracle.c -- plain, single-threaded CPU oracle for the hybrid voxel-point
 * octree of "GPU-Accelerated LOD Generation for Point Clouds" (Schuetz, Kerbl,
 * Klaus, Wimmer; arXiv 2302.14801).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  The GPU product path
 * never calls it and shares no code, header, table or helper with it.
 *
 * What it computes, step by step (each step cites the passage it follows):
 *   1. validate input                      (Sec. 3 data structure; Sec. 7 point struct)
 *   2. axis-aligned bounding box            (implicit in Sec. 4.1.1 "project into the counting grid")
 *   3. bounding cube and scale              (Sec. 4.1.1; reading: min-anchored cube, side = max extent)
 *   4. quantize to 2^21 cells per axis      (Sec. 4.1.1 / 4.1.4 projection; reading: double, floor, clamp)
 *   5. Morton key, 63 bits, x lowest        (reading: every level's grid is a key prefix)
 *   6. octree: node inner iff count > T and level < max_level, else leaf
 *                                           (Sec. 4.1.2 merging + 4.1.5 recursion; equals the
 *                                            top-down rule because counts are monotone)
 *   7. leaf membership                      (Sec. 3, Sec. 4.1.4)
 *   8. bottom-up voxel sampling into each inner node's 128^3 grid, one child
 *      octant per child                     (Sec. 4.2, Fig. 1 caption on octants)
 *        AVERAGE: per cell floor(sum/n) of R, G, B over samples, A = 255
 *                                           (Sec. 4.2.3, each sample adds one to the counter)
 *        FIRST:   sample with the smallest input index  (Sec. 4.2.1, made order-free)
 *        RANDOM:  sample with the largest (h(id,seed) << 32 | id), h from the
 *                 SplitMix64 output function (Steele, Lea, Flood, OOPSLA 2014)
 *                                           (Sec. 4.2.2, Listing 1, made order-free)
 *        WEIGHTED: every sample adds w * RGB and w to the 2x2x2 cells around it,
 *                 w = 1 - (distance to the cell centre in cells), clamped at 0;
 *                 only the cell containing a sample is occupied; colour =
 *                 floor(sum(w * c) / sum(w)), A = 255   (Sec. 4.2.4)
 *                 Reading, to make it exact: positions on the half-cell lattice
 *                 of the 2^21 quantization grid (a point at its quantization
 *                 cell's centre, a child voxel at its cell's centre), weights in
 *                 16-bit fixed point, w = 65536 - floor(65536 * distance), from
 *                 an exact integer square root.
 *
 * Arithmetic: IEEE double for the one float->int projection, compiled with
 * -ffp-contract=off; everything after quantization is integer.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "lod_oracle.h"

#define KEY_LEVELS 21
#define GRID_LEVELS 7 /* 128 = 2^7 cells per axis in every inner node */
#define GRID_CELLS (1u << (3 * GRID_LEVELS))

/* ---------------------------------------------------------------- helpers */

/* SplitMix64 output function applied to one 64-bit counter value. */
static uint64_t splitmix64(uint64_t x) {
  uint64_t z = x + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

uint32_t lod_oracle_hash(uint32_t id, uint32_t seed) {
  return (uint32_t)(splitmix64(((uint64_t)seed << 32) | (uint64_t)id) >> 32);
}

/* Morton code of three coordinates with `bits` bits each; x is the lowest bit
 * of every 3-bit group.  A plain per-bit loop. */
static uint64_t morton_bits(uint32_t x, uint32_t y, uint32_t z, int bits) {
  uint64_t k = 0;
  for (int i = 0; i < bits; ++i) {
    k |= (uint64_t)((x >> i) & 1u) << (3 * i);
    k |= (uint64_t)((y >> i) & 1u) << (3 * i + 1);
    k |= (uint64_t)((z >> i) & 1u) << (3 * i + 2);
  }
  return k;
}

static uint32_t quantize_axis(float p, float lo, double scale) {
  double v = ((double)p - (double)lo) * scale;
  double f = floor(v);
  if (f > 2097151.0) f = 2097151.0; /* the far face of the cube maps to the last cell */
  if (f < 0.0) f = 0.0;             /* unreachable for finite input (p >= lo) */
  return (uint32_t)f;
}

typedef struct {
  uint64_t key;
  uint32_t id;
} keyed;

static int cmp_keyed(const void* a, const void* b) {
  const keyed* x = (const keyed*)a;
  const keyed* y = (const keyed*)b;
  if (x->key != y->key) return x->key < y->key ? -1 : 1;
  if (x->id != y->id) return x->id < y->id ? -1 : 1;
  return 0;
}

static int cmp_u32(const void* a, const void* b) {
  uint32_t x = *(const uint32_t*)a, y = *(const uint32_t*)b;
  return x < y ? -1 : (x > y ? 1 : 0);
}

/* --------------------------------------------------------- result memory */

void lod_oracle_free(lod_oracle_tree* t) {
  if (!t) return;
  free(t->level); free(t->is_leaf); free(t->child_mask); free(t->key);
  free(t->npoints); free(t->count); free(t->first_child); free(t->offset);
  free(t->point_ids); free(t->voxels); free(t->voxel_ids);
  memset(t, 0, sizeof(*t));
}

/* --------------------------------------------------------- steps 1 - 5 */

int lod_oracle_cube(const lod_oracle_point* pts, uint64_t n, float lo[3], float hi[3],
                    double* side, double* scale) {
  for (int a = 0; a < 3; ++a) { lo[a] = INFINITY; hi[a] = -INFINITY; }
  for (uint64_t i = 0; i < n; ++i) {
    const float c[3] = {pts[i].x, pts[i].y, pts[i].z};
    for (int a = 0; a < 3; ++a) {
      if (!isfinite(c[a])) return LOD_ORACLE_ERR_NONFINITE;
      if (c[a] < lo[a]) lo[a] = c[a];
      if (c[a] > hi[a]) hi[a] = c[a];
    }
  }
  if (n == 0) { for (int a = 0; a < 3; ++a) { lo[a] = 0.f; hi[a] = 0.f; } }
  double s = 0.0;
  for (int a = 0; a < 3; ++a) {
    double e = (double)hi[a] - (double)lo[a];
    if (e > s) s = e;
  }
  if (s == 0.0) s = 1.0;
  *side = s;
  *scale = 2097152.0 / s;
  return LOD_ORACLE_OK;
}

int lod_oracle_keys_in_cube(const lod_oracle_point* pts, uint64_t n, const float lo[3], double side,
                            uint64_t* keys) {
  const double scale = 2097152.0 / side;
  for (uint64_t i = 0; i < n; ++i) {
    uint32_t qx = quantize_axis(pts[i].x, lo[0], scale);
    uint32_t qy = quantize_axis(pts[i].y, lo[1], scale);
    uint32_t qz = quantize_axis(pts[i].z, lo[2], scale);
    keys[i] = morton_bits(qx, qy, qz, KEY_LEVELS);
  }
  return LOD_ORACLE_OK;
}

int lod_oracle_keys(const lod_oracle_point* pts, uint64_t n, uint64_t* keys) {
  float lo[3], hi[3];
  double side, scale;
  int st = lod_oracle_cube(pts, n, lo, hi, &side, &scale);
  if (st) return st;
  for (uint64_t i = 0; i < n; ++i) {
    uint32_t qx = quantize_axis(pts[i].x, lo[0], scale);
    uint32_t qy = quantize_axis(pts[i].y, lo[1], scale);
    uint32_t qz = quantize_axis(pts[i].z, lo[2], scale);
    keys[i] = morton_bits(qx, qy, qz, KEY_LEVELS);
  }
  return LOD_ORACLE_OK;
}

/* --------------------------------------------------------- step 6: octree */

typedef struct {
  uint32_t level;
  uint64_t key;   /* prefix: key >> 3*(21-level) of every member */
  uint64_t lo, hi; /* range in the sorted (key, id) array */
} pending;

/* --------------------------------------------------------- step 8 grids */

typedef struct {
  /* AVERAGE: per-cell sums of R, G, B and the sample counter */
  uint64_t* sum_r; uint64_t* sum_g; uint64_t* sum_b; uint64_t* n;
  /* PICK: best ordering key, its colour and its id */
  uint64_t* best; uint32_t* best_rgba; uint32_t* best_id;
  uint32_t* occupied; uint32_t num_occupied;
} grid128;

static uint64_t pick_key(int sampling, uint32_t id, uint32_t seed) {
  if (sampling == LOD_ORACLE_FIRST) return (uint64_t)id;
  return ((uint64_t)lod_oracle_hash(id, seed) << 32) | (uint64_t)id;
}

/* A sample (a child's point or a child's voxel) lands in cell (x, y, z) of the
 * node's 128^3 grid: accumulate it. */
static void grid_add(grid128* g, int sampling, uint32_t seed, uint32_t x, uint32_t y, uint32_t z,
                     const uint8_t rgba[4], uint32_t id) {
  uint32_t c = (z * 128u + y) * 128u + x;
  int fresh;
  if (sampling == LOD_ORACLE_AVERAGE) {
    fresh = g->n[c] == 0;
    g->sum_r[c] += rgba[0];
    g->sum_g[c] += rgba[1];
    g->sum_b[c] += rgba[2];
    g->n[c] += 1;
  } else {
    uint64_t k = pick_key(sampling, id, seed);
    fresh = g->n[c] == 0;
    int better = fresh || (sampling == LOD_ORACLE_FIRST ? k < g->best[c] : k > g->best[c]);
    if (better) {
      g->best[c] = k;
      g->best_rgba[c] = (uint32_t)rgba[0] | ((uint32_t)rgba[1] << 8) | ((uint32_t)rgba[2] << 16) |
                        ((uint32_t)rgba[3] << 24);
      g->best_id[c] = id;
    }
    g->n[c] += 1;
  }
  if (fresh) g->occupied[g->num_occupied++] = c;
}

/* Exact floor(sqrt(x)) for x < 2^52: a double estimate, then integer
 * corrections (the estimate is within one of the answer). */
static uint64_t isqrt_u64(uint64_t x) {
  uint64_t r = (uint64_t)sqrt((double)x);
  while (r * r > x) --r;
  while ((r + 1) * (r + 1) <= x) ++r;
  return r;
}

/* Coordinate along one axis (0 = x) of the cell a Morton key names. */
static uint32_t key_axis(uint64_t key, int axis) {
  uint32_t c = 0;
  for (int i = 0; i < KEY_LEVELS; ++i) c |= (uint32_t)((key >> (3 * i + axis)) & 1u) << i;
  return c;
}

/* WEIGHTED (Sec. 4.2.4): per-cell weighted sums over the whole 128^3 grid of
 * the node being sampled, and the list of cells touched (for clearing). */
typedef struct {
  uint64_t* wr; uint64_t* wg; uint64_t* wb; uint64_t* w;
  uint8_t* touched; uint32_t* touched_list; uint32_t num_touched;
} wgrid128;

/* A sample of node (L, key) at position pos2 (per axis, in units of half a
 * cell of the 2^21 grid) splats onto the 2x2x2 cells of the node's grid whose
 * centres surround it.  A cell at distance d (in cells of the node's grid,
 * 2^(15-L) units) gets weight max(0, 65536 - floor(65536 d)). */
static void wgrid_splat(wgrid128* g, int L, const uint32_t node_xyz[3], const uint64_t pos2[3], const uint8_t rgba[4]) {
  const int cs = 15 - L; /* log2 of the node's cell size in pos2 units */
  int64_t cand[3][2];
  for (int a = 0; a < 3; ++a) {
    int64_t k = (int64_t)(pos2[a] >> cs);                    /* containing cell, global index */
    int64_t f = (int64_t)pos2[a] - (k << cs);                /* offset inside it */
    cand[a][0] = k;
    cand[a][1] = f < ((int64_t)1 << (cs - 1)) ? k - 1 : k + 1; /* the other neighbour on this axis */
  }
  for (int m = 0; m < 8; ++m) {
    int64_t c[3];
    int inside = 1;
    for (int a = 0; a < 3; ++a) {
      c[a] = cand[a][(m >> a) & 1];
      int64_t local = c[a] - ((int64_t)node_xyz[a] << 7);
      if (local < 0 || local > 127) inside = 0;
    }
    if (!inside) continue;
    uint64_t d2 = 0;
    for (int a = 0; a < 3; ++a) {
      int64_t d = (int64_t)pos2[a] - ((2 * c[a] + 1) << (cs - 1));
      d2 += (uint64_t)(d * d);
    }
    uint64_t r = isqrt_u64(d2 << (2 * L + 2)); /* floor(65536 * distance) */
    if (r >= 65536) continue;
    uint64_t w = 65536 - r;
    uint32_t x = (uint32_t)(c[0] - ((int64_t)node_xyz[0] << 7));
    uint32_t y = (uint32_t)(c[1] - ((int64_t)node_xyz[1] << 7));
    uint32_t z = (uint32_t)(c[2] - ((int64_t)node_xyz[2] << 7));
    uint32_t cell = (z * 128u + y) * 128u + x;
    if (!g->touched[cell]) {
      g->touched[cell] = 1;
      g->touched_list[g->num_touched++] = cell;
    }
    g->wr[cell] += w * rgba[0];
    g->wg[cell] += w * rgba[1];
    g->wb[cell] += w * rgba[2];
    g->w[cell] += w;
  }
}

typedef struct {
  uint64_t code;
  uint32_t cell;
} coded_cell;

static int cmp_coded(const void* a, const void* b) {
  const coded_cell* x = (const coded_cell*)a;
  const coded_cell* y = (const coded_cell*)b;
  return x->code < y->code ? -1 : (x->code > y->code ? 1 : 0);
}

/* ---------------------------------------------------------------- build */

/* The build with the cube either computed from the points (steps 2-3) or
 * supplied by the caller (cube_lo != NULL), so that the subtree of any node of
 * a large cloud can be rebuilt from that node's points alone: below a node,
 * the octree and its voxels depend only on the node's own points. */
static int build_impl(const lod_oracle_point* pts, uint64_t n, uint32_t leaf_cap, uint32_t max_level, int sampling,
                      uint32_t seed, const float* cube_lo, double cube_side, lod_oracle_tree* out) {
  memset(out, 0, sizeof(*out));
  if (leaf_cap == 0 || max_level > 14 || sampling < 0 || sampling > 3) return LOD_ORACLE_ERR_INVALID;
  /* WEIGHTED marks occupancy like AVERAGE and keeps its own weighted sums */
  const int weighted = sampling == LOD_ORACLE_WEIGHTED;
  if (weighted) sampling = LOD_ORACLE_AVERAGE;
  if (n > 0xFFFFFFFFull) return LOD_ORACLE_ERR_INVALID;
  if (n > 0 && !pts) return LOD_ORACLE_ERR_INVALID;

  /* Steps 2-3 */
  int st = lod_oracle_cube(pts, n, out->aabb_min, out->aabb_max, &out->side, &out->scale);
  if (st) return st;
  if (cube_lo) {
    for (int a = 0; a < 3; ++a) out->aabb_min[a] = cube_lo[a];
    out->side = cube_side;
    out->scale = 2097152.0 / cube_side;
  }
  if (n == 0) return LOD_ORACLE_OK; /* empty tree: no nodes */

  /* Steps 4-5: key per point, then sort (key, id) ascending. */
  keyed* kv = (keyed*)malloc(sizeof(keyed) * n);
  if (!kv) return LOD_ORACLE_ERR_OOM;
  for (uint64_t i = 0; i < n; ++i) {
    uint32_t qx = quantize_axis(pts[i].x, out->aabb_min[0], out->scale);
    uint32_t qy = quantize_axis(pts[i].y, out->aabb_min[1], out->scale);
    uint32_t qz = quantize_axis(pts[i].z, out->aabb_min[2], out->scale);
    kv[i].key = morton_bits(qx, qy, qz, KEY_LEVELS);
    kv[i].id = (uint32_t)i;
  }
  qsort(kv, n, sizeof(keyed), cmp_keyed);

  /* Step 6: breadth-first, so nodes come out in ascending (level, key) order
   * and the children of a node are consecutive.  A node holding more than T
   * points below the depth limit is inner; otherwise it is a leaf. */
  uint64_t cap = 1024;
  pending* q = (pending*)malloc(sizeof(pending) * cap);
  uint64_t qn = 0;
  q[qn++] = (pending){0, 0, 0, n};
  uint8_t* is_leaf = NULL; uint32_t* first_child = NULL; uint8_t* child_mask = NULL;
  uint64_t ncap = 0;
  for (uint64_t h = 0; h < qn; ++h) {
    if (qn + 8 > cap) { cap *= 2; q = (pending*)realloc(q, sizeof(pending) * cap); }
    if (h >= ncap) {
      ncap = cap;
      is_leaf = (uint8_t*)realloc(is_leaf, ncap);
      first_child = (uint32_t*)realloc(first_child, ncap * 4);
      child_mask = (uint8_t*)realloc(child_mask, ncap);
    }
    pending nd = q[h];
    uint64_t cnt = nd.hi - nd.lo;
    int inner = cnt > leaf_cap && nd.level < max_level;
    is_leaf[h] = (uint8_t)!inner;
    first_child[h] = 0;
    child_mask[h] = 0;
    if (!inner) continue;
    first_child[h] = (uint32_t)qn;
    int shift = 3 * (KEY_LEVELS - (int)nd.level - 1);
    uint64_t i = nd.lo;
    while (i < nd.hi) {
      uint64_t child_key = kv[i].key >> shift;
      uint64_t j = i;
      while (j < nd.hi && (kv[j].key >> shift) == child_key) ++j;
      child_mask[h] |= (uint8_t)(1u << (child_key & 7u));
      q[qn++] = (pending){nd.level + 1, child_key, i, j};
      i = j;
    }
  }
  uint32_t nn = (uint32_t)qn;
  out->num_nodes = nn;
  out->level = (uint8_t*)malloc(nn);
  out->key = (uint64_t*)malloc(8ull * nn);
  out->npoints = (uint32_t*)malloc(4ull * nn);
  out->count = (uint32_t*)calloc(nn, 4);
  out->offset = (uint64_t*)calloc(nn, 8);
  out->is_leaf = is_leaf; out->first_child = first_child; out->child_mask = child_mask;
  for (uint32_t h = 0; h < nn; ++h) {
    out->level[h] = (uint8_t)q[h].level;
    out->key[h] = q[h].key;
    out->npoints[h] = (uint32_t)(q[h].hi - q[h].lo);
  }

  /* Step 7: every point goes to the one leaf whose prefix it shares.  Leaves
   * are laid out in node order; inside a leaf the ids are ascending. */
  out->num_points = n;
  out->point_ids = (uint32_t*)malloc(4ull * n);
  uint64_t pos = 0;
  for (uint32_t h = 0; h < nn; ++h) {
    if (!out->is_leaf[h]) continue;
    out->offset[h] = pos;
    out->count[h] = out->npoints[h];
    for (uint64_t i = q[h].lo; i < q[h].hi; ++i) out->point_ids[pos++] = kv[i].id;
    qsort(out->point_ids + out->offset[h], out->count[h], 4, cmp_u32);
  }

  /* Step 8: bottom-up voxel sampling.  Per-node voxel lists are built
   * deepest level first (children before parents) and concatenated in node
   * order at the end. */
  uint8_t** node_vox = (uint8_t**)calloc(nn, sizeof(uint8_t*));
  uint32_t** node_vid = (uint32_t**)calloc(nn, sizeof(uint32_t*));
  grid128 g;
  memset(&g, 0, sizeof(g));
  g.n = (uint64_t*)calloc(GRID_CELLS, 8);
  g.occupied = (uint32_t*)malloc(4ull * GRID_CELLS);
  if (sampling == LOD_ORACLE_AVERAGE) {
    g.sum_r = (uint64_t*)calloc(GRID_CELLS, 8);
    g.sum_g = (uint64_t*)calloc(GRID_CELLS, 8);
    g.sum_b = (uint64_t*)calloc(GRID_CELLS, 8);
  } else {
    g.best = (uint64_t*)calloc(GRID_CELLS, 8);
    g.best_rgba = (uint32_t*)calloc(GRID_CELLS, 4);
    g.best_id = (uint32_t*)calloc(GRID_CELLS, 4);
  }
  coded_cell* order = (coded_cell*)malloc(sizeof(coded_cell) * GRID_CELLS);
  wgrid128 wg;
  memset(&wg, 0, sizeof(wg));
  if (weighted) {
    wg.wr = (uint64_t*)calloc(GRID_CELLS, 8);
    wg.wg = (uint64_t*)calloc(GRID_CELLS, 8);
    wg.wb = (uint64_t*)calloc(GRID_CELLS, 8);
    wg.w = (uint64_t*)calloc(GRID_CELLS, 8);
    wg.touched = (uint8_t*)calloc(GRID_CELLS, 1);
    wg.touched_list = (uint32_t*)malloc(4ull * GRID_CELLS);
  }

  int deepest = 0;
  for (uint32_t h = 0; h < nn; ++h) if (out->level[h] > deepest) deepest = out->level[h];
  uint64_t total_vox = 0;
  for (int L = deepest; L >= 0; --L) {
    for (uint32_t h = 0; h < nn; ++h) {
      if (out->level[h] != (uint8_t)L || out->is_leaf[h]) continue;
      g.num_occupied = 0;
      wg.num_touched = 0;
      const uint32_t node_xyz[3] = {key_axis(out->key[h], 0), key_axis(out->key[h], 1), key_axis(out->key[h], 2)};
      /* The 8 children, in octant order; child octant o covers cells
       * [64*ox, 64*ox+64) x [64*oy, ..) x [64*oz, ..) of this node's grid. */
      for (uint32_t c = out->first_child[h]; c < nn && out->level[c] == (uint8_t)(L + 1) &&
                                             (out->key[c] >> 3) == out->key[h];
           ++c) {
        uint32_t o = (uint32_t)(out->key[c] & 7u);
        uint32_t ox = o & 1u, oy = (o >> 1) & 1u, oz = (o >> 2) & 1u;
        if (out->is_leaf[c]) {
          /* samples are the child's original points; cell = quantized
           * position at resolution 2^(L+7) per axis, relative to this node */
          int sh = KEY_LEVELS - (L + GRID_LEVELS);
          for (uint64_t i = q[c].lo; i < q[c].hi; ++i) {
            const lod_oracle_point* p = &pts[kv[i].id];
            uint32_t qx = quantize_axis(p->x, out->aabb_min[0], out->scale);
            uint32_t qy = quantize_axis(p->y, out->aabb_min[1], out->scale);
            uint32_t qz = quantize_axis(p->z, out->aabb_min[2], out->scale);
            uint8_t rgba[4] = {p->r, p->g, p->b, p->a};
            grid_add(&g, sampling, seed, (qx >> sh) & 127u, (qy >> sh) & 127u, (qz >> sh) & 127u, rgba,
                     kv[i].id);
            if (weighted) {
              /* a point sits at the centre of its 2^21-grid cell */
              const uint64_t pos2[3] = {2ull * qx + 1, 2ull * qy + 1, 2ull * qz + 1};
              wgrid_splat(&wg, L, node_xyz, pos2, rgba);
            }
          }
        } else {
          /* samples are the child's voxels; the child's 128^3 grid folds
           * 2x2x2 -> 1 into this node's octant o */
          for (uint32_t v = 0; v < out->count[c]; ++v) {
            const uint8_t* vx = node_vox[c] + 8ull * v;
            uint8_t rgba[4] = {vx[4], vx[5], vx[6], vx[7]};
            uint32_t id = node_vid[c] ? node_vid[c][v] : 0u;
            grid_add(&g, sampling, seed, ox * 64u + (vx[0] >> 1), oy * 64u + (vx[1] >> 1),
                     oz * 64u + (vx[2] >> 1), rgba, id);
            if (weighted) {
              /* a child voxel sits at the centre of its cell (level L + 8):
               * global index j = child coordinate * 128 + voxel coordinate */
              uint64_t pos2[3];
              for (int a = 0; a < 3; ++a) {
                const uint64_t j = ((uint64_t)key_axis(out->key[c], a) << 7) + vx[a];
                pos2[a] = (2 * j + 1) << (13 - L);
              }
              wgrid_splat(&wg, L, node_xyz, pos2, rgba);
            }
          }
        }
      }
      /* extraction: one voxel per occupied cell, listed in Morton order */
      uint32_t m = g.num_occupied;
      for (uint32_t k = 0; k < m; ++k) {
        uint32_t cell = g.occupied[k];
        uint32_t x = cell & 127u, y = (cell >> 7) & 127u, z = cell >> 14;
        order[k].code = morton_bits(x, y, z, GRID_LEVELS);
        order[k].cell = cell;
      }
      qsort(order, m, sizeof(coded_cell), cmp_coded);
      uint8_t* vox = (uint8_t*)malloc(8ull * (m ? m : 1));
      uint32_t* vid = sampling == LOD_ORACLE_AVERAGE ? NULL : (uint32_t*)malloc(4ull * (m ? m : 1));
      for (uint32_t k = 0; k < m; ++k) {
        uint32_t cell = order[k].cell;
        uint8_t* v = vox + 8ull * k;
        v[0] = (uint8_t)(cell & 127u);
        v[1] = (uint8_t)((cell >> 7) & 127u);
        v[2] = (uint8_t)(cell >> 14);
        v[3] = 0;
        if (weighted) {
          /* the containing sample has weight > 0.13, so the sum is positive */
          uint64_t ws = wg.w[cell];
          v[4] = (uint8_t)(wg.wr[cell] / ws); /* weighted mean, truncated */
          v[5] = (uint8_t)(wg.wg[cell] / ws);
          v[6] = (uint8_t)(wg.wb[cell] / ws);
          v[7] = 255;
          g.sum_r[cell] = g.sum_g[cell] = g.sum_b[cell] = 0;
        } else if (sampling == LOD_ORACLE_AVERAGE) {
          uint64_t cnt = g.n[cell];
          v[4] = (uint8_t)(g.sum_r[cell] / cnt); /* arithmetic mean, truncated */
          v[5] = (uint8_t)(g.sum_g[cell] / cnt);
          v[6] = (uint8_t)(g.sum_b[cell] / cnt);
          v[7] = 255;
          g.sum_r[cell] = g.sum_g[cell] = g.sum_b[cell] = 0;
        } else {
          uint32_t c4 = g.best_rgba[cell];
          v[4] = (uint8_t)c4; v[5] = (uint8_t)(c4 >> 8); v[6] = (uint8_t)(c4 >> 16); v[7] = (uint8_t)(c4 >> 24);
          vid[k] = g.best_id[cell];
          g.best[cell] = 0;
        }
        g.n[cell] = 0; /* only occupied cells are cleared for reuse */
      }
      for (uint32_t k = 0; k < wg.num_touched; ++k) {
        uint32_t cell = wg.touched_list[k];
        wg.wr[cell] = wg.wg[cell] = wg.wb[cell] = wg.w[cell] = 0;
        wg.touched[cell] = 0;
      }
      node_vox[h] = vox;
      node_vid[h] = vid;
      out->count[h] = m;
      total_vox += m;
    }
  }
  out->num_voxels = total_vox;
  out->voxels = (uint8_t*)malloc(8ull * (total_vox ? total_vox : 1));
  out->voxel_ids = sampling == LOD_ORACLE_AVERAGE ? NULL : (uint32_t*)malloc(4ull * (total_vox ? total_vox : 1));
  uint64_t vpos = 0;
  for (uint32_t h = 0; h < nn; ++h) {
    if (out->is_leaf[h]) continue;
    out->offset[h] = vpos;
    memcpy(out->voxels + 8ull * vpos, node_vox[h], 8ull * out->count[h]);
    if (out->voxel_ids) memcpy(out->voxel_ids + vpos, node_vid[h], 4ull * out->count[h]);
    vpos += out->count[h];
    free(node_vox[h]);
    free(node_vid[h]);
  }
  free(node_vox); free(node_vid);
  free(g.sum_r); free(g.sum_g); free(g.sum_b); free(g.n); free(g.best); free(g.best_rgba);
  free(g.best_id); free(g.occupied); free(order);
  free(wg.wr); free(wg.wg); free(wg.wb); free(wg.w); free(wg.touched); free(wg.touched_list);
  free(q); free(kv);
  return LOD_ORACLE_OK;
}

int lod_oracle_build(const lod_oracle_point* pts, uint64_t n, uint32_t leaf_cap, uint32_t max_level, int sampling,
                     uint32_t seed, lod_oracle_tree* out) {
  return build_impl(pts, n, leaf_cap, max_level, sampling, seed, NULL, 0.0, out);
}

int lod_oracle_build_in_cube(const lod_oracle_point* pts, uint64_t n, uint32_t leaf_cap, uint32_t max_level,
                             int sampling, uint32_t seed, const float lo[3], double side, lod_oracle_tree* out) {
  return build_impl(pts, n, leaf_cap, max_level, sampling, seed, lo, side, out);
}
