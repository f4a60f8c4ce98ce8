// k_split.hip -- bounding box, cube, and the hierarchical counting sort that
// splits the input into octree cells (Sec. 4.1: counting, creating target
// offsets, insert; Sec. 4.1.5: repeated for cells that need more depth).
//
// A "partition" call takes a list of segments (contiguous point ranges, each
// the points of one octree node) and sorts every segment by the next e levels
// of the Morton key: one dense 8^e counting grid per segment (Sec. 4.1.1),
// exclusive prefix sums as target offsets (Sec. 4.1.3), and an insert pass
// that moves every point to its cell (Sec. 4.1.4).  On gfx950 the per-point
// counting and the insert are privatised in LDS: a workgroup counts a chunk
// of a segment in LDS and writes one histogram row, and the insert stages a
// round of points in LDS sorted by cell so that the global stores come out as
// contiguous runs instead of single 16-byte writes (global atomics and
// scattered 16-byte stores both run at ~25-40 G ops/s on this part, far below
// what the 8 TB/s memory can stream).
#include <algorithm>

#include "common.h"
#include "launch.h"
#include "scan.h"

namespace lod {

// ------------------------------------------------------------ bounding box

__global__ void k_bbox_init(BBoxAcc* acc, uint32_t nclouds) {
  const uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nclouds) return;
  for (int a = 0; a < 3; ++a) {
    acc[c].lo[a] = 0xffffffffu;
    acc[c].hi[a] = 0u;
  }
  acc[c].nonfinite = 0u;
}

constexpr int kBBoxWG = 256;
constexpr uint32_t kBBoxTile = kBBoxWG * 64;  // points per workgroup

// Cloud of a bounding-box tile: the last cloud whose first tile is <= t.
__device__ __forceinline__ uint32_t tile_cloud(const CloudInfo* __restrict__ clouds, uint32_t nclouds, uint32_t t) {
  uint32_t lo = 0, hi = nclouds;  // answer in [lo, hi)
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) / 2;
    if (clouds[mid].tile_base <= t) lo = mid;
    else hi = mid;
  }
  return lo;
}

// One tile of at most kBBoxTile points of one cloud per workgroup; per-cloud
// minima and maxima of the order-preserving integer images of x, y, z.
__global__ void __launch_bounds__(kBBoxWG) k_bbox(const uint4* __restrict__ pts, const CloudInfo* __restrict__ clouds,
                                                  uint32_t nclouds, BBoxAcc* acc) {
  const uint32_t c = tile_cloud(clouds, nclouds, blockIdx.x);
  const CloudInfo ci = clouds[c];
  const uint64_t t0 = (uint64_t)ci.start + (uint64_t)(blockIdx.x - ci.tile_base) * kBBoxTile;
  const uint64_t n = min((uint64_t)ci.start + ci.count, t0 + kBBoxTile);
  acc += c;
  uint32_t lo0 = 0xffffffffu, lo1 = 0xffffffffu, lo2 = 0xffffffffu;
  uint32_t hi0 = 0u, hi1 = 0u, hi2 = 0u, bad = 0u;
  const uint64_t stride = kBBoxWG;
  uint64_t i = t0 + threadIdx.x;
  auto acc1 = [&](const uint4& v) {
    // exponent all ones = Inf or NaN
    uint32_t nf = ((v.x & 0x7f800000u) == 0x7f800000u) | ((v.y & 0x7f800000u) == 0x7f800000u) |
                  ((v.z & 0x7f800000u) == 0x7f800000u);
    bad |= nf;
    if (!nf) {
      uint32_t a = float_order(__uint_as_float(v.x)), b = float_order(__uint_as_float(v.y)),
               c = float_order(__uint_as_float(v.z));
      lo0 = min(lo0, a); hi0 = max(hi0, a);
      lo1 = min(lo1, b); hi1 = max(hi1, b);
      lo2 = min(lo2, c); hi2 = max(hi2, c);
    }
  };
  for (; i + 7 * stride < n; i += 8 * stride) {
    uint4 v[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) v[k] = pts[i + k * stride];
#pragma unroll
    for (int k = 0; k < 8; ++k) acc1(v[k]);
  }
  for (; i < n; i += stride) acc1(pts[i]);
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) {
    lo0 = min(lo0, (uint32_t)__shfl_xor((int)lo0, d, 64));
    lo1 = min(lo1, (uint32_t)__shfl_xor((int)lo1, d, 64));
    lo2 = min(lo2, (uint32_t)__shfl_xor((int)lo2, d, 64));
    hi0 = max(hi0, (uint32_t)__shfl_xor((int)hi0, d, 64));
    hi1 = max(hi1, (uint32_t)__shfl_xor((int)hi1, d, 64));
    hi2 = max(hi2, (uint32_t)__shfl_xor((int)hi2, d, 64));
    bad |= (uint32_t)__shfl_xor((int)bad, d, 64);
  }
  __shared__ uint32_t sh[7][kBBoxWG / 64];
  const int w = threadIdx.x / 64;
  if (lane_id() == 0) {
    sh[0][w] = lo0; sh[1][w] = lo1; sh[2][w] = lo2;
    sh[3][w] = hi0; sh[4][w] = hi1; sh[5][w] = hi2; sh[6][w] = bad;
  }
  __syncthreads();
  if (threadIdx.x < 7) {
    uint32_t r = sh[threadIdx.x][0];
    for (int k = 1; k < kBBoxWG / 64; ++k) {
      uint32_t t = sh[threadIdx.x][k];
      r = threadIdx.x < 3 ? min(r, t) : (threadIdx.x < 6 ? max(r, t) : (r | t));
    }
    if (threadIdx.x < 3) atomicMin(&acc->lo[threadIdx.x], r);
    else if (threadIdx.x < 6) atomicMax(&acc->hi[threadIdx.x - 3], r);
    else if (r) atomicOr(&acc->nonfinite, 1u);
  }
}

// The bounding cube of every cloud: anchored at the minimum, side = largest
// extent (1 if all points coincide).
__global__ void k_cube(const BBoxAcc* acc, const CloudInfo* clouds, uint32_t nclouds, Cube* cube) {
  const uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nclouds) return;
  const uint32_t n = clouds[c].count;
  double side = 0.0;
  for (int a = 0; a < 3; ++a) {
    float lo = n ? order_float(acc[c].lo[a]) : 0.f;
    float hi = n ? order_float(acc[c].hi[a]) : 0.f;
    if (acc[c].lo[a] == 0xffffffffu) lo = hi = 0.f;  // every point rejected
    cube[c].lo[a] = lo;
    cube[c].hi[a] = hi;
    double e = __dsub_rn((double)hi, (double)lo);
    if (e > side) side = e;
  }
  if (side == 0.0) side = 1.0;
  cube[c].side = side;
  cube[c].scale = 2097152.0 / side;
  cube[c].nonfinite = acc[c].nonfinite;
}

// ------------------------------------------------------------ partition

// Split every segment into chunks of at most `chunk` points and the chunks
// into groups of at most kGroupChunks (one workgroup: prefix sums only).
constexpr int kChunkWG = 1024;
__global__ void __launch_bounds__(kChunkWG) k_chunk_scan(Segment* segs, const uint32_t* nseg_ptr, uint32_t chunk,
                                                         uint32_t* nchunk_ptr, uint32_t max_chunks,
                                                         uint32_t* ngroup_ptr, uint32_t max_groups) {
  __shared__ uint32_t sh[kChunkWG / 64 + 1];
  const uint32_t nseg = *nseg_ptr;
  uint32_t cbase = 0, gbase = 0;
  for (uint32_t s0 = 0; s0 < nseg; s0 += kChunkWG) {
    const uint32_t s = s0 + threadIdx.x;
    uint32_t cnt = 0, grp = 0;
    if (s < nseg) {
      cnt = (segs[s].count + chunk - 1) / chunk;
      grp = (cnt + kGroupChunks - 1) / kGroupChunks;
    }
    uint32_t ctot, gtot;
    const uint32_t cex = block_excl_scan<kChunkWG>(cnt, sh, &ctot);
    const uint32_t gex = block_excl_scan<kChunkWG>(grp, sh, &gtot);
    if (s < nseg) {
      segs[s].chunk_begin = cbase + cex;
      segs[s].chunk_count = cnt;
      segs[s].group_begin = gbase + gex;
      segs[s].group_count = grp;
    }
    cbase += ctot;
    gbase += gtot;
  }
  if (threadIdx.x == 0) {
    *nchunk_ptr = min(cbase, max_chunks);
    *ngroup_ptr = min(gbase, max_groups);
  }
}

// Largest segment index whose `first` field is <= x (segments are ordered).
__device__ __forceinline__ uint32_t find_segment(const Segment* segs, uint32_t nseg, uint32_t x, bool groups) {
  uint32_t lo = 0, hi = nseg - 1;
  while (lo < hi) {
    const uint32_t mid = (lo + hi + 1) >> 1;
    const uint32_t f = groups ? segs[mid].group_begin : segs[mid].chunk_begin;
    if (f <= x) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

__global__ void k_chunk_fill(const Segment* __restrict__ segs, const uint32_t* nseg_ptr, uint32_t chunk,
                             Chunk* chunks, const uint32_t* nchunk_ptr, ChunkGroup* groups,
                             const uint32_t* ngroup_ptr) {
  const uint32_t nseg = *nseg_ptr, nchunk = *nchunk_ptr, ngroup = *ngroup_ptr;
  if (nseg == 0) return;
  const uint32_t stride = gridDim.x * blockDim.x;
  for (uint32_t c = blockIdx.x * blockDim.x + threadIdx.x; c < nchunk; c += stride) {
    const uint32_t s = find_segment(segs, nseg, c, false);
    const Segment sg = segs[s];
    const uint32_t k = c - sg.chunk_begin;
    Chunk ch;
    ch.seg = s;
    ch.start = sg.start + k * chunk;
    ch.count = min(chunk, sg.count - k * chunk);
    ch.pad = 0;
    chunks[c] = ch;
  }
  for (uint32_t g = blockIdx.x * blockDim.x + threadIdx.x; g < ngroup; g += stride) {
    const uint32_t s = find_segment(segs, nseg, g, true);
    const Segment sg = segs[s];
    const uint32_t k = g - sg.group_begin;
    ChunkGroup gr;
    gr.seg = s;
    gr.first = sg.chunk_begin + k * kGroupChunks;
    gr.count = min(kGroupChunks, sg.chunk_count - k * kGroupChunks);
    gr.index = k;
    groups[g] = gr;
  }
}

// Count one chunk into an LDS histogram of B = 8^E cells and write the row
// (each workgroup takes chunks blockIdx.x, blockIdx.x + gridDim.x, ... of the
// device-side chunk count).
constexpr int kCountWG = 1024;
template <int E>
__global__ void __launch_bounds__(kCountWG) k_part_count(const uint4* __restrict__ pts, const Cube* cube,
                                                         const Segment* __restrict__ segs,
                                                         const Chunk* __restrict__ chunks,
                                                         const uint32_t* nchunk_ptr, uint32_t* __restrict__ hist) {
  constexpr uint32_t B = 1u << (3 * E);
  __shared__ uint32_t h[B];
  const uint32_t nchunk = *nchunk_ptr;
  for (uint32_t c = blockIdx.x; c < nchunk; c += gridDim.x) {
  const Chunk ch = chunks[c];
  const Segment sg = segs[ch.seg];
  for (uint32_t j = threadIdx.x; j < B; j += kCountWG) h[j] = 0;
  lds_barrier();
  uint32_t i = threadIdx.x;
  const CubeD cd = load_cube(cube + sg.cloud);
  const uint32_t lvl_bit = kKeyLevels - (sg.level + E);  // the E levels below the segment's level
  const uint4* p = pts + ch.start;
  for (; i + 7 * kCountWG < ch.count; i += 8 * kCountWG) {
    uint4 v[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) v[k] = p[i + k * kCountWG];
#pragma unroll
    for (int k = 0; k < 8; ++k)
      atomicAdd(&h[point_cell(__uint_as_float(v[k].x), __uint_as_float(v[k].y), __uint_as_float(v[k].z), cd, lvl_bit, E)],
                1u);
  }
  for (; i < ch.count; i += kCountWG) {
    uint4 v = p[i];
    atomicAdd(&h[point_cell(__uint_as_float(v.x), __uint_as_float(v.y), __uint_as_float(v.z), cd, lvl_bit, E)], 1u);
  }
  lds_barrier();
  uint32_t* row = hist + (uint64_t)c * B;
  for (uint32_t j = threadIdx.x; j < B; j += kCountWG) row[j] = h[j];
  lds_barrier();
  }
}

// k_part_count() from the cells the previous insert stored beside the
// records (one 16-bit cell per record, in the records' order).
template <int E>
__global__ void __launch_bounds__(kCountWG) k_part_count_dig(const uint16_t* __restrict__ dig,
                                                             const Chunk* __restrict__ chunks,
                                                             const uint32_t* nchunk_ptr, uint32_t* __restrict__ hist) {
  constexpr uint32_t B = 1u << (3 * E);
  __shared__ uint32_t h[B];
  const uint32_t nchunk = *nchunk_ptr;
  for (uint32_t c = blockIdx.x; c < nchunk; c += gridDim.x) {
    const Chunk ch = chunks[c];
    for (uint32_t j = threadIdx.x; j < B; j += kCountWG) h[j] = 0;
    lds_barrier();
    const uint16_t* p = dig + ch.start;
    uint32_t i = threadIdx.x;
    for (; i + 7 * kCountWG < ch.count; i += 8 * kCountWG) {
      uint32_t d[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) d[k] = p[i + k * kCountWG];
#pragma unroll
      for (int k = 0; k < 8; ++k) atomicAdd(&h[d[k]], 1u);
    }
    for (; i < ch.count; i += kCountWG) atomicAdd(&h[p[i]], 1u);
    lds_barrier();
    uint32_t* row = hist + (uint64_t)c * B;
    for (uint32_t j = threadIdx.x; j < B; j += kCountWG) row[j] = h[j];
    lds_barrier();
  }
}

// Column scan of the chunk rows, in three steps so that no thread walks more
// than kGroupChunks rows: (1) per (group, cell) sums, (2) per (segment, cell)
// exclusive scan over the segment's groups, whose total is the segment's cell
// count (the finest level of its grid), (3) per (group, cell) rewrite of the
// rows as exclusive offsets within the segment.
__global__ void k_colscan_groups(const ChunkGroup* __restrict__ groups, const uint32_t* ngroup_ptr, uint32_t E,
                                 const uint32_t* __restrict__ hist, uint32_t* __restrict__ gsum) {
  const uint32_t B = 1u << (3 * E);
  const uint64_t total = (uint64_t)*ngroup_ptr << (3 * E);
  for (uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (uint64_t)gridDim.x * blockDim.x) {
    const uint32_t g = (uint32_t)(t >> (3 * E)), b = (uint32_t)(t & (B - 1));
    const ChunkGroup gr = groups[g];
    uint32_t s = 0;
    for (uint32_t k = 0; k < gr.count; ++k) s += hist[(uint64_t)(gr.first + k) * B + b];
    gsum[(uint64_t)g * B + b] = s;
  }
}

__global__ void k_colscan_segments(const Segment* __restrict__ segs, const uint32_t* nseg_ptr, uint32_t E,
                                   uint32_t* __restrict__ gsum, const GridDesc* __restrict__ grids, uint32_t* pool) {
  const uint32_t B = 1u << (3 * E);
  const uint64_t total = (uint64_t)*nseg_ptr << (3 * E);
  for (uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (uint64_t)gridDim.x * blockDim.x) {
    const uint32_t s = (uint32_t)(t >> (3 * E)), b = (uint32_t)(t & (B - 1));
    const Segment sg = segs[s];
    uint32_t run = 0;
    for (uint32_t k = 0; k < sg.group_count; ++k) {
      uint32_t* cell = gsum + (uint64_t)(sg.group_begin + k) * B + b;
      const uint32_t v = *cell;
      *cell = run;
      run += v;
    }
    pool[grids[sg.grid].pyr + pyr_level_offset(E) + b] = run;
  }
}

__global__ void k_colscan_apply(const ChunkGroup* __restrict__ groups, const uint32_t* ngroup_ptr, uint32_t E,
                                uint32_t* __restrict__ hist, const uint32_t* __restrict__ gsum) {
  const uint32_t B = 1u << (3 * E);
  const uint64_t total = (uint64_t)*ngroup_ptr << (3 * E);
  for (uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (uint64_t)gridDim.x * blockDim.x) {
    const uint32_t g = (uint32_t)(t >> (3 * E)), b = (uint32_t)(t & (B - 1));
    const ChunkGroup gr = groups[g];
    uint32_t run = gsum[(uint64_t)g * B + b];
    for (uint32_t k = 0; k < gr.count; ++k) {
      uint32_t* cell = hist + (uint64_t)(gr.first + k) * B + b;
      const uint32_t v = *cell;
      *cell = run;
      run += v;
    }
  }
}

// Finish the grids of a partition: finest-cell offsets (exclusive prefix sum
// plus the segment start: the target offsets of counting sort, Sec. 4.1.3),
// the count pyramid above (Sec. 4.1.2 merges 2x2x2 groups level by level),
// and no child grids yet.
constexpr int kGridWG = 1024;
__global__ void __launch_bounds__(kGridWG) k_grid_finish(const Segment* __restrict__ segs, const uint32_t* nseg_ptr,
                                                         const GridDesc* __restrict__ grids, uint32_t* pool) {
  __shared__ uint32_t sh[kGridWG / 64 + 1];
  const uint32_t nseg = *nseg_ptr;
  for (uint32_t s = blockIdx.x; s < nseg; s += gridDim.x) {
  const Segment sg = segs[s];
  const GridDesc g = grids[sg.grid];
  const uint32_t E = g.e;
  const uint32_t B = 1u << (3 * E);
  uint32_t* fin = pool + g.pyr + pyr_level_offset(E);
  uint32_t* off = pool + g.off;
  int32_t* child = (int32_t*)(pool + g.child);
  // exclusive scan, each thread owning a contiguous run of B / kGridWG cells
  const uint32_t per = (B + kGridWG - 1) / kGridWG;
  const uint32_t b0 = threadIdx.x * per;
  uint32_t local = 0;
  for (uint32_t k = 0; k < per; ++k)
    if (b0 + k < B) local += fin[b0 + k];
  uint32_t tot;
  uint32_t ex = block_excl_scan<kGridWG>(local, sh, &tot);
  uint32_t run = sg.start + ex;
  for (uint32_t k = 0; k < per; ++k)
    if (b0 + k < B) {
      off[b0 + k] = run;
      run += fin[b0 + k];
      child[b0 + k] = -1;
    }
  __syncthreads();
  for (int j = (int)E - 1; j >= 0; --j) {
    uint32_t* up = pool + g.pyr + pyr_level_offset((uint32_t)j);
    const uint32_t* dn = pool + g.pyr + pyr_level_offset((uint32_t)j + 1);
    const uint32_t nj = 1u << (3 * j);
    for (uint32_t i = threadIdx.x; i < nj; i += kGridWG) {
      uint32_t v = 0;
      for (int o = 0; o < 8; ++o) v += dn[8 * i + o];
      up[i] = v;
    }
    __syncthreads();
  }
  }
}

// Insert (Sec. 4.1.4): move every point of a chunk to its cell.  A round of
// R = WG * PPT points is sorted by cell in LDS (counting sort: LDS histogram,
// workgroup prefix sum, staging), then written out so that consecutive lanes
// store consecutive records of the same cell.  The per-cell output cursors
// start at the chunk's target offsets and advance round by round; they live
// in registers (thread t owns cells t*BPT .. t*BPT+BPT-1), so that a single
// LDS array of cell counts serves the histogram, the staging offsets and the
// output deltas, and the rest of LDS holds as large a round as possible: the
// stores of a round are runs of consecutive records per cell, and longer runs
// write HBM more efficiently.
constexpr int kScatWG = 1024;
// Workgroups of a count or insert launch at most; each takes every
// gridDim.x-th chunk of the device-side chunk list.
constexpr uint32_t kMaxPartBlocks = 4096;
// Workgroups of the one-chunk insert launch at most (a launch holds fewer
// than 2^32 threads).
constexpr uint32_t kMaxOneChunkBlocks = 1u << 20;
#define PAD(b) ((b) + ((b) >> 5))
template <bool IDS>
struct ScatShape {
  static constexpr int PPT = IDS ? 6 : 7;  // LDS: R*(16 + 2 + 4*IDS) bytes of staging + 16.5 KB of counts
  static constexpr int R = kScatWG * PPT;
};

// Workgroup b takes chunk c0 + b; with LOOP also c0 + b + gridDim.x, ...
// (looping keeps more registers live: the one-chunk form covers the chunks
// a partition can be expected to have, the looping form any beyond).
template <int E, bool IDS, bool LOOP>
__global__ void __launch_bounds__(kScatWG) k_part_scatter(const uint4* __restrict__ src, const uint32_t* __restrict__ src_ids,
                                                          uint4* __restrict__ dst, uint32_t* __restrict__ dst_ids,
                                                          const Cube* cube, const Segment* __restrict__ segs,
                                                          const Chunk* __restrict__ chunks, const uint32_t* nchunk_ptr,
                                                          const uint32_t* __restrict__ hist,
                                                          const GridDesc* __restrict__ grids, const uint32_t* __restrict__ pool,
                                                          uint16_t* __restrict__ dig, uint32_t c0) {
  constexpr int PPT = ScatShape<IDS>::PPT;
  constexpr uint32_t R = ScatShape<IDS>::R;
  constexpr uint32_t B = 1u << (3 * E);
  constexpr uint32_t BPT = (B + kScatWG - 1) / kScatWG;  // cells per thread in the scan
  // one padding word per 32 cells: the scan's per-thread runs of BPT cells
  // then fall on distinct LDS banks
  constexpr uint32_t BP = B + B / 32 + 1;
  __shared__ uint32_t cnt[BP];
  __shared__ uint4 stage[R];
  __shared__ uint16_t stage_b[R];
  __shared__ uint32_t stage_id[IDS ? R : 1];
  __shared__ uint32_t sh[kScatWG / 64 + 1];
  const uint32_t nchunk = *nchunk_ptr;
  for (uint32_t c = c0 + blockIdx.x; c < nchunk; c += gridDim.x) {
  if (LOOP) lds_barrier();  // the previous chunk's last reads of LDS are done
  const Chunk ch = chunks[c];
  const Segment sg = segs[ch.seg];
  const GridDesc g = grids[sg.grid];
  const CubeD cd = load_cube(cube + sg.cloud);
  const uint32_t lvl_bit = kKeyLevels - (sg.level + E);  // the E levels below the segment's level
  const uint32_t* row = hist + (uint64_t)c * B;
  const uint32_t* goff = pool + g.off;
  // without source ids (the first pass over the input, one segment per
  // cloud) a point's id is its index in its cloud
  const uint32_t ch_cloud_start = sg.start;
  uint32_t cur[BPT];
#pragma unroll
  for (uint32_t k = 0; k < BPT; ++k) {
    const uint32_t b = threadIdx.x * BPT + k;
    cur[k] = b < B ? goff[b] + row[b] : 0u;
  }
  for (uint32_t j = threadIdx.x; j < B; j += kScatWG) cnt[PAD(j)] = 0;
  lds_barrier();
  // software pipeline: the records of round r + 1 are loaded while round r is
  // sorted in LDS and written out
  uint4 v[PPT];
  uint32_t id[PPT];
  auto load_round = [&](uint32_t base, uint4* vv, uint32_t* ii) {
    const uint32_t nround = base < ch.count ? min(R, ch.count - base) : 0u;
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
      const uint32_t j = k * kScatWG + threadIdx.x;
      if (j < nround) {
        const uint32_t gi = ch.start + base + j;
        vv[k] = src[gi];
        if (IDS) ii[k] = src_ids ? src_ids[gi] : gi - ch_cloud_start;
      }
    }
  };
  load_round(0, v, id);
  for (uint32_t base = 0; base < ch.count; base += R) {
    const uint32_t nround = min(R, ch.count - base);
    uint32_t bk[PPT], rk[PPT];
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
      const uint32_t j = k * kScatWG + threadIdx.x;
      if (j < nround) {
        bk[k] = point_cell(__uint_as_float(v[k].x), __uint_as_float(v[k].y), __uint_as_float(v[k].z), cd, lvl_bit, E);
        rk[k] = atomicAdd(&cnt[PAD(bk[k])], 1u);
      }
    }
    uint4 vn[PPT];
    uint32_t idn[PPT];
    load_round(base + R, vn, idn);
    lds_barrier();
    // exclusive scan of the round's cell counts (in place); counts and
    // prefixes stay in registers
    uint32_t mine[BPT], exk[BPT];
    uint32_t local = 0;
#pragma unroll
    for (uint32_t k = 0; k < BPT; ++k) {
      const uint32_t b = threadIdx.x * BPT + k;
      mine[k] = b < B ? cnt[PAD(b)] : 0u;
      local += mine[k];
    }
    uint32_t tot;
    uint32_t ex = block_excl_scan<kScatWG>(local, sh, &tot);
#pragma unroll
    for (uint32_t k = 0; k < BPT; ++k) {
      const uint32_t b = threadIdx.x * BPT + k;
      exk[k] = ex;
      if (b < B) cnt[PAD(b)] = ex;
      ex += mine[k];
    }
    lds_barrier();
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
      const uint32_t j = k * kScatWG + threadIdx.x;
      if (j < nround) {
        const uint32_t pos = cnt[PAD(bk[k])] + rk[k];
        stage[pos] = v[k];
        stage_b[pos] = (uint16_t)bk[k];
        if (IDS) stage_id[pos] = id[k];
      }
    }
    lds_barrier();
    // staged position j of cell b goes to cursor(b) + (j - prefix(b))
#pragma unroll
    for (uint32_t k = 0; k < BPT; ++k) {
      const uint32_t b = threadIdx.x * BPT + k;
      if (b < B) cnt[PAD(b)] = cur[k] - exk[k];
      cur[k] += mine[k];
    }
    lds_barrier();
    for (uint32_t j = threadIdx.x; j < nround; j += kScatWG) {
      const uint32_t d = cnt[PAD(stage_b[j])] + j;
      const uint4 r = stage[j];
      dst[d] = r;
      if (IDS) dst_ids[d] = stage_id[j];
      // the record's cell in the next partition (E levels further down),
      // stored beside it so that the next count need not read the records
      if (dig) dig[d] = (uint16_t)point_cell(__uint_as_float(r.x), __uint_as_float(r.y), __uint_as_float(r.z), cd,
                                             lvl_bit - E, E);
    }
    lds_barrier();
#pragma unroll
    for (uint32_t k = 0; k < BPT; ++k) {
      const uint32_t b = threadIdx.x * BPT + k;
      if (b < B) cnt[PAD(b)] = 0;
    }
    lds_barrier();
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
      v[k] = vn[k];
      if (IDS) id[k] = idn[k];
    }
  }
  if (!LOOP) break;
  }
}

uint32_t scatter_round(bool ids) { return ids ? (uint32_t)ScatShape<true>::R : (uint32_t)ScatShape<false>::R; }

// Copy the points (and ids) of every segment from one buffer to the other;
// kCopySplit workgroups share a segment (refinement lists are short and
// their segments large).
constexpr uint32_t kCopySplit = 64;
__global__ void __launch_bounds__(256) k_copy_segments(const uint4* __restrict__ src, const uint32_t* __restrict__ src_ids,
                                                       uint4* __restrict__ dst, uint32_t* __restrict__ dst_ids,
                                                       const Segment* __restrict__ segs, const uint32_t* nseg_ptr) {
  const uint32_t nseg = *nseg_ptr;
  for (uint32_t s = blockIdx.x; s < nseg; s += gridDim.x) {
    const Segment sg = segs[s];
    for (uint32_t i = blockIdx.y * 256 + threadIdx.x; i < sg.count; i += kCopySplit * 256) {
      dst[sg.start + i] = src[sg.start + i];
      if (dst_ids) dst_ids[sg.start + i] = src_ids[sg.start + i];
    }
  }
}

// One segment per non-empty finest cell of every root grid (grids 0 ..
// ngrids-1, one workgroup each), each with its own grid descriptor, to be
// partitioned by E2 more levels.  Segments are appended in any order; the
// segment counter must start at 0.
__global__ void __launch_bounds__(kChunkWG) k_segments_from_grid(GridDesc* grids, uint32_t* pool, uint32_t E2,
                                                                 uint64_t slot_base, uint32_t first_grid,
                                                                 Segment* segs, uint32_t* nseg_ptr) {
  __shared__ uint32_t sh[kChunkWG / 64 + 1];
  __shared__ uint32_t s_base;
  const uint32_t g0 = blockIdx.x;
  const GridDesc g = grids[g0];
  const uint32_t B = 1u << (3 * g.e);
  const uint32_t* fin = pool + g.pyr + pyr_level_offset(g.e);
  const uint32_t* off = pool + g.off;
  int32_t* child = (int32_t*)(pool + g.child);
  const uint64_t words = grid_words(E2);
  for (uint32_t b0 = 0; b0 < B; b0 += kChunkWG) {
    const uint32_t b = b0 + threadIdx.x;
    const uint32_t cnt = b < B ? fin[b] : 0u;
    uint32_t tot;
    const uint32_t ex = block_excl_scan<kChunkWG>(cnt ? 1u : 0u, sh, &tot);
    if (threadIdx.x == 0) s_base = tot ? atomicAdd(nseg_ptr, tot) : 0u;
    __syncthreads();
    if (cnt) {
      const uint32_t s = s_base + ex;
      const uint32_t gi = first_grid + s;
      Segment sg;
      sg.start = off[b];
      sg.count = cnt;
      sg.grid = gi;
      sg.level = g.base_level + g.e;
      sg.chunk_begin = 0;
      sg.chunk_count = 0;
      sg.key = (g.base_key << (3 * g.e)) | b;
      sg.group_begin = 0;
      sg.group_count = 0;
      sg.cloud = g0;
      sg.pad = 0;
      segs[s] = sg;
      GridDesc d;
      d.base_level = sg.level;
      d.e = E2;
      d.base_key = sg.key;
      d.pyr = slot_base + (uint64_t)s * words;
      d.off = d.pyr + pyr_level_offset(E2 + 1);
      d.child = d.off + ((uint64_t)1 << (3 * E2));
      d.seg_start = sg.start;
      d.seg_count = cnt;
      grids[gi] = d;
      child[b] = (int32_t)gi;
    }
    __syncthreads();
  }
}

// One root segment and root grid (E0 levels, pool slot c) per cloud.
__global__ void k_init_roots(const CloudInfo* clouds, uint32_t nclouds, uint32_t E0, Segment* segs, uint32_t* nseg_ptr,
                             GridDesc* grids) {
  const uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c == 0) *nseg_ptr = nclouds;
  if (c >= nclouds) return;
  Segment sg;
  sg.start = clouds[c].start;
  sg.count = clouds[c].count;
  sg.grid = c;
  sg.level = 0;
  sg.chunk_begin = 0;
  sg.chunk_count = 0;
  sg.key = 0;
  sg.group_begin = 0;
  sg.group_count = 0;
  sg.cloud = c;
  sg.pad = 0;
  segs[c] = sg;
  GridDesc d;
  d.base_level = 0;
  d.e = E0;
  d.base_key = 0;
  d.pyr = (uint64_t)c * grid_words(E0);
  d.off = d.pyr + pyr_level_offset(E0 + 1);
  d.child = d.off + ((uint64_t)1 << (3 * E0));
  d.seg_start = sg.start;
  d.seg_count = sg.count;
  grids[c] = d;
}

// ------------------------------------------------------------ fills

__global__ void k_fill_u32(uint32_t* p, uint32_t v, uint64_t n) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ void k_build_init(BuildState* bs, uint32_t num_grids, uint64_t used_words) {
  BuildState z;
  memset(&z, 0, sizeof(z));
  z.num_grids = z.need_grids = num_grids;
  z.used_words = z.need_words = used_words;
  *bs = z;
}

// ------------------------------------------------------------ launchers

void launch_fill_u32(uint32_t* p, uint32_t v, uint64_t n, hipStream_t st) {
  if (!n) return;
  hipLaunchKernelGGL(k_fill_u32, dim3((uint32_t)std::min<uint64_t>((n + 255) / 256, 4096)), dim3(256), 0, st, p, v, n);
}

void launch_build_init(BuildState* bs, uint32_t num_grids, uint64_t used_words, hipStream_t st) {
  hipLaunchKernelGGL(k_build_init, dim3(1), dim3(1), 0, st, bs, num_grids, used_words);
}

uint32_t bbox_tiles(uint32_t count) { return (count + kBBoxTile - 1) / kBBoxTile; }

void launch_bbox(const void* pts, const CloudInfo* clouds, uint32_t nclouds, uint32_t ntiles, BBoxAcc* acc, Cube* cube,
                 hipStream_t st) {
  const uint32_t cb = (nclouds + 255) / 256;
  hipLaunchKernelGGL(k_bbox_init, dim3(cb), dim3(256), 0, st, acc, nclouds);
  if (ntiles) hipLaunchKernelGGL(k_bbox, dim3(ntiles), dim3(kBBoxWG), 0, st, (const uint4*)pts, clouds, nclouds, acc);
  hipLaunchKernelGGL(k_cube, dim3(cb), dim3(256), 0, st, acc, clouds, nclouds, cube);
}

void launch_bbox_reset(BBoxAcc* acc, hipStream_t st) {
  hipLaunchKernelGGL(k_bbox_init, dim3(1), dim3(256), 0, st, acc, 1u);
}

void launch_bbox_add(const void* pts, const CloudInfo* piece, uint32_t ntiles, BBoxAcc* acc, hipStream_t st) {
  if (ntiles) hipLaunchKernelGGL(k_bbox, dim3(ntiles), dim3(kBBoxWG), 0, st, (const uint4*)pts, piece, 1u, acc);
}

void launch_bbox_cube(const BBoxAcc* acc, const CloudInfo* whole, Cube* cube, hipStream_t st) {
  hipLaunchKernelGGL(k_cube, dim3(1), dim3(256), 0, st, acc, whole, 1u, cube);
}

void launch_init_roots(const CloudInfo* clouds, uint32_t nclouds, uint32_t E0, Segment* segs, uint32_t* nseg,
                       GridDesc* grids, hipStream_t st) {
  hipLaunchKernelGGL(k_init_roots, dim3((nclouds + 255) / 256), dim3(256), 0, st, clouds, nclouds, E0, segs, nseg,
                     grids);
}

void launch_make_chunks(Segment* segs, const uint32_t* nseg, uint32_t max_segs, uint32_t chunk, Chunk* chunks,
                        uint32_t* nchunk, uint32_t max_chunks, ChunkGroup* groups, uint32_t* ngroup,
                        uint32_t max_groups, hipStream_t st) {
  hipLaunchKernelGGL(k_chunk_scan, dim3(1), dim3(kChunkWG), 0, st, segs, nseg, chunk, nchunk, max_chunks, ngroup,
                     max_groups);
  uint32_t blocks = (max_chunks + max_segs + 255) / 256;
  if (blocks > 2048) blocks = 2048;
  hipLaunchKernelGGL(k_chunk_fill, dim3(blocks ? blocks : 1), dim3(256), 0, st, segs, nseg, chunk, chunks, nchunk,
                     groups, ngroup);
}

template <int E>
static void count_e(const void* pts, const uint16_t* dig, const Cube* cube, const Segment* segs, const Chunk* chunks,
                    const uint32_t* nchunk, uint32_t max_chunks, uint32_t* hist, hipStream_t st) {
  const uint32_t blocks = std::min<uint32_t>(max_chunks, kMaxPartBlocks);
  if (dig)
    hipLaunchKernelGGL((k_part_count_dig<E>), dim3(blocks), dim3(kCountWG), 0, st, dig, chunks, nchunk, hist);
  else
    hipLaunchKernelGGL((k_part_count<E>), dim3(blocks), dim3(kCountWG), 0, st, (const uint4*)pts, cube, segs, chunks,
                       nchunk, hist);
}

void launch_part_count(uint32_t E, const void* pts, const uint16_t* dig, const Cube* cube, const Segment* segs,
                       const Chunk* chunks, const uint32_t* nchunk, uint32_t max_chunks, uint32_t* hist,
                       hipStream_t st) {
  if (!max_chunks) return;
  switch (E) {
    case 1: count_e<1>(pts, dig, cube, segs, chunks, nchunk, max_chunks, hist, st); break;
    case 2: count_e<2>(pts, dig, cube, segs, chunks, nchunk, max_chunks, hist, st); break;
    case 3: count_e<3>(pts, dig, cube, segs, chunks, nchunk, max_chunks, hist, st); break;
    case 4: count_e<4>(pts, dig, cube, segs, chunks, nchunk, max_chunks, hist, st); break;
    default: break;
  }
}

static uint32_t stride_blocks(uint64_t threads) {
  return (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>((threads + 255) / 256, 8192));
}

void launch_part_colscan(const Segment* segs, const uint32_t* nseg, uint32_t max_segs, const ChunkGroup* groups,
                         const uint32_t* ngroup, uint32_t max_groups, uint32_t E, uint32_t* hist, uint32_t* gsum,
                         const GridDesc* grids, uint32_t* pool, hipStream_t st) {
  if (!max_segs) return;
  const uint64_t tg = (uint64_t)max_groups << (3 * E);
  const uint64_t ts = (uint64_t)max_segs << (3 * E);
  hipLaunchKernelGGL(k_colscan_groups, dim3(stride_blocks(tg)), dim3(256), 0, st, groups, ngroup, E, hist, gsum);
  hipLaunchKernelGGL(k_colscan_segments, dim3(stride_blocks(ts)), dim3(256), 0, st, segs, nseg, E, gsum, grids, pool);
  hipLaunchKernelGGL(k_colscan_apply, dim3(stride_blocks(tg)), dim3(256), 0, st, groups, ngroup, E, hist, gsum);
}

void launch_grid_finish(const Segment* segs, const uint32_t* nseg, uint32_t max_segs, const GridDesc* grids,
                        uint32_t* pool, hipStream_t st) {
  if (!max_segs) return;
  hipLaunchKernelGGL(k_grid_finish, dim3(std::min<uint32_t>(max_segs, 2048)), dim3(kGridWG), 0, st, segs, nseg, grids,
                     pool);
}

template <int E, bool IDS>
static void scatter_e(const void* src, const uint32_t* src_ids, void* dst, uint32_t* dst_ids, uint16_t* dig,
                      const Cube* cube, const Segment* segs, const Chunk* chunks, const uint32_t* nchunk,
                      uint32_t max_chunks, uint32_t expect_chunks, const uint32_t* hist, const GridDesc* grids,
                      const uint32_t* pool, hipStream_t st) {
  // one workgroup per expected chunk (those past the real count return at
  // once), then a grid that loops over any chunks beyond
  const uint32_t g1 = std::max<uint32_t>(1, std::min(std::min(max_chunks, expect_chunks), kMaxOneChunkBlocks));
  hipLaunchKernelGGL((k_part_scatter<E, IDS, false>), dim3(g1), dim3(kScatWG), 0, st, (const uint4*)src, src_ids,
                     (uint4*)dst, dst_ids, cube, segs, chunks, nchunk, hist, grids, pool, dig, 0u);
  if (max_chunks > g1)
    hipLaunchKernelGGL((k_part_scatter<E, IDS, true>), dim3(std::min<uint32_t>(max_chunks - g1, kMaxPartBlocks)),
                       dim3(kScatWG), 0, st, (const uint4*)src, src_ids, (uint4*)dst, dst_ids, cube, segs, chunks,
                       nchunk, hist, grids, pool, dig, g1);
}

void launch_part_scatter(uint32_t E, bool ids, const void* src, const uint32_t* src_ids, void* dst, uint32_t* dst_ids,
                         uint16_t* dig, const Cube* cube, const Segment* segs, const Chunk* chunks,
                         const uint32_t* nchunk, uint32_t max_chunks, uint32_t expect_chunks, const uint32_t* hist,
                         const GridDesc* grids, const uint32_t* pool, hipStream_t st) {
  if (!max_chunks) return;
#define LOD_SCAT(EE)                                                                                                   \
  case EE:                                                                                                             \
    if (ids) scatter_e<EE, true>(src, src_ids, dst, dst_ids, dig, cube, segs, chunks, nchunk, max_chunks,             \
                                 expect_chunks, hist, grids, pool, st);                                                \
    else scatter_e<EE, false>(src, src_ids, dst, dst_ids, dig, cube, segs, chunks, nchunk, max_chunks, expect_chunks, \
                              hist, grids, pool, st);                                                                  \
    break;
  switch (E) {
    LOD_SCAT(1)
    LOD_SCAT(2)
    LOD_SCAT(3)
    LOD_SCAT(4)
    default: break;
  }
#undef LOD_SCAT
}

void launch_copy_segments(const void* src, const uint32_t* src_ids, void* dst, uint32_t* dst_ids, const Segment* segs,
                          const uint32_t* nseg, uint32_t max_segs, hipStream_t st) {
  if (!max_segs) return;
  hipLaunchKernelGGL(k_copy_segments, dim3(std::min<uint32_t>(max_segs, 256), kCopySplit), dim3(256), 0, st,
                     (const uint4*)src, src_ids,
                     (uint4*)dst, dst_ids, segs, nseg);
}

void launch_segments_from_grid(GridDesc* grids, uint32_t ngrids, uint32_t* pool, uint32_t E2, uint64_t slot_base,
                               uint32_t first_grid, Segment* segs, uint32_t* nseg, hipStream_t st) {
  hipLaunchKernelGGL(k_segments_from_grid, dim3(ngrids), dim3(kChunkWG), 0, st, grids, pool, E2, slot_base, first_grid,
                     segs, nseg);
}

}  // namespace lod
