// k_merge.hip -- kernels of the chunked build (Sec. 7: chunks of a bottom-up
// out-of-core pipeline, merged into one octree).
//
// The input is cut along the cells of one level b of the common bounding
// cube: each piece of the input that passes through the GPU is counted and
// sorted by cell here (a counting sort; with few cells, counts and ranks in
// LDS), so that a cell's points are one run per piece.  A cell with more
// than T points is an inner node of the whole tree at level b, and its
// subtree depends on its own points only, so it is built as a chunk.  The
// levels above b are then sampled here from the chunk roots'
// voxels and the points of the small leaves above them, with the cell
// average and pick rules of Sec. 4.2:
//   * every (parent, child octant) pair is a job with a dense grid of the
//     64^3 parent cells that the octant covers;
//   * each sample (a child voxel: 2x2x2 child cells per parent cell; or a
//     point) adds to its cell: R, G, B sums and a count, or the best pick
//     order; a second pass lets the winning sample write its colour and id;
//   * each grid's occupied cells are emitted in Morton order, so a parent's
//     voxel list is its jobs' outputs in octant order;
//   * the weighted average (Sec. 4.2.4) counts samples per cell the same way
//     (its occupied cells are the average's), then every sample splats onto
//     the up to 2x2x2 cells around it in its parent's grid -- also across
//     octants, so a parent's eight jobs share a launch -- with the exact
//     integer weights of the in-core weighted pass.
#include "common.h"
#include "launch.h"
#include "scan.h"
#include "weighted.h"

namespace lod {

// The level-h cell (h <= 7) of each of n points, and a histogram of them.
__global__ void __launch_bounds__(256) k_cells(const uint4* __restrict__ pts, uint32_t n, const Cube* cube, uint32_t h,
                                               uint32_t* __restrict__ cell, uint32_t* hist) {
  const uint32_t i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const CubeD cd = load_cube(cube);
  const uint4 v = pts[i];
  const uint32_t s = kKeyLevels - h;
  const uint32_t c = morton7(quantize(__uint_as_float(v.x), cd.lo[0], cd.scale) >> s,
                             quantize(__uint_as_float(v.y), cd.lo[1], cd.scale) >> s,
                             quantize(__uint_as_float(v.z), cd.lo[2], cd.scale) >> s);
  cell[i] = c;
  atomicAdd(hist + c, 1u);
}

// The same for levels of at most 4096 cells (h <= 4): a workgroup counts a
// tile of 4096 points in LDS and adds each cell once, so few cells do not
// serialize millions of global atomics.
constexpr uint32_t kCellTile = 4096;  // 16 points per thread
constexpr uint32_t kLdsCells = 4096;

__global__ void __launch_bounds__(256) k_cells_lds(const uint4* __restrict__ pts, uint32_t n, const Cube* cube,
                                                   uint32_t h, uint32_t* __restrict__ cell, uint32_t* hist) {
  __shared__ uint32_t lh[kLdsCells];
  const uint32_t nb = 1u << (3 * h), t = threadIdx.x;
  for (uint32_t c = t; c < nb; c += 256) lh[c] = 0;
  __syncthreads();
  const CubeD cd = load_cube(cube);
  const uint32_t s = kKeyLevels - h;
  for (uint32_t k = 0; k < kCellTile / 256; ++k) {
    const uint32_t i = blockIdx.x * kCellTile + k * 256 + t;
    if (i >= n) break;
    const uint4 v = pts[i];
    const uint32_t c = morton7(quantize(__uint_as_float(v.x), cd.lo[0], cd.scale) >> s,
                               quantize(__uint_as_float(v.y), cd.lo[1], cd.scale) >> s,
                               quantize(__uint_as_float(v.z), cd.lo[2], cd.scale) >> s);
    cell[i] = c;
    atomicAdd(&lh[c], 1u);
  }
  __syncthreads();
  for (uint32_t c = t; c < nb; c += 256)
    if (lh[c]) atomicAdd(hist + c, lh[c]);
}

void launch_cells(const void* pts, uint32_t n, const Cube* cube, uint32_t h, uint32_t* cell, uint32_t* hist,
                  hipStream_t s) {
  if (!n) return;
  if ((1u << (3 * h)) <= kLdsCells)
    hipLaunchKernelGGL(k_cells_lds, dim3((n + kCellTile - 1) / kCellTile), dim3(256), 0, s, (const uint4*)pts, n,
                       cube, h, cell, hist);
  else
    hipLaunchKernelGGL(k_cells, dim3((n + 255) / 256), dim3(256), 0, s, (const uint4*)pts, n, cube, h, cell, hist);
}

// Counting sort of a piece by cell: exclusive prefix of the histogram (a
// workgroup per tile of 4096 bins, a one-workgroup pass over the tile sums,
// then the bins), then every point to its cell's next slot.  The order inside
// a cell is free (the build does not depend on it; ids travel along).
constexpr uint32_t kBinTile = 4096;  // 16 bins per thread

__global__ void __launch_bounds__(256) k_bin_tiles(const uint32_t* __restrict__ hist, uint32_t nbins,
                                                   uint32_t* __restrict__ tile_sum) {
  __shared__ uint32_t sh[256 / 64 + 1];
  const uint32_t b0 = blockIdx.x * kBinTile + threadIdx.x * 16;
  uint32_t sum = 0;
  for (uint32_t k = 0; k < 16; ++k)
    if (b0 + k < nbins) sum += hist[b0 + k];
  uint32_t tot;
  (void)block_excl_scan<256>(sum, sh, &tot);
  if (threadIdx.x == 0) tile_sum[blockIdx.x] = tot;
}

// In place: tile sums -> exclusive tile offsets (ntiles <= 256 * 4).
__global__ void __launch_bounds__(256) k_tile_offsets(uint32_t* tile_sum, uint32_t ntiles) {
  __shared__ uint32_t sh[256 / 64 + 1];
  const uint32_t t0 = threadIdx.x * 4;
  uint32_t v[4], sum = 0;
  for (uint32_t k = 0; k < 4; ++k) {
    v[k] = t0 + k < ntiles ? tile_sum[t0 + k] : 0u;
    sum += v[k];
  }
  uint32_t tot;
  uint32_t run = block_excl_scan<256>(sum, sh, &tot);
  for (uint32_t k = 0; k < 4; ++k) {
    if (t0 + k < ntiles) tile_sum[t0 + k] = run;
    run += v[k];
  }
}

__global__ void __launch_bounds__(256) k_bin_cursors(const uint32_t* __restrict__ hist, uint32_t nbins,
                                                     const uint32_t* __restrict__ tile_off, uint32_t* __restrict__ cursor) {
  __shared__ uint32_t sh[256 / 64 + 1];
  const uint32_t b0 = blockIdx.x * kBinTile + threadIdx.x * 16;
  uint32_t v[16], sum = 0;
  for (uint32_t k = 0; k < 16; ++k) {
    v[k] = b0 + k < nbins ? hist[b0 + k] : 0u;
    sum += v[k];
  }
  uint32_t tot;
  uint32_t run = tile_off[blockIdx.x] + block_excl_scan<256>(sum, sh, &tot);
  for (uint32_t k = 0; k < 16; ++k) {
    if (b0 + k < nbins) cursor[b0 + k] = run;
    run += v[k];
  }
}

__global__ void __launch_bounds__(256) k_scatter_cells(const uint4* __restrict__ pts, const uint32_t* __restrict__ cell,
                                                       uint32_t n, uint32_t id0, uint32_t* cursor,
                                                       uint4* __restrict__ out, uint32_t* __restrict__ out_ids) {
  const uint32_t i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const uint32_t pos = atomicAdd(cursor + cell[i], 1u);
  out[pos] = pts[i];
  if (out_ids) out_ids[pos] = id0 + i;
}

// Few cells: a workgroup ranks a tile of 4096 points per cell in LDS, then
// reserves each cell's slots with one global atomic.
__global__ void __launch_bounds__(256) k_scatter_cells_lds(const uint4* __restrict__ pts,
                                                           const uint32_t* __restrict__ cell, uint32_t n,
                                                           uint32_t nbins, uint32_t id0, uint32_t* cursor,
                                                           uint4* __restrict__ out, uint32_t* __restrict__ out_ids) {
  __shared__ uint32_t lc[kLdsCells], lb[kLdsCells];
  const uint32_t t = threadIdx.x;
  for (uint32_t c = t; c < nbins; c += 256) lc[c] = 0;
  __syncthreads();
  constexpr uint32_t K = kCellTile / 256;
  uint32_t cc[K], rk[K];
#pragma unroll
  for (uint32_t k = 0; k < K; ++k) {
    const uint32_t i = blockIdx.x * kCellTile + k * 256 + t;
    cc[k] = 0;
    rk[k] = 0;
    if (i < n) {
      cc[k] = cell[i];
      rk[k] = atomicAdd(&lc[cc[k]], 1u);
    }
  }
  __syncthreads();
  for (uint32_t c = t; c < nbins; c += 256) lb[c] = lc[c] ? atomicAdd(cursor + c, lc[c]) : 0u;
  __syncthreads();
#pragma unroll
  for (uint32_t k = 0; k < K; ++k) {
    const uint32_t i = blockIdx.x * kCellTile + k * 256 + t;
    if (i < n) {
      const uint32_t pos = lb[cc[k]] + rk[k];
      out[pos] = pts[i];
      if (out_ids) out_ids[pos] = id0 + i;
    }
  }
}

void launch_sort_by_cell(const void* pts, const uint32_t* cell, uint32_t n, uint32_t id0, const uint32_t* hist,
                         uint32_t nbins, uint32_t* tiles, uint32_t* cursor, void* out, uint32_t* out_ids,
                         hipStream_t s) {
  if (!n) return;
  const uint32_t ntiles = (nbins + kBinTile - 1) / kBinTile;
  hipLaunchKernelGGL(k_bin_tiles, dim3(ntiles), dim3(256), 0, s, hist, nbins, tiles);
  hipLaunchKernelGGL(k_tile_offsets, dim3(1), dim3(256), 0, s, tiles, ntiles);
  hipLaunchKernelGGL(k_bin_cursors, dim3(ntiles), dim3(256), 0, s, hist, nbins, (const uint32_t*)tiles, cursor);
  if (nbins <= kLdsCells)
    hipLaunchKernelGGL(k_scatter_cells_lds, dim3((n + kCellTile - 1) / kCellTile), dim3(256), 0, s,
                       (const uint4*)pts, cell, n, nbins, id0, cursor, (uint4*)out, out_ids);
  else
    hipLaunchKernelGGL(k_scatter_cells, dim3((n + 255) / 256), dim3(256), 0, s, (const uint4*)pts, cell, n, id0,
                       cursor, (uint4*)out, out_ids);
}

// ------------------------------------------------------------ top levels

// FIRST keeps the minimum pick order (a starts at ~0); the average's sums and
// RANDOM's maximum start at 0.
__global__ void __launch_bounds__(256) k_top_clear(TopCell* g, uint64_t ncells, unsigned long long a0) {
  for (uint64_t i = blockIdx.x * 256ull + threadIdx.x; i < ncells; i += (uint64_t)gridDim.x * 256) {
    TopCell c;
    c.a = a0;
    c.b = c.c = c.w = 0;
    c.n = 0;
    c.mid = 0xffffffffu;
    g[i] = c;
  }
}

// Cell (18-bit Morton code inside the job's octant) and colour of sample i.
__device__ __forceinline__ void top_sample(const TopJob& j, uint32_t i, const CubeD& cd, uint32_t& m, uint32_t& rgba) {
  if (j.kind == 0) {
    // a voxel of the child's 128^3 grid: two child cells per parent cell
    const uint64_t v = ((const uint64_t*)j.src)[i];
    m = morton7(((uint32_t)v & 0xffu) >> 1, ((uint32_t)(v >> 8) & 0xffu) >> 1, ((uint32_t)(v >> 16) & 0xffu) >> 1);
    rgba = (uint32_t)(v >> 32);
  } else {
    // a point: its cell at level L + 7, inside the child's octant
    const uint4 v = ((const uint4*)j.src)[i];
    const uint32_t s = kKeyLevels - (j.level + 7);
    m = morton7((quantize(__uint_as_float(v.x), cd.lo[0], cd.scale) >> s) & 63u,
                (quantize(__uint_as_float(v.y), cd.lo[1], cd.scale) >> s) & 63u,
                (quantize(__uint_as_float(v.z), cd.lo[2], cd.scale) >> s) & 63u);
    rgba = v.w;
  }
}

// MODE: 0 average, 1 first, 2 random, 3 count only (the weighted mode's
// occupancy).  Grid (x: slices of the samples, y: job).
template <int MODE>
__global__ void __launch_bounds__(256) k_top_splat(const TopJob* __restrict__ jobs, const Cube* cube, uint32_t seed,
                                                   bool full, TopCell* grids) {
  const TopJob j = jobs[blockIdx.y];
  TopCell* g = grids + (uint64_t)blockIdx.y * kTopCells;
  const CubeD cd = load_cube(cube);
  for (uint32_t i = blockIdx.x * 256 + threadIdx.x; i < j.count; i += gridDim.x * 256) {
    uint32_t m, rgba;
    top_sample(j, i, cd, m, rgba);
    TopCell* c = g + m;
    atomicAdd(&c->n, 1u);
    // full precision in the average modes: the cell's smallest input index
    if ((MODE == 0 || MODE == 3) && full) atomicMin(&c->mid, j.ids[i]);
    if (MODE == 3) continue;
    if (MODE == 0) {
      atomicAdd(&c->a, (unsigned long long)(rgba & 0xffu));
      atomicAdd(&c->b, (unsigned long long)((rgba >> 8) & 0xffu));
      atomicAdd(&c->c, (unsigned long long)((rgba >> 16) & 0xffu));
    } else {
      const unsigned long long k = pick_order(j.ids[i], seed, MODE == 2);
      if (MODE == 1) atomicMin(&c->a, k);
      else atomicMax(&c->a, k);
    }
  }
}

// Pick modes: the one sample whose order won its cell (ids are distinct)
// writes its colour and id.
template <int MODE>
__global__ void __launch_bounds__(256) k_top_pick(const TopJob* __restrict__ jobs, const Cube* cube, uint32_t seed,
                                                  TopCell* grids) {
  const TopJob j = jobs[blockIdx.y];
  TopCell* g = grids + (uint64_t)blockIdx.y * kTopCells;
  const CubeD cd = load_cube(cube);
  for (uint32_t i = blockIdx.x * 256 + threadIdx.x; i < j.count; i += gridDim.x * 256) {
    uint32_t m, rgba;
    top_sample(j, i, cd, m, rgba);
    const uint32_t id = j.ids[i];
    if (pick_order(id, seed, MODE == 2) == g[m].a) g[m].b = (unsigned long long)rgba | ((unsigned long long)id << 32);
  }
}

// Weighted mode: every sample's splats onto the occupied cells of its parent's
// grid, in whichever octant's job they fall.
__global__ void __launch_bounds__(256) k_top_wsplat(const TopJob* __restrict__ jobs, const Cube* cube,
                                                    TopCell* grids) {
  const TopJob j = jobs[blockIdx.y];
  const CubeD cd = load_cube(cube);
  const uint32_t L = j.level;
  for (uint32_t i = blockIdx.x * 256 + threadIdx.x; i < j.count; i += gridDim.x * 256) {
    uint64_t pos2[3];
    uint32_t rgba;
    if (j.kind == 0) {
      // a child voxel at the centre of its cell (level L + 8)
      const uint64_t v = ((const uint64_t*)j.src)[i];
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const uint64_t jj = ((uint64_t)j.C[a] << 7) + ((v >> (8 * a)) & 0xffu);
        pos2[a] = (2 * jj + 1) << (13 - L);
      }
      rgba = (uint32_t)(v >> 32);
    } else {
      // a point at the centre of its 2^21-grid cell
      const uint4 v = ((const uint4*)j.src)[i];
      pos2[0] = 2ull * quantize(__uint_as_float(v.x), cd.lo[0], cd.scale) + 1;
      pos2[1] = 2ull * quantize(__uint_as_float(v.y), cd.lo[1], cd.scale) + 1;
      pos2[2] = 2ull * quantize(__uint_as_float(v.z), cd.lo[2], cd.scale) + 1;
      rgba = v.w;
    }
    const uint64_t R = rgba & 0xffu, Gc = (rgba >> 8) & 0xffu, B = (rgba >> 16) & 0xffu;
    wtargets(L, j.G, pos2, [&](uint32_t code, uint64_t w) {
      const int32_t jb = j.sib[code >> 18];
      if (jb < 0) return;  // no child there: no occupied cell
      TopCell* c = grids + (uint64_t)jb * kTopCells + (code & (kTopCells - 1));
      if (c->n == 0u) return;  // not an occupied cell
      atomicAdd(&c->a, (unsigned long long)(w * R));
      atomicAdd(&c->b, (unsigned long long)(w * Gc));
      atomicAdd(&c->c, (unsigned long long)(w * B));
      atomicAdd(&c->w, (unsigned long long)w);
    });
  }
}

// Occupied cells of each 4096-cell slice of every job's grid.
__global__ void __launch_bounds__(256) k_top_count(const TopCell* __restrict__ grids, uint32_t* slice_cnt) {
  __shared__ uint32_t sh[256 / 64 + 1];
  const TopCell* g = grids + (uint64_t)blockIdx.y * kTopCells + (uint64_t)blockIdx.x * kTopSlice;
  uint32_t c = 0;
  for (uint32_t k = threadIdx.x; k < kTopSlice; k += 256) c += g[k].n != 0u;
  uint32_t tot;
  (void)block_excl_scan<256>(c, sh, &tot);
  if (threadIdx.x == 0) slice_cnt[blockIdx.y * kTopSlices + blockIdx.x] = tot;
}

// Voxels (and ids) of every job's occupied cells in Morton order, slice s of
// job j starting at slice_off[j * kTopSlices + s].
template <int MODE>
__global__ void __launch_bounds__(256) k_top_emit(const TopJob* __restrict__ jobs, const TopCell* __restrict__ grids,
                                                  const uint64_t* __restrict__ slice_off, uint64_t* vox,
                                                  uint32_t* vid) {
  __shared__ uint32_t sh[256 / 64 + 1];
  const uint32_t oct = jobs[blockIdx.y].oct;
  const uint32_t m0 = blockIdx.x * kTopSlice;
  const TopCell* g = grids + (uint64_t)blockIdx.y * kTopCells + m0;
  uint64_t pos = slice_off[blockIdx.y * kTopSlices + blockIdx.x];
  for (uint32_t r = 0; r < kTopSlice; r += 256) {
    const TopCell c = g[r + threadIdx.x];
    const bool occ = c.n != 0u;
    uint32_t tot;
    const uint32_t ex = block_excl_scan<256>((uint32_t)occ, sh, &tot);
    if (occ) {
      uint32_t rgba, id = 0;
      if (MODE == 0) {
        rgba = (uint32_t)(c.a / c.n) | ((uint32_t)(c.b / c.n) << 8) | ((uint32_t)(c.c / c.n) << 16) | (255u << 24);
        id = c.mid;
      } else if (MODE == 3) {
        // a cell's own sample weighs more than 0.13, so c.w > 0
        const unsigned long long w = c.w ? c.w : 1ull;
        rgba = (uint32_t)(c.a / w) | ((uint32_t)(c.b / w) << 8) | ((uint32_t)(c.c / w) << 16) | (255u << 24);
        id = c.mid;
      } else {
        rgba = (uint32_t)c.b;
        id = (uint32_t)(c.b >> 32);
      }
      vox[pos + ex] = make_voxel((oct << 18) | (m0 + r + threadIdx.x), rgba);
      if (vid) vid[pos + ex] = id;
    }
    pos += tot;
  }
}

void launch_top_clear(TopCell* grids, uint32_t njobs, uint32_t mode, hipStream_t s) {
  const uint64_t cells = (uint64_t)njobs * kTopCells;
  hipLaunchKernelGGL(k_top_clear, dim3(2048), dim3(256), 0, s, grids, cells, mode == 1 ? ~0ull : 0ull);
}

void launch_top_splat(const TopJob* jobs, uint32_t njobs, uint32_t max_count, const Cube* cube, uint32_t mode,
                      uint32_t seed, bool full, TopCell* grids, hipStream_t s) {
  if (!njobs || !max_count) return;
  const dim3 grid(std::min<uint32_t>((max_count + 255) / 256, 512), njobs);
  switch (mode) {
    case 0:
      hipLaunchKernelGGL(k_top_splat<0>, grid, dim3(256), 0, s, jobs, cube, seed, full, grids);
      break;
    case 1:
      hipLaunchKernelGGL(k_top_splat<1>, grid, dim3(256), 0, s, jobs, cube, seed, full, grids);
      hipLaunchKernelGGL(k_top_pick<1>, grid, dim3(256), 0, s, jobs, cube, seed, grids);
      break;
    case 2:
      hipLaunchKernelGGL(k_top_splat<2>, grid, dim3(256), 0, s, jobs, cube, seed, full, grids);
      hipLaunchKernelGGL(k_top_pick<2>, grid, dim3(256), 0, s, jobs, cube, seed, grids);
      break;
    default:
      hipLaunchKernelGGL(k_top_splat<3>, grid, dim3(256), 0, s, jobs, cube, seed, full, grids);
      hipLaunchKernelGGL(k_top_wsplat, grid, dim3(256), 0, s, jobs, cube, grids);
      break;
  }
}

void launch_top_count(const TopCell* grids, uint32_t njobs, uint32_t* slice_cnt, hipStream_t s) {
  if (!njobs) return;
  hipLaunchKernelGGL(k_top_count, dim3(kTopSlices, njobs), dim3(256), 0, s, grids, slice_cnt);
}

void launch_top_emit(const TopJob* jobs, uint32_t njobs, const TopCell* grids, const uint64_t* slice_off,
                     uint32_t mode, uint64_t* vox, uint32_t* vid, hipStream_t s) {
  if (!njobs) return;
  if (mode == 0)
    hipLaunchKernelGGL(k_top_emit<0>, dim3(kTopSlices, njobs), dim3(256), 0, s, jobs, grids, slice_off, vox, vid);
  else if (mode == 3)
    hipLaunchKernelGGL(k_top_emit<3>, dim3(kTopSlices, njobs), dim3(256), 0, s, jobs, grids, slice_off, vox, vid);
  else
    hipLaunchKernelGGL(k_top_emit<1>, dim3(kTopSlices, njobs), dim3(256), 0, s, jobs, grids, slice_off, vox, vid);
}

// ------------------------------------------------------------ copies

// Full-precision records: the accepted samples' input records (gathered by
// id) with the voxels' colours.
__global__ void __launch_bounds__(256) k_voxel_records(const uint4* __restrict__ rec, const uint64_t* __restrict__ vox,
                                                       uint64_t n, uint4* __restrict__ out) {
  for (uint64_t i = blockIdx.x * 256ull + threadIdx.x; i < n; i += (uint64_t)gridDim.x * 256) {
    const uint4 r = rec[i];
    out[i] = make_uint4(r.x, r.y, r.z, (uint32_t)(vox[i] >> 32));
  }
}

void launch_voxel_records(const void* rec, const uint64_t* vox, uint64_t n, void* out, hipStream_t s) {
  if (!n) return;
  const uint64_t blocks = std::min<uint64_t>((n + 255) / 256, 65536);
  hipLaunchKernelGGL(k_voxel_records, dim3((uint32_t)blocks), dim3(256), 0, s, (const uint4*)rec, vox, n, (uint4*)out);
}

// out[i] = {pts[ids[i]].x, .y, .z, colour of vox[i]}: the input records of
// accepted samples gathered by id from a cloud on the device; an id beyond the
// cloud raises *bad and writes nothing.
__global__ void __launch_bounds__(256) k_voxel_records_by_id(const uint4* __restrict__ pts, uint32_t npts,
                                                             const uint32_t* __restrict__ ids,
                                                             const uint64_t* __restrict__ vox, uint64_t n,
                                                             uint4* __restrict__ out, uint32_t* bad) {
  for (uint64_t i = blockIdx.x * 256ull + threadIdx.x; i < n; i += (uint64_t)gridDim.x * 256) {
    const uint32_t id = ids[i];
    if (id >= npts) {
      atomicOr(bad, 1u);
      continue;
    }
    const uint4 r = pts[id];
    out[i] = make_uint4(r.x, r.y, r.z, (uint32_t)(vox[i] >> 32));
  }
}

void launch_voxel_records_by_id(const void* pts, uint32_t npts, const uint32_t* ids, const uint64_t* vox, uint64_t n,
                                void* out, uint32_t* bad, hipStream_t s) {
  if (!n) return;
  const uint64_t blocks = std::min<uint64_t>((n + 255) / 256, 65536);
  hipLaunchKernelGGL(k_voxel_records_by_id, dim3((uint32_t)blocks), dim3(256), 0, s, (const uint4*)pts, npts, ids, vox,
                     n, (uint4*)out, bad);
}

// Run r copies runs[r].len elements from the device address runs[r].src to
// dst + runs[r].dst.
template <typename T>
__global__ void __launch_bounds__(256) k_copy_runs(const CopyRun* __restrict__ runs, T* dst) {
  const CopyRun r = runs[blockIdx.x];
  const T* src = (const T*)r.src;
  for (uint64_t i = (uint64_t)blockIdx.y * 256 + threadIdx.x; i < r.len; i += (uint64_t)gridDim.y * 256)
    dst[r.dst + i] = src[i];
}

void launch_copy_runs(const CopyRun* runs, uint32_t nruns, uint32_t elem_bytes, void* dst, hipStream_t s) {
  if (!nruns) return;
  const dim3 grid(nruns, 16);
  if (elem_bytes == 16) hipLaunchKernelGGL(k_copy_runs<uint4>, grid, dim3(256), 0, s, runs, (uint4*)dst);
  else if (elem_bytes == 8) hipLaunchKernelGGL(k_copy_runs<uint64_t>, grid, dim3(256), 0, s, runs, (uint64_t*)dst);
  else hipLaunchKernelGGL(k_copy_runs<uint32_t>, grid, dim3(256), 0, s, runs, (uint32_t*)dst);
}

}  // namespace lod
