// lod_api.cpp -- host orchestration and C ABI of the gfx950 octree builder.
//
// One build call handles any number of independent clouds (lod_build: one,
// lod_build_batch: one per chunk) with the same launches: every kernel works
// on lists of segments, trees or work items that may belong to any cloud.
// Pipeline (all kernels on the caller's stream):
//   1. bounding box and cube of every cloud        (k_split.hip)
//   2. partition by the first E0 levels            (a root counting grid per
//                                                   cloud, Sec. 4.1.1-4.1.4)
//   3. partition every root cell by E1 more levels (extended counting grids,
//                                                   Sec. 4.1.5)
//   4. node enumeration, one workgroup per tree; nodes whose region is not
//      sorted deep enough are partitioned again (4 more levels) and
//      enumeration resumes                          (k_tree.hip)
//   5. voxels of every leaf for all its ancestors up to 6 levels above it,
//      then offsets and the gather into each tree's voxel list (Sec. 4.2,
//      k_voxel.hip)
// The host synchronises the stream once per enumeration round (to size and
// launch refinements), once to size the voxel output, and at the end: a
// constant number of times per call, however many clouds it builds.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <condition_variable>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <deque>
#include <exception>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "../../include/lod.h"
#include "common.h"
#include "internal.h"
#include "launch.h"

using namespace lod;

// ------------------------------------------------------------------ errors

static thread_local char g_err[512] = "";

void lod_set_error(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
}
#define set_err lod_set_error
using lodint::cache;

static void fail(lod_status st, const char* msg) { lod_fail(st, msg); }

namespace {

// Grow-only scratch buffer owned by a workspace.
// Grow-only scratch buffer owned by a workspace.  A block outgrown during a
// build may still be read by kernels queued on the build's stream, and the
// device cache is shared by every thread (the server builds on several
// streams at once), so outgrown blocks are retired to the workspace and only
// returned to the cache once the build's stream has drained.
struct Scratch {
  void* p = nullptr;
  size_t cap = 0;
  std::vector<void*>* retired = nullptr;
  template <typename T>
  T* get(int dev, size_t count) {
    size_t bytes = count * sizeof(T);
    if (bytes > cap) {
      if (p) {
        if (retired) retired->push_back(p);
        else cache().release(dev, p);
      }
      p = cache().alloc(dev, bytes);
      cap = bytes;
    }
    return (T*)p;
  }
  void drop(int dev) {
    cache().release(dev, p);
    p = nullptr;
    cap = 0;
  }
};

// Growable pinned host buffer for small tables exchanged with the device.
struct Pinned {
  void* p = nullptr;
  size_t cap = 0;
  template <typename T>
  T* get(size_t count) {
    const size_t bytes = std::max<size_t>(count * sizeof(T), 64);
    if (bytes > cap) {
      if (p) (void)hipHostFree(p);
      p = nullptr;
      cap = 0;
      const size_t c = std::max<size_t>(bytes, 4096);
      if (hipHostMalloc(&p, c, hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        p = nullptr;
        set_err("pinned host allocation failed");
        throw LodError{LOD_ERR_OOM};
      }
      cap = c;
    }
    return (T*)p;
  }
  ~Pinned() {
    if (p) (void)hipHostFree(p);
  }
};

struct Workspace {
  int dev = 0;
  Scratch X, Xid, bbox, cube, segs, chunks, counters, hist, grids, pool, pool2, refine, leaf_refine;
  Scratch groups, gsum;
  Scratch n_level, n_leaf, n_mask, n_key, n_npts, n_count, n_first, n_off, n_cover, n_grid, n_parent, n_tree;
  Scratch c_level, c_leaf, c_mask, c_key, c_npts, c_count, c_first, c_off, c_cover, c_grid, c_parent, c_tree;
  Scratch t2, t2id, icnt, idesc, iself, v_sz, v_dfs, v_dfsn, v_psize, v_poff, v_selfc, v_selfid;
  Scratch state, bstate, clouds, trees, nbeg, wslot, wlist, wbits, wpre, wacc, wseg, wblk;
  Pinned h_clouds, h_nbeg, h_states, h_trees, h_cubes, h_bs, h_wlist, h_wblk;
  std::vector<void*> retired;  // outgrown blocks, released when the build's stream has drained
  hipEvent_t ev[16] = {};
  bool ev_ready = false;
  std::vector<Scratch*> scratches() {
    return {&X,       &Xid,     &bbox,    &cube,    &segs,     &chunks,  &counters, &hist,    &grids,
            &pool,    &pool2,   &refine,  &leaf_refine, &groups, &gsum,     &n_level, &n_leaf,  &n_mask,
            &n_key,   &n_npts,  &n_count, &n_first, &n_off,    &n_cover, &n_grid,   &n_parent, &n_tree,
            &c_level, &c_leaf,  &c_mask,  &c_key,   &c_npts,   &c_count, &c_first,  &c_off,   &c_cover,
            &c_grid,  &c_parent, &c_tree, &t2,      &t2id,     &icnt,    &idesc,    &iself,   &v_sz,
            &v_dfs,   &v_dfsn,  &v_psize, &v_poff,  &v_selfc,  &v_selfid, &state,   &bstate,  &clouds,
            &trees,   &nbeg,    &wslot,   &wlist,   &wbits,   &wpre,    &wacc,    &wseg,    &wblk};
  }
  Workspace() {
    for (Scratch* sc : scratches()) sc->retired = &retired;
  }
  // only once nothing queued by the last build can still touch them
  void flush_retired() {
    for (void* q : retired) cache().release(dev, q);
    retired.clear();
  }
  ~Workspace() {
    if (ev_ready)
      for (hipEvent_t& e : ev) (void)hipEventDestroy(e);
    flush_retired();
    for (Scratch* sc : scratches()) sc->drop(dev);
  }
};

std::mutex g_ws_mu;
std::vector<Workspace*> g_ws_free;

Workspace* acquire_ws(int dev) {
  {
    std::lock_guard<std::mutex> g(g_ws_mu);
    for (size_t i = 0; i < g_ws_free.size(); ++i)
      if (g_ws_free[i]->dev == dev) {
        Workspace* w = g_ws_free[i];
        g_ws_free.erase(g_ws_free.begin() + (long)i);
        return w;
      }
  }
  Workspace* w = new Workspace();
  w->dev = dev;
  return w;
}

void release_ws(Workspace* w) {
  w->flush_retired();
  std::lock_guard<std::mutex> g(g_ws_mu);
  g_ws_free.push_back(w);
}

struct WsGuard {
  Workspace* w;
  explicit WsGuard(int dev) : w(acquire_ws(dev)) {}
  ~WsGuard() { release_ws(w); }
};

// When a build ends by an exception, kernels may still be queued on its
// stream: drain it before device memory goes back to the shared cache
// (declared after the owners of that memory, so it runs first).
struct DrainOnUnwind {
  hipStream_t s;
  int pending;
  explicit DrainOnUnwind(hipStream_t st) : s(st), pending(std::uncaught_exceptions()) {}
  ~DrainOnUnwind() {
    if (std::uncaught_exceptions() > pending) {
      (void)hipStreamSynchronize(s);
      (void)hipGetLastError();
    }
  }
};

// Stage timer: events recorded on the build stream (no effect when disabled).
enum { EV_START, EV_BBOX, EV_COUNT0, EV_OFF0, EV_SCAT0, EV_COUNT1, EV_OFF1, EV_SCAT1, EV_TREE, EV_LEAF, EV_LEVELS,
       EV_NUM };
struct StageTimer {
  Workspace& w;
  hipStream_t s;
  bool on;
  StageTimer(Workspace& ws, hipStream_t st, bool enabled) : w(ws), s(st), on(enabled) {
    if (on && !w.ev_ready) {
      for (int i = 0; i < EV_NUM; ++i)
        if (hipEventCreate(&w.ev[i]) != hipSuccess) {
          (void)hipGetLastError();
          on = false;
          return;
        }
      w.ev_ready = true;
    }
  }
  void mark(int i) {
    if (on) (void)hipEventRecord(w.ev[i], s);
  }
  float ms(int a, int b) {
    float t = 0.f;
    if (on && hipEventElapsedTime(&t, w.ev[a], w.ev[b]) != hipSuccess) {
      (void)hipGetLastError();
      t = 0.f;
    }
    return t;
  }
};

}  // namespace

// -------------------------------------------------------------- parameters

namespace {

struct Plan {
  uint32_t E0, E1;
  uint32_t chunk0, chunk1, chunk_ref;
  uint32_t mode;  // voxel-stage mode: the sampling strategy, or 3 (average with accepted ids)
  bool ids;
  bool full;      // full-precision records of the voxels
  bool weighted;  // neighbourhood-weighted colours, rewritten after the average build
};

uint32_t ceil_div(uint64_t a, uint64_t b) { return (uint32_t)((a + b - 1) / b); }

// E0/E1 follow the typical (median) cloud, chunk sizes the total: chunks set
// the parallelism of a pass over all clouds.
Plan make_plan(uint64_t n_typical, uint64_t n_total, const lod_params& p) {
  Plan pl;
  const uint64_t n = n_typical;
  pl.E0 = n >= (4u << 20) ? 4 : (n >= (256u << 10) ? 3 : 2);
  pl.E1 = n >= (4u << 20) ? 4 : (n >= (64u << 10) ? 3 : 2);
  if (p.tune_levels0) pl.E0 = std::min<uint32_t>(4, p.tune_levels0);
  if (p.tune_levels1) pl.E1 = std::min<uint32_t>(4, p.tune_levels1);
  pl.full = (p.flags & LOD_FLAG_FULL_PRECISION) != 0;
  pl.weighted = p.sampling == LOD_WEIGHTED;
  const bool averaging = p.sampling == LOD_AVERAGE || pl.weighted;
  pl.mode = averaging ? (pl.full ? 3u : 0u) : p.sampling;
  pl.ids = !averaging || (p.flags & LOD_FLAG_POINT_IDS) || pl.full;
  // chunks are whole numbers of insert rounds (about 64k points for large
  // inputs, two rounds in the middle range and for refinements)
  const uint32_t R = scatter_round(pl.ids);
  const uint64_t N = n_total;
  pl.chunk0 = N >= (64u << 20) ? R * ((65536 + R / 2) / R) : (N >= (4u << 20) ? 2 * R : 4096);
  if (p.tune_chunk) pl.chunk0 = std::max<uint32_t>(1, (p.tune_chunk + R / 2) / R) * R;
  pl.chunk1 = pl.chunk0;
  pl.chunk_ref = 2 * R;
  return pl;
}

Nodes node_ptrs(Workspace& w, uint32_t cap) {
  Nodes nd;
  nd.level = w.n_level.get<uint8_t>(w.dev, cap);
  nd.is_leaf = w.n_leaf.get<uint8_t>(w.dev, cap);
  nd.child_mask = w.n_mask.get<uint8_t>(w.dev, cap);
  nd.key = w.n_key.get<uint64_t>(w.dev, cap);
  nd.npoints = w.n_npts.get<uint32_t>(w.dev, cap);
  nd.count = w.n_count.get<uint32_t>(w.dev, cap);
  nd.first_child = w.n_first.get<uint32_t>(w.dev, cap);
  nd.offset = w.n_off.get<uint64_t>(w.dev, cap);
  nd.cover = w.n_cover.get<int32_t>(w.dev, cap);
  nd.grid = w.n_grid.get<int32_t>(w.dev, cap);
  nd.parent = w.n_parent.get<uint32_t>(w.dev, cap);
  nd.tree = w.n_tree.get<uint32_t>(w.dev, cap);
  return nd;
}

Nodes compact_ptrs(Workspace& w, uint32_t cap) {
  Nodes nd;
  nd.level = w.c_level.get<uint8_t>(w.dev, cap);
  nd.is_leaf = w.c_leaf.get<uint8_t>(w.dev, cap);
  nd.child_mask = w.c_mask.get<uint8_t>(w.dev, cap);
  nd.key = w.c_key.get<uint64_t>(w.dev, cap);
  nd.npoints = w.c_npts.get<uint32_t>(w.dev, cap);
  nd.count = w.c_count.get<uint32_t>(w.dev, cap);
  nd.first_child = w.c_first.get<uint32_t>(w.dev, cap);
  nd.offset = w.c_off.get<uint64_t>(w.dev, cap);
  nd.cover = w.c_cover.get<int32_t>(w.dev, cap);
  nd.grid = w.c_grid.get<int32_t>(w.dev, cap);
  nd.parent = w.c_parent.get<uint32_t>(w.dev, cap);
  nd.tree = w.c_tree.get<uint32_t>(w.dev, cap);
  return nd;
}

VoxTree vox_ptrs(Workspace& w, uint32_t num_nodes) {
  VoxTree vt;
  const size_t c = std::max<uint32_t>(num_nodes, 1);
  vt.sz = w.v_sz.get<uint32_t>(w.dev, c);
  vt.dfs = w.v_dfs.get<uint32_t>(w.dev, c);
  vt.dfs_node = w.v_dfsn.get<uint32_t>(w.dev, c);
  vt.psize = w.v_psize.get<uint32_t>(w.dev, 8 * c);
  vt.poff = w.v_poff.get<uint64_t>(w.dev, 8 * c);
  vt.selfc = w.v_selfc.get<uint32_t>(w.dev, c);
  vt.selfid = w.v_selfid.get<uint32_t>(w.dev, c);
  return vt;
}

// Grid storage grows on demand; descriptors hold offsets, so relocation is a copy.
struct GridPool {
  Workspace& w;
  uint64_t used_words = 0;
  uint32_t num_grids = 0;
  uint32_t cap_grids = 0;
  uint64_t cap_words = 0;
  GridDesc* grids = nullptr;
  uint32_t* pool = nullptr;
  hipStream_t s;
  GridPool(Workspace& ws, hipStream_t st) : w(ws), s(st) {}
  void reserve(uint32_t grids_needed, uint64_t words_needed) {
    if (grids_needed > cap_grids) {
      uint32_t nc = std::max<uint32_t>(grids_needed, cap_grids * 2);
      if (w.grids.cap >= (size_t)nc * sizeof(GridDesc) || num_grids == 0) {
        grids = w.grids.get<GridDesc>(w.dev, nc);
      } else {
        GridDesc* old = grids;
        Scratch tmp;
        GridDesc* nw = tmp.get<GridDesc>(w.dev, nc);
        HIPCHK(hipMemcpyAsync(nw, old, sizeof(GridDesc) * num_grids, hipMemcpyDeviceToDevice, s));
        HIPCHK(hipStreamSynchronize(s));
        w.grids.drop(w.dev);
        tmp.retired = w.grids.retired;
        w.grids = tmp;
        grids = nw;
      }
      cap_grids = nc;
    }
    if (words_needed > cap_words) {
      uint64_t nc = std::max<uint64_t>(words_needed, cap_words * 2);
      if (w.pool.cap >= nc * 4 || used_words == 0) {
        pool = w.pool.get<uint32_t>(w.dev, nc);
      } else {
        uint32_t* old = pool;
        Scratch tmp;
        uint32_t* nw = tmp.get<uint32_t>(w.dev, nc);
        HIPCHK(hipMemcpyAsync(nw, old, 4ull * used_words, hipMemcpyDeviceToDevice, s));
        HIPCHK(hipStreamSynchronize(s));
        w.pool.drop(w.dev);
        tmp.retired = w.pool.retired;
        w.pool = tmp;
        pool = nw;
      }
      cap_words = nc;
    }
  }
};

// Partition `nseg` segments (device list, at most max_segs, covering at most
// max_points points) by E levels from src into dst.
void partition(Workspace& w, GridPool& gp, uint32_t E, uint32_t chunk, uint32_t max_segs, uint64_t max_points,
               const void* src, const uint32_t* src_ids, void* dst, uint32_t* dst_ids, bool ids, Segment* segs,
               uint32_t* nseg, const Cube* cube, hipStream_t s, StageTimer* tm = nullptr, int ev0 = 0) {
  uint32_t* nchunk = nseg + 1;
  uint32_t* ngroup = nseg + 2;
  const uint32_t max_chunks = ceil_div(max_points, chunk) + max_segs;
  const uint32_t max_groups = ceil_div(max_chunks, kGroupChunks) + max_segs;
  Chunk* chunks = w.chunks.get<Chunk>(w.dev, max_chunks);
  ChunkGroup* groups = w.groups.get<ChunkGroup>(w.dev, max_groups);
  uint32_t* hist = w.hist.get<uint32_t>(w.dev, (size_t)max_chunks << (3 * E));
  uint32_t* gsum = w.gsum.get<uint32_t>(w.dev, (size_t)max_groups << (3 * E));
  launch_make_chunks(segs, nseg, max_segs, chunk, chunks, nchunk, max_chunks, groups, ngroup, max_groups, s);
  launch_part_count(E, src, cube, segs, chunks, nchunk, max_chunks, hist, s);
  if (tm) tm->mark(ev0);
  launch_part_colscan(segs, nseg, max_segs, groups, ngroup, max_groups, E, hist, gsum, gp.grids, gp.pool, s);
  launch_grid_finish(segs, nseg, max_segs, gp.grids, gp.pool, s);
  if (tm) tm->mark(ev0 + 1);
  launch_part_scatter(E, ids, src, src_ids, dst, dst_ids, cube, segs, chunks, nchunk, max_chunks, hist, gp.grids,
                      gp.pool, s);
  if (tm) tm->mark(ev0 + 2);
  HIPCHK(hipGetLastError());
}

// Refine the nodes in `list` (count known on the host): partition their
// points by 4 more levels (Y -> X), copy back, attach the new grids.
void refine_nodes(Workspace& w, GridPool& gp, const Nodes& nd, uint32_t* list, uint32_t count, uint64_t n, void* Y,
                  uint32_t* Yid, bool ids, const Cube* cube, uint32_t chunk, hipStream_t s) {
  const uint32_t E = 4;
  const uint32_t first = gp.num_grids;
  const uint64_t slot = gp.used_words;
  gp.reserve(first + count, slot + (uint64_t)count * grid_words(E));
  Segment* segs = w.segs.get<Segment>(w.dev, std::max<uint32_t>(count, 1));
  uint32_t* ctr = w.counters.get<uint32_t>(w.dev, 16);
  uint32_t* nseg = ctr + 4;
  HIPCHK(hipMemcpyAsync(nseg, &count, 4, hipMemcpyHostToDevice, s));
  launch_refine_segments(nd, list, nseg, count, E, first, slot, gp.grids, segs, nseg, s);
  partition(w, gp, E, chunk, count, n, Y, Yid, w.X.p, (uint32_t*)w.Xid.p, ids, segs, nseg, cube, s);
  launch_copy_segments(w.X.p, (const uint32_t*)w.Xid.p, Y, ids ? Yid : nullptr, segs, nseg, count, s);
  HIPCHK(hipGetLastError());
  gp.num_grids = first + count;
  gp.used_words = slot + (uint64_t)count * grid_words(E);
}

}  // namespace

std::vector<lod_tree*> lod_build_clouds(const lod_point* d_points, const uint64_t* offs, uint32_t nchunks,
                                        const lod_params& prm, hipStream_t s, const BuildExtras* x) {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  const uint64_t N = offs[nchunks] - offs[0];
  const lod_point* in = d_points + offs[0];
  // empty chunks get empty trees and take no part in the build
  std::vector<uint32_t> active;
  for (uint32_t i = 0; i < nchunks; ++i)
    if (offs[i + 1] > offs[i]) active.push_back(i);
  const uint32_t nc = (uint32_t)active.size();
  std::vector<std::unique_ptr<lod_tree>> trees(nchunks);
  for (uint32_t i = 0; i < nchunks; ++i) {
    trees[i].reset(new lod_tree());
    trees[i]->dev = dev;
    trees[i]->v.cube_side = 1.0;
  }
  auto release_all = [&]() {
    std::vector<lod_tree*> out(nchunks);
    for (uint32_t i = 0; i < nchunks; ++i) out[i] = trees[i].release();
    return out;
  };
  if (nc == 0) return release_all();

  WsGuard guard(dev);
  Workspace& w = *guard.w;
  std::vector<uint64_t> sizes(nc);
  for (uint32_t c = 0; c < nc; ++c) sizes[c] = offs[active[c] + 1] - offs[active[c]];
  std::vector<uint64_t> sorted = sizes;
  std::nth_element(sorted.begin(), sorted.begin() + nc / 2, sorted.end());
  const Plan pl = make_plan(sorted[nc / 2], N, prm);
  const bool ids = pl.ids;

  // cloud table
  CloudInfo* hci = w.h_clouds.get<CloudInfo>(nc);
  uint32_t ntiles = 0;
  uint64_t passb_bound = 0;
  const uint64_t root_cells = 1ull << (3 * pl.E0);
  for (uint32_t c = 0; c < nc; ++c) {
    hci[c].start = (uint32_t)(offs[active[c]] - offs[0]);
    hci[c].count = (uint32_t)sizes[c];
    hci[c].tile_base = ntiles;
    hci[c].pad = 0;
    ntiles += bbox_tiles(hci[c].count);
    passb_bound += std::min<uint64_t>(root_cells, sizes[c]);
  }
  CloudInfo* clouds = w.clouds.get<CloudInfo>(dev, nc);
  HIPCHK(hipMemcpyAsync(clouds, hci, sizeof(CloudInfo) * nc, hipMemcpyHostToDevice, s));

  // outputs that do not depend on the tree shapes
  std::shared_ptr<LodArena> arena = std::make_shared<LodArena>();
  arena->dev = dev;
  DrainOnUnwind drain(s);
  lod_point* Y = arena->alloc<lod_point>(N);
  uint32_t* Yid = ids ? arena->alloc<uint32_t>(N) : nullptr;
  // scratch
  void* X = w.X.get<uint4>(dev, N);
  uint32_t* Xid = w.Xid.get<uint32_t>(dev, ids ? N : 1);
  BBoxAcc* bb = w.bbox.get<BBoxAcc>(dev, nc);
  Cube* cube = w.cube.get<Cube>(dev, nc);
  uint32_t* ctr = w.counters.get<uint32_t>(dev, 16);
  BuildState* bs = w.bstate.get<BuildState>(dev, 1);
  HIPCHK(hipMemsetAsync(bs, 0, sizeof(BuildState), s));

  GridPool gp(w, s);
  gp.reserve((uint32_t)(nc + passb_bound), (uint64_t)nc * grid_words(pl.E0) + passb_bound * grid_words(pl.E1));

  StageTimer tm(w, s, (prm.flags & LOD_FLAG_TIMING) != 0);
  tm.mark(EV_START);
  // 1. bounding boxes and cubes (or the one cube given for all clouds)
  if (x && x->cube) {
    Cube* hgc = w.h_cubes.get<Cube>(nc);
    for (uint32_t c = 0; c < nc; ++c) hgc[c] = *(const Cube*)x->cube;
    HIPCHK(hipMemcpyAsync(cube, hgc, sizeof(Cube) * nc, hipMemcpyHostToDevice, s));
    HIPCHK(hipStreamSynchronize(s));  // the pinned table is refilled below
  } else {
    launch_bbox(in, clouds, nc, ntiles, bb, cube, s);
  }
  tm.mark(EV_BBOX);
  // 2. root partition, input -> X
  Segment* segs = w.segs.get<Segment>(dev, std::max<uint64_t>(std::max<uint64_t>(passb_bound, nc), 1));
  uint32_t* nseg = ctr;
  launch_init_roots(clouds, nc, pl.E0, segs, nseg, gp.grids, s);
  const uint32_t* in_ids = x && x->d_ids ? x->d_ids + offs[0] : nullptr;
  partition(w, gp, pl.E0, pl.chunk0, nc, N, in, in_ids, X, Xid, ids, segs, nseg, cube, s, &tm, EV_COUNT0);
  gp.num_grids = nc;
  gp.used_words = (uint64_t)nc * grid_words(pl.E0);
  // 3. every root cell by E1 more levels, X -> Y
  HIPCHK(hipMemsetAsync(nseg, 0, sizeof(uint32_t), s));
  launch_segments_from_grid(gp.grids, nc, gp.pool, pl.E1, gp.used_words, nc, segs, nseg, s);
  partition(w, gp, pl.E1, pl.chunk1, (uint32_t)passb_bound, N, X, Xid, Y, Yid, ids, segs, nseg, cube, s, &tm,
            EV_COUNT1);
  gp.num_grids = (uint32_t)(nc + passb_bound);  // descriptors past the real count are never referenced
  gp.used_words += passb_bound * grid_words(pl.E1);

  // 4. nodes: one region of slots per tree
  uint32_t* hnb = w.h_nbeg.get<uint32_t>(2 * (size_t)nc);
  uint64_t cap_total = 0;
  for (uint32_t c = 0; c < nc; ++c) {
    const uint64_t inner_max = sizes[c] / ((uint64_t)prm.leaf_cap + 1);
    const uint64_t cap = 1 + 8ull * inner_max * std::max<uint32_t>(prm.max_level, 1) + 8;
    hnb[c] = (uint32_t)cap_total;
    cap_total += cap;
    if (cap_total >= 0x7fffffffull) fail(LOD_ERR_CAPACITY, "node table capacity exceeded");
    hnb[nc + c] = (uint32_t)cap_total;
  }
  uint32_t* nbeg = w.nbeg.get<uint32_t>(dev, 2 * (size_t)nc);
  HIPCHK(hipMemcpyAsync(nbeg, hnb, 8ull * nc, hipMemcpyHostToDevice, s));
  const uint32_t max_nodes = (uint32_t)cap_total;
  Nodes nd = node_ptrs(w, max_nodes);
  TreeState* st = w.state.get<TreeState>(dev, nc);
  uint32_t* refine = w.refine.get<uint32_t>(dev, max_nodes);
  uint32_t* leaf_refine = w.leaf_refine.get<uint32_t>(dev, max_nodes);
  launch_tree_init(prm.leaf_cap, prm.max_level, gp.grids, gp.pool, nd, st, nbeg, nbeg + nc, nc, s);
  BuildState* hbs = w.h_bs.get<BuildState>(1);
  TreeState* hst = w.h_states.get<TreeState>(nc);
  Cube* hcube = w.h_cubes.get<Cube>(nc);
  HIPCHK(hipMemcpyAsync(hcube, cube, sizeof(Cube) * nc, hipMemcpyDeviceToHost, s));
  for (;;) {
    HIPCHK(hipMemsetAsync(&bs->nref, 0, sizeof(uint32_t), s));
    launch_tree_build(prm.leaf_cap, prm.max_level, gp.grids, gp.pool, nd, st, nc, refine, leaf_refine, bs, s);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(hbs, bs, sizeof(BuildState), hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(hst, st, sizeof(TreeState) * nc, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    for (uint32_t c = 0; c < nc; ++c)
      if (hcube[c].nonfinite) fail(LOD_ERR_NONFINITE, "input contains a NaN or infinite coordinate");
    if (hbs->overflow) fail(LOD_ERR_CAPACITY, "node table capacity exceeded");
    if (hbs->nref) {
      refine_nodes(w, gp, nd, refine, hbs->nref, N, Y, Yid, ids, cube, pl.chunk_ref, s);
      continue;
    }
    break;
  }
  if (hbs->nlref) refine_nodes(w, gp, nd, leaf_refine, hbs->nlref, N, Y, Yid, ids, cube, pl.chunk_ref, s);

  // per-tree placement in the compact node table
  TreeInfo* hti = w.h_trees.get<TreeInfo>(nc);
  uint32_t num_nodes = 0;
  for (uint32_t c = 0; c < nc; ++c) {
    TreeInfo& ti = hti[c];
    memset(&ti, 0, sizeof(ti));
    const TreeState& ts = hst[c];
    ti.node_base = num_nodes;
    ti.num_nodes = ts.num_nodes - ts.node_begin;
    ti.point_base = hci[c].start;
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
    num_nodes += ti.num_nodes;
  }
  TreeInfo* tinfo = w.trees.get<TreeInfo>(dev, nc);
  HIPCHK(hipMemcpyAsync(tinfo, hti, sizeof(TreeInfo) * nc, hipMemcpyHostToDevice, s));
  if (nc > 1) {
    const Nodes cn = compact_ptrs(w, num_nodes);
    launch_compact_nodes(nd, cn, tinfo, nbeg, nc, num_nodes, s);
    nd = cn;
  }
  tm.mark(EV_TREE);

  // 5. voxels: every leaf's lists for its ancestors up to 6 levels above it
  // (depth 1 into X, coarser ones into t2), then the tree pass and the node
  // offsets, one sync to size the output, then piece offsets and the gather
  const uint32_t items = 8 * num_nodes;
  uint64_t* T1 = (uint64_t*)X;
  uint32_t* icnt = w.icnt.get<uint32_t>(dev, 6ull * items);
  void* desc = w.idesc.get<uint4>(dev, 4ull * items);
  uint64_t* iself = w.iself.get<uint64_t>(dev, items);
  const uint64_t t2cap = coarse_space_bound(N, num_nodes);
  uint64_t* T2 = w.t2.get<uint64_t>(dev, t2cap);
  uint32_t* T2id = pl.mode ? w.t2id.get<uint32_t>(dev, t2cap) : nullptr;
  const VoxTree vt = vox_ptrs(w, num_nodes);
  launch_item_desc(nd, num_nodes, gp.grids, gp.pool, bs, desc, s);
  launch_leaf_voxels(pl.mode, num_nodes, desc, Y, Yid, cube, T1, Xid, T2, T2id, icnt, iself, prm.seed, s);
  tm.mark(EV_LEAF);
  launch_voxel_tree(pl.mode, nd, vt, num_nodes, tinfo, nc, icnt, iself, prm.seed, s);
  HIPCHK(hipGetLastError());
  HIPCHK(hipMemcpyAsync(hti, tinfo, sizeof(TreeInfo) * nc, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  uint64_t vtotal = 0;
  for (uint32_t c = 0; c < nc; ++c) {
    hti[c].vbase = vtotal;
    vtotal += hti[c].vtotal;
  }
  HIPCHK(hipMemcpyAsync(tinfo, hti, sizeof(TreeInfo) * nc, hipMemcpyHostToDevice, s));
  uint64_t* vox = arena->alloc<uint64_t>(std::max<uint64_t>(vtotal, 1));
  uint32_t* vids = pl.mode ? arena->alloc<uint32_t>(std::max<uint64_t>(vtotal, 1)) : nullptr;
  launch_voxel_gather(pl.mode, nd, vt, num_nodes, tinfo, icnt, desc, T1, Xid, T2, T2id, vox, vids, s);
  if (pl.weighted && vtotal) {
    if (vtotal > 0xffffffffull) fail(LOD_ERR_INVALID, "weighted sampling handles at most 2^32 - 1 voxels per call");
    // the nodes of the call grouped by level (each tree's levels are
    // contiguous in the node table); one occupancy bitmap slot per inner node
    // of a level: at most the widest level's node count, and at most
    // n / (T + 1) per tree (inner nodes of one level are disjoint and hold
    // more than T points each)
    uint32_t deepest = 0;
    for (uint32_t c = 0; c < nc; ++c) deepest = std::max(deepest, hti[c].deepest);
    uint32_t* hl = w.h_wlist.get<uint32_t>(num_nodes);
    uint64_t loff[25] = {};
    uint64_t slots = 1, k = 0;
    for (uint32_t L = 0; L <= deepest; ++L) {
      loff[L] = k;
      for (uint32_t c = 0; c < nc; ++c) {
        if (k + (hti[c].level_end[L] - hti[c].level_begin[L]) > num_nodes)
          fail(LOD_ERR_CAPACITY, "level ranges exceed the node table");
        for (uint32_t i = hti[c].level_begin[L]; i < hti[c].level_end[L]; ++i) hl[k++] = i;
      }
      slots = std::max<uint64_t>(slots, k - loff[L]);
    }
    loff[deepest + 1] = k;
    uint64_t inner_bound = 0;
    for (uint32_t c = 0; c < nc; ++c) inner_bound += hci[c].count / ((uint64_t)prm.leaf_cap + 1);
    slots = std::max<uint64_t>(1, std::min(slots, inner_bound));
    const uint64_t words = slots * weighted_bitmap_words();
    uint32_t* wlist = w.wlist.get<uint32_t>(dev, num_nodes);
    uint32_t* wslot = w.wslot.get<uint32_t>(dev, num_nodes);
    unsigned long long* wbits = w.wbits.get<unsigned long long>(dev, words);
    uint32_t* wpre = w.wpre.get<uint32_t>(dev, words);
    unsigned long long* wacc = w.wacc.get<unsigned long long>(dev, 4 * vtotal);
    uint2* wseg = w.wseg.get<uint2>(dev, 64ull * num_nodes);
    uint32_t* wblk = w.wblk.get<uint32_t>(dev, 64ull * num_nodes + 2);
    HIPCHK(hipMemcpyAsync(wlist, hl, sizeof(uint32_t) * k, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemsetAsync(wbits, 0, 8 * words, s));
    HIPCHK(hipMemsetAsync(wacc, 0, 32 * vtotal, s));
    HIPCHK(hipMemsetAsync(wseg, 0, 64ull * sizeof(uint2) * num_nodes, s));
    HIPCHK(launch_weighted(nd, wlist, loff, deepest, tinfo, cube, desc, Y, vox, wslot, wbits, wpre, wseg, wacc,
                           wblk + 2, wblk, w.h_wblk.get<uint32_t>(1), wblk + 1, s));
  }
  lod_point* vpts = nullptr;
  if (pl.full && !(x && x->ids_only)) {
    vpts = arena->alloc<lod_point>(std::max<uint64_t>(vtotal, 1));
    launch_voxel_points(vox, vids, vtotal, tinfo, clouds, nc, in, vpts, s);
  }
  HIPCHK(hipGetLastError());
  tm.mark(EV_LEVELS);

  // 6. output node tables (per-tree indices and offsets)
  uint8_t* o_level = arena->alloc<uint8_t>(num_nodes);
  uint8_t* o_leaf = arena->alloc<uint8_t>(num_nodes);
  uint8_t* o_mask = arena->alloc<uint8_t>(num_nodes);
  uint64_t* o_key = arena->alloc<uint64_t>(num_nodes);
  uint32_t* o_npts = arena->alloc<uint32_t>(num_nodes);
  uint32_t* o_count = arena->alloc<uint32_t>(num_nodes);
  uint32_t* o_first = arena->alloc<uint32_t>(num_nodes);
  uint64_t* o_off = arena->alloc<uint64_t>(num_nodes);
  launch_finalize_nodes(nd, tinfo, num_nodes, o_level, o_leaf, o_mask, o_key, o_npts, o_count, o_first, o_off, s);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(s));

  lod_timings T{};
  if (tm.on) {
    T.bbox = tm.ms(EV_START, EV_BBOX);
    T.count0 = tm.ms(EV_BBOX, EV_COUNT0);
    T.offsets0 = tm.ms(EV_COUNT0, EV_OFF0);
    T.scatter0 = tm.ms(EV_OFF0, EV_SCAT0);
    T.count1 = tm.ms(EV_SCAT0, EV_COUNT1);
    T.offsets1 = tm.ms(EV_COUNT1, EV_OFF1);
    T.scatter1 = tm.ms(EV_OFF1, EV_SCAT1);
    T.tree = tm.ms(EV_SCAT1, EV_TREE);
    T.leaf_voxels = tm.ms(EV_TREE, EV_LEAF);
    T.levels = tm.ms(EV_LEAF, EV_LEVELS);
    T.total = tm.ms(EV_START, EV_LEVELS);
  }
  for (uint32_t c = 0; c < nc; ++c) {
    lod_tree& t = *trees[active[c]];
    const TreeInfo& ti = hti[c];
    t.arena = arena;
    t.timings = T;
    t.footprint = (uint64_t)((double)arena->bytes * (double)hci[c].count / (double)N);
    lod_tree_view& v = t.v;
    for (int a = 0; a < 3; ++a) {
      v.aabb_min[a] = hcube[c].lo[a];
      v.aabb_max[a] = hcube[c].hi[a];
    }
    v.cube_side = hcube[c].side;
    v.num_nodes = ti.num_nodes;
    v.num_points = hci[c].count;
    v.num_voxels = ti.vtotal;
    v.node_level = o_level + ti.node_base;
    v.node_is_leaf = o_leaf + ti.node_base;
    v.node_child_mask = o_mask + ti.node_base;
    v.node_key = o_key + ti.node_base;
    v.node_npoints = o_npts + ti.node_base;
    v.node_count = o_count + ti.node_base;
    v.node_first_child = o_first + ti.node_base;
    v.node_offset = o_off + ti.node_base;
    v.points = Y + ti.point_base;
    v.point_ids = Yid ? Yid + ti.point_base : nullptr;
    v.voxels = (const lod_voxel*)(vox + ti.vbase);
    v.voxel_ids = vids ? vids + ti.vbase : nullptr;
    v.voxel_points = vpts ? vpts + ti.vbase : nullptr;
  }
  return release_all();
}

lod_tree* lod_build_tree(const lod_point* d_points, uint64_t n, const lod_params& prm, hipStream_t s) {
  const uint64_t offs[2] = {0, n};
  std::vector<lod_tree*> t = lod_build_clouds(d_points, offs, 1, prm, s);
  return t[0];
}

namespace {

lod_status check_params(const lod_params* p) {
  if (!p) return LOD_ERR_INVALID;
  if (p->leaf_cap == 0 || p->max_level > 14 || p->sampling > 3) return LOD_ERR_INVALID;
  if (p->tune_levels0 > 4 || p->tune_levels1 > 4) return LOD_ERR_INVALID;
  return LOD_OK;
}

}  // namespace

// ----------------------------------------------------------------- C ABI

extern "C" {

void lod_params_default(lod_params* p) {
  if (!p) return;
  memset(p, 0, sizeof(*p));
  p->leaf_cap = 50000;
  p->max_level = 12;
  p->sampling = LOD_AVERAGE;
}

lod_status lod_build(const lod_point* d_points, uint64_t n, const lod_params* p, void* hip_stream, lod_tree** out) {
  if (!out) {
    set_err("out is NULL");
    return LOD_ERR_INVALID;
  }
  *out = nullptr;
  if (check_params(p) != LOD_OK) {
    set_err("invalid parameters");
    return LOD_ERR_INVALID;
  }
  if (n >= 0xffffffffull || (n && !d_points)) {
    set_err("n must be below 2^32 and d_points non-NULL");
    return LOD_ERR_INVALID;
  }
  try {
    *out = lod_build_tree(d_points, n, *p, (hipStream_t)hip_stream);
    return LOD_OK;
  } catch (const LodError& e) {
    (void)hipGetLastError();
    return e.st;
  } catch (...) {
    set_err("unexpected host exception");
    return LOD_ERR_OOM;
  }
}

lod_status lod_build_batch(const lod_point* d_points, const uint64_t* h_offsets, uint32_t num_chunks,
                           const lod_params* p, void* hip_stream, lod_tree** out) {
  if (!out || (num_chunks && !h_offsets)) {
    set_err("out/h_offsets is NULL");
    return LOD_ERR_INVALID;
  }
  for (uint32_t i = 0; i < num_chunks; ++i) out[i] = nullptr;
  if (check_params(p) != LOD_OK) {
    set_err("invalid parameters");
    return LOD_ERR_INVALID;
  }
  for (uint32_t i = 0; i < num_chunks; ++i)
    if (h_offsets[i + 1] < h_offsets[i] || h_offsets[i + 1] - h_offsets[i] >= 0xffffffffull) {
      set_err("offsets must be non-decreasing and chunks below 2^32 points");
      return LOD_ERR_INVALID;
    }
  if (num_chunks && h_offsets[num_chunks] - h_offsets[0] >= 0xffffffffull) {
    set_err("a batch holds fewer than 2^32 points");
    return LOD_ERR_INVALID;
  }
  if (num_chunks && h_offsets[num_chunks] > h_offsets[0] && !d_points) {
    set_err("d_points is NULL");
    return LOD_ERR_INVALID;
  }
  if (num_chunks == 0) return LOD_OK;
  try {
    std::vector<lod_tree*> t = lod_build_clouds(d_points, h_offsets, num_chunks, *p, (hipStream_t)hip_stream);
    for (uint32_t i = 0; i < num_chunks; ++i) out[i] = t[i];
    return LOD_OK;
  } catch (const LodError& e) {
    (void)hipGetLastError();
    return e.st;
  } catch (...) {
    set_err("unexpected host exception");
    return LOD_ERR_OOM;
  }
}

lod_status lod_tree_view_get(const lod_tree* t, lod_tree_view* v) {
  if (!t || !v) {
    set_err("tree or view is NULL");
    return LOD_ERR_INVALID;
  }
  *v = t->v;
  return LOD_OK;
}

void lod_tree_free(lod_tree* t) { delete t; }

lod_status lod_tree_timings(const lod_tree* t, lod_timings* out) {
  if (!t || !out) {
    set_err("tree or output is NULL");
    return LOD_ERR_INVALID;
  }
  *out = t->timings;
  return LOD_OK;
}

const char* lod_status_str(lod_status s) {
  switch (s) {
    case LOD_OK: return "LOD_OK";
    case LOD_PENDING: return "LOD_PENDING";
    case LOD_ERR_INVALID: return "LOD_ERR_INVALID";
    case LOD_ERR_NONFINITE: return "LOD_ERR_NONFINITE";
    case LOD_ERR_OOM: return "LOD_ERR_OOM";
    case LOD_ERR_CAPACITY: return "LOD_ERR_CAPACITY";
    case LOD_ERR_TOO_LARGE: return "LOD_ERR_TOO_LARGE";
    case LOD_ERR_UNKNOWN_TICKET: return "LOD_ERR_UNKNOWN_TICKET";
    case LOD_ERR_HIP: return "LOD_ERR_HIP";
  }
  return "unknown status";
}

const char* lod_last_error(void) { return g_err; }

}  // extern "C"
