// lod_api.cpp -- host orchestration and C ABI of the gfx950 octree builder.
//
// Pipeline of one build (all kernels on the caller's stream):
//   1. bounding box and cube                       (k_split.hip)
//   2. partition by the first E0 levels            (root counting grid, Sec. 4.1.1-4.1.4)
//   3. partition every root cell by E1 more levels (extended counting grids, Sec. 4.1.5)
//   4. node enumeration; nodes whose region is not sorted deep enough are
//      partitioned again (4 more levels) and enumeration resumes
//   5. leaf voxels for all leaves at once, then the inner levels bottom-up
//      (Sec. 4.2)
// The host synchronises the stream a few times: after node enumeration (to
// size the node table and handle refinements), after the leaf voxels (to size
// the voxel buffer) and at the end.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <condition_variable>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <deque>
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

#define HIPCHK(x)                                                                    \
  do {                                                                               \
    hipError_t e_ = (x);                                                             \
    if (e_ != hipSuccess) {                                                          \
      set_err("%s failed: %s (%s:%d)", #x, hipGetErrorString(e_), __FILE__, __LINE__); \
      throw LodError{e_ == hipErrorOutOfMemory ? LOD_ERR_OOM : LOD_ERR_HIP};          \
    }                                                                                \
  } while (0)

static void fail(lod_status st, const char* msg) {
  set_err("%s", msg);
  throw LodError{st};
}

namespace {

// Grow-only scratch buffer owned by a workspace.
struct Scratch {
  void* p = nullptr;
  size_t cap = 0;
  template <typename T>
  T* get(int dev, size_t count) {
    size_t bytes = count * sizeof(T);
    if (bytes > cap) {
      cache().release(dev, p);
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

struct HostStage {
  TreeState st;
  Cube cube;
};

struct Workspace {
  int dev = 0;
  Scratch X, Xid, bbox, cube, segs, chunks, counters, hist, grids, pool, pool2, refine, leaf_refine;
  Scratch groups, gsum, tilesum, runidx, inner_ids, inner_voff, starts;
  Scratch n_level, n_leaf, n_mask, n_key, n_npts, n_count, n_first, n_off, n_cover, n_grid, n_parent, n_aux, n_jobofs;
  Scratch n_dstbase, n_firstrun, runpos, gcount, gstart;
  Scratch state;
  HostStage* host = nullptr;
  hipEvent_t ev[16] = {};
  bool ev_ready = false;
  ~Workspace() {
    if (ev_ready)
      for (hipEvent_t& e : ev) (void)hipEventDestroy(e);
    Scratch* all[] = {&X, &Xid, &bbox, &cube, &segs, &chunks, &counters, &hist, &grids, &pool, &pool2, &refine,
                      &leaf_refine, &groups, &gsum, &tilesum, &runidx, &inner_ids, &inner_voff, &starts, &n_level, &n_leaf, &n_mask, &n_key, &n_npts, &n_count, &n_first, &n_off,
                      &n_cover, &n_grid, &n_parent, &n_aux, &n_jobofs, &state, &n_dstbase, &n_firstrun, &runpos, &gcount, &gstart};
    for (Scratch* s : all) s->drop(dev);
    if (host) (void)hipHostFree(host);
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
  if (hipHostMalloc((void**)&w->host, sizeof(HostStage), hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    delete w;
    set_err("pinned host allocation failed");
    throw LodError{LOD_ERR_OOM};
  }
  return w;
}

void release_ws(Workspace* w) {
  std::lock_guard<std::mutex> g(g_ws_mu);
  g_ws_free.push_back(w);
}

struct WsGuard {
  Workspace* w;
  explicit WsGuard(int dev) : w(acquire_ws(dev)) {}
  ~WsGuard() { release_ws(w); }
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
  uint32_t mode;
  bool ids;
};

uint32_t ceil_div(uint64_t a, uint64_t b) { return (uint32_t)((a + b - 1) / b); }

Plan make_plan(uint64_t n, const lod_params& p) {
  Plan pl;
  pl.E0 = n >= (4u << 20) ? 4 : (n >= (256u << 10) ? 3 : 2);
  pl.E1 = n >= (4u << 20) ? 4 : (n >= (64u << 10) ? 3 : 2);
  if (p.tune_levels0) pl.E0 = std::min<uint32_t>(4, p.tune_levels0);
  if (p.tune_levels1) pl.E1 = std::min<uint32_t>(4, p.tune_levels1);
  pl.chunk0 = n >= (64u << 20) ? 65536 : (n >= (4u << 20) ? 16384 : 4096);
  pl.chunk1 = pl.chunk0;
  pl.chunk_ref = 16384;
  pl.mode = p.sampling;
  pl.ids = p.sampling != LOD_AVERAGE || (p.flags & LOD_FLAG_POINT_IDS);
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
  nd.aux = w.n_aux.get<uint32_t>(w.dev, cap);
  nd.jobofs = w.n_jobofs.get<uint32_t>(w.dev, cap);
  nd.dstbase = w.n_dstbase.get<uint64_t>(w.dev, cap);
  nd.firstrun = w.n_firstrun.get<uint32_t>(w.dev, cap);
  return nd;
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

lod_tree* lod_build_tree(const lod_point* d_points, uint64_t n, const lod_params& prm, hipStream_t s) {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  std::unique_ptr<lod_tree> t(new lod_tree());
  t->dev = dev;
  t->v.num_points = n;
  if (n == 0) {
    t->v.cube_side = 1.0;
    return t.release();
  }
  WsGuard guard(dev);
  Workspace& w = *guard.w;
  const Plan pl = make_plan(n, prm);
  const bool ids = pl.ids;

  // outputs that do not depend on the tree shape
  lod_point* Y = t->alloc<lod_point>(n);
  uint32_t* Yid = ids ? t->alloc<uint32_t>(n) : nullptr;
  // scratch
  void* X = w.X.get<uint4>(dev, n);
  uint32_t* Xid = w.Xid.get<uint32_t>(dev, ids ? n : 1);
  BBoxAcc* bb = w.bbox.get<BBoxAcc>(dev, 1);
  Cube* cube = w.cube.get<Cube>(dev, 1);
  uint32_t* ctr = w.counters.get<uint32_t>(dev, 16);
  TreeState* st = w.state.get<TreeState>(dev, 1);

  GridPool gp(w, s);
  const uint32_t root_cells = 1u << (3 * pl.E0);
  const uint32_t max_segs1 = (uint32_t)std::min<uint64_t>(root_cells, n);
  gp.reserve(1 + max_segs1, grid_words(pl.E0) + (uint64_t)max_segs1 * grid_words(pl.E1));

  StageTimer tm(w, s, (prm.flags & LOD_FLAG_TIMING) != 0);
  tm.mark(EV_START);
  // 1. bounding box and cube
  launch_bbox(d_points, n, bb, cube, s);
  tm.mark(EV_BBOX);
  // 2. root partition, input -> X
  Segment* segs = w.segs.get<Segment>(dev, std::max<uint32_t>(max_segs1, 1));
  uint32_t* nseg = ctr;
  launch_init_root((uint32_t)n, pl.E0, segs, nseg, gp.grids, s);
  partition(w, gp, pl.E0, pl.chunk0, 1, n, d_points, nullptr, X, Xid, ids, segs, nseg, cube, s, &tm, EV_COUNT0);
  gp.num_grids = 1;
  gp.used_words = grid_words(pl.E0);
  // 3. every root cell by E1 more levels, X -> Y
  launch_segments_from_grid(gp.grids, 0, gp.pool, pl.E1, gp.used_words, 1, segs, nseg, s);
  partition(w, gp, pl.E1, pl.chunk1, max_segs1, n, X, Xid, Y, Yid, ids, segs, nseg, cube, s, &tm, EV_COUNT1);
  gp.num_grids = 1 + max_segs1;  // descriptors past the real count are never referenced
  gp.used_words += (uint64_t)max_segs1 * grid_words(pl.E1);

  // 4. nodes
  const uint64_t inner_max = n / ((uint64_t)prm.leaf_cap + 1);
  const uint64_t cap64 = 1 + 8ull * inner_max * std::max<uint32_t>(prm.max_level, 1) + 8;
  const uint32_t max_nodes = (uint32_t)std::min<uint64_t>(cap64, 0x7fffffffu);
  Nodes nd = node_ptrs(w, max_nodes);
  uint32_t* refine = w.refine.get<uint32_t>(dev, max_nodes);
  uint32_t* leaf_refine = w.leaf_refine.get<uint32_t>(dev, max_nodes);
  launch_tree_init(prm.leaf_cap, prm.max_level, gp.grids, gp.pool, nd, st, s);
  HostStage* hs = w.host;
  for (;;) {
    launch_tree_build(prm.leaf_cap, prm.max_level, gp.grids, gp.pool, nd, st, refine, leaf_refine, max_nodes, s);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(&hs->st, st, sizeof(TreeState), hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(&hs->cube, cube, sizeof(Cube), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (hs->cube.nonfinite) fail(LOD_ERR_NONFINITE, "input contains a NaN or infinite coordinate");
    if (hs->st.overflow) fail(LOD_ERR_CAPACITY, "node table capacity exceeded");
    if (hs->st.status == 2) {
      refine_nodes(w, gp, nd, refine, hs->st.num_refine, n, Y, Yid, ids, cube, pl.chunk_ref, s);
      continue;
    }
    break;
  }
  if (hs->st.num_leaf_refine)
    refine_nodes(w, gp, nd, leaf_refine, hs->st.num_leaf_refine, n, Y, Yid, ids, cube, pl.chunk_ref, s);
  const uint32_t num_nodes = hs->st.num_nodes;
  TreeState levels = hs->st;
  tm.mark(EV_TREE);

  // 5. voxels: leaves (all levels at once) into X, then the bound, then levels bottom-up
  uint64_t* temp = (uint64_t*)X;
  uint32_t* gcount = w.gcount.get<uint32_t>(dev, 8ull * num_nodes);
  uint32_t* gstart = w.gstart.get<uint32_t>(dev, 8ull * num_nodes);
  launch_leaf_voxels(pl.mode, nd, num_nodes, gp.grids, gp.pool, Y, Yid, cube, temp, Xid, gcount, gstart, prm.seed, s);
  tm.mark(EV_LEAF);
  launch_voxel_bound(nd, st, s);
  HIPCHK(hipGetLastError());
  HIPCHK(hipMemcpyAsync(&hs->st, st, sizeof(TreeState), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  const uint64_t vcap = hs->st.voxel_bound;
  uint64_t* vox = t->alloc<uint64_t>(std::max<uint64_t>(vcap, 1));
  uint32_t* vids = pl.mode ? t->alloc<uint32_t>(std::max<uint64_t>(vcap, 1)) : nullptr;
  int deepest_inner = -1;
  for (int L = 0; L < 22; ++L)
    if (levels.level_end[L + 1] > levels.level_begin[L + 1]) deepest_inner = L;
  uint32_t* tilesum = w.tilesum.get<uint32_t>(dev, (vcap + 4095) / 4096 + 2);
  uint32_t* runidx = w.runidx.get<uint32_t>(dev, vcap + 2);
  uint8_t* vflag = w.starts.get<uint8_t>(dev, vcap + 8);
  uint32_t* vowner = w.inner_ids.get<uint32_t>(dev, vcap + 1);
  uint32_t* runpos = w.runpos.get<uint32_t>(dev, vcap + 1);
  for (int L = deepest_inner; L >= 0; --L)
    launch_level(pl.mode, nd, (uint32_t)L, levels.level_begin[L], levels.level_end[L], levels.level_begin[L + 1],
                 levels.level_end[L + 1], vcap, temp, Xid, vox, vids, st, tilesum, runidx, runpos, vflag, vowner,
                 gcount, gstart, prm.seed, s);
  HIPCHK(hipGetLastError());
  tm.mark(EV_LEVELS);

  // 6. exact-size node table for the tree
  uint8_t* o_level = t->alloc<uint8_t>(num_nodes);
  uint8_t* o_leaf = t->alloc<uint8_t>(num_nodes);
  uint8_t* o_mask = t->alloc<uint8_t>(num_nodes);
  uint64_t* o_key = t->alloc<uint64_t>(num_nodes);
  uint32_t* o_npts = t->alloc<uint32_t>(num_nodes);
  uint32_t* o_count = t->alloc<uint32_t>(num_nodes);
  uint32_t* o_first = t->alloc<uint32_t>(num_nodes);
  uint64_t* o_off = t->alloc<uint64_t>(num_nodes);
  HIPCHK(hipMemcpyAsync(o_level, nd.level, num_nodes, hipMemcpyDeviceToDevice, s));
  HIPCHK(hipMemcpyAsync(o_leaf, nd.is_leaf, num_nodes, hipMemcpyDeviceToDevice, s));
  HIPCHK(hipMemcpyAsync(o_mask, nd.child_mask, num_nodes, hipMemcpyDeviceToDevice, s));
  HIPCHK(hipMemcpyAsync(o_key, nd.key, 8ull * num_nodes, hipMemcpyDeviceToDevice, s));
  HIPCHK(hipMemcpyAsync(o_npts, nd.npoints, 4ull * num_nodes, hipMemcpyDeviceToDevice, s));
  HIPCHK(hipMemcpyAsync(o_count, nd.count, 4ull * num_nodes, hipMemcpyDeviceToDevice, s));
  HIPCHK(hipMemcpyAsync(o_first, nd.first_child, 4ull * num_nodes, hipMemcpyDeviceToDevice, s));
  HIPCHK(hipMemcpyAsync(o_off, nd.offset, 8ull * num_nodes, hipMemcpyDeviceToDevice, s));
  HIPCHK(hipMemcpyAsync(&hs->st, st, sizeof(TreeState), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));

  if (tm.on) {
    lod_timings& T = t->timings;
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
  lod_tree_view& v = t->v;
  for (int a = 0; a < 3; ++a) {
    v.aabb_min[a] = hs->cube.lo[a];
    v.aabb_max[a] = hs->cube.hi[a];
  }
  v.cube_side = hs->cube.side;
  v.num_nodes = num_nodes;
  v.num_points = n;
  v.num_voxels = hs->st.voxel_total;
  v.node_level = o_level;
  v.node_is_leaf = o_leaf;
  v.node_child_mask = o_mask;
  v.node_key = o_key;
  v.node_npoints = o_npts;
  v.node_count = o_count;
  v.node_first_child = o_first;
  v.node_offset = o_off;
  v.points = Y;
  v.point_ids = Yid;
  v.voxels = (const lod_voxel*)vox;
  v.voxel_ids = vids;
  return t.release();
}

namespace {

lod_status check_params(const lod_params* p) {
  if (!p) return LOD_ERR_INVALID;
  if (p->leaf_cap == 0 || p->max_level > 14 || p->sampling > 2) return LOD_ERR_INVALID;
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
  for (uint32_t i = 0; i < num_chunks; ++i) {
    lod_status stt = lod_build(d_points + h_offsets[i], h_offsets[i + 1] - h_offsets[i], p, hip_stream, &out[i]);
    if (stt != LOD_OK) {
      for (uint32_t k = 0; k < i; ++k) {
        lod_tree_free(out[k]);
        out[k] = nullptr;
      }
      return stt;
    }
  }
  return LOD_OK;
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
