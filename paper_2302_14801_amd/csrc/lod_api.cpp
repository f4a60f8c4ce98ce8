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
// Nothing is read back while the build runs.  Every capacity (segments,
// chunks, grids, node slots, work items, voxel output) is fixed on the host
// from the input sizes before the first kernel; the refinement rounds are
// unrolled to the number the depth limit allows; counts that size later
// work stay on the device, and launches are sized by the capacities with
// kernels looping over the device counts.  The host reads the build state
// once, after the last kernel: if a capacity chosen from an estimate (the
// refinement grids, the voxel output) was too small, the build flagged it,
// every later kernel returned at once, and the build runs again with the
// capacities it reported.  Because the whole build is one sequence of
// launches without host decisions, a batch is captured into a HIP graph and
// launched as one graph.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
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

// Grow-only device buffer owned by a workspace.  A block outgrown during a
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
      p = nullptr;
      cap = 0;
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
  Scratch S;  // the device scratch region of a build
  Pinned H;   // the host tables of a build (copied to the device, read back)
  Scratch wslot, wlist, wbits, wpre, wacc, wseg, wblk;  // the weighted pass
  Pinned h_wlist;
  // capacities learned from earlier builds (grow-only; they change only how
  // often a build has to be repeated, never its result)
  double voxels_per_point = 0.0, coarse_per_point = 0.0;
  hipStream_t capture = nullptr;   // stream used only to record graphs
  hipGraphExec_t exec = nullptr;   // the last graph instantiated here
  std::vector<void*> retired;  // outgrown blocks, released when the build's stream has drained
  hipEvent_t ev[16] = {};
  bool ev_ready = false;
  std::vector<Scratch*> scratches() { return {&S, &wslot, &wlist, &wbits, &wpre, &wacc, &wseg, &wblk}; }
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
    if (exec) (void)hipGraphExecDestroy(exec);
    if (capture) (void)hipStreamDestroy(capture);
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
  hipEvent_t* ev;
  hipStream_t s;
  bool on;
  StageTimer(Workspace& w, hipStream_t st, bool enabled) : ev(w.ev), s(st), on(enabled) {
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
    if (on) (void)hipEventRecord(ev[i], s);
  }
  float ms(int a, int b) {
    float t = 0.f;
    if (on && hipEventElapsedTime(&t, ev[a], ev[b]) != hipSuccess) {
      (void)hipGetLastError();
      t = 0.f;
    }
    return t;
  }
};
void mark(StageTimer* tm, int i) {
  if (tm) tm->mark(i);
}

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
  bool digits;    // the first insert stores each record's cell of the second partition for its count
};

uint32_t ceil_div(uint64_t a, uint64_t b) { return (uint32_t)((a + b - 1) / b); }

// Compute units of the current device (cached per device).
static uint32_t device_cus() {
  static std::atomic<int> cached[64];
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) dev = 0;
  int v = cached[dev].load();
  if (v <= 0) {
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v <= 0) v = 256;
    cached[dev].store(v);
  }
  return (uint32_t)v;
}

// Insert rounds per chunk of a large first partition.  The insert runs one
// workgroup per chunk and compute unit, the count two per compute unit, so
// the last wave of workgroups of either pass can be nearly empty; m is chosen
// to keep both passes' makespans close to their averages without making
// chunks too short.
static uint32_t rounds_per_chunk(uint64_t n, uint32_t R) {
  const uint64_t cus = device_cus();
  const uint64_t rounds = (n + R - 1) / R;
  uint32_t best = 9;
  uint64_t best_cost = ~0ull;
  for (uint32_t m = 4; m <= 12; ++m) {
    const uint64_t chunks = (rounds + m - 1) / m;
    // (a round takes a count workgroup about 7/12 of the time it takes an
    // insert workgroup; plus a small cost per chunk: its histogram row and scans)
    const uint64_t cost =
        12 * cus * ((chunks + cus - 1) / cus) * m + 7 * cus * ((chunks + 2 * cus - 1) / (2 * cus)) * m + 4 * chunks;
    if (cost < best_cost) {
      best_cost = cost;
      best = m;
    }
  }
  return best;
}

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
  // chunks are whole numbers of insert rounds (4 to 12 of them for large
  // inputs, two rounds in the middle range and for refinements)
  const uint32_t R = scatter_round(pl.ids);
  const uint64_t N = n_total;
  pl.chunk0 = N >= (64u << 20) ? R * rounds_per_chunk(N, R) : (N >= (4u << 20) ? 2 * R : 4096);
  if (p.tune_chunk) pl.chunk0 = std::max<uint32_t>(1, (p.tune_chunk + R / 2) / R) * R;
  pl.chunk1 = pl.chunk0;
  pl.chunk_ref = 2 * R;
  // large inputs: the second count reads 2 bytes per point instead of the
  // 16-byte record (both partitions take the same number of levels)
  pl.digits = N >= (64u << 20) && pl.E0 == pl.E1;
  return pl;
}

// Node slots a tree of n points can need: every inner node has more than T
// points, so a level holds at most n / (T + 1) of them (and at most 8^L),
// and every node but the root is the child of an inner node.
uint64_t tree_node_cap(uint64_t n, uint32_t T, uint32_t ML) {
  const uint64_t inner = n / ((uint64_t)T + 1);
  uint64_t s = 0, p = 1;
  for (uint32_t L = 0; L < ML; ++L) {
    s += std::min(p, inner);
    if (p < (1ull << 40)) p *= 8;
  }
  return 1 + 8 * s + 8;
}

// Capacities of one build call, fixed before anything is enqueued.
struct Caps {
  uint64_t N = 0;
  uint32_t nc = 0;
  uint64_t passb = 0;     // segments of the second partition (one per possible root cell)
  uint32_t rounds = 0;    // refinement rounds of inner nodes
  uint32_t ref_inner = 0; // grids of inner-node refinements (4 levels), all rounds
  uint32_t ref_leaf = 0;  // grids of leaf refinements (2 levels)
  uint32_t segs = 0, chunks = 0, groups = 0;
  uint64_t hist = 0, gsum = 0;  // words of histogram rows and group sums
  uint32_t grids0 = 0;    // grid descriptors of the two main partitions
  uint64_t words0 = 0;    // their pool words
  uint32_t grids = 0;     // all grid descriptors
  uint64_t words = 0;     // all pool words
  uint32_t max_nodes = 0; // node slots of all trees
  uint64_t t2cap = 0;     // coarse-list entries
  uint64_t vcap = 0;      // output voxels (estimate)
  uint32_t items = 0;     // work items of the leaf kernel that get a workgroup each (estimate)
};

void part_caps(Caps& c, uint64_t N, uint32_t chunk, uint32_t max_segs, uint32_t E) {
  const uint64_t chunks = (uint64_t)ceil_div(N, chunk) + max_segs;
  const uint64_t groups = (uint64_t)ceil_div(chunks, kGroupChunks) + max_segs;
  if (chunks >= 0xffffffffull || groups >= 0xffffffffull) fail(LOD_ERR_CAPACITY, "partition work list too long");
  c.chunks = std::max<uint32_t>(c.chunks, (uint32_t)chunks);
  c.groups = std::max<uint32_t>(c.groups, (uint32_t)groups);
  c.hist = std::max<uint64_t>(c.hist, chunks << (3 * E));
  c.gsum = std::max<uint64_t>(c.gsum, groups << (3 * E));
  c.segs = std::max<uint32_t>(c.segs, max_segs);
}

// sizes: points of every (non-empty) cloud; vcap, t2cap: capacities of the
// estimated pools (0 = default estimate).
Caps make_caps(const Plan& pl, const uint64_t* sizes, uint32_t nc, uint64_t N, const lod_params& p, uint64_t vcap,
               uint64_t t2cap = 0) {
  Caps c;
  c.N = N;
  c.nc = nc;
  const uint64_t root_cells = 1ull << (3 * pl.E0);
  uint64_t nodes = 0, inner_per_level = 0;
  for (uint32_t i = 0; i < nc; ++i) {
    c.passb += std::min<uint64_t>(root_cells, sizes[i]);
    nodes += tree_node_cap(sizes[i], p.leaf_cap, p.max_level);
    inner_per_level += sizes[i] / ((uint64_t)p.leaf_cap + 1);
  }
  if (nodes >= 0x7fffffffull) fail(LOD_ERR_CAPACITY, "node table capacity exceeded");
  c.max_nodes = (uint32_t)nodes;
  const uint32_t D0 = pl.E0 + pl.E1;
  c.rounds = p.max_level > D0 ? (p.max_level - D0 + 3) / 4 : 0;
  // refinement grids, bounded exactly: a round refines inner nodes of one
  // level per tree (at most n / (T + 1) of them), a leaf at most once (it
  // needs its points sorted two levels below it), so the leaf grids sort 2
  // levels only (8^2 cells instead of 8^4 for the inner nodes' grids)
  c.ref_inner = (uint32_t)std::min<uint64_t>(std::min<uint64_t>((uint64_t)c.rounds * inner_per_level, nodes),
                                             0x7fffffffull);
  c.ref_leaf = (uint32_t)nodes;
  part_caps(c, N, pl.chunk0, nc, pl.E0);
  part_caps(c, N, pl.chunk1, (uint32_t)c.passb, pl.E1);
  part_caps(c, N, pl.chunk_ref, c.ref_inner, kRefineInnerE);
  part_caps(c, N, pl.chunk_ref, c.ref_leaf, kRefineLeafE);
  c.segs = std::max<uint32_t>(c.segs, 1);
  c.grids0 = (uint32_t)(nc + c.passb);
  c.words0 = (uint64_t)nc * grid_words(pl.E0) + c.passb * grid_words(pl.E1);
  if ((uint64_t)c.grids0 + c.ref_inner + c.ref_leaf >= 0x7fffffffull) fail(LOD_ERR_CAPACITY, "too many grids");
  c.grids = c.grids0 + c.ref_inner + c.ref_leaf;
  c.words = c.words0 + (uint64_t)c.ref_inner * grid_words(kRefineInnerE) +
            (uint64_t)c.ref_leaf * grid_words(kRefineLeafE);
  // coarse lists: at most min(5p, 4681) entries per item of p points; the
  // pool is an estimate (about one entry per point), checked on the device
  const uint64_t t2max = coarse_space_bound(N, c.max_nodes);
  c.t2cap = std::min<uint64_t>(t2max, t2cap ? t2cap : N + N / 2 + 65536);
  c.vcap = vcap ? vcap : N + 64;
  // leaf-kernel items (8 per node): about 8 nodes per T points plus a few per
  // tree; only the launch shape depends on it
  uint64_t est = 0;
  for (uint32_t i = 0; i < nc; ++i) est += 8 * (8 * sizes[i] / p.leaf_cap + 64);
  c.items = (uint32_t)std::min<uint64_t>(est, 8ull * c.max_nodes);
  return c;
}

// Bump allocation of the buffers of one build in a region (256-byte
// aligned); with a null base only the size is computed.
struct Carve {
  char* base;
  uint64_t off = 0;
  explicit Carve(void* b) : base((char*)b) {}
  template <typename T>
  T* take(uint64_t count) {
    off = (off + 255) & ~255ull;
    T* p = base ? (T*)(base + off) : nullptr;
    off += std::max<uint64_t>(count, 1) * sizeof(T);
    return p;
  }
};

// Every buffer of a build: device scratch (S), device output owned by the
// trees (O), host tables (H).
struct Bufs {
  uint4* X;
  uint32_t* Xid;
  uint16_t* dig;  // per record of X: its cell in the second partition (or null)
  BBoxAcc* bbox;
  Cube* cube;
  CloudInfo* clouds;
  Segment* segs;
  uint32_t* ctr;
  Chunk* chunks;
  ChunkGroup* groups;
  uint32_t *hist, *gsum;
  GridDesc* grids;
  uint32_t* pool;
  Nodes nd, cn;  // node slots per tree; compact table (the same with one tree)
  uint32_t *refine, *leaf_refine;
  TreeState* st;
  BuildState* bs;
  uint32_t* nbeg;
  TreeInfo* tinfo;
  ItemDesc* desc;
  uint32_t* icnt;
  uint64_t* iself;
  uint32_t* redo;
  uint32_t* slist;
  uint64_t* T2;
  uint32_t* T2id;
  VoxTree vt;
  lod_point* Y;
  uint32_t* Yid;
  uint64_t* vox;
  uint32_t* vids;
  lod_point* vpts;
  uint8_t *o_level, *o_leaf, *o_mask;
  uint64_t* o_key;
  uint32_t *o_npts, *o_count, *o_first;
  uint64_t* o_off;
  CloudInfo* h_clouds;
  uint32_t* h_nbeg;
  Cube* h_cube_in;
  BuildState* h_bs;
  TreeInfo* h_trees;
  Cube* h_cubes;
};

void take_nodes(Carve& s, Nodes& nd, uint32_t cap) {
  nd.level = s.take<uint8_t>(cap);
  nd.is_leaf = s.take<uint8_t>(cap);
  nd.child_mask = s.take<uint8_t>(cap);
  nd.key = s.take<uint64_t>(cap);
  nd.npoints = s.take<uint32_t>(cap);
  nd.count = s.take<uint32_t>(cap);
  nd.first_child = s.take<uint32_t>(cap);
  nd.offset = s.take<uint64_t>(cap);
  nd.cover = s.take<int32_t>(cap);
  nd.grid = s.take<int32_t>(cap);
  nd.parent = s.take<uint32_t>(cap);
  nd.tree = s.take<uint32_t>(cap);
}

struct RegionSizes {
  uint64_t scratch, out, host;
};

RegionSizes layout(Bufs& b, const Caps& c, const Plan& pl, bool cube_given, bool want_vpts, void* S, void* O, void* H) {
  Carve s(S), o(O), h(H);
  b.X = s.take<uint4>(c.N);
  b.Xid = s.take<uint32_t>(pl.ids ? c.N : 1);
  b.dig = pl.digits ? s.take<uint16_t>(c.N) : nullptr;
  b.bbox = s.take<BBoxAcc>(c.nc);
  b.cube = s.take<Cube>(c.nc);
  b.clouds = s.take<CloudInfo>(c.nc);
  b.segs = s.take<Segment>(c.segs);
  b.ctr = s.take<uint32_t>(16);
  b.chunks = s.take<Chunk>(c.chunks);
  b.groups = s.take<ChunkGroup>(c.groups);
  b.hist = s.take<uint32_t>(c.hist);
  b.gsum = s.take<uint32_t>(c.gsum);
  b.grids = s.take<GridDesc>(c.grids);
  b.pool = s.take<uint32_t>(c.words);
  take_nodes(s, b.nd, c.max_nodes);
  if (c.nc > 1) take_nodes(s, b.cn, c.max_nodes);
  else b.cn = b.nd;
  b.refine = s.take<uint32_t>(c.max_nodes);
  b.leaf_refine = s.take<uint32_t>(c.max_nodes);
  b.st = s.take<TreeState>(c.nc);
  b.bs = s.take<BuildState>(1);
  b.nbeg = s.take<uint32_t>(2ull * c.nc);
  b.tinfo = s.take<TreeInfo>(c.nc);
  const uint64_t items = 8ull * c.max_nodes;
  b.desc = s.take<ItemDesc>(items);
  b.icnt = s.take<uint32_t>(6 * items);
  b.iself = s.take<uint64_t>(items);
  b.redo = s.take<uint32_t>(items);
  b.slist = s.take<uint32_t>(pl.mode == 0 || pl.mode == 3 ? items : 1);
  b.T2 = s.take<uint64_t>(c.t2cap);
  b.T2id = pl.mode ? s.take<uint32_t>(c.t2cap) : nullptr;
  b.vt.sz = s.take<uint32_t>(c.max_nodes);
  b.vt.dfs = s.take<uint32_t>(c.max_nodes);
  b.vt.dfs_node = s.take<uint32_t>(c.max_nodes);
  b.vt.psize = s.take<uint32_t>(8ull * c.max_nodes);
  b.vt.poff = s.take<uint64_t>(8ull * c.max_nodes);
  b.vt.selfc = s.take<uint32_t>(c.max_nodes);
  b.vt.selfid = s.take<uint32_t>(c.max_nodes);
  b.Y = o.take<lod_point>(c.N);
  b.Yid = pl.ids ? o.take<uint32_t>(c.N) : nullptr;
  b.vox = o.take<uint64_t>(c.vcap);
  b.vids = pl.mode ? o.take<uint32_t>(c.vcap) : nullptr;
  b.vpts = want_vpts ? o.take<lod_point>(c.vcap) : nullptr;
  b.o_level = o.take<uint8_t>(c.max_nodes);
  b.o_leaf = o.take<uint8_t>(c.max_nodes);
  b.o_mask = o.take<uint8_t>(c.max_nodes);
  b.o_key = o.take<uint64_t>(c.max_nodes);
  b.o_npts = o.take<uint32_t>(c.max_nodes);
  b.o_count = o.take<uint32_t>(c.max_nodes);
  b.o_first = o.take<uint32_t>(c.max_nodes);
  b.o_off = o.take<uint64_t>(c.max_nodes);
  b.h_clouds = h.take<CloudInfo>(c.nc);
  b.h_nbeg = h.take<uint32_t>(2ull * c.nc);
  b.h_cube_in = cube_given ? h.take<Cube>(c.nc) : nullptr;
  b.h_bs = h.take<BuildState>(1);
  b.h_trees = h.take<TreeInfo>(c.nc);
  b.h_cubes = h.take<Cube>(c.nc);
  return {s.off, o.off, h.off};
}

// Partition `nseg` segments (device count, at most max_segs, expected about
// expect_segs, covering at most max_points points) by E levels from src into
// dst.  dig_in: the cells of src's records, stored by the previous insert
// (counted instead of the records); dig_out: where this insert stores each
// record's cell E levels further down (either may be null).
void partition(const Bufs& b, uint32_t E, uint32_t chunk, uint32_t max_segs, uint32_t expect_segs, uint64_t max_points,
               const void* src, const uint32_t* src_ids, void* dst, uint32_t* dst_ids, bool ids, uint32_t* nseg,
               const uint16_t* dig_in, uint16_t* dig_out, hipStream_t s, StageTimer* tm, int ev0) {
  uint32_t* nchunk = nseg + 1;
  uint32_t* ngroup = nseg + 2;
  const uint32_t max_chunks = ceil_div(max_points, chunk) + max_segs;
  const uint32_t expect_chunks = ceil_div(max_points, chunk) + std::min(max_segs, expect_segs);
  const uint32_t max_groups = ceil_div(max_chunks, kGroupChunks) + max_segs;
  launch_make_chunks(b.segs, nseg, max_segs, chunk, b.chunks, nchunk, max_chunks, b.groups, ngroup, max_groups, s);
  launch_part_count(E, src, dig_in, b.cube, b.segs, b.chunks, nchunk, max_chunks, b.hist, s);
  if (ev0) mark(tm, ev0);
  launch_part_colscan(b.segs, nseg, max_segs, b.groups, ngroup, max_groups, E, b.hist, b.gsum, b.grids, b.pool, s);
  launch_grid_finish(b.segs, nseg, max_segs, b.grids, b.pool, s);
  if (ev0) mark(tm, ev0 + 1);
  launch_part_scatter(E, ids, src, src_ids, dst, dst_ids, dig_out, b.cube, b.segs, b.chunks, nchunk, max_chunks,
                      expect_chunks, b.hist, b.grids, b.pool, s);
  if (ev0) mark(tm, ev0 + 2);
  HIPCHK(hipGetLastError());
}

// Refine the nodes of `list` (*nlist of them, a device count, at most
// max_segs): partition their points by E more levels (Y -> X), copy back,
// attach the new grids.
void refine(const Bufs& b, const Caps& c, const Plan& pl, const uint32_t* list, const uint32_t* nlist, uint32_t E,
            uint32_t max_segs, hipStream_t s) {
  uint32_t* nseg = b.ctr + 4;
  launch_refine_segments(b.nd, list, nlist, c.max_nodes, E, b.bs, c.grids, c.words, b.grids, b.segs, nseg, s);
  // refinements are few (none at all in most large builds): a workgroup
  // each for a thousand segments' chunks, the rest to the looping grid
  partition(b, E, pl.chunk_ref, max_segs, 1024, c.N, b.Y, b.Yid, b.X, b.Xid, pl.ids, nseg, nullptr, nullptr, s,
            nullptr, 0);
  launch_copy_segments(b.X, b.Xid, b.Y, pl.ids ? b.Yid : nullptr, b.segs, nseg, max_segs, s);
  launch_refine_commit(b.bs, nseg, E, s);
  HIPCHK(hipGetLastError());
}

// The whole build, from the host tables to the read-back of the build state:
// launches and copies only, no synchronisation (so it can be captured).
void enqueue(const Bufs& b, const Caps& c, const Plan& pl, const lod_params& prm, const lod_point* in,
             const uint32_t* in_ids, uint32_t ntiles, bool cube_given, hipStream_t s, StageTimer* tm) {
  const uint32_t nc = c.nc;
  mark(tm, EV_START);
  launch_build_init(b.bs, c.grids0, c.words0, s);
  HIPCHK(hipMemcpyAsync(b.clouds, b.h_clouds, sizeof(CloudInfo) * nc, hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(b.nbeg, b.h_nbeg, 8ull * nc, hipMemcpyHostToDevice, s));
  // 1. bounding boxes and cubes (or the one cube given for all clouds)
  if (cube_given) HIPCHK(hipMemcpyAsync(b.cube, b.h_cube_in, sizeof(Cube) * nc, hipMemcpyHostToDevice, s));
  else launch_bbox(in, b.clouds, nc, ntiles, b.bbox, b.cube, s);
  mark(tm, EV_BBOX);
  // 2. root partition, input -> X
  uint32_t* nseg = b.ctr;
  launch_init_roots(b.clouds, nc, pl.E0, b.segs, nseg, b.grids, s);
  partition(b, pl.E0, pl.chunk0, nc, nc, c.N, in, in_ids, b.X, b.Xid, pl.ids, nseg, nullptr, b.dig, s, tm,
            EV_COUNT0);
  // 3. every root cell by E1 more levels, X -> Y
  launch_fill_u32(nseg, 0, 1, s);
  launch_segments_from_grid(b.grids, nc, b.pool, pl.E1, (uint64_t)nc * grid_words(pl.E0), nc, b.segs, nseg, s);
  partition(b, pl.E1, pl.chunk1, (uint32_t)c.passb, (uint32_t)c.passb, c.N, b.X, b.Xid, b.Y, b.Yid, pl.ids, nseg,
            b.dig, nullptr, s, tm, EV_COUNT1);
  // 4. nodes: one region of slots per tree, enumeration resumed after each
  // refinement round (a round without nodes to refine does nothing)
  launch_tree_init(prm.leaf_cap, prm.max_level, b.grids, b.pool, b.nd, b.st, b.nbeg, b.nbeg + nc, nc, s);
  for (uint32_t r = 0; r <= c.rounds; ++r) {
    launch_fill_u32(&b.bs->nref, 0, 1, s);
    launch_tree_build(prm.leaf_cap, prm.max_level, b.grids, b.pool, b.nd, b.st, nc, b.refine, b.leaf_refine, b.bs, s);
    if (r < c.rounds) refine(b, c, pl, b.refine, &b.bs->nref, kRefineInnerE, c.ref_inner, s);
  }
  refine(b, c, pl, b.leaf_refine, &b.bs->nlref, kRefineLeafE, c.ref_leaf, s);
  launch_tree_info(b.st, b.clouds, nc, b.tinfo, b.bs, s);
  if (nc > 1) launch_compact_nodes(b.nd, b.cn, b.tinfo, b.nbeg, nc, c.max_nodes, b.bs, s);
  HIPCHK(hipGetLastError());
  mark(tm, EV_TREE);
  // 5. voxels: every leaf's lists for its ancestors up to 6 levels above it
  // (depth 1 into X, coarser ones into T2), the tree pass and the offsets,
  // then the pieces' positions and the gather
  uint64_t* T1 = (uint64_t*)b.X;
  launch_item_desc(b.cn, c.max_nodes, b.grids, b.pool, b.bs, b.desc, c.t2cap, pl.mode == 0 || pl.mode == 3, b.icnt,
                   b.slist, b.redo,
                   s);
  launch_leaf_voxels(pl.mode, c.max_nodes, c.items, b.desc, b.Y, b.Yid, b.cube, T1, b.Xid, b.T2, b.T2id, b.icnt, b.iself,
                     prm.seed, b.bs, b.slist, b.redo, s);
  mark(tm, EV_LEAF);
  launch_voxel_tree(pl.mode, b.cn, b.vt, c.max_nodes, b.tinfo, nc, c.vcap, b.icnt, b.iself, prm.seed, b.bs, s);
  launch_voxel_gather(pl.mode, b.cn, b.vt, c.max_nodes, b.tinfo, b.icnt, b.desc, T1, b.Xid, b.T2, b.T2id, b.vox,
                      b.vids, b.bs, s);
  // full-precision records take the voxel colours: after the weighted pass
  if (b.vpts && !pl.weighted)
    launch_voxel_points(b.vox, b.vids, c.vcap, b.bs, b.tinfo, b.clouds, nc, in, b.vpts, s);
  HIPCHK(hipGetLastError());
  mark(tm, EV_LEVELS);
  // 6. output node tables (per-tree indices and offsets)
  launch_finalize_nodes(b.cn, b.tinfo, c.max_nodes, b.bs, b.o_level, b.o_leaf, b.o_mask, b.o_key, b.o_npts,
                        b.o_count, b.o_first, b.o_off, s);
  HIPCHK(hipGetLastError());
  // 7. the one read-back of the build
  HIPCHK(hipMemcpyAsync(b.h_bs, b.bs, sizeof(BuildState), hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(b.h_trees, b.tinfo, sizeof(TreeInfo) * nc, hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(b.h_cubes, b.cube, sizeof(Cube) * nc, hipMemcpyDeviceToHost, s));
}

// Record the build into a graph on the workspace's capture stream and run it
// on `s` as one graph launch.  The executable graph is kept and updated in
// place for the next build of the same shape (only pointers and sizes
// differ), or instantiated again.
void run_as_graph(Workspace& w, const Bufs& b, const Caps& c, const Plan& pl, const lod_params& prm,
                  const lod_point* in, const uint32_t* in_ids, uint32_t ntiles, bool cube_given, hipStream_t s) {
  if (!w.capture) HIPCHK(hipStreamCreateWithFlags(&w.capture, hipStreamNonBlocking));
  HIPCHK(hipStreamBeginCapture(w.capture, hipStreamCaptureModeRelaxed));
  hipGraph_t g = nullptr;
  try {
    enqueue(b, c, pl, prm, in, in_ids, ntiles, cube_given, w.capture, nullptr);
  } catch (...) {
    (void)hipStreamEndCapture(w.capture, &g);
    if (g) (void)hipGraphDestroy(g);
    (void)hipGetLastError();
    throw;
  }
  HIPCHK(hipStreamEndCapture(w.capture, &g));
  struct GraphGuard {
    hipGraph_t g;
    ~GraphGuard() {
      if (g) (void)hipGraphDestroy(g);
    }
  } guard{g};
  if (w.exec) {
    hipGraphNode_t err_node = nullptr;
    hipGraphExecUpdateResult res;
    if (hipGraphExecUpdate(w.exec, g, &err_node, &res) != hipSuccess || res != hipGraphExecUpdateSuccess) {
      (void)hipGetLastError();
      (void)hipGraphExecDestroy(w.exec);
      w.exec = nullptr;
    }
  }
  if (!w.exec) HIPCHK(hipGraphInstantiate(&w.exec, g, nullptr, nullptr, 0));
  HIPCHK(hipGraphLaunch(w.exec, s));
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
  const bool cube_given = x && x->cube;
  const bool want_vpts = pl.full && !(x && x->ids_only);
  const uint32_t* in_ids = x && x->d_ids ? x->d_ids + offs[0] : nullptr;
  const bool graph = nc > 1 && !(prm.flags & (LOD_FLAG_NO_GRAPH | LOD_FLAG_TIMING)) && !pl.weighted;

  uint64_t vcap = (uint64_t)std::ceil(w.voxels_per_point * (double)N);
  uint64_t t2cap = (uint64_t)std::ceil(w.coarse_per_point * (double)N);
  std::shared_ptr<LodArena> arena;
  Bufs b{};
  Caps c;
  DrainOnUnwind drain(s);
  StageTimer tm(w, s, (prm.flags & LOD_FLAG_TIMING) != 0);
  for (int attempt = 0;; ++attempt) {
    c = make_caps(pl, sizes.data(), nc, N, prm, vcap, t2cap);
    const RegionSizes rs = layout(b, c, pl, cube_given, want_vpts, nullptr, nullptr, nullptr);
    arena = std::make_shared<LodArena>();
    arena->dev = dev;
    void* O = arena->alloc<char>(rs.out);
    layout(b, c, pl, cube_given, want_vpts, w.S.get<char>(dev, rs.scratch), O, w.H.get<char>(rs.host));
    // host tables: clouds, node regions, the given cube
    uint32_t ntiles = 0;
    uint64_t cap_total = 0;
    for (uint32_t i = 0; i < nc; ++i) {
      b.h_clouds[i].start = (uint32_t)(offs[active[i]] - offs[0]);
      b.h_clouds[i].count = (uint32_t)sizes[i];
      b.h_clouds[i].tile_base = ntiles;
      b.h_clouds[i].pad = 0;
      ntiles += bbox_tiles(b.h_clouds[i].count);
      b.h_nbeg[i] = (uint32_t)cap_total;
      cap_total += tree_node_cap(sizes[i], prm.leaf_cap, prm.max_level);
      b.h_nbeg[nc + i] = (uint32_t)cap_total;
      if (cube_given) b.h_cube_in[i] = *(const Cube*)x->cube;
    }
    if (graph) {
      run_as_graph(w, b, c, pl, prm, in, in_ids, ntiles, cube_given, s);
    } else {
      enqueue(b, c, pl, prm, in, in_ids, ntiles, cube_given, s, &tm);
    }
    HIPCHK(hipStreamSynchronize(s));
    for (uint32_t i = 0; i < nc; ++i)
      if (b.h_cubes[i].nonfinite) fail(LOD_ERR_NONFINITE, "input contains a NaN or infinite coordinate");
    const BuildState& hb = *b.h_bs;
    // node slots and refinement grids are bounded exactly
    if (hb.overflow & (kOverNodes | kOverGrids)) fail(LOD_ERR_CAPACITY, "node table or grid capacity exceeded");
    if (!hb.overflow) break;
    // a capacity estimate was too small: build again with what was asked for
    if (attempt >= 4) fail(LOD_ERR_CAPACITY, "build capacities still exceeded after re-planning");
    if (hb.overflow & kOverVoxels) {
      vcap = hb.vtotal + 64;
      w.voxels_per_point = std::max(w.voxels_per_point, (double)vcap / (double)N);
    }
    if (hb.overflow & kOverCoarse) {
      t2cap = hb.coarse_used + hb.coarse_used / 16 + 4096;
      w.coarse_per_point = std::max(w.coarse_per_point, (double)t2cap / (double)N);
    }
  }
  const uint32_t num_nodes = b.h_bs->total_nodes;
  const uint64_t vtotal = b.h_bs->vtotal;
  TreeInfo* hti = b.h_trees;
  if (pl.weighted && vtotal) {
    if (vtotal > 0xffffffffull) fail(LOD_ERR_INVALID, "weighted sampling handles at most 2^32 - 1 voxels per call");
    // the nodes of the call grouped by level (each tree's levels are
    // contiguous in the node table); one occupancy bitmap slot per inner node
    // of a level: at most the widest level's node count, and at most
    // n / (T + 1) per tree (inner nodes of one level are disjoint and hold
    // more than T points each)
    uint32_t deepest = 0;
    for (uint32_t i = 0; i < nc; ++i) deepest = std::max(deepest, hti[i].deepest);
    uint32_t* hl = w.h_wlist.get<uint32_t>(num_nodes);
    uint64_t loff[25] = {};
    uint64_t slots = 1, k = 0;
    for (uint32_t L = 0; L <= deepest; ++L) {
      loff[L] = k;
      for (uint32_t i = 0; i < nc; ++i) {
        if (k + (hti[i].level_end[L] - hti[i].level_begin[L]) > num_nodes)
          fail(LOD_ERR_CAPACITY, "level ranges exceed the node table");
        for (uint32_t j = hti[i].level_begin[L]; j < hti[i].level_end[L]; ++j) hl[k++] = j;
      }
      slots = std::max<uint64_t>(slots, k - loff[L]);
    }
    loff[deepest + 1] = k;
    uint64_t inner_bound = 0;
    for (uint32_t i = 0; i < nc; ++i) inner_bound += sizes[i] / ((uint64_t)prm.leaf_cap + 1);
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
    HIPCHK(launch_weighted(b.cn, wlist, loff, deepest, b.tinfo, b.cube, b.desc, b.Y, b.vox, wslot, wbits, wpre, wseg,
                           wacc, wblk + 2, wblk, wblk + 1, s));
    if (b.vpts) launch_voxel_points(b.vox, b.vids, c.vcap, b.bs, b.tinfo, b.clouds, nc, in, b.vpts, s);
    HIPCHK(hipGetLastError());
    tm.mark(EV_LEVELS);
    HIPCHK(hipStreamSynchronize(s));
  }

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
  for (uint32_t i = 0; i < nc; ++i) {
    lod_tree& t = *trees[active[i]];
    const TreeInfo& ti = hti[i];
    const Cube& cb = b.h_cubes[i];
    t.arena = arena;
    t.timings = T;
    t.footprint = (uint64_t)((double)arena->bytes * (double)sizes[i] / (double)N);
    lod_tree_view& v = t.v;
    for (int a = 0; a < 3; ++a) {
      v.aabb_min[a] = cb.lo[a];
      v.aabb_max[a] = cb.hi[a];
    }
    v.cube_side = cb.side;
    v.num_nodes = ti.num_nodes;
    v.num_points = sizes[i];
    v.num_voxels = ti.vtotal;
    v.node_level = b.o_level + ti.node_base;
    v.node_is_leaf = b.o_leaf + ti.node_base;
    v.node_child_mask = b.o_mask + ti.node_base;
    v.node_key = b.o_key + ti.node_base;
    v.node_npoints = b.o_npts + ti.node_base;
    v.node_count = b.o_count + ti.node_base;
    v.node_first_child = b.o_first + ti.node_base;
    v.node_offset = b.o_off + ti.node_base;
    v.points = b.Y + ti.point_base;
    v.point_ids = b.Yid ? b.Yid + ti.point_base : nullptr;
    v.voxels = (const lod_voxel*)(b.vox + ti.vbase);
    v.voxel_ids = b.vids ? b.vids + ti.vbase : nullptr;
    v.voxel_points = b.vpts ? b.vpts + ti.vbase : nullptr;
  }
  return release_all();
}

uint64_t lod_plan_bytes(const uint64_t* sizes, uint32_t n, const lod_params& p) {
  std::vector<uint64_t> nz;
  uint64_t N = 0;
  for (uint32_t i = 0; i < n; ++i)
    if (sizes[i]) {
      nz.push_back(sizes[i]);
      N += sizes[i];
    }
  if (nz.empty()) return 0;
  std::vector<uint64_t> sorted = nz;
  std::nth_element(sorted.begin(), sorted.begin() + sorted.size() / 2, sorted.end());
  const Plan pl = make_plan(sorted[sorted.size() / 2], N, p);
  const Caps c = make_caps(pl, nz.data(), (uint32_t)nz.size(), N, p, 0);
  Bufs b{};
  const RegionSizes rs = layout(b, c, pl, false, pl.full, nullptr, nullptr, nullptr);
  uint64_t weighted = 0;
  if (pl.weighted) {
    // 32 B of sums per voxel, an occupancy bitmap and prefixes per inner
    // node of the widest level (at most n / (T + 1) per tree), per-node
    // block lists
    uint64_t slots = 1;
    for (uint64_t v : nz) slots += v / ((uint64_t)p.leaf_cap + 1);
    weighted = 32 * c.vcap + slots * weighted_bitmap_words() * 12 + 800ull * c.max_nodes;
  }
  return rs.scratch + rs.out + weighted;
}

lod_tree* lod_build_tree(const lod_point* d_points, uint64_t n, const lod_params& prm, hipStream_t s) {
  const uint64_t offs[2] = {0, n};
  std::vector<lod_tree*> t = lod_build_clouds(d_points, offs, 1, prm, s);
  return t[0];
}

// ------------------------------------------------------ allocation-free build
//
// lod_build_noalloc is the one-cloud build with its device scratch in the
// file-scope array below instead of blocks from the device cache, its output
// in the caller's buffer and its few host tables in a static host buffer.
// Each GPU the library runs on holds its own copy of the array until the
// process ends.  In host code the name `scratch` denotes a host-side
// stand-in, never the device memory: its device address is looked up once
// per device (hipGetSymbolAddress, with the device current) and only that
// address reaches kernels and copies.
static __device__ __align__(256) unsigned char scratch[LOD_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kNaMaxDevices = 64;
std::mutex g_na_mu;                        // one allocation-free build at a time per process
void* g_na_ptr[kNaMaxDevices] = {};        // device address of `scratch`, per device
alignas(256) unsigned char g_na_host[16384];  // host tables of one build (one cloud)

void* noalloc_scratch(int dev) {
  if (dev < 0 || dev >= kNaMaxDevices) fail(LOD_ERR_INVALID, "device index out of range");
  if (!g_na_ptr[dev]) {
    void* ptr = nullptr;
    HIPCHK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) fail(LOD_ERR_HIP, "no device address for the allocation-free build's scratch");
    g_na_ptr[dev] = ptr;
  }
  return g_na_ptr[dev];
}

// Output bytes of a one-cloud build with room for vcap voxels.
uint64_t noalloc_out_bytes(const Caps& c, const Plan& pl) {
  Bufs b{};
  return layout(b, c, pl, false, pl.full, nullptr, nullptr, nullptr).out;
}

// Caller holds g_na_mu.  *out_bytes: capacity of d_out in, bytes used (or,
// with LOD_ERR_CAPACITY for voxels, bytes needed) out.
void build_noalloc(const lod_point* in, uint64_t n, const lod_params& prm, hipStream_t s, void* d_out,
                   uint64_t* out_bytes, lod_tree_view* view) {
  memset(view, 0, sizeof(*view));
  view->cube_side = 1.0;
  if (n == 0) {
    *out_bytes = 0;
    return;
  }
  const Plan pl = make_plan(n, n, prm);
  const uint64_t sizes[1] = {n};
  uint64_t t2cap = 0;
  // the voxel capacity: as many as the caller's buffer holds (n + 64 for a
  // size query)
  Caps c = make_caps(pl, sizes, 1, n, prm, n + 64);
  {
    Bufs q{};
    if (layout(q, c, pl, false, pl.full, nullptr, nullptr, nullptr).scratch > LOD_NOALLOC_SCRATCH_BYTES)
      fail(LOD_ERR_TOO_LARGE, "the build does not fit the allocation-free build's scratch (LOD_NOALLOC_SCRATCH_BYTES)");
  }
  const uint64_t fixed = noalloc_out_bytes(make_caps(pl, sizes, 1, n, prm, 1), pl);
  if (!d_out) {
    *out_bytes = noalloc_out_bytes(c, pl);
    return;
  }
  if ((uintptr_t)d_out & 255) fail(LOD_ERR_INVALID, "d_out must be 256-byte aligned");
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  void* S = noalloc_scratch(dev);
  const uint64_t per_voxel = 8 + (pl.mode ? 4 : 0) + (pl.full ? 16 : 0);
  if (*out_bytes < fixed) {
    *out_bytes = noalloc_out_bytes(c, pl);
    fail(LOD_ERR_CAPACITY, "output buffer too small for the points and node tables");
  }
  // the largest voxel capacity whose layout fits (sizes grow with it)
  uint64_t vlo = 1, vhi = *out_bytes / per_voxel + 2;
  while (vhi - vlo > 1) {
    const uint64_t m = vlo + (vhi - vlo) / 2;
    if (noalloc_out_bytes(make_caps(pl, sizes, 1, n, prm, m, 0), pl) <= *out_bytes) vlo = m;
    else vhi = m;
  }
  const uint64_t vcap = vlo;
  DrainOnUnwind drain(s);
  Bufs b{};
  for (int attempt = 0;; ++attempt) {
    c = make_caps(pl, sizes, 1, n, prm, vcap, t2cap);
    const RegionSizes rs = layout(b, c, pl, false, pl.full, nullptr, nullptr, nullptr);
    if (rs.out > *out_bytes) fail(LOD_ERR_CAPACITY, "output buffer too small for the points and node tables");
    if (rs.scratch > LOD_NOALLOC_SCRATCH_BYTES)
      fail(attempt ? LOD_ERR_CAPACITY : LOD_ERR_TOO_LARGE,
           "the build does not fit the allocation-free build's scratch (LOD_NOALLOC_SCRATCH_BYTES)");
    if (rs.host > sizeof(g_na_host)) fail(LOD_ERR_CAPACITY, "host tables exceed their static buffer");
    layout(b, c, pl, false, pl.full, S, d_out, g_na_host);
    b.h_clouds[0].start = 0;
    b.h_clouds[0].count = (uint32_t)n;
    b.h_clouds[0].tile_base = 0;
    b.h_clouds[0].pad = 0;
    b.h_nbeg[0] = 0;
    b.h_nbeg[1] = (uint32_t)tree_node_cap(n, prm.leaf_cap, prm.max_level);
    enqueue(b, c, pl, prm, in, nullptr, bbox_tiles((uint32_t)n), false, s, nullptr);
    HIPCHK(hipStreamSynchronize(s));
    if (b.h_cubes[0].nonfinite) fail(LOD_ERR_NONFINITE, "input contains a NaN or infinite coordinate");
    const BuildState& hb = *b.h_bs;
    if (hb.overflow & (kOverNodes | kOverGrids)) fail(LOD_ERR_CAPACITY, "node table or grid capacity exceeded");
    if (!hb.overflow) break;
    if (hb.overflow & kOverVoxels) {
      *out_bytes = noalloc_out_bytes(make_caps(pl, sizes, 1, n, prm, hb.vtotal, t2cap), pl);
      fail(LOD_ERR_CAPACITY, "output buffer too small for the voxels (its required size is in *out_bytes)");
    }
    // a scratch estimate was too small: again with what the build asked for,
    // while it still fits the array
    if (attempt >= 4) fail(LOD_ERR_CAPACITY, "build capacities still exceeded after re-planning");
    if (hb.overflow & kOverCoarse) t2cap = hb.coarse_used + hb.coarse_used / 16 + 4096;
  }
  const TreeInfo& ti = b.h_trees[0];
  const Cube& cb = b.h_cubes[0];
  for (int a = 0; a < 3; ++a) {
    view->aabb_min[a] = cb.lo[a];
    view->aabb_max[a] = cb.hi[a];
  }
  view->cube_side = cb.side;
  view->num_nodes = ti.num_nodes;
  view->num_points = n;
  view->num_voxels = ti.vtotal;
  view->node_level = b.o_level;
  view->node_is_leaf = b.o_leaf;
  view->node_child_mask = b.o_mask;
  view->node_key = b.o_key;
  view->node_npoints = b.o_npts;
  view->node_count = b.o_count;
  view->node_first_child = b.o_first;
  view->node_offset = b.o_off;
  view->points = b.Y;
  view->point_ids = b.Yid;
  view->voxels = (const lod_voxel*)b.vox;
  view->voxel_ids = b.vids;
  view->voxel_points = b.vpts;
  *out_bytes = noalloc_out_bytes(c, pl);
}

}  // namespace

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
    const uint64_t offs[2] = {0, n};
    const lod_params q =
        (p->flags & LOD_FLAG_AUTOTUNE) ? tune_batch(d_points, offs, 1, *p, (hipStream_t)hip_stream, nullptr) : *p;
    *out = lod_build_tree(d_points, n, q, (hipStream_t)hip_stream);
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
    const lod_params q = (p->flags & LOD_FLAG_AUTOTUNE)
                             ? tune_batch(d_points, h_offsets, num_chunks, *p, (hipStream_t)hip_stream, nullptr)
                             : *p;
    std::vector<lod_tree*> t = lod_build_clouds(d_points, h_offsets, num_chunks, q, (hipStream_t)hip_stream);
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

lod_status lod_build_noalloc(const lod_point* d_points, uint64_t n, const lod_params* p, void* hip_stream,
                             void* d_out, uint64_t* out_bytes, lod_tree_view* view) {
  if (!out_bytes || !view) {
    set_err("out_bytes/view is NULL");
    return LOD_ERR_INVALID;
  }
  if (check_params(p) != LOD_OK) {
    set_err("invalid parameters");
    return LOD_ERR_INVALID;
  }
  if (p->sampling == LOD_WEIGHTED) {
    set_err("lod_build_noalloc does not take LOD_WEIGHTED (its pass needs scratch beyond the static array)");
    return LOD_ERR_INVALID;
  }
  if (n >= 0xffffffffull || (n && !d_points)) {
    set_err("n must be below 2^32 and d_points non-NULL");
    return LOD_ERR_INVALID;
  }
  try {
    std::lock_guard<std::mutex> g(g_na_mu);
    lod_params q = *p;
    q.flags &= ~(uint32_t)(LOD_FLAG_TIMING | LOD_FLAG_AUTOTUNE);
    build_noalloc(d_points, n, q, (hipStream_t)hip_stream, d_out, out_bytes, view);
    return LOD_OK;
  } catch (const LodError& e) {
    (void)hipGetLastError();
    memset(view, 0, sizeof(*view));
    return e.st;
  } catch (...) {
    set_err("unexpected host exception");
    memset(view, 0, sizeof(*view));
    return LOD_ERR_OOM;
  }
}

lod_status lod_tune_batch(const lod_point* d_points, const uint64_t* h_offsets, uint32_t num_chunks,
                          const lod_params* p, void* hip_stream, lod_params* tuned, lod_tune_info* info) {
  if (!tuned || (num_chunks && !h_offsets)) {
    set_err("tuned/h_offsets is NULL");
    return LOD_ERR_INVALID;
  }
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
  try {
    *tuned = tune_batch(d_points, h_offsets, num_chunks, *p, (hipStream_t)hip_stream, info);
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
