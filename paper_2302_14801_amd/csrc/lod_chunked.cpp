// lod_chunked.cpp -- the chunked (out-of-core) build: the tree of a host
// point cloud, equal to the in-core build, made from chunks of a bounded size
// (Sec. 7: a bottom-up out-of-core pipeline cuts the input into chunks of
// about 10M points, builds each on the GPU and combines them).
//
//   1. the bounding cube of the whole cloud, piece by piece on the GPU;
//   2. each piece sorted by cell on the GPU, so that a cell's points are one
//      run per piece; the same pass counts the level-h cells (h <= 7), which
//      give the split level b, the shallowest level whose cells hold at most
//      chunk_points points.  When the cloud fits in device memory it stays
//      there (one host -> device pass for everything); otherwise the pieces
//      stream: each is uploaded for the cube, uploaded again to be sorted,
//      and sent back sorted, and chunks are uploaded batch by batch;
//   4. the nodes of levels 0..b from the counts alone: a node at level L is
//      inner iff it holds more than T points and L < max_level, exactly the
//      in-core rule;
//   5. every level-b cell that is an inner node is a chunk root: its subtree
//      depends on its own points only, so the cells are built in batches of
//      about chunk_points points with the common cube (lod_build_clouds),
//      and their nodes at levels >= b are the whole tree's;
//   6. leaves at levels <= b (at most T points each) are copied from the
//      sorted pieces;
//   7. the voxels of the inner nodes above b, level by level from b - 1 up,
//      from their children's samples (k_merge.hip);
//   8. one tree: nodes in (level, key) order, leaf points in Morton order of
//      the leaves, voxels in node order, as the in-core build lays them out.
#include <algorithm>
#include <atomic>
#include <cstring>
#include <memory>
#include <thread>
#include <vector>

#include "common.h"
#include "internal.h"
#include "launch.h"

using namespace lod;

namespace {

// Device memory from the cache for the duration of the build.
struct DevBuf {
  int dev = 0;
  void* p = nullptr;
  size_t cap = 0;
  explicit DevBuf(int d) : dev(d) {}
  DevBuf(const DevBuf&) = delete;
  template <typename T>
  T* get(size_t count) {
    const size_t bytes = std::max<size_t>(count * sizeof(T), 256);
    if (bytes > cap) {
      release();
      p = lodint::cache().alloc(dev, bytes);
      cap = bytes;
    }
    return (T*)p;
  }
  void release() {
    if (p) lodint::cache().release(dev, p);
    p = nullptr;
    cap = 0;
  }
  ~DevBuf() { release(); }
};

// Pinned host memory for the duration of the build.
struct HostBuf {
  void* p = nullptr;
  HostBuf() = default;
  HostBuf(const HostBuf&) = delete;
  template <typename T>
  T* get(size_t count) {
    if (p) (void)hipHostFree(p);
    p = nullptr;
    if (hipHostMalloc(&p, std::max<size_t>(count * sizeof(T), 64), hipHostMallocDefault) != hipSuccess) {
      (void)hipGetLastError();
      p = nullptr;
      lod_fail(LOD_ERR_OOM, "pinned host allocation failed");
    }
    return (T*)p;
  }
  ~HostBuf() {
    if (p) (void)hipHostFree(p);
  }
};

// A second stream (default priority) for the sorted pieces' way back, with
// an event per buffer pair: sorted (ready to copy), done (copied back).
struct SideStream {
  hipStream_t s = nullptr;
  hipEvent_t sorted[2] = {}, done[2] = {};
  SideStream() {
    HIPCHK(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    for (int i = 0; i < 2; ++i) {
      HIPCHK(hipEventCreateWithFlags(&sorted[i], hipEventDisableTiming));
      HIPCHK(hipEventCreateWithFlags(&done[i], hipEventDisableTiming));
    }
  }
  SideStream(const SideStream&) = delete;
  ~SideStream() {
    if (s) (void)hipStreamSynchronize(s);
    for (int i = 0; i < 2; ++i) {
      if (sorted[i]) (void)hipEventDestroy(sorted[i]);
      if (done[i]) (void)hipEventDestroy(done[i]);
    }
    if (s) (void)hipStreamDestroy(s);
  }
};

// Waits for the stream before the buffers above it are released (also when
// the build unwinds).
struct Drain {
  hipStream_t s;
  ~Drain() { (void)hipStreamSynchronize(s); }
};

struct TreeDel {
  void operator()(lod_tree* t) const { lod_tree_free(t); }
};
using TreePtr = std::unique_ptr<lod_tree, TreeDel>;

// A node of the merged tree and where its payload comes from.
struct MNode {
  uint32_t level;
  uint64_t key;
  bool leaf;
  uint64_t npoints;
  uint32_t count = 0;    // points (leaf) or voxels (inner)
  // top leaf: host range of sorted points; top inner: level buffer range;
  // chunk node: tree and its node index
  int src = 0;           // 0 top leaf, 1 top inner, 2 chunk node
  uint64_t c0 = 0, c1 = 0;  // top leaf: its level-b cells
  uint32_t tree = 0;     // chunk node: root index
  uint64_t soff = 0;     // chunk node: offset in its tree; top inner: offset in its level buffer
  uint64_t off = 0;      // output offset
  uint8_t mask = 0;
  uint32_t first = 0;
};

uint64_t morton_order(uint32_t level, uint64_t key) { return key << (3 * (kKeyLevels - level)); }

}  // namespace

lod_tree* lod_build_chunked_tree(const lod_point* hin, uint64_t n, const lod_params& prm, uint64_t chunk,
                                 hipStream_t s) {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  const uint32_t T = prm.leaf_cap;
  const uint32_t mode = prm.sampling;  // 0 average, 1 first, 2 random, 3 weighted
  const bool pick = mode == LOD_PICK_FIRST || mode == LOD_PICK_RANDOM;
  const bool full = (prm.flags & LOD_FLAG_FULL_PRECISION) != 0;
  const bool ids = pick || full || (prm.flags & LOD_FLAG_POINT_IDS);
  const bool vids_out = pick || full;  // voxel ids: pick winners, or accepted samples

  DevBuf d_stage(dev), d_ids(dev), d_cell(dev), d_hist(dev), d_small(dev), d_grids(dev), d_jobs(dev), d_cnt(dev),
      d_soff(dev), d_runs(dev), d_sorted(dev), d_sorted2(dev), d_sids(dev), d_sids2(dev), d_cursor(dev),
      d_tiles(dev), d_hist2(dev);
  HostBuf h_ci, h_cube, h_sorted, h_sids, h_vid, h_rec;
  DevBuf d_rec(dev), d_res(dev), d_ress(dev), d_resid(dev), d_bruns(dev), d_bad(dev);
  std::vector<std::unique_ptr<DevBuf>> lvox, lvid;  // voxels of the levels above b
  Drain drain{s};  // declared last: the stream drains before any buffer above is released

  // everything in one chunk, or no level to split at: the in-core build
  if (n <= chunk || prm.max_level < 2) {
    lod_point* dp = d_stage.get<lod_point>(n);
    if (n) HIPCHK(hipMemcpyAsync(dp, hin, 16ull * n, hipMemcpyHostToDevice, s));
    return lod_build_tree(dp, n, prm, s);
  }

  // The cloud stays on the device when it fits in half of the free device
  // memory: the input, its pieces sorted by cell and their ids.
  size_t free_b = 0, total_b = 0;
  HIPCHK(hipMemGetInfo(&free_b, &total_b));
  const bool resident =
      !(prm.flags & LOD_FLAG_LOW_MEMORY) && n * (32ull + (ids ? 8 : 0)) + (1ull << 30) <= free_b / 2;
  lod_point* R = resident ? d_res.get<lod_point>(n) : nullptr;            // the input
  lod_point* RS = resident ? d_ress.get<lod_point>(n) : nullptr;          // pieces sorted by cell
  uint32_t* RSid = resident && ids ? d_resid.get<uint32_t>(n) : nullptr;  // their input indices

  // 1. the bounding cube, piece by piece (pieces of at least 2^20 points)
  const uint64_t P = std::min<uint64_t>(n, std::max<uint64_t>(chunk, 1u << 20));
  const uint64_t npieces = (n + P - 1) / P;
  lod_point* stage = resident ? nullptr : d_stage.get<lod_point>(P);
  CloudInfo* hci = h_ci.get<CloudInfo>(npieces + 1);
  for (uint64_t k = 0; k < npieces; ++k) {
    const uint64_t m = std::min<uint64_t>(P, n - k * P);
    hci[k] = CloudInfo{0u, (uint32_t)m, 0u, 0u};
  }
  hci[npieces] = CloudInfo{0u, (uint32_t)n, 0u, 0u};
  char* small = d_small.get<char>(4096 + sizeof(CloudInfo) * (npieces + 1));
  BBoxAcc* acc = (BBoxAcc*)small;
  Cube* dcube = (Cube*)(small + 256);
  CloudInfo* dci = (CloudInfo*)(small + 4096);
  HIPCHK(hipMemcpyAsync(dci, hci, sizeof(CloudInfo) * (npieces + 1), hipMemcpyHostToDevice, s));
  launch_bbox_reset(acc, s);
  for (uint64_t k = 0; k < npieces; ++k) {
    const uint64_t m = hci[k].count;
    lod_point* dst = resident ? R + k * P : stage;
    HIPCHK(hipMemcpyAsync(dst, hin + k * P, 16ull * m, hipMemcpyHostToDevice, s));
    launch_bbox_add(dst, dci + k, bbox_tiles((uint32_t)m), acc, s);
  }
  launch_bbox_cube(acc, dci + npieces, dcube, s);
  Cube* hc = h_cube.get<Cube>(1);
  HIPCHK(hipMemcpyAsync(hc, dcube, sizeof(Cube), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  if (hc->nonfinite) lod_fail(LOD_ERR_NONFINITE, "input contains a NaN or infinite coordinate");

  // 2. every piece sorted by cell on the GPU (and sent back when streaming),
  // so that a cell's points are one run per piece.  Pieces are sorted by level s = min(h, 4)
  // cells (at most 4096: counts and ranks in LDS), h = min(7, max_level - 1).
  // The sort's counts give the split level b, the shallowest level whose
  // cells hold at most chunk_points points, when that is level s or above;
  // otherwise a pass counts the level-h cells and the pieces are sorted
  // again by level-b cells.  pst[k][c]: first
  // point of cell c in piece k (piece k starts at k * PS of the sorted
  // arrays).  When streaming, the sorted pieces return on a second stream
  // while the next piece is uploaded and sorted.
  const uint32_t h = std::min<uint32_t>(7, prm.max_level - 1);
  const uint32_t nh = 1u << (3 * h);
  // the sorted pieces on the host when streaming; input indices travel only
  // when used
  lod_point* sp = resident ? nullptr : h_sorted.get<lod_point>(n);
  uint32_t* sid = !resident && ids ? h_sids.get<uint32_t>(n) : nullptr;
  std::vector<std::vector<uint32_t>> pst;
  uint32_t* hist_h = d_hist.get<uint32_t>(nh);
  uint64_t PS = 0, npieces_s = 0;
  uint32_t sorted_level = 0;
  auto sort_pass = [&](uint32_t level) {
    const uint32_t ns = 1u << (3 * level);
    // at least 16 points per cell: the per-piece tables stay at n / 4 bytes
    PS = std::min<uint64_t>(n, std::max<uint64_t>(P, 16ull * ns));
    npieces_s = (n + PS - 1) / PS;
    sorted_level = level;
    pst.assign(npieces_s, std::vector<uint32_t>((size_t)ns + 1));
    uint32_t* hist_s = d_hist2.get<uint32_t>(ns);
    uint32_t* dcell = d_cell.get<uint32_t>(PS);
    uint32_t* cursor = d_cursor.get<uint32_t>(ns);
    uint32_t* tiles = d_tiles.get<uint32_t>(1024);
    if (resident) {
      // every piece from the resident input into the resident sorted array
      for (uint64_t k = 0; k < npieces_s; ++k) {
        const uint64_t m = std::min<uint64_t>(PS, n - k * PS);
        HIPCHK(hipMemsetAsync(hist_s, 0, 4ull * ns, s));
        launch_cells(R + k * PS, (uint32_t)m, dcube, level, dcell, hist_s, s);
        HIPCHK(hipMemcpyAsync(pst[k].data(), hist_s, 4ull * ns, hipMemcpyDeviceToHost, s));
        launch_sort_by_cell(R + k * PS, dcell, (uint32_t)m, (uint32_t)(k * PS), hist_s, ns, tiles, cursor, RS + k * PS,
                            RSid ? RSid + k * PS : nullptr, s);
        HIPCHK(hipGetLastError());
      }
      HIPCHK(hipStreamSynchronize(s));
    }
    stage = resident ? nullptr : d_stage.get<lod_point>(PS);
    lod_point* dsorted[2] = {resident ? nullptr : d_sorted.get<lod_point>(PS),
                             resident ? nullptr : d_sorted2.get<lod_point>(PS)};
    uint32_t* dsids[2] = {resident ? nullptr : d_sids.get<uint32_t>(PS),
                          resident ? nullptr : d_sids2.get<uint32_t>(PS)};
    SideStream s2;
    for (uint64_t k = 0; !resident && k < npieces_s; ++k) {
      const uint64_t m = std::min<uint64_t>(PS, n - k * PS);
      const int q = (int)(k & 1);
      HIPCHK(hipMemcpyAsync(stage, hin + k * PS, 16ull * m, hipMemcpyHostToDevice, s));
      HIPCHK(hipMemsetAsync(hist_s, 0, 4ull * ns, s));
      launch_cells(stage, (uint32_t)m, dcube, level, dcell, hist_s, s);
      HIPCHK(hipMemcpyAsync(pst[k].data(), hist_s, 4ull * ns, hipMemcpyDeviceToHost, s));
      // the buffers of piece k - 2 are free once their copy back has ended
      if (k >= 2) HIPCHK(hipStreamWaitEvent(s, s2.done[q], 0));
      launch_sort_by_cell(stage, dcell, (uint32_t)m, (uint32_t)(k * PS), hist_s, ns, tiles, cursor, dsorted[q],
                          dsids[q], s);
      HIPCHK(hipGetLastError());
      HIPCHK(hipEventRecord(s2.sorted[q], s));
      HIPCHK(hipStreamWaitEvent(s2.s, s2.sorted[q], 0));
      HIPCHK(hipMemcpyAsync(sp + k * PS, dsorted[q], 16ull * m, hipMemcpyDeviceToHost, s2.s));
      if (sid) HIPCHK(hipMemcpyAsync(sid + k * PS, dsids[q], 4ull * m, hipMemcpyDeviceToHost, s2.s));
      HIPCHK(hipEventRecord(s2.done[q], s2.s));
    }
    HIPCHK(hipStreamSynchronize(s2.s));
    HIPCHK(hipStreamSynchronize(s));
    for (uint64_t k = 0; k < npieces_s; ++k) {
      uint32_t run = 0;
      for (uint32_t c = 0; c <= ns; ++c) {
        const uint32_t v = c < ns ? pst[k][c] : 0u;
        pst[k][c] = run;
        run += v;
      }
    }
  };
  const uint32_t s_level = std::min<uint32_t>(h, 4);
  sort_pass(s_level);
  // counts of the levels 0..top (Morton-contiguous sums), top = s_level from
  // the sort's per-piece counts, or h from a counting pass
  std::vector<std::vector<uint64_t>> cnt;
  auto levels_from = [&](uint32_t top) {
    cnt.resize(top + 1);
    for (int L = (int)top - 1; L >= 0; --L) {
      cnt[L].assign(1ull << (3 * L), 0);
      for (uint64_t c = 0; c < cnt[L + 1].size(); ++c) cnt[L][c >> 3] += cnt[L + 1][c];
    }
  };
  auto split_level = [&](uint32_t top) -> uint32_t {
    for (uint32_t L = 1; L <= top; ++L)
      if (*std::max_element(cnt[L].begin(), cnt[L].end()) <= chunk) return L;
    return top;
  };
  cnt.assign(s_level + 1, {});
  cnt[s_level].assign(1ull << (3 * s_level), 0);
  for (uint64_t k = 0; k < npieces_s; ++k)
    for (uint32_t c = 0; c < (1u << (3 * s_level)); ++c) cnt[s_level][c] += pst[k][c + 1] - pst[k][c];
  levels_from(s_level);
  uint32_t b = split_level(s_level);
  if (b == s_level && s_level < h &&
      *std::max_element(cnt[s_level].begin(), cnt[s_level].end()) > chunk) {
    // level s is not fine enough: count the level-h cells, then sort again
    HIPCHK(hipMemsetAsync(hist_h, 0, 4ull * nh, s));
    uint32_t* dcell = d_cell.get<uint32_t>(P);
    stage = resident ? nullptr : d_stage.get<lod_point>(P);
    for (uint64_t k = 0; k < npieces; ++k) {
      const uint64_t m = hci[k].count;
      if (!resident) HIPCHK(hipMemcpyAsync(stage, hin + k * P, 16ull * m, hipMemcpyHostToDevice, s));
      launch_cells(resident ? R + k * P : stage, (uint32_t)m, dcube, h, dcell, hist_h, s);
      HIPCHK(hipGetLastError());
    }
    std::vector<uint32_t> hh(nh);
    HIPCHK(hipMemcpyAsync(hh.data(), hist_h, 4ull * nh, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    cnt.assign(h + 1, {});
    cnt[h].assign(hh.begin(), hh.end());
    levels_from(h);
    b = split_level(h);
    sort_pass(b);
  }
  d_sorted.release();
  d_sorted2.release();
  d_sids.release();
  d_sids2.release();
  d_cell.release();
  // the points of level-b cells [c0, c1): one run per piece
  const uint32_t sh = 3 * (sorted_level - b);
  auto for_runs = [&](uint64_t c0, uint64_t c1, auto&& f) {
    uint64_t o = 0;
    for (uint64_t k = 0; k < npieces_s; ++k) {
      const uint64_t beg = k * PS + pst[k][c0 << sh], len = pst[k][c1 << sh] - pst[k][c0 << sh];
      if (len) f(beg, len, o);
      o += len;
    }
  };

  // 4. nodes of levels 0..b
  std::vector<MNode> nodes;
  std::vector<uint64_t> roots;  // level-b cells that are inner nodes
  {
    std::vector<uint64_t> cur{0};
    for (uint32_t L = 0; L <= b && !cur.empty(); ++L) {
      std::vector<uint64_t> next;
      for (uint64_t key : cur) {
        MNode m;
        m.level = L;
        m.key = key;
        m.npoints = cnt[L][key];
        m.leaf = !(m.npoints > T && L < prm.max_level);
        if (m.leaf) {
          // a top leaf: its level-b cells are contiguous in the sorted points
          m.src = 0;
          m.c0 = key << (3 * (b - L));
          m.c1 = (key + 1) << (3 * (b - L));
          m.count = (uint32_t)m.npoints;
          nodes.push_back(m);
        } else if (L == b) {
          roots.push_back(key);  // its node comes from the chunk tree
        } else {
          m.src = 1;
          nodes.push_back(m);
          for (uint32_t o = 0; o < 8; ++o)
            if (cnt[L + 1][(key << 3) | o]) next.push_back((key << 3) | o);
        }
      }
      cur.swap(next);
    }
  }

  // 5. chunk builds: the root cells in batches of about chunk points
  lod_params cp = prm;
  if (ids) cp.flags |= LOD_FLAG_POINT_IDS;
  std::vector<TreePtr> rtrees(roots.size());
  struct HTree {
    std::vector<uint8_t> level, leaf;
    std::vector<uint64_t> key, off;
    std::vector<uint32_t> npts, count;
  };
  std::vector<HTree> ht(roots.size());
  // batches [bstart[i], bstart[i + 1]) of roots; batch i + 1 is uploaded on
  // the side stream (into the other buffer pair) while batch i is built
  std::vector<size_t> bstart{0};
  uint64_t max_pts = 0;
  for (size_t r0 = 0; r0 < roots.size();) {
    size_t r1 = r0;
    uint64_t pts = 0;
    while (r1 < roots.size() && (r1 == r0 || pts + cnt[b][roots[r1]] <= chunk)) pts += cnt[b][roots[r1++]];
    bstart.push_back(r1);
    max_pts = std::max(max_pts, pts);
    r0 = r1;
  }
  lod_point* bpts[2] = {d_stage.get<lod_point>(max_pts), d_sorted.get<lod_point>(max_pts)};
  uint32_t* bids[2] = {ids ? d_ids.get<uint32_t>(max_pts) : nullptr, ids ? d_sids.get<uint32_t>(max_pts) : nullptr};
  SideStream up;
  // resident: a batch's points gathered from the sorted pieces on the device
  // (one run per root cell and piece) on the build stream
  std::vector<CopyRun> pr, ir;  // read by the copies until the batch's closing synchronisation
  auto gather = [&](size_t i) {
    const int q = (int)(i & 1);
    pr.clear();
    ir.clear();
    uint64_t o = 0;
    for (size_t r = bstart[i]; r < bstart[i + 1]; ++r) {
      const uint64_t c = roots[r];
      for_runs(c, c + 1, [&](uint64_t beg, uint64_t len, uint64_t at) {
        pr.push_back(CopyRun{RS + beg, o + at, len});
        if (RSid) ir.push_back(CopyRun{RSid + beg, o + at, len});
      });
      o += cnt[b][c];
    }
    CopyRun* dr = d_bruns.get<CopyRun>(pr.size() + ir.size());
    if (pr.empty()) return;
    HIPCHK(hipMemcpyAsync(dr, pr.data(), sizeof(CopyRun) * pr.size(), hipMemcpyHostToDevice, s));
    if (!ir.empty())
      HIPCHK(hipMemcpyAsync(dr + pr.size(), ir.data(), sizeof(CopyRun) * ir.size(), hipMemcpyHostToDevice, s));
    launch_copy_runs(dr, (uint32_t)pr.size(), 16, bpts[q], s);
    if (!ir.empty()) launch_copy_runs(dr + pr.size(), (uint32_t)ir.size(), 4, bids[q], s);
    HIPCHK(hipGetLastError());
  };
  auto upload = [&](size_t i) {
    const int q = (int)(i & 1);
    uint64_t o = 0;
    for (size_t r = bstart[i]; r < bstart[i + 1]; ++r) {
      const uint64_t c = roots[r];
      for_runs(c, c + 1, [&](uint64_t beg, uint64_t len, uint64_t at) {
        HIPCHK(hipMemcpyAsync(bpts[q] + o + at, sp + beg, 16ull * len, hipMemcpyHostToDevice, up.s));
        if (sid) HIPCHK(hipMemcpyAsync(bids[q] + o + at, sid + beg, 4ull * len, hipMemcpyHostToDevice, up.s));
      });
      o += cnt[b][c];
    }
    HIPCHK(hipEventRecord(up.done[q], up.s));
  };
  const size_t nbatches = bstart.size() - 1;
  if (nbatches && !resident) upload(0);
  for (size_t i = 0; i < nbatches; ++i) {
    const size_t r0 = bstart[i], r1 = bstart[i + 1];
    const int q = (int)(i & 1);
    if (resident) {
      gather(i);  // the run table is free: the previous batch ended with a synchronisation
    } else {
      // the other buffer pair was last read by batch i - 1, whose build has ended
      if (i + 1 < nbatches) upload(i + 1);
      HIPCHK(hipStreamWaitEvent(s, up.done[q], 0));
    }
    lod_point* bp = bpts[q];
    uint32_t* bid = bids[q];
    std::vector<uint64_t> offs(r1 - r0 + 1, 0);
    for (size_t r = r0; r < r1; ++r) offs[r - r0 + 1] = offs[r - r0] + cnt[b][roots[r]];
    BuildExtras x;
    x.cube = hc;
    x.d_ids = bid;
    x.ids_only = true;  // full-precision records are gathered once for the whole tree
    std::vector<lod_tree*> t = lod_build_clouds(bp, offs.data(), (uint32_t)(r1 - r0), cp, s, &x);
    for (size_t r = r0; r < r1; ++r) rtrees[r].reset(t[r - r0]);
    // node tables of the new trees
    for (size_t r = r0; r < r1; ++r) {
      const lod_tree_view& v = rtrees[r]->v;
      HTree& q = ht[r];
      const uint32_t nn = v.num_nodes;
      q.level.resize(nn); q.leaf.resize(nn); q.key.resize(nn); q.off.resize(nn); q.npts.resize(nn); q.count.resize(nn);
      HIPCHK(hipMemcpyAsync(q.level.data(), v.node_level, nn, hipMemcpyDeviceToHost, s));
      HIPCHK(hipMemcpyAsync(q.leaf.data(), v.node_is_leaf, nn, hipMemcpyDeviceToHost, s));
      HIPCHK(hipMemcpyAsync(q.key.data(), v.node_key, 8ull * nn, hipMemcpyDeviceToHost, s));
      HIPCHK(hipMemcpyAsync(q.off.data(), v.node_offset, 8ull * nn, hipMemcpyDeviceToHost, s));
      HIPCHK(hipMemcpyAsync(q.npts.data(), v.node_npoints, 4ull * nn, hipMemcpyDeviceToHost, s));
      HIPCHK(hipMemcpyAsync(q.count.data(), v.node_count, 4ull * nn, hipMemcpyDeviceToHost, s));
    }
    HIPCHK(hipStreamSynchronize(s));
    for (size_t r = r0; r < r1; ++r) {
      const HTree& q = ht[r];
      bool found = false;
      for (uint32_t i = 0; i < q.level.size(); ++i) {
        if (q.level[i] < b) continue;
        if (q.level[i] == b) {
          if (q.key[i] != roots[r] || q.leaf[i]) lod_fail(LOD_ERR_CAPACITY, "chunk root differs from the cell counts");
          found = true;
        }
        MNode m;
        m.level = q.level[i];
        m.key = q.key[i];
        m.leaf = q.leaf[i] != 0;
        m.npoints = q.npts[i];
        m.count = q.count[i];
        m.src = 2;
        m.tree = (uint32_t)r;
        m.soff = q.off[i];
        nodes.push_back(m);
      }
      if (!found) lod_fail(LOD_ERR_CAPACITY, "chunk tree without its root cell");
    }
  }
  HIPCHK(hipStreamSynchronize(up.s));
  d_ids.release();
  d_sids.release();
  d_sorted.release();

  // 8a. node order, children, leaf point offsets
  std::sort(nodes.begin(), nodes.end(), [](const MNode& a, const MNode& c) {
    return a.level != c.level ? a.level < c.level : a.key < c.key;
  });
  const uint32_t num_nodes = (uint32_t)nodes.size();
  {
    // children of node i: the next level's nodes whose key >> 3 is its key,
    // consecutive in (level, key) order
    size_t j = 0;
    for (uint32_t i = 0; i < num_nodes; ++i) {
      MNode& m = nodes[i];
      if (m.leaf) continue;
      while (j < num_nodes && (nodes[j].level < m.level + 1 ||
                               (nodes[j].level == m.level + 1 && (nodes[j].key >> 3) < m.key)))
        ++j;
      m.first = (uint32_t)j;
      for (size_t k = j; k < num_nodes && nodes[k].level == m.level + 1 && (nodes[k].key >> 3) == m.key; ++k)
        m.mask |= (uint8_t)(1u << (nodes[k].key & 7u));
    }
    std::vector<uint32_t> leaves;
    for (uint32_t i = 0; i < num_nodes; ++i)
      if (nodes[i].leaf) leaves.push_back(i);
    std::sort(leaves.begin(), leaves.end(), [&](uint32_t a, uint32_t c) {
      return morton_order(nodes[a].level, nodes[a].key) < morton_order(nodes[c].level, nodes[c].key);
    });
    uint64_t run = 0;
    for (uint32_t i : leaves) {
      nodes[i].off = run;
      run += nodes[i].count;
    }
    if (run != n) lod_fail(LOD_ERR_CAPACITY, "leaf points do not add up to the input");
  }

  // 6. output points: top leaves from the sorted pieces (on the device, or
  // on the host when streaming), chunk leaves from their trees
  std::shared_ptr<LodArena> arena = std::make_shared<LodArena>();
  arena->dev = dev;
  lod_point* Y = arena->alloc<lod_point>(n);
  uint32_t* Yid = ids ? arena->alloc<uint32_t>(n) : nullptr;
  std::vector<CopyRun> prun, irun;
  for (const MNode& m : nodes) {
    if (!m.leaf || !m.count) continue;
    if (m.src == 0 && resident) {
      for_runs(m.c0, m.c1, [&](uint64_t beg, uint64_t len, uint64_t at) {
        prun.push_back(CopyRun{RS + beg, m.off + at, len});
        if (Yid) irun.push_back(CopyRun{RSid + beg, m.off + at, len});
      });
    } else if (m.src == 0) {
      for_runs(m.c0, m.c1, [&](uint64_t beg, uint64_t len, uint64_t at) {
        HIPCHK(hipMemcpyAsync(Y + m.off + at, sp + beg, 16ull * len, hipMemcpyHostToDevice, s));
        if (Yid) HIPCHK(hipMemcpyAsync(Yid + m.off + at, sid + beg, 4ull * len, hipMemcpyHostToDevice, s));
      });
    } else {
      const lod_tree_view& v = rtrees[m.tree]->v;
      prun.push_back(CopyRun{v.points + m.soff, m.off, m.count});
      if (Yid) irun.push_back(CopyRun{v.point_ids + m.soff, m.off, m.count});
    }
  }
  auto run_copies = [&](const std::vector<CopyRun>& runs, uint32_t bytes, void* dst) {
    if (runs.empty()) return;
    CopyRun* dr = d_runs.get<CopyRun>(runs.size());
    HIPCHK(hipMemcpyAsync(dr, runs.data(), sizeof(CopyRun) * runs.size(), hipMemcpyHostToDevice, s));
    launch_copy_runs(dr, (uint32_t)runs.size(), bytes, dst, s);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(s));  // the run table is reused
  };
  run_copies(prun, 16, Y);
  if (Yid) run_copies(irun, 4, Yid);

  // 7. voxels of the inner nodes above b, level by level
  std::vector<uint32_t> node_at;  // (level, key) -> node index for the levels <= b
  lvox.resize(b);
  lvid.resize(b);
  auto find = [&](uint32_t level, uint64_t key) -> const MNode& {
    auto it = std::lower_bound(nodes.begin(), nodes.end(), std::make_pair(level, key),
                               [](const MNode& a, const std::pair<uint32_t, uint64_t>& k) {
                                 return a.level != k.first ? a.level < k.first : a.key < k.second;
                               });
    return *it;
  };
  const uint32_t kMaxJobs = 64;  // 64 dense grids of 10 MB
  TopCell* grids = d_grids.get<TopCell>((size_t)kMaxJobs * kTopCells);
  for (int L = (int)b - 1; L >= 0; --L) {
    std::vector<TopJob> jobs;
    std::vector<uint32_t> owner;  // node index of each job's parent
    std::vector<size_t> first;    // a parent's first job (launches never split a parent)
    uint64_t bound = 0;
    for (uint32_t i = 0; i < num_nodes; ++i) {
      const MNode& a = nodes[i];
      if (a.level != (uint32_t)L || a.leaf) continue;
      first.push_back(jobs.size());
      for (uint32_t o = 0; o < 8; ++o) {
        if (!(a.mask >> o & 1u)) continue;
        const MNode& c = find(L + 1, (a.key << 3) | o);
        TopJob j{};
        j.oct = o;
        j.level = (uint32_t)L;
        for (int x = 0; x < 3; ++x) {
          j.G[x] = compact21(a.key >> x);
          j.C[x] = compact21(c.key >> x);
        }
        if (c.leaf) {
          j.kind = 1;
          j.src = Y + c.off;
          j.ids = Yid ? Yid + c.off : nullptr;
          j.count = c.count;
        } else if (c.src == 2) {
          const lod_tree_view& v = rtrees[c.tree]->v;
          j.kind = 0;
          j.src = (const uint64_t*)v.voxels + c.soff;
          j.ids = v.voxel_ids ? v.voxel_ids + c.soff : nullptr;
          j.count = c.count;
        } else {
          j.kind = 0;
          j.src = (const uint64_t*)lvox[L + 1]->p + c.soff;
          j.ids = vids_out ? (const uint32_t*)lvid[L + 1]->p + c.soff : nullptr;
          j.count = c.count;
        }
        bound += std::min<uint64_t>(kTopCells, j.count);
        jobs.push_back(j);
        owner.push_back(i);
      }
    }
    lvox[L].reset(new DevBuf(dev));
    lvid[L].reset(new DevBuf(dev));
    uint64_t* vox = lvox[L]->get<uint64_t>(bound);
    uint32_t* vid = vids_out ? lvid[L]->get<uint32_t>(bound) : nullptr;
    first.push_back(jobs.size());
    uint64_t pos = 0;
    for (size_t f = 0, j0 = 0; j0 < jobs.size(); j0 = first[f]) {
      // whole parents, at most kMaxJobs jobs (a parent has at most 8)
      while (f + 1 < first.size() && first[f + 1] - j0 <= kMaxJobs) ++f;
      const uint32_t nj = (uint32_t)(first[f] - j0);
      // the jobs of each parent's octants in this launch
      for (size_t q = j0; q < j0 + nj; ++q) {
        for (int o = 0; o < 8; ++o) jobs[q].sib[o] = -1;
        for (size_t r = j0; r < j0 + nj; ++r)
          if (owner[r] == owner[q]) jobs[q].sib[jobs[r].oct] = (int32_t)(r - j0);
      }
      uint32_t maxc = 0;
      for (uint32_t k = 0; k < nj; ++k) maxc = std::max(maxc, jobs[j0 + k].count);
      TopJob* dj = d_jobs.get<TopJob>(nj);
      uint32_t* dcnt = d_cnt.get<uint32_t>((size_t)nj * kTopSlices);
      uint64_t* dsoff = d_soff.get<uint64_t>((size_t)nj * kTopSlices);
      HIPCHK(hipMemcpyAsync(dj, jobs.data() + j0, sizeof(TopJob) * nj, hipMemcpyHostToDevice, s));
      launch_top_clear(grids, nj, mode, s);
      launch_top_splat(dj, nj, maxc, dcube, mode, prm.seed, full, grids, s);
      launch_top_count(grids, nj, dcnt, s);
      HIPCHK(hipGetLastError());
      std::vector<uint32_t> hcnt((size_t)nj * kTopSlices);
      std::vector<uint64_t> hsoff((size_t)nj * kTopSlices);
      HIPCHK(hipMemcpyAsync(hcnt.data(), dcnt, 4ull * hcnt.size(), hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      for (uint32_t k = 0; k < nj; ++k) {
        uint32_t jc = 0;
        for (uint32_t q = 0; q < kTopSlices; ++q) {
          hsoff[(size_t)k * kTopSlices + q] = pos;
          pos += hcnt[(size_t)k * kTopSlices + q];
          jc += hcnt[(size_t)k * kTopSlices + q];
        }
        MNode& a = nodes[owner[j0 + k]];
        if (a.count == 0) a.soff = pos - jc;  // the parent's first job
        a.count += jc;
      }
      HIPCHK(hipMemcpyAsync(dsoff, hsoff.data(), 8ull * hsoff.size(), hipMemcpyHostToDevice, s));
      launch_top_emit(dj, nj, grids, dsoff, mode, vox, vid, s);
      HIPCHK(hipGetLastError());
      HIPCHK(hipStreamSynchronize(s));  // the host tables are refilled
    }
  }
  d_grids.release();

  // 8b. voxels in node order
  uint64_t vtotal = 0;
  for (MNode& m : nodes)
    if (!m.leaf) {
      m.off = vtotal;
      vtotal += m.count;
    }
  uint64_t* vox = arena->alloc<uint64_t>(std::max<uint64_t>(vtotal, 1));
  uint32_t* vids = vids_out ? arena->alloc<uint32_t>(std::max<uint64_t>(vtotal, 1)) : nullptr;
  std::vector<CopyRun> vrun, vidrun;
  for (const MNode& m : nodes) {
    if (m.leaf || !m.count) continue;
    if (m.src == 2) {
      const lod_tree_view& v = rtrees[m.tree]->v;
      vrun.push_back(CopyRun{(const uint64_t*)v.voxels + m.soff, m.off, m.count});
      if (vids) vidrun.push_back(CopyRun{v.voxel_ids + m.soff, m.off, m.count});
    } else {
      vrun.push_back(CopyRun{(const uint64_t*)lvox[m.level]->p + m.soff, m.off, m.count});
      if (vids) vidrun.push_back(CopyRun{(const uint32_t*)lvid[m.level]->p + m.soff, m.off, m.count});
    }
  }
  run_copies(vrun, 8, vox);
  if (vids) run_copies(vidrun, 4, vids);

  // full precision: the accepted samples' input records, gathered by id from
  // the resident cloud or from the host cloud, with the voxels' colours
  lod_point* vpts = nullptr;
  if (full && vtotal && resident) {
    vpts = arena->alloc<lod_point>(vtotal);
    uint32_t* bad = d_bad.get<uint32_t>(1);
    HIPCHK(hipMemsetAsync(bad, 0, 4, s));
    launch_voxel_records_by_id(R, (uint32_t)n, vids, vox, vtotal, vpts, bad, s);
    HIPCHK(hipGetLastError());
    uint32_t hbad = 0;
    HIPCHK(hipMemcpyAsync(&hbad, bad, 4, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (hbad) lod_fail(LOD_ERR_CAPACITY, "an accepted sample id lies outside the input");
  } else if (full && vtotal) {
    uint32_t* hv = h_vid.get<uint32_t>(vtotal);
    lod_point* hr = h_rec.get<lod_point>(vtotal);
    HIPCHK(hipMemcpyAsync(hv, vids, 4ull * vtotal, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    const uint32_t nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    std::vector<std::thread> th;
    std::atomic<bool> bad{false};
    for (uint32_t t = 0; t < nt; ++t)
      th.emplace_back([&, t] {
        for (uint64_t i = vtotal * t / nt; i < vtotal * (t + 1) / nt; ++i) {
          if (hv[i] >= n) {
            bad = true;
            return;
          }
          hr[i] = hin[hv[i]];
        }
      });
    for (auto& x : th) x.join();
    if (bad) lod_fail(LOD_ERR_CAPACITY, "an accepted sample id lies outside the input");
    lod_point* drec = d_rec.get<lod_point>(vtotal);
    vpts = arena->alloc<lod_point>(vtotal);
    HIPCHK(hipMemcpyAsync(drec, hr, 16ull * vtotal, hipMemcpyHostToDevice, s));
    launch_voxel_records(drec, vox, vtotal, vpts, s);
    HIPCHK(hipGetLastError());
  }

  // 8c. node table
  uint8_t* o_level = arena->alloc<uint8_t>(num_nodes);
  uint8_t* o_leaf = arena->alloc<uint8_t>(num_nodes);
  uint8_t* o_mask = arena->alloc<uint8_t>(num_nodes);
  uint64_t* o_key = arena->alloc<uint64_t>(num_nodes);
  uint32_t* o_npts = arena->alloc<uint32_t>(num_nodes);
  uint32_t* o_count = arena->alloc<uint32_t>(num_nodes);
  uint32_t* o_first = arena->alloc<uint32_t>(num_nodes);
  uint64_t* o_off = arena->alloc<uint64_t>(num_nodes);
  {
    std::vector<uint8_t> lv(num_nodes), lf(num_nodes), mk(num_nodes);
    std::vector<uint64_t> ky(num_nodes), of(num_nodes);
    std::vector<uint32_t> np(num_nodes), ct(num_nodes), fc(num_nodes);
    for (uint32_t i = 0; i < num_nodes; ++i) {
      const MNode& m = nodes[i];
      lv[i] = (uint8_t)m.level;
      lf[i] = m.leaf ? 1 : 0;
      mk[i] = m.mask;
      ky[i] = m.key;
      of[i] = m.off;
      np[i] = (uint32_t)m.npoints;
      ct[i] = m.count;
      fc[i] = m.leaf ? 0u : m.first;
    }
    HIPCHK(hipMemcpyAsync(o_level, lv.data(), num_nodes, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(o_leaf, lf.data(), num_nodes, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(o_mask, mk.data(), num_nodes, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(o_key, ky.data(), 8ull * num_nodes, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(o_npts, np.data(), 4ull * num_nodes, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(o_count, ct.data(), 4ull * num_nodes, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(o_first, fc.data(), 4ull * num_nodes, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(o_off, of.data(), 8ull * num_nodes, hipMemcpyHostToDevice, s));
    HIPCHK(hipStreamSynchronize(s));
  }

  std::unique_ptr<lod_tree> t(new lod_tree());
  t->dev = dev;
  t->arena = arena;
  t->footprint = arena->bytes;
  lod_tree_view& v = t->v;
  for (int a = 0; a < 3; ++a) {
    v.aabb_min[a] = hc->lo[a];
    v.aabb_max[a] = hc->hi[a];
  }
  v.cube_side = hc->side;
  v.num_nodes = num_nodes;
  v.num_points = n;
  v.num_voxels = vtotal;
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
  v.voxel_points = vpts;
  return t.release();
}

extern "C" lod_status lod_build_chunked(const lod_point* h_points, uint64_t n, const lod_params* p,
                                        uint64_t chunk_points, void* hip_stream, lod_tree** out) {
  if (!out) {
    lod_set_error("out is NULL");
    return LOD_ERR_INVALID;
  }
  *out = nullptr;
  if (!p || p->leaf_cap == 0 || p->max_level > 14 || p->sampling > 3 || p->tune_levels0 > 4 ||
      p->tune_levels1 > 4) {
    lod_set_error("invalid parameters");
    return LOD_ERR_INVALID;
  }
  if (n >= 0xffffffffull || (n && !h_points) || chunk_points == 0) {
    lod_set_error("n must be below 2^32, h_points non-NULL and chunk_points positive");
    return LOD_ERR_INVALID;
  }
  try {
    *out = lod_build_chunked_tree(h_points, n, *p, chunk_points, (hipStream_t)hip_stream);
    return LOD_OK;
  } catch (const LodError& e) {
    (void)hipGetLastError();
    return e.st;
  } catch (...) {
    lod_set_error("unexpected host exception");
    return LOD_ERR_OOM;
  }
}
