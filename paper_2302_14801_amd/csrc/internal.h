// internal.h -- library-internal host structures shared by the C ABI files.
#pragma once
#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdarg>
#include <cstdio>
#include <map>
#include <memory>
#include <mutex>
#include <vector>

#include "../../include/lod.h"

struct LodError {
  lod_status st;
};

void lod_set_error(const char* fmt, ...);

// Throw LodError (HIP failure, or an out-of-memory status) after recording the
// failing call.
#define HIPCHK(x)                                                                          \
  do {                                                                                     \
    hipError_t e_ = (x);                                                                   \
    if (e_ != hipSuccess) {                                                                \
      lod_set_error("%s failed: %s (%s:%d)", #x, hipGetErrorString(e_), __FILE__, __LINE__); \
      throw LodError{e_ == hipErrorOutOfMemory ? LOD_ERR_OOM : LOD_ERR_HIP};                \
    }                                                                                      \
  } while (0)

[[noreturn]] inline void lod_fail(lod_status st, const char* msg) {
  lod_set_error("%s", msg);
  throw LodError{st};
}

// ---------------------------------------------------------- device memory
//
// A small caching allocator: freed blocks are kept per device and reused for
// requests of at least half their size, so steady-state builds do not call
// hipMalloc.  Trees hold blocks until lod_tree_free.

namespace lodint {

struct Block {
  void* p = nullptr;
  size_t cap = 0;
};

class DeviceCache {
 public:
  void* alloc(int dev, size_t bytes) {
    if (bytes == 0) bytes = 256;
    {
      std::lock_guard<std::mutex> g(mu_);
      auto& m = free_[dev];
      auto it = m.lower_bound(bytes);
      if (it != m.end() && it->first <= 2 * bytes + (4u << 20)) {
        void* p = it->second;
        size_t cap = it->first;
        m.erase(it);
        used_[p] = cap;
        return p;
      }
    }
    size_t cap = (bytes + (2u << 20) - 1) & ~(size_t)((2u << 20) - 1);
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, cap);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      trim(dev);
      e = hipMalloc(&p, cap);
      if (e != hipSuccess) {
        (void)hipGetLastError();
        lod_set_error("device allocation of %zu bytes failed: %s", cap, hipGetErrorString(e));
        throw LodError{LOD_ERR_OOM};
      }
    }
    std::lock_guard<std::mutex> g(mu_);
    used_[p] = cap;
    return p;
  }
  void release(int dev, void* p) {
    if (!p) return;
    std::lock_guard<std::mutex> g(mu_);
    auto it = used_.find(p);
    if (it == used_.end()) return;
    free_[dev].emplace(it->second, p);
    used_.erase(it);
  }
  void trim(int dev) {
    std::lock_guard<std::mutex> g(mu_);
    for (auto& kv : free_[dev]) (void)hipFree(kv.second);
    free_[dev].clear();
  }

 private:
  std::mutex mu_;
  std::map<int, std::multimap<size_t, void*>> free_;
  std::map<void*, size_t> used_;
};

// One process-wide cache, never destroyed (frees after runtime teardown are unsafe).
inline DeviceCache& cache() {
  static DeviceCache* c = new DeviceCache();
  return *c;
}
}  // namespace lodint

// ---------------------------------------------------------------- the tree

// Device memory of the trees of one build call (one tree for lod_build, the
// chunks of lod_build_batch), released with the last of them.
struct LodArena {
  int dev = 0;
  std::vector<void*> blocks;
  uint64_t bytes = 0;
  ~LodArena() {
    for (void* p : blocks) lodint::cache().release(dev, p);
  }
  template <typename T>
  T* alloc(size_t count) {
    void* p = lodint::cache().alloc(dev, count * sizeof(T));
    blocks.push_back(p);
    bytes += count * sizeof(T);
    return (T*)p;
  }
};

struct lod_tree {
  int dev = 0;
  lod_tree_view v{};
  lod_timings timings{};
  std::shared_ptr<LodArena> arena;
  uint64_t footprint = 0;                              // device bytes accounted to this tree
  std::shared_ptr<std::atomic<uint64_t>> budget_used;  // server accounting, if any
  ~lod_tree() {
    if (budget_used) budget_used->fetch_sub(footprint);
  }
};

// Build the trees of `nclouds` independent clouds, cloud i being points
// [offs[i], offs[i+1]) of d_points (offs on the host), on `stream`, blocking
// until complete; throws LodError.  One tree per cloud, in order.
// Options of the chunked build: one bounding cube for every cloud (a host
// pointer to a lod::Cube, instead of each cloud's own cube; every point must
// lie in it), the input index of every point (a device array parallel to
// d_points, instead of the index within its cloud), and, with full precision,
// the accepted samples' ids without their records (the caller gathers them).
struct BuildExtras {
  const void* cube = nullptr;
  const uint32_t* d_ids = nullptr;
  bool ids_only = false;
};
std::vector<lod_tree*> lod_build_clouds(const lod_point* d_points, const uint64_t* offs, uint32_t nclouds,
                                        const lod_params& p, hipStream_t stream, const BuildExtras* x = nullptr);
// The chunked build of n host points (lod_build_chunked); throws LodError.
lod_tree* lod_build_chunked_tree(const lod_point* h_points, uint64_t n, const lod_params& p, uint64_t chunk_points,
                                 hipStream_t stream);
// One cloud.
lod_tree* lod_build_tree(const lod_point* d_points, uint64_t n, const lod_params& p, hipStream_t stream);
// The plan tuner (lod_tune.cpp): p with its tune_* fields chosen for batches
// like (offs, n) (kept if p sets any of them); throws LodError.
lod_params tune_batch(const lod_point* d_points, const uint64_t* offs, uint32_t n, const lod_params& p,
                      hipStream_t s, lod_tune_info* info);
// Device bytes a build of clouds of these sizes lays out (scratch and output,
// with the default estimates; the weighted pass's scratch included): the
// server admits requests by it.  Throws LodError.
uint64_t lod_plan_bytes(const uint64_t* sizes, uint32_t n, const lod_params& p);
