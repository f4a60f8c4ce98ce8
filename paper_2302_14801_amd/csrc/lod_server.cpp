// lod_server.cpp -- request server with continuous batching.
//
// Chunks arrive as host point arrays (the bottom-up out-of-core use of
// Sec. 7: independent chunks of a larger cloud, each built on the GPU).
// Up to `max_inflight` worker threads, each with its own HIP stream and
// device input buffer, take requests from a FIFO queue.  A request is
// admitted when its estimated device footprint fits in the budget next to the
// requests already running and the trees still resident; admitted requests
// run concurrently, so their kernels overlap on the device, and new requests
// join as soon as a worker and memory free up.  Finished trees stay resident
// (and count against the budget) until the client frees them.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "internal.h"

namespace {

struct Request {
  uint64_t ticket = 0;
  const lod_point* h = nullptr;
  uint64_t n = 0;
  uint64_t estimate = 0;
  bool done = false;
  lod_status status = LOD_PENDING;
  lod_tree* tree = nullptr;
  char err[256] = "";
};

// Device bytes a build of n points may hold at its peak: the input copy
// (16 B/pt), the partition scratch and staged voxels (20 B/pt), the tree's
// points and ids (20 B/pt), voxel lists (at most ~8 B per point per inner
// level, 24 B/pt is a safe typical bound) plus fixed-size grids and tables.
// Full-precision records add 20 B per voxel (record and id), bounded the same
// way by 24 B/pt.
uint64_t footprint_estimate(uint64_t n, const lod_params& p) {
  const uint64_t full = (p.flags & LOD_FLAG_FULL_PRECISION) ? 24ull * n : 0ull;
  // weighted: 32 B of sums per voxel (at most about half a voxel per point)
  // and a 384 KB bitmap per node of the widest level (at most about 2 n / T)
  const uint64_t weighted =
      p.sampling == LOD_WEIGHTED ? 16ull * n + (385ull << 10) * (2ull * n / std::max(p.leaf_cap, 1u) + 8ull) : 0ull;
  return 80ull * n + full + weighted + (96ull << 20);
}

}  // namespace

struct lod_server {
  int dev = 0;
  lod_params params{};
  uint64_t budget = 0;
  std::shared_ptr<std::atomic<uint64_t>> used = std::make_shared<std::atomic<uint64_t>>(0);
  std::mutex mu;
  std::condition_variable cv;
  std::deque<Request*> queue;
  std::map<uint64_t, Request*> requests;
  uint64_t next_ticket = 1;
  bool stop = false;
  std::vector<std::thread> workers;

  void worker() {
    (void)hipSetDevice(dev);
    hipStream_t s = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return;
    void* dbuf = nullptr;
    size_t dcap = 0;
    for (;;) {
      Request* r = nullptr;
      {
        std::unique_lock<std::mutex> lk(mu);
        // trees freed by the client release budget without notifying, so re-check periodically
        while (!cv.wait_for(lk, std::chrono::milliseconds(1), [&] {
          if (stop) return true;
          if (queue.empty()) return false;
          return used->load() + queue.front()->estimate <= budget;
        })) {
        }
        if (stop) break;
        r = queue.front();
        queue.pop_front();
        used->fetch_add(r->estimate);
      }
      lod_status st = LOD_OK;
      lod_tree* t = nullptr;
      try {
        const size_t bytes = r->n * sizeof(lod_point);
        if (bytes > dcap) {
          lodint::cache().release(dev, dbuf);
          dbuf = lodint::cache().alloc(dev, bytes);
          dcap = bytes;
        }
        if (bytes && hipMemcpyAsync(dbuf, r->h, bytes, hipMemcpyHostToDevice, s) != hipSuccess) {
          (void)hipGetLastError();
          lod_set_error("host-to-device copy of the request failed");
          throw LodError{LOD_ERR_HIP};
        }
        t = lod_build_tree((const lod_point*)dbuf, r->n, params, s);
      } catch (const LodError& e) {
        st = e.st;
      } catch (...) {
        st = LOD_ERR_OOM;
      }
      {
        std::lock_guard<std::mutex> lk(mu);
        used->fetch_sub(r->estimate);
        if (t) {
          used->fetch_add(t->footprint);
          t->budget_used = used;
        }
        r->tree = t;
        r->status = st;
        if (st != LOD_OK) snprintf(r->err, sizeof(r->err), "%s", lod_last_error());
        r->done = true;
      }
      cv.notify_all();
    }
    lodint::cache().release(dev, dbuf);
    (void)hipStreamDestroy(s);
  }
};

extern "C" {

lod_status lod_server_create(uint64_t hbm_budget_bytes, uint32_t max_inflight, const lod_params* p,
                             lod_server** out) {
  if (!out || !p || p->leaf_cap == 0 || p->max_level > 14 || p->sampling > 3 || max_inflight == 0 ||
      max_inflight > 64 || hbm_budget_bytes == 0) {
    lod_set_error("invalid server arguments");
    if (out) *out = nullptr;
    return LOD_ERR_INVALID;
  }
  auto* s = new lod_server();
  (void)hipGetDevice(&s->dev);
  s->params = *p;
  s->budget = hbm_budget_bytes;
  for (uint32_t i = 0; i < max_inflight; ++i) s->workers.emplace_back([s] { s->worker(); });
  *out = s;
  return LOD_OK;
}

lod_status lod_submit(lod_server* s, const lod_point* h_points, uint64_t n, uint64_t* ticket) {
  if (!s || !ticket || (n && !h_points) || n >= 0xffffffffull) {
    lod_set_error("invalid submit arguments");
    return LOD_ERR_INVALID;
  }
  const uint64_t est = footprint_estimate(n, s->params);
  if (est > s->budget) {
    lod_set_error("request of %llu points needs about %llu bytes, more than the whole budget",
                  (unsigned long long)n, (unsigned long long)est);
    return LOD_ERR_TOO_LARGE;
  }
  auto* r = new Request();
  r->h = h_points;
  r->n = n;
  r->estimate = est;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    r->ticket = s->next_ticket++;
    s->requests[r->ticket] = r;
    s->queue.push_back(r);
    *ticket = r->ticket;
  }
  s->cv.notify_all();
  return LOD_OK;
}

lod_status lod_poll(lod_server* s, uint64_t ticket, lod_tree** out) {
  if (!s || !out) {
    lod_set_error("invalid poll arguments");
    return LOD_ERR_INVALID;
  }
  *out = nullptr;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->requests.find(ticket);
  if (it == s->requests.end()) {
    lod_set_error("unknown ticket %llu", (unsigned long long)ticket);
    return LOD_ERR_UNKNOWN_TICKET;
  }
  Request* r = it->second;
  if (!r->done) return LOD_PENDING;
  lod_status st = r->status;
  *out = r->tree;
  if (st != LOD_OK) lod_set_error("%s", r->err);
  s->requests.erase(it);
  delete r;
  return st;
}

void lod_server_destroy(lod_server* s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv.notify_all();
  for (auto& th : s->workers) th.join();
  for (auto& kv : s->requests) {
    if (kv.second->tree) lod_tree_free(kv.second->tree);
    delete kv.second;
  }
  delete s;
}

}  // extern "C"
