// lod_server.cpp -- request server with continuous batching.
//
// Chunks arrive as host point arrays (the bottom-up out-of-core use of
// Sec. 7: independent chunks of a larger cloud, each built on the GPU).
// Up to `max_inflight` worker threads, each with its own HIP stream and
// device input buffer, take requests from a FIFO queue.  A worker that is
// free takes the request at the head of the queue and every further queued
// request that still fits -- in the memory budget, next to the builds running
// and the trees still resident, and in a batch of at most kMaxBatch requests
// and kMaxBatchPoints points -- copies them into one device buffer and builds
// them together as one multi-cloud build (one graph launch).  Admission is by
// the bytes the build lays out (its input copy, scratch and output, from the
// same capacity plan the build uses), not a per-point guess.  Several workers
// run at once, so batches overlap on the device, and new requests join as
// soon as a worker and memory free up.  Finished trees stay resident (and
// count against the budget with their share of the output) until the client
// frees them.  A request's tree is the one lod_build makes of it alone;
// if a batch fails (for example a request with a non-finite coordinate), its
// requests are built again one by one, so an error stays with its request.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "internal.h"

namespace {

constexpr size_t kMaxBatch = 64;
constexpr uint64_t kMaxBatchPoints = 64ull << 20;

struct Request {
  uint64_t ticket = 0;
  const lod_point* h = nullptr;
  uint64_t n = 0;
  bool done = false;
  lod_status status = LOD_PENDING;
  lod_tree* tree = nullptr;
  char err[256] = "";
};

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

  // Device bytes a batch of these request sizes holds while it builds: the
  // input copy plus the laid-out scratch and output.
  uint64_t batch_bytes(const std::vector<uint64_t>& sizes) {
    uint64_t n = 0;
    for (uint64_t v : sizes) n += v;
    return 16 * n + lod_plan_bytes(sizes.data(), (uint32_t)sizes.size(), params);
  }

  // Take the head of the queue and whatever else fits (with the lock held);
  // returns the batch (empty if the head does not fit yet) and its bytes.
  std::vector<Request*> take_batch(uint64_t& bytes) {
    std::vector<Request*> batch;
    std::vector<uint64_t> sizes;
    uint64_t points = 0;
    bytes = 0;
    const uint64_t free_bytes = budget > used->load() ? budget - used->load() : 0;
    for (size_t i = 0; i < queue.size() && batch.size() < kMaxBatch; ++i) {
      Request* r = queue[i];
      if (!batch.empty() && points + r->n > kMaxBatchPoints) break;
      sizes.push_back(r->n);
      uint64_t b = 0;
      try {
        b = batch_bytes(sizes);
      } catch (const LodError&) {
        b = ~0ull;
      }
      if (b > free_bytes) {
        sizes.pop_back();
        // the head alone is admitted only into an otherwise idle budget if it
        // could never fit next to anything (it fits the whole budget: checked
        // at submission)
        if (batch.empty() && used->load() == 0) {
          batch.push_back(r);
          bytes = b == ~0ull ? budget : b;
        }
        break;
      }
      batch.push_back(r);
      points += r->n;
      bytes = b;
    }
    queue.erase(queue.begin(), queue.begin() + (long)batch.size());
    return batch;
  }

  void finish(Request* r, lod_tree* t, lod_status st, const char* err) {
    if (t) {
      used->fetch_add(t->footprint);
      t->budget_used = used;
    }
    r->tree = t;
    r->status = st;
    if (st != LOD_OK) snprintf(r->err, sizeof(r->err), "%s", err);
    r->done = true;
  }

  void worker() {
    (void)hipSetDevice(dev);
    hipStream_t s = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return;
    void* dbuf = nullptr;
    size_t dcap = 0;
    for (;;) {
      std::vector<Request*> batch;
      uint64_t reserved = 0;
      {
        std::unique_lock<std::mutex> lk(mu);
        // trees freed by the client release budget without notifying, so re-check periodically
        for (;;) {
          if (stop) break;
          if (!queue.empty()) {
            batch = take_batch(reserved);
            if (!batch.empty()) break;
          }
          cv.wait_for(lk, std::chrono::milliseconds(1));
        }
        if (stop) break;
        used->fetch_add(reserved);
      }
      std::vector<uint64_t> offs(batch.size() + 1, 0);
      for (size_t i = 0; i < batch.size(); ++i) offs[i + 1] = offs[i] + batch[i]->n;
      std::vector<lod_tree*> trees;
      lod_status st = LOD_OK;
      char err[256] = "";
      try {
        const size_t bytes = offs.back() * sizeof(lod_point);
        if (bytes > dcap) {
          lodint::cache().release(dev, dbuf);
          dbuf = nullptr;
          dcap = 0;
          dbuf = lodint::cache().alloc(dev, bytes);
          dcap = bytes;
        }
        for (size_t i = 0; i < batch.size(); ++i)
          if (batch[i]->n &&
              hipMemcpyAsync((lod_point*)dbuf + offs[i], batch[i]->h, batch[i]->n * sizeof(lod_point),
                             hipMemcpyHostToDevice, s) != hipSuccess) {
            (void)hipGetLastError();
            lod_set_error("host-to-device copy of a request failed");
            throw LodError{LOD_ERR_HIP};
          }
        trees = lod_build_clouds((const lod_point*)dbuf, offs.data(), (uint32_t)batch.size(), params, s);
      } catch (const LodError& e) {
        st = e.st;
        snprintf(err, sizeof(err), "%s", lod_last_error());
      } catch (...) {
        st = LOD_ERR_OOM;
        snprintf(err, sizeof(err), "unexpected host exception");
      }
      if (st != LOD_OK && batch.size() > 1 && st != LOD_ERR_HIP) {
        // one request may be at fault: build each alone for its own status
        for (size_t i = 0; i < batch.size(); ++i) {
          lod_tree* t = nullptr;
          lod_status si = LOD_OK;
          try {
            t = lod_build_tree((const lod_point*)dbuf + offs[i], batch[i]->n, params, s);
          } catch (const LodError& e) {
            si = e.st;
          } catch (...) {
            si = LOD_ERR_OOM;
          }
          std::lock_guard<std::mutex> lk(mu);
          finish(batch[i], t, si, lod_last_error());
        }
        std::lock_guard<std::mutex> lk(mu);
        used->fetch_sub(reserved);
      } else {
        std::lock_guard<std::mutex> lk(mu);
        used->fetch_sub(reserved);
        for (size_t i = 0; i < batch.size(); ++i)
          finish(batch[i], st == LOD_OK ? trees[i] : nullptr, st, err);
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
  s->params.flags &= ~(uint32_t)LOD_FLAG_AUTOTUNE;
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
  uint64_t est = 0;
  try {
    est = s->batch_bytes(std::vector<uint64_t>{n});
  } catch (const LodError& e) {
    return e.st;
  }
  if (est > s->budget) {
    lod_set_error("request of %llu points needs %llu bytes, more than the whole budget", (unsigned long long)n,
                  (unsigned long long)est);
    return LOD_ERR_TOO_LARGE;
  }
  auto* r = new Request();
  r->h = h_points;
  r->n = n;
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
