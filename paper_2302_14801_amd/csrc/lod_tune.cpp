// lod_tune.cpp -- the plan autotuner of batched builds (lod_tune_batch,
// LOD_FLAG_AUTOTUNE).
//
// A build's plan -- levels sorted by the first and the second partition pass
// (the resolutions of the root and the extended counting grids, 8^E cells
// each) and points per partition work item -- decides only how the work is
// cut, never what is computed.  The tuner times lod_build_batch with a small
// set of candidate plans on a sample of the caller's chunks (already on the
// device), keeps the fastest, and caches it for the process per workload
// class: chunk count, median and total chunk size (each rounded to a power of
// two), sampling mode and the flags that change the work (ids, full
// precision).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "internal.h"

namespace {

struct Plan3 {
  uint32_t l0, l1, chunk;
};

// (0, 0, 0) is the library's automatic choice.
std::vector<Plan3> candidates() {
  std::vector<Plan3> c{{0, 0, 0}};
  for (uint32_t e0 = 2; e0 <= 4; ++e0)
    for (uint32_t e1 = 2; e1 <= 4; ++e1)
      if (e0 + e1 >= 5)
        for (uint32_t ch : {14336u, 64512u}) c.push_back({e0, e1, ch});
  return c;
}

struct Entry {
  Plan3 plan;
  float best_ms, default_ms;
  uint32_t sample_chunks;
};

std::mutex g_mu;
std::map<std::string, Entry>& cache() {
  static auto* m = new std::map<std::string, Entry>();
  return *m;
}

int log2_round(double v) { return (int)std::lround(std::log2(std::max(v, 1.0))); }

std::string signature(const uint64_t* offs, uint32_t n, const lod_params& p) {
  std::vector<uint64_t> sizes;
  uint64_t total = 0;
  for (uint32_t i = 0; i < n; ++i)
    if (offs[i + 1] > offs[i]) {
      sizes.push_back(offs[i + 1] - offs[i]);
      total += offs[i + 1] - offs[i];
    }
  char buf[160];
  if (sizes.empty()) {
    snprintf(buf, sizeof(buf), "empty/s%u", p.sampling);
    return buf;
  }
  std::nth_element(sizes.begin(), sizes.begin() + sizes.size() / 2, sizes.end());
  const uint32_t work_flags = p.flags & (LOD_FLAG_POINT_IDS | LOD_FLAG_FULL_PRECISION);
  snprintf(buf, sizeof(buf), "k%d/m%d/t%d/s%u/f%u/T%u/L%u", log2_round((double)sizes.size()),
           log2_round((double)sizes[sizes.size() / 2]), log2_round((double)total), p.sampling, work_flags, p.leaf_cap,
           p.max_level);
  return buf;
}

// Milliseconds of one batch build of the sample (trees freed), median of
// `reps` after one warm-up.
float time_plan(const lod_point* d_points, const uint64_t* offs, uint32_t k, const lod_params& p, hipStream_t s,
                int reps) {
  std::vector<lod_tree*> trees(k);
  std::vector<float> t;
  for (int r = 0; r <= reps; ++r) {
    const auto t0 = std::chrono::steady_clock::now();
    std::vector<lod_tree*> out = lod_build_clouds(d_points, offs, k, p, s);
    const auto t1 = std::chrono::steady_clock::now();
    for (lod_tree* x : out) lod_tree_free(x);
    if (r) t.push_back(std::chrono::duration<float, std::milli>(t1 - t0).count());
  }
  std::sort(t.begin(), t.end());
  return t[t.size() / 2];
}

}  // namespace

// The tuned copy of p for batches like (offs, n); info may be NULL.
lod_params tune_batch(const lod_point* d_points, const uint64_t* offs, uint32_t n, const lod_params& p,
                      hipStream_t s, lod_tune_info* info) {
  lod_params out = p;
  out.flags &= ~(uint32_t)LOD_FLAG_AUTOTUNE;
  if (info) *info = lod_tune_info{};
  if (p.tune_levels0 || p.tune_levels1 || p.tune_chunk || n == 0) return out;  // an explicit plan is kept
  const std::string sig = signature(offs, n, p);
  {
    std::lock_guard<std::mutex> g(g_mu);
    auto it = cache().find(sig);
    if (it != cache().end()) {
      const Entry& e = it->second;
      out.tune_levels0 = e.plan.l0;
      out.tune_levels1 = e.plan.l1;
      out.tune_chunk = e.plan.chunk;
      if (info) *info = lod_tune_info{1u, e.sample_chunks, e.plan.l0, e.plan.l1, e.plan.chunk, e.best_ms, e.default_ms};
      return out;
    }
  }
  const uint32_t k = std::min<uint32_t>(64, n);
  lod_params q = out;
  q.flags &= ~(uint32_t)LOD_FLAG_TIMING;
  Entry best{{0, 0, 0}, 0.f, 0.f, k};
  bool first = true;
  for (const Plan3& c : candidates()) {
    q.tune_levels0 = c.l0;
    q.tune_levels1 = c.l1;
    q.tune_chunk = c.chunk;
    const float ms = time_plan(d_points, offs, k, q, s, 2);
    if (c.l0 == 0 && c.l1 == 0 && c.chunk == 0) best.default_ms = ms;
    if (first || ms < best.best_ms) {
      best.plan = c;
      best.best_ms = ms;
      first = false;
    }
  }
  {
    std::lock_guard<std::mutex> g(g_mu);
    cache()[sig] = best;
  }
  out.tune_levels0 = best.plan.l0;
  out.tune_levels1 = best.plan.l1;
  out.tune_chunk = best.plan.chunk;
  if (info) *info = lod_tune_info{0u, k, best.plan.l0, best.plan.l1, best.plan.chunk, best.best_ms, best.default_ms};
  return out;
}
