"""Autotuner for the partition plan of batched builds.

What a build computes never depends on its plan, only how fast it runs.  The
plan has three knobs, all fields of lod_params:
  tune_levels0  levels sorted by the first partition pass: the resolution of
                the per-cloud root counting grid (8^E cells, one LDS
                histogram of that size per workgroup);
  tune_levels1  levels sorted by the second pass (the extended grids);
  tune_chunk    points per partition work item, i.e. per workgroup of the
                counting and insert kernels.
tune_batch() times lod_build_batch for a small set of candidate plans on a
sample of the caller's chunks (already on the device) and keeps the fastest,
cached per workload signature: chunk count, median and total chunk size
(each rounded to a power of two) and the sampling mode.  The cache lives in
memory and, if a path is given, in a JSON file.
"""
from __future__ import annotations

import json
import math
import os
import time

import numpy as np

from . import binding

# (levels0, levels1, chunk); 0 = the library's automatic choice
CANDIDATES = [(0, 0, 0)] + [(e0, e1, ch) for e0 in (2, 3, 4) for e1 in (2, 3, 4) if 5 <= e0 + e1 <= 8
                            for ch in (14336, 64512)]

_memo: dict = {}


def signature(offsets, sampling: int) -> str:
    """Workload class of a batch: chunk count, median and total size (powers of two), mode."""
    sizes = np.diff(np.asarray(offsets, np.int64))
    sizes = sizes[sizes > 0]
    if len(sizes) == 0:
        return f"empty/s{sampling}"
    p2 = lambda v: int(round(math.log2(max(float(v), 1.0))))
    return f"k{p2(len(sizes))}/m{p2(np.median(sizes))}/t{p2(sizes.sum())}/s{sampling}"


def _load(path):
    if path and os.path.exists(path):
        try:
            with open(path) as f:
                return json.load(f)
        except (OSError, ValueError):
            return {}
    return {}


def _params(base: binding.lod_params, plan) -> binding.lod_params:
    p = binding.lod_params()
    for name, _ in binding.lod_params._fields_:
        setattr(p, name, getattr(base, name))
    p.tune_levels0, p.tune_levels1, p.tune_chunk = plan
    return p


def time_plan(points, offsets, params, reps: int = 2, stream=None) -> float:
    """Median seconds of lod_build_batch (trees freed) after one warm-up."""
    import torch

    def once():
        for t in binding.lod_build_batch(points, offsets, params=params, stream=stream):
            t.free()

    once()
    times = []
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        once()
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    return float(np.median(times))


def tune_batch(points, offsets, base: binding.lod_params, sample_chunks: int = 64, reps: int = 2,
               cache_path: str | None = None, stream=None):
    """Best plan for batches like (points, offsets); returns (lod_params, info).

    points: device tensor of all chunks, offsets: host offsets (chunks + 1).
    The candidates run on the first `sample_chunks` chunks."""
    sig = signature(offsets, base.sampling)
    cache = _load(cache_path)
    cache.update(_memo)
    if sig in cache:
        plan = tuple(cache[sig]["plan"])
        return _params(base, plan), {"signature": sig, "plan": list(plan), "cached": True}
    offs = np.asarray(offsets, np.int64)
    k = min(sample_chunks, len(offs) - 1)
    sub = offs[:k + 1] - offs[0]
    sample = points[int(offs[0]) * 16:int(offs[k]) * 16]
    results = []
    for plan in CANDIDATES:
        results.append((time_plan(sample, sub, _params(base, plan), reps, stream), plan))
    results.sort()
    best_t, best = results[0]
    default_t = next(t for t, p in results if p == (0, 0, 0))
    entry = {"plan": list(best), "sample_s": best_t, "default_sample_s": default_t}
    _memo[sig] = entry
    if cache_path:
        cache[sig] = entry
        os.makedirs(os.path.dirname(os.path.abspath(cache_path)), exist_ok=True)
        with open(cache_path, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
    return _params(base, best), {"signature": sig, "plan": list(best), "cached": False,
                                 "sample_chunks": k, "sample_s": round(best_t, 6),
                                 "default_sample_s": round(default_t, 6), "candidates": len(CANDIDATES)}
