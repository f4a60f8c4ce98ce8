"""Plan autotuner of batched builds: a thin wrapper of the library's
lod_tune_batch (the tuning itself -- candidate plans timed on a sample of the
chunks, a per-process cache by workload class -- runs in liblod.so, so C
callers reach it too, also through LOD_FLAG_AUTOTUNE).

A plan (the tune_* fields of lod_params: levels of the two partition passes
and points per partition work item) changes only how the work is cut, never
the result."""
from __future__ import annotations

from . import binding


def tune_batch(points, offsets, base: binding.lod_params, stream=None):
    """Best plan for batches like (points, offsets): (lod_params, info)."""
    tuned, info = binding.lod_tune_batch(points, offsets, base, stream=stream)
    info = dict(info)
    info["plan"] = [info.pop("levels0"), info.pop("levels1"), info.pop("chunk")]
    return tuned, info
