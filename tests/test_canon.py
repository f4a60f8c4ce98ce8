"""The tree comparison used by every parity test, checked on the CPU: it
accepts a tree that differs from the oracle's only in what is free (point
order inside a leaf) and rejects planted differences."""
from __future__ import annotations

import numpy as np
import pytest

import canon
import oracle
import synth


def _as_gpu_layout(o: dict, points: np.ndarray, keep_ids: bool, seed: int = 0) -> dict:
    """The oracle's tree in the GPU's layout: leaf records instead of ids
    (ids only if kept), points shuffled inside every leaf."""
    raw = np.ascontiguousarray(points).view(np.uint8).reshape(-1, 16)
    rng = np.random.default_rng(seed)
    ids = o["point_ids"].copy()
    for i in np.nonzero(o["is_leaf"])[0]:
        a, c = int(o["offset"][i]), int(o["count"][i])
        ids[a:a + c] = rng.permutation(ids[a:a + c])
    g = dict(o)
    g["points"] = raw[ids.astype(np.int64)]
    g["point_ids"] = ids if keep_ids else None
    return g


@pytest.mark.parametrize("keep_ids", [False, True])
def test_equal_up_to_leaf_order_passes(keep_ids):
    p = synth.aerial(40_000, seed=3)
    o = oracle.build(p, leaf_cap=500, max_level=12)
    canon.compare_trees(_as_gpu_layout(o, p, keep_ids), o, p)


def test_duplicate_records_pass():
    p = synth.uniform_cloud(3000, 5)
    p[1000:1500] = p[0]
    o = oracle.build(p, leaf_cap=100, max_level=12)
    canon.compare_trees(_as_gpu_layout(o, p, False, seed=2), o, p)


@pytest.mark.parametrize("keep_ids", [False, True])
def test_point_moved_to_another_leaf_fails(keep_ids):
    p = synth.aerial(40_000, seed=3)
    o = oracle.build(p, leaf_cap=500, max_level=12)
    g = _as_gpu_layout(o, p, keep_ids)
    leaves = np.nonzero(o["is_leaf"])[0]
    a, b = int(o["offset"][leaves[3]]), int(o["offset"][leaves[7]])
    g["points"] = g["points"].copy()
    g["points"][[a, b]] = g["points"][[b, a]]
    if keep_ids:
        g["point_ids"] = g["point_ids"].copy()
        g["point_ids"][[a, b]] = g["point_ids"][[b, a]]
    with pytest.raises(AssertionError):
        canon.compare_trees(g, o, p)


def test_changed_record_fails():
    p = synth.aerial(40_000, seed=3)
    o = oracle.build(p, leaf_cap=500, max_level=12)
    g = _as_gpu_layout(o, p, False)
    g["points"] = g["points"].copy()
    g["points"][123, 13] ^= 1  # one colour bit of one record
    with pytest.raises(AssertionError):
        canon.compare_trees(g, o, p)


def test_changed_voxel_and_node_field_fail():
    p = synth.aerial(40_000, seed=3)
    o = oracle.build(p, leaf_cap=500, max_level=12)
    g = _as_gpu_layout(o, p, False)
    g["voxels"] = g["voxels"].copy()
    g["voxels"][len(g["voxels"]) // 2, 5] ^= 4
    with pytest.raises(AssertionError):
        canon.compare_trees(g, o, p)
    g = _as_gpu_layout(o, p, False)
    g["count"] = g["count"].copy()
    g["count"][0] += 1
    with pytest.raises(AssertionError):
        canon.compare_trees(g, o, p)
