"""Comparison of a GPU tree (binding ``Tree.to_host()``) with the oracle's.

What is unique is compared exactly: the node table (both sides list nodes in
ascending (level, key) order with children consecutive), per-leaf point
multisets, and per-node voxel lists (both sides list voxels in Morton order).
What is free -- the order of points inside a leaf -- is compared as a sorted
multiset."""
from __future__ import annotations

import numpy as np

NODE_FIELDS = ("level", "key", "is_leaf", "npoints", "child_mask", "first_child", "count")


def rows_sorted(rows: np.ndarray) -> np.ndarray:
    """Sort 16-byte records lexicographically (as two little-endian u64 words)."""
    r = np.ascontiguousarray(rows).view(np.uint64).reshape(-1, 2)
    order = np.lexsort((r[:, 0], r[:, 1]))
    return r[order]


def compare_trees(g: dict, o: dict, points: np.ndarray, ids: bool = None):
    raw = np.ascontiguousarray(points).view(np.uint8).reshape(-1, 16)
    assert g["num_nodes"] == o["num_nodes"], (g["num_nodes"], o["num_nodes"])
    assert g["num_points"] == o["num_points"]
    for f in NODE_FIELDS:
        if not np.array_equal(g[f], o[f]):
            bad = np.nonzero(g[f] != o[f])[0][:10]
            raise AssertionError(f"node field {f} differs at {bad.tolist()}: gpu {g[f][bad].tolist()} "
                                 f"oracle {o[f][bad].tolist()}")
    if g["num_nodes"]:
        assert np.all(g["aabb_min"] == o["aabb_min"]) and np.all(g["aabb_max"] == o["aabb_max"])
        assert g["side"] == o["side"]
    assert g["num_voxels"] == o["num_voxels"], (g["num_voxels"], o["num_voxels"])
    for i in np.nonzero(g["is_leaf"])[0]:
        go, gc = int(g["offset"][i]), int(g["count"][i])
        oo, oc = int(o["offset"][i]), int(o["count"][i])
        assert gc == oc
        oid = o["point_ids"][oo:oo + oc]
        if g.get("point_ids") is not None:
            gid = g["point_ids"][go:go + gc]
            assert np.array_equal(np.sort(gid), np.sort(oid)), f"leaf {i} ids differ"
            assert np.array_equal(g["points"][go:go + gc], raw[gid]), f"leaf {i} records do not match ids"
        else:
            assert np.array_equal(rows_sorted(g["points"][go:go + gc]), rows_sorted(raw[oid])), \
                f"leaf {i} point multiset differs"
    for i in np.nonzero(g["is_leaf"] == 0)[0]:
        go, gc = int(g["offset"][i]), int(g["count"][i])
        oo, oc = int(o["offset"][i]), int(o["count"][i])
        gv, ov = g["voxels"][go:go + gc], o["voxels"][oo:oo + oc]
        if not np.array_equal(gv, ov):
            bad = np.nonzero(np.any(gv != ov, axis=1))[0][:5]
            raise AssertionError(f"voxels of node {i} (level {g['level'][i]}) differ at {bad.tolist()}: "
                                 f"gpu {gv[bad].tolist()} oracle {ov[bad].tolist()}")
        if o.get("voxel_ids") is not None:
            assert g.get("voxel_ids") is not None
            assert np.array_equal(g["voxel_ids"][go:go + gc], o["voxel_ids"][oo:oo + oc]), f"voxel ids of {i}"


def subtree_indices(t: dict, root: int) -> list:
    """Indices of the nodes of the subtree rooted at `root`, level by level."""
    out, frontier = [root], [root]
    while frontier:
        nxt = []
        for i in frontier:
            if not t["is_leaf"][i]:
                fc = int(t["first_child"][i])
                nxt.extend(range(fc, fc + bin(int(t["child_mask"][i])).count("1")))
        out.extend(nxt)
        frontier = nxt
    return out
