"""Comparison of a GPU tree (binding ``Tree.to_host()``) with the oracle's.

What is unique is compared exactly: the node table (both sides list nodes in
ascending (level, key) order with children consecutive), per-leaf point
multisets, and per-node voxel lists (both sides list voxels in Morton order).
What is free -- the order of points inside a leaf -- is compared as a
multiset: both sides are put in one canonical order (by leaf, then by a hash
of the record or by the id) and then compared record for record, so a pass
means the multisets are equal.  Vectorised, so whole trees of 10^8 points
compare in seconds."""
from __future__ import annotations

import numpy as np

NODE_FIELDS = ("level", "key", "is_leaf", "npoints", "child_mask", "first_child", "count")


def rows_sorted(rows: np.ndarray) -> np.ndarray:
    """Sort 16-byte records lexicographically (as two little-endian u64 words)."""
    r = np.ascontiguousarray(rows).view(np.uint64).reshape(-1, 2)
    order = np.lexsort((r[:, 0], r[:, 1]))
    return r[order]


def _mix(w: np.ndarray) -> np.ndarray:
    """64-bit hash of 16-byte records given as (n, 2) u64 words."""
    with np.errstate(over="ignore"):
        h = (w[:, 0] * np.uint64(0x9E3779B97F4A7C15)) ^ (w[:, 1] + np.uint64(0xD1B54A32D192ED03))
        h ^= h >> np.uint64(31)
        h *= np.uint64(0xBF58476D1CE4E5B9)
        h ^= h >> np.uint64(29)
        h *= np.uint64(0x94D049BB133111EB)
        h ^= h >> np.uint64(32)
    return h


def _leaf_owner(t: dict, leaves: np.ndarray) -> tuple:
    """For the points of `leaves` (node indices, in node order): the positions
    in t's point arrays and the rank of the owning leaf, leaf by leaf."""
    off = t["offset"][leaves].astype(np.int64)
    cnt = t["count"][leaves].astype(np.int64)
    total = int(cnt.sum())
    rank = np.repeat(np.arange(len(leaves), dtype=np.uint64), cnt)
    start = np.repeat(off - np.concatenate([[0], np.cumsum(cnt)[:-1]]), cnt)
    pos = np.arange(total, dtype=np.int64) + start
    return pos, rank


def _canonical(rank: np.ndarray, sub: np.ndarray, nleaves: int) -> np.ndarray:
    """Order putting points by leaf rank, then by `sub` (u64) inside a leaf."""
    bits = max(1, int(nleaves - 1).bit_length())
    key = (rank << np.uint64(64 - bits)) | (sub >> np.uint64(bits))
    return np.argsort(key, kind="stable")


def compare_leaves(g: dict, o: dict, raw: np.ndarray):
    """Every leaf holds the same multiset of input records on both sides (and
    the same ids where the GPU kept them)."""
    leaves = np.nonzero(g["is_leaf"])[0]
    if len(leaves) == 0:
        return
    gpos, grank = _leaf_owner(g, leaves)
    opos, orank = _leaf_owner(o, leaves)
    assert np.array_equal(grank, orank)
    oid = o["point_ids"][opos].astype(np.int64)
    if g.get("point_ids") is not None:
        gid = g["point_ids"][gpos].astype(np.uint64)
        og = _canonical(grank, gid << np.uint64(32), len(leaves))
        oo = _canonical(orank, oid.astype(np.uint64) << np.uint64(32), len(leaves))
        if not np.array_equal(gid[og], oid[oo].astype(np.uint64)):
            bad = np.nonzero(gid[og] != oid[oo].astype(np.uint64))[0][:5]
            raise AssertionError(f"leaf point ids differ at sorted positions {bad.tolist()} "
                                 f"(leaves {leaves[grank[og][bad].astype(np.int64)].tolist()})")
        grec = g["points"][gpos]
        if not np.array_equal(grec, raw[g["point_ids"][gpos].astype(np.int64)]):
            raise AssertionError("leaf records do not match their ids")
        return
    gw = np.ascontiguousarray(g["points"][gpos]).view(np.uint64).reshape(-1, 2)
    ow = np.ascontiguousarray(raw[oid]).view(np.uint64).reshape(-1, 2)
    og = _canonical(grank, _mix(gw), len(leaves))
    oo = _canonical(orank, _mix(ow), len(leaves))
    differ = np.nonzero(np.any(gw[og] != ow[oo], axis=1))[0]
    # two different records of one leaf whose truncated hashes tie may sit in
    # either order: those leaves are compared again by a full sort
    for r in np.unique(grank[og][differ]).tolist():
        i = int(leaves[r])
        go, gc = int(g["offset"][i]), int(g["count"][i])
        ids = o["point_ids"][int(o["offset"][i]):int(o["offset"][i]) + int(o["count"][i])]
        if not np.array_equal(rows_sorted(g["points"][go:go + gc]), rows_sorted(raw[ids])):
            raise AssertionError(f"leaf {i} point multiset differs")


def compare_voxels(g: dict, o: dict):
    inner = np.nonzero(g["is_leaf"] == 0)[0]
    assert g["num_voxels"] == o["num_voxels"], (g["num_voxels"], o["num_voxels"])
    same_layout = np.array_equal(g["offset"][inner], o["offset"][inner])
    if same_layout and np.array_equal(g["voxels"], o["voxels"]):
        if o.get("voxel_ids") is not None:
            assert g.get("voxel_ids") is not None
            if not np.array_equal(g["voxel_ids"], o["voxel_ids"]):
                bad = np.nonzero(g["voxel_ids"] != o["voxel_ids"])[0][:5]
                raise AssertionError(f"voxel ids differ at {bad.tolist()}")
        return
    for i in inner:
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
    compare_voxels(g, o)
    compare_leaves(g, o, raw)


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
