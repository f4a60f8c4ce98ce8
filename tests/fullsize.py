"""Parity checks for builds too large for the oracle to rebuild whole.

Two parts:
  * properties that hold at any size, checked on every point and node:
    bounding box, node-table invariants, every output point inside the leaf
    whose prefix it carries, output points a permutation of the input;
  * sampled subtrees: below a node, the octree and its voxels depend only on
    the node's own points, so the oracle rebuilds a few nodes' subtrees from
    those points alone (selected from the input by their keys in the global
    cube) and the subtrees are compared bit for bit."""
from __future__ import annotations

import os
import time

import numpy as np

import canon
import oracle

CHUNK = 50_000_000  # rows per step of the whole-cloud passes (bounded host memory)


def log(msg):
    """Progress line on stdout and, if LOD_PROGRESS_FILE names a file, appended
    there too (pytest holds a test's stdout until the test ends)."""
    line = f"[full-size] {time.strftime('%H:%M:%S')} {msg}"
    print(line, flush=True)
    path = os.environ.get("LOD_PROGRESS_FILE")
    if path:
        with open(path, "a") as f:
            f.write(line + "\n")


def multiset_hash(rows: np.ndarray) -> tuple:
    """Order-independent digest of 16-byte records: sum and xor of a mixed
    64-bit value per record (two independent aggregations), in chunks."""
    s, x = np.uint64(0), np.uint64(0)
    for i in range(0, len(rows), CHUNK):
        if i and i % (10 * CHUNK) == 0:
            log(f"  hashed {i} records")
        w = np.ascontiguousarray(rows[i:i + CHUNK]).view(np.uint64).reshape(-1, 2)
        with np.errstate(over="ignore"):
            h = (w[:, 0] * np.uint64(0x9E3779B97F4A7C15)) ^ (w[:, 1] + np.uint64(0xD1B54A32D192ED03))
            h ^= h >> np.uint64(29)
            h *= np.uint64(0xBF58476D1CE4E5B9)
            h ^= h >> np.uint64(32)
            s = s + h.sum(dtype=np.uint64)
            x ^= np.bitwise_xor.reduce(h)
    return int(s), int(x)


def check_build(g: dict, pts: np.ndarray, T: int, ML: int, subtree_picks: int = 4, seed: int = 7,
                leaf_sample: int | None = None, sampling: int = 0):
    """g: the GPU tree copied to the host; pts: the input records; sampling:
    the mode of the build (the subtrees are rebuilt with it)."""
    N = len(pts)
    lo = np.array([pts["x"].min(), pts["y"].min(), pts["z"].min()], np.float32)
    hi = np.array([pts["x"].max(), pts["y"].max(), pts["z"].max()], np.float32)
    assert np.array_equal(g["aabb_min"], lo) and np.array_equal(g["aabb_max"], hi)
    side = max(float(hi[a]) - float(lo[a]) for a in range(3))
    assert g["side"] == side
    log("bounding box ok")

    lv, leaf, npt, key = g["level"], g["is_leaf"].astype(bool), g["npoints"].astype(np.int64), g["key"]
    assert lv[0] == 0 and npt[0] == N and npt[leaf].sum() == N
    assert np.all((lv[1:] > lv[:-1]) | ((lv[1:] == lv[:-1]) & (key[1:] > key[:-1])))
    assert np.all(lv[leaf & (npt > T)] == ML)
    assert np.all(npt[~leaf] > T)
    inner = np.nonzero(~leaf)[0]
    nch = np.array([bin(int(m)).count("1") for m in g["child_mask"][inner]])
    for i, k in zip(inner, nch):
        fc = int(g["first_child"][i])
        ch = np.arange(fc, fc + k)
        assert np.all(key[ch] >> np.uint64(3) == key[i]) and np.all(lv[ch] == lv[i] + 1)
        assert npt[ch].sum() == npt[i]
    log("node invariants ok")

    leaves = np.nonzero(leaf)[0]
    cnt = g["count"][leaves].astype(np.int64)
    off = g["offset"][leaves].astype(np.int64)
    order = np.argsort(off)
    assert np.array_equal(off[order], np.concatenate([[0], np.cumsum(cnt[order])[:-1]]))
    check = leaves if leaf_sample is None else np.random.default_rng(seed).choice(
        leaves, size=min(leaf_sample, len(leaves)), replace=False)
    for li in check:
        o_, c_, l_, k_ = int(g["offset"][li]), int(g["count"][li]), int(lv[li]), key[li]
        gk = oracle.keys_in_cube(g["points"][o_:o_ + c_], lo, side)
        assert np.all(gk >> np.uint64(3 * (21 - l_)) == k_), f"leaf {li}"
    log(f"leaf membership ok ({len(check)} leaves)")
    assert multiset_hash(g["points"]) == multiset_hash(pts.view(np.uint8).reshape(-1, 16))
    log("output points are a permutation of the input")

    cand = [i for i in inner if 150_000 <= npt[i] <= 2_500_000]
    rng = np.random.default_rng(seed)
    picks = sorted(set(rng.choice(cand, size=min(subtree_picks, len(cand)), replace=False).tolist())) if cand else []
    deep = [i for i in range(g["num_nodes"]) if lv[i] == lv.max() - 1 and not leaf[i]]
    if deep:
        picks.append(int(deep[len(deep) // 2]))
    assert picks
    # each picked node's points, selected from the input by key prefix
    want = {x: (int(lv[x]), np.uint64(int(key[x]))) for x in picks}
    sel = {x: [] for x in picks}
    for i in range(0, N, CHUNK):
        if i and i % (10 * CHUNK) == 0:
            log(f"  keyed {i} input points")
        ik = oracle.keys_in_cube(pts[i:i + CHUNK], lo, side)
        for x, (L, kx) in want.items():
            sel[x].append(np.nonzero((ik >> np.uint64(3 * (21 - L))) == kx)[0] + i)
    for x in picks:
        L, kx = want[x]
        s = np.concatenate(sel[x])
        assert len(s) == npt[x]
        sub = np.ascontiguousarray(pts[s])
        o = oracle.build(sub, leaf_cap=T, max_level=ML, sampling=sampling, cube_lo=lo, cube_side=side)
        ox = int(np.nonzero((o["level"] == L) & (o["key"] == kx))[0][0])
        gi, oi = canon.subtree_indices(g, x), canon.subtree_indices(o, ox)
        assert len(gi) == len(oi)
        for f in canon.NODE_FIELDS[:5] + ("count",):
            assert np.array_equal(g[f][gi], o[f][oi]), f
        for a, b in zip(gi, oi):
            ga, gc = int(g["offset"][a]), int(g["count"][a])
            ob, oc = int(o["offset"][b]), int(o["count"][b])
            if g["is_leaf"][a]:
                ids = s[o["point_ids"][ob:ob + oc]]
                assert np.array_equal(canon.rows_sorted(g["points"][ga:ga + gc]),
                                      canon.rows_sorted(pts.view(np.uint8).reshape(-1, 16)[ids]))
            else:
                assert np.array_equal(g["voxels"][ga:ga + gc], o["voxels"][ob:ob + oc]), f"voxels of node {a}"
        log(f"subtree at level {L} with {npt[x]} points ({len(gi)} nodes) matches the oracle")
