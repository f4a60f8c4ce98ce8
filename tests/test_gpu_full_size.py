"""GPU parity at the benchmark's full size: the 100M-point aerial plain build
(T = 50 000, 128^3, colour-filtered), built exactly as bench.py builds it.

The oracle cannot rebuild 100M points in seconds, so the check has two parts:
  * properties that hold at any size, checked on every point and node:
    bounding box, node-table invariants, every output point inside the leaf
    whose prefix it carries, output points a permutation of the input;
  * sampled subtrees: below a node, the octree and its voxels depend only on
    the node's own points, so the oracle rebuilds a few nodes' subtrees from
    those points alone (in the global cube) and the subtrees are compared
    bit for bit."""
from __future__ import annotations

import time

import numpy as np
import pytest

import canon
import oracle
import synth

pytestmark = pytest.mark.gpu

N = 100_000_000
T = 50_000
ML = 12


def log(msg):
    print(f"[full-size] {time.strftime('%H:%M:%S')} {msg}", flush=True)


def multiset_hash(rows: np.ndarray) -> tuple:
    """Order-independent digest of 16-byte records: sum and xor of a mixed
    64-bit value per record (two independent aggregations)."""
    w = np.ascontiguousarray(rows).view(np.uint64).reshape(-1, 2)
    with np.errstate(over="ignore"):
        h = (w[:, 0] * np.uint64(0x9E3779B97F4A7C15)) ^ (w[:, 1] + np.uint64(0xD1B54A32D192ED03))
        h ^= h >> np.uint64(29)
        h *= np.uint64(0xBF58476D1CE4E5B9)
        h ^= h >> np.uint64(32)
        return int(h.sum(dtype=np.uint64)), int(np.bitwise_xor.reduce(h))


def test_aerial_100m_bench_configuration():
    import torch

    import paper_2302_14801_amd as lod

    log("generating")
    host = torch.empty(N * 16, dtype=torch.uint8, pin_memory=True)
    pts = host.numpy().view(synth.POINT_DTYPE)
    synth.aerial(N, seed=2, out=pts)
    dev = host.to("cuda:0")
    log("building on the GPU")
    params = lod.make_params(leaf_cap=T, max_level=ML, timing=True)
    t = lod.lod_build(dev, params=params)
    g = t.to_host()
    t.free()
    del dev
    log(f"{g['num_nodes']} nodes, {g['num_voxels']} voxels")

    # bounding cube
    lo = np.array([pts["x"].min(), pts["y"].min(), pts["z"].min()], np.float32)
    hi = np.array([pts["x"].max(), pts["y"].max(), pts["z"].max()], np.float32)
    assert np.array_equal(g["aabb_min"], lo) and np.array_equal(g["aabb_max"], hi)
    side = max(float(hi[a]) - float(lo[a]) for a in range(3))
    assert g["side"] == side

    # node table invariants
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

    # every output point lies in the leaf whose prefix it carries; output = permutation of input
    gk = oracle.keys_in_cube(g["points"], lo, side)
    leaves = np.nonzero(leaf)[0]
    cnt = g["count"][leaves].astype(np.int64)
    off = g["offset"][leaves].astype(np.int64)
    assert np.array_equal(np.sort(off), np.concatenate([[0], np.cumsum(cnt[np.argsort(off)])[:-1]]))
    owner_level = np.zeros(N, np.uint64)
    owner_key = np.zeros(N, np.uint64)
    for o_, c_, l_, k_ in zip(off, cnt, lv[leaves], key[leaves]):
        owner_level[o_:o_ + c_] = l_
        owner_key[o_:o_ + c_] = k_
    shift = np.uint64(3) * (np.uint64(21) - owner_level)
    assert np.array_equal(gk >> shift, owner_key)
    del gk, owner_level, owner_key, shift
    assert multiset_hash(g["points"]) == multiset_hash(pts.view(np.uint8).reshape(-1, 16))
    log("leaf membership and permutation ok")

    # sampled subtrees against the oracle
    ik = oracle.keys_in_cube(pts, lo, side)
    cand = [i for i in inner if 150_000 <= npt[i] <= 2_500_000]
    rng = np.random.default_rng(7)
    picks = sorted(set(rng.choice(cand, size=min(4, len(cand)), replace=False).tolist()))
    deep = [i for i in range(g["num_nodes"]) if lv[i] == lv.max() - 1 and not leaf[i]]
    if deep:
        picks.append(int(deep[len(deep) // 2]))
    assert picks
    for x in picks:
        L, kx = int(lv[x]), int(key[x])
        sel = np.nonzero((ik >> np.uint64(3 * (21 - L))) == np.uint64(kx))[0]
        assert len(sel) == npt[x]
        sub = np.ascontiguousarray(pts[sel])
        o = oracle.build(sub, leaf_cap=T, max_level=ML, cube_lo=lo, cube_side=side)
        ox = int(np.nonzero((o["level"] == L) & (o["key"] == np.uint64(kx)))[0][0])
        gi, oi = canon.subtree_indices(g, x), canon.subtree_indices(o, ox)
        assert len(gi) == len(oi)
        for f in canon.NODE_FIELDS[:5] + ("count",):
            assert np.array_equal(g[f][gi], o[f][oi]), f
        for a, b in zip(gi, oi):
            ga, gc = int(g["offset"][a]), int(g["count"][a])
            ob, oc = int(o["offset"][b]), int(o["count"][b])
            if g["is_leaf"][a]:
                ids = sel[o["point_ids"][ob:ob + oc]]
                assert np.array_equal(canon.rows_sorted(g["points"][ga:ga + gc]),
                                      canon.rows_sorted(pts.view(np.uint8).reshape(-1, 16)[ids]))
            else:
                assert np.array_equal(g["voxels"][ga:ga + gc], o["voxels"][ob:ob + oc]), f"voxels of node {a}"
        log(f"subtree at level {L} with {npt[x]} points ({len(gi)} nodes) matches the oracle")
