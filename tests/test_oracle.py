"""Pins for the CPU oracle (no GPU).  Each test checks the oracle against
something other than itself: the paper's own bottom-up merge procedure, closed
forms, invariants, a hand-worked example and published generator outputs."""
from __future__ import annotations

import json
import os
from fractions import Fraction

import numpy as np
import pytest

import brute
import oracle
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _pts(rows):
    a = np.zeros(len(rows), synth.POINT_DTYPE)
    for i, r in enumerate(rows):
        a[i] = (r[0], r[1], r[2], r[3], r[4], r[5], r[6])
    return a


# --------------------------------------------------------------- cube, keys

def test_cube_matches_numpy_min_max():
    p = synth.uniform_cloud(1000, 3, lo=(-5, 2, 100), hi=(7, 3, 101))
    lo, hi, side, scale = oracle.cube(p)
    assert np.array_equal(lo, np.array([p["x"].min(), p["y"].min(), p["z"].min()], np.float32))
    assert np.array_equal(hi, np.array([p["x"].max(), p["y"].max(), p["z"].max()], np.float32))
    assert side == max(float(hi[a]) - float(lo[a]) for a in range(3))
    assert scale == 2097152.0 / side


def test_degenerate_extent_uses_unit_side():
    p = _pts([[3.0, 3.0, 3.0, 1, 2, 3, 4]] * 5)
    _, _, side, scale = oracle.cube(p)
    assert side == 1.0 and scale == 2097152.0
    assert np.all(oracle.keys(p) == 0)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_keys_match_bitwise_interleave(seed):
    p = synth.uniform_cloud(3000, seed, lo=(-100, 0, 5), hi=(100, 50, 6))
    k = oracle.keys(p)
    q = brute.quantize(p)
    assert np.array_equal(k, brute.morton(q))
    assert np.array_equal(brute.demorton(k), q)


def test_quantization_within_one_cell_of_exact_rational():
    p = synth.uniform_cloud(400, 9, lo=(-1e3, 1e-3, 7), hi=(1e3, 2e-3, 8))
    lo, hi, side, _ = oracle.cube(p)
    q = brute.demorton(oracle.keys(p))
    for i in range(len(p)):
        for a, ax in enumerate("xyz"):
            exact = (Fraction(float(p[ax][i])) - Fraction(float(lo[a]))) * (1 << 21) / Fraction(side)
            e = min(int(exact), (1 << 21) - 1)
            assert abs(int(q[i, a]) - e) <= 1


def test_extreme_faces_and_monotonicity():
    p = synth.uniform_cloud(2000, 5, lo=(0, 0, 0), hi=(10, 10, 10))
    q = brute.demorton(oracle.keys(p))
    for a, ax in enumerate("xyz"):
        imin, imax = np.argmin(p[ax]), np.argmax(p[ax])
        assert q[imin, a] == 0
        order = np.argsort(p[ax], kind="stable")
        assert np.all(np.diff(q[order, a].astype(np.int64)) >= 0)
    # the longest axis' far face maps to the last cell
    lo, hi, side, _ = oracle.cube(p)
    a = int(np.argmax(hi.astype(np.float64) - lo.astype(np.float64)))
    assert q[np.argmax(p["xyz"[a]]), a] == (1 << 21) - 1


def test_nested_prefixes():
    p = synth.uniform_cloud(500, 11)
    k = oracle.keys(p)
    q = brute.demorton(k)
    for L in range(0, 22):
        cell = q >> np.uint32(21 - L)
        assert np.array_equal(brute.prefix(k, L), brute.morton(cell) if L else np.zeros(len(k), np.uint64))


def test_nonfinite_rejected():
    p = synth.uniform_cloud(10, 1)
    p["y"][3] = np.nan
    with pytest.raises(oracle.OracleError) as e:
        oracle.build(p)
    assert e.value.status == oracle.ERR_NONFINITE
    p["y"][3] = np.inf
    with pytest.raises(oracle.OracleError):
        oracle.build(p)


def test_invalid_params_rejected():
    p = synth.uniform_cloud(10, 1)
    for kw in ({"leaf_cap": 0}, {"max_level": 15}, {"sampling": 4}):
        with pytest.raises(oracle.OracleError) as e:
            oracle.build(p, **kw)
        assert e.value.status == oracle.ERR_INVALID


# --------------------------------------------------------------- hash

def test_splitmix_published_vectors():
    g = json.load(open(os.path.join(GOLDEN, "splitmix64_vectors.json")))
    gamma = int(g["gamma"], 16)
    outs = [int(v, 16) for v in g["outputs"]]
    for k, out in enumerate(outs):
        x = (k * gamma) & ((1 << 64) - 1)  # the output function adds one more gamma
        assert brute.splitmix64(x) == out
        seed, pid = x >> 32, x & 0xFFFFFFFF
        assert int(oracle.point_hash([pid], seed)[0]) == out >> 32


# --------------------------------------------------------------- tree

def _tree_invariants(t, n, T, max_level):
    nn = t["num_nodes"]
    if n == 0:
        assert nn == 0
        return
    lv, leaf, npts, key = t["level"], t["is_leaf"].astype(bool), t["npoints"].astype(np.int64), t["key"]
    assert lv[0] == 0 and key[0] == 0 and npts[0] == n
    order = list(zip(lv.tolist(), key.tolist()))
    assert order == sorted(order) and len(set(order)) == nn
    assert npts[leaf].sum() == n
    assert np.all(npts > 0)
    for i in range(nn):
        if leaf[i]:
            assert npts[i] <= T or lv[i] == max_level
            assert t["count"][i] == npts[i]
        else:
            assert npts[i] > T and lv[i] < max_level
            fc = int(t["first_child"][i])
            ch = [c for c in range(fc, nn) if lv[c] == lv[i] + 1 and key[c] >> np.uint64(3) == key[i]]
            assert ch == list(range(fc, fc + len(ch))) and len(ch) >= 1
            assert npts[ch].sum() == npts[i]
            mask = 0
            for c in ch:
                mask |= 1 << int(key[c] & np.uint64(7))
            assert mask == t["child_mask"][i]


def _membership(t, p):
    k = oracle.keys(p)
    seen = np.zeros(len(p), np.int64)
    for i in np.nonzero(t["is_leaf"])[0]:
        ids = t["point_ids"][t["offset"][i]:t["offset"][i] + t["count"][i]]
        seen[ids] += 1
        assert np.all(brute.prefix(k[ids], int(t["level"][i])) == t["key"][i])
    assert np.all(seen == 1)


CASES = [(n, T, ml, seed) for (n, T, ml) in [(50, 1, 2), (300, 3, 4), (800, 7, 12), (2000, 50, 12),
                                             (1500, 1, 6), (2000, 100, 3)] for seed in (0, 1)]


@pytest.mark.parametrize("n,T,ml,seed", CASES)
def test_tree_equals_paper_merge_procedure(n, T, ml, seed):
    p = synth.uniform_cloud(n, seed + 17 * n)
    t = oracle.build(p, leaf_cap=T, max_level=ml)
    _tree_invariants(t, n, T, ml)
    _membership(t, p)
    assert brute.tree_nodes(t) == brute.paper_merge_tree(oracle.keys(p), T, ml)


def test_tree_on_clustered_input_matches_merge_procedure():
    # "teapot in a stadium": a dense cluster inside a sparse cloud
    a = synth.uniform_cloud(400, 1, lo=(0, 0, 0), hi=(100, 100, 100))
    b = synth.uniform_cloud(1600, 2, lo=(40, 40, 40), hi=(40.01, 40.01, 40.01))
    p = np.concatenate([a, b])
    t = oracle.build(p, leaf_cap=20, max_level=14)
    _tree_invariants(t, len(p), 20, 14)
    assert t["level"].max() >= 12
    assert brute.tree_nodes(t) == brute.paper_merge_tree(oracle.keys(p), 20, 14)


def test_small_input_is_one_root_leaf():
    p = synth.uniform_cloud(50, 4)
    t = oracle.build(p, leaf_cap=50)
    assert t["num_nodes"] == 1 and t["is_leaf"][0] == 1 and t["num_voxels"] == 0
    assert sorted(t["point_ids"].tolist()) == list(range(50))


def test_empty_input():
    t = oracle.build(np.zeros(0, synth.POINT_DTYPE))
    assert t["num_nodes"] == 0 and t["num_points"] == 0 and t["num_voxels"] == 0


@pytest.mark.parametrize("k", [1, 2, 3])
def test_lattice_gives_complete_octree(k):
    s = 2 ** k
    g = (np.arange(s, dtype=np.float32) + 0.5)
    xs, ys, zs = np.meshgrid(g, g, g, indexing="ij")
    p = np.zeros(s ** 3, synth.POINT_DTYPE)
    p["x"], p["y"], p["z"] = xs.ravel(), ys.ravel(), zs.ravel()
    p["r"] = np.arange(s ** 3) % 256
    t = oracle.build(p, leaf_cap=1, max_level=12)
    for L in range(k + 1):
        assert np.sum(t["level"] == L) == 8 ** L
    assert np.all(t["is_leaf"][t["level"] == k]) and not np.any(t["is_leaf"][t["level"] < k])


def test_identical_points_give_chain_to_depth_limit():
    p = _pts([[1.0, 2.0, 3.0, 9, 9, 9, 9]] * 10 + [[5.0, 2.0, 3.0, 1, 1, 1, 1]])
    t = oracle.build(p, leaf_cap=3, max_level=9)
    deep = t["level"] == 9
    assert np.sum(deep & (t["is_leaf"] == 1)) == 1 and t["npoints"][deep & (t["is_leaf"] == 1)][0] == 10
    for L in range(1, 9):
        inner = (t["level"] == L) & (t["is_leaf"] == 0)
        assert np.sum(inner) == 1  # one single-child inner node per level


# --------------------------------------------------------------- voxels

def test_hand_worked_example():
    g = json.load(open(os.path.join(GOLDEN, "tiny_hand_worked.json")))
    p = _pts(g["points"])
    T, ml = g["params"]["leaf_cap"], g["params"]["max_level"]
    for sampling, field in ((oracle.AVERAGE, "average_voxels"), (oracle.FIRST, "first_voxels")):
        t = oracle.build(p, leaf_cap=T, max_level=ml, sampling=sampling)
        got = [{"level": int(t["level"][i]), "key": int(t["key"][i]), "leaf": bool(t["is_leaf"][i]),
                "npoints": int(t["npoints"][i]), "child_mask": int(t["child_mask"][i])} for i in range(t["num_nodes"])]
        assert got == g["nodes"]
        for i in range(t["num_nodes"]):
            name = f"{t['level'][i]}:{t['key'][i]}"
            if t["is_leaf"][i]:
                ids = sorted(t["point_ids"][t["offset"][i]:t["offset"][i] + t["count"][i]].tolist())
                assert ids == g["leaf_ids"][name]
            else:
                v = t["voxels"][t["offset"][i]:t["offset"][i] + t["count"][i]].astype(int)
                rows = [[r[0], r[1], r[2], r[4], r[5], r[6], r[7]] for r in v]
                if sampling == oracle.FIRST:
                    ids = t["voxel_ids"][t["offset"][i]:t["offset"][i] + t["count"][i]].tolist()
                    rows = [r + [d] for r, d in zip(rows, ids)]
                assert sorted(rows) == sorted(g[field][name])


VOX_CASES = [(600, 5, 12, 0), (1500, 40, 12, 1), (3000, 200, 6, 2), (1200, 1, 5, 3)]


@pytest.mark.parametrize("n,T,ml,seed", VOX_CASES)
def test_voxel_positions_are_occupied_cells(n, T, ml, seed):
    p = synth.uniform_cloud(n, seed)
    t = oracle.build(p, leaf_cap=T, max_level=ml)
    k = oracle.keys(p)
    q = brute.demorton(k)
    for i in np.nonzero(t["is_leaf"] == 0)[0]:
        got = set(brute.tree_voxels(t, i).keys())
        assert got == brute.closed_form_cells(q, k, int(t["level"][i]), int(t["key"][i]))


@pytest.mark.parametrize("n,T,ml,seed", VOX_CASES)
def test_average_matches_recursion_and_leaf_closed_form(n, T, ml, seed):
    p = synth.uniform_cloud(n, seed)
    t = oracle.build(p, leaf_cap=T, max_level=ml)
    k = oracle.keys(p)
    q = brute.demorton(k)
    nodes = brute.tree_nodes(t)
    rec = brute.recursive_voxels(p, q, k, nodes, T, ml)
    checked_closed = 0
    for i in np.nonzero(t["is_leaf"] == 0)[0]:
        L, key = int(t["level"][i]), int(t["key"][i])
        got = brute.tree_voxels(t, i)
        assert got == rec[(L, key)]
        fc = int(t["first_child"][i])
        kids = [c for c in range(fc, t["num_nodes"]) if t["level"][c] == L + 1 and int(t["key"][c]) >> 3 == key]
        if all(t["is_leaf"][c] for c in kids):
            cf = brute.closed_form_leaf_means(p, q, k, L, key)
            assert {c: v[:3] for c, v in got.items()} == cf
            checked_closed += 1
    assert checked_closed > 0


@pytest.mark.parametrize("sampling", [oracle.FIRST, oracle.RANDOM])
@pytest.mark.parametrize("n,T,ml,seed", VOX_CASES[:3])
def test_pick_equals_argmin_argmax_over_subtree(sampling, n, T, ml, seed):
    p = synth.uniform_cloud(n, seed)
    t = oracle.build(p, leaf_cap=T, max_level=ml, sampling=sampling, seed=1234 + seed)
    k = oracle.keys(p)
    q = brute.demorton(k)
    for i in np.nonzero(t["is_leaf"] == 0)[0]:
        got = brute.tree_voxels(t, i)
        cf = brute.closed_form_pick(p, q, k, int(t["level"][i]), int(t["key"][i]), sampling, 1234 + seed)
        assert {c: v[4] for c, v in got.items()} == cf
        for c, v in got.items():
            pid = v[4]
            assert v[:4] == (int(p["r"][pid]), int(p["g"][pid]), int(p["b"][pid]), int(p["a"][pid]))


@pytest.mark.parametrize("sampling", [oracle.AVERAGE, oracle.FIRST, oracle.RANDOM])
@pytest.mark.parametrize("n,T,ml,seed", VOX_CASES[:3])
def test_full_precision_records_hold_the_accepted_sample(sampling, n, T, ml, seed):
    """Sec. 7: a full-precision record is an input point of the voxel's cell --
    the pick of the pick modes, the smallest-index point under the node in
    the cell for the average -- with the voxel's colour."""
    p = synth.uniform_cloud(n, seed)
    raw = p.view(np.uint8).reshape(-1, 16)
    t = oracle.build(p, leaf_cap=T, max_level=ml, sampling=sampling, seed=99, full_precision=True)
    k = oracle.keys(p)
    q = brute.demorton(k)
    rec = t["voxel_points"]
    assert rec.shape == (t["num_voxels"], 16) and len(t["voxel_ids"]) == t["num_voxels"]
    for i in np.nonzero(t["is_leaf"] == 0)[0]:
        L, key = int(t["level"][i]), int(t["key"][i])
        off, cnt = int(t["offset"][i]), int(t["count"][i])
        want = brute.closed_form_pick(p, q, k, L, key, oracle.FIRST if sampling == oracle.AVERAGE else sampling, 99)
        for j in range(off, off + cnt):
            v = t["voxels"][j]
            pid = int(t["voxel_ids"][j])
            assert want[(int(v[0]), int(v[1]), int(v[2]))] == pid
            # the accepted point lies in the voxel's cell and keeps its coordinates
            assert tuple(brute._point_cell(q[pid:pid + 1], L)[0].tolist()) == (int(v[0]), int(v[1]), int(v[2]))
            assert np.array_equal(rec[j, :12], raw[pid, :12])
            assert np.array_equal(rec[j, 12:], v[4:8])
            if sampling != oracle.AVERAGE:
                assert np.array_equal(rec[j], raw[pid])


def test_full_precision_leaves_the_voxels_alone():
    p = synth.uniform_cloud(2000, 6)
    a = oracle.build(p, leaf_cap=20, max_level=12)
    b = oracle.build(p, leaf_cap=20, max_level=12, full_precision=True)
    for f in ("level", "key", "count", "offset", "voxels"):
        assert np.array_equal(a[f], b[f])
    assert a["voxel_ids"] is None and b["voxel_ids"] is not None


WEIGHTED_CASES = [(150, 3, 12, 0), (250, 10, 12, 1), (200, 1, 5, 2), (120, 7, 14, 3)]


@pytest.mark.parametrize("n,T,ml,seed", WEIGHTED_CASES)
def test_weighted_equals_gather_form(n, T, ml, seed):
    """Sec. 4.2.4: the oracle scatters every sample onto its 2x2x2 cells; the
    brute-force form gathers, for every occupied cell, all samples of the node."""
    p = synth.uniform_cloud(n, seed)
    t = oracle.build(p, leaf_cap=T, max_level=ml, sampling=oracle.WEIGHTED)
    k = oracle.keys(p)
    q = brute.demorton(k)
    want = brute.recursive_weighted(p, q, k, brute.tree_nodes(t))
    for i in np.nonzero(t["is_leaf"] == 0)[0]:
        got = {c: v[:4] for c, v in brute.tree_voxels(t, i).items()}
        assert got == want[(int(t["level"][i]), int(t["key"][i]))]


@pytest.mark.parametrize("n,T,ml,seed", WEIGHTED_CASES[:3])
def test_weighted_within_bound_of_real_weights(n, T, ml, seed):
    """Fixed-point weights against float64 weights on the same samples (the
    oracle's child voxels): each fixed weight exceeds the real one by less than
    one unit of 2^-16 and the sum of weights is at least that of the
    containing sample (> 0.13), so a colour moves by less than
    1 + 255 * samples / (0.13 * 65536) steps."""
    p = synth.uniform_cloud(n, seed)
    t = oracle.build(p, leaf_cap=T, max_level=ml, sampling=oracle.WEIGHTED)
    k = oracle.keys(p)
    q = brute.demorton(k)
    nodes = brute.tree_nodes(t)
    mine = {(int(t["level"][i]), int(t["key"][i])): {c: v[:4] for c, v in brute.tree_voxels(t, i).items()}
            for i in np.nonzero(t["is_leaf"] == 0)[0]}
    real = brute.recursive_weighted(p, q, k, nodes, real=True, child_voxels=mine)
    bound = int(np.ceil(1 + 255 * n / (0.13 * 65536)))
    worst = 0
    for node, vox in mine.items():
        for c, v in vox.items():
            worst = max(worst, max(abs(v[a] - real[node][c][a]) for a in range(3)))
    assert worst <= bound


def test_weighted_keeps_cells_and_constant_colour():
    p = synth.uniform_cloud(3000, 8)
    a = oracle.build(p, leaf_cap=30, max_level=12)
    p2 = p.copy()
    p2["r"], p2["g"], p2["b"] = 7, 130, 251
    w = oracle.build(p2, leaf_cap=30, max_level=12, sampling=oracle.WEIGHTED)
    for f in ("level", "key", "count", "offset"):
        assert np.array_equal(a[f], w[f])
    assert np.array_equal(a["voxels"][:, :4], w["voxels"][:, :4])
    assert np.all(w["voxels"][:, 4:] == np.array([7, 130, 251, 255], np.uint8))


def test_weighted_differs_from_average_where_neighbours_overlap():
    # a surface with several samples per cell and two halves of different
    # colour: cells along the seam mix both sides, cells far from it do not
    p = synth.terrain(60_000, seed=4)
    p["r"] = np.where(p["x"] < np.median(p["x"]), 0, 240)
    p["g"] = 100
    a = oracle.build(p, leaf_cap=2000, max_level=12)
    w = oracle.build(p, leaf_cap=2000, max_level=12, sampling=oracle.WEIGHTED)
    assert np.array_equal(a["voxels"][:, :4], w["voxels"][:, :4])
    assert np.all(w["voxels"][:, 5] == 100)
    mixed = (w["voxels"][:, 4] != 0) & (w["voxels"][:, 4] != 240)
    mixed_avg = (a["voxels"][:, 4] != 0) & (a["voxels"][:, 4] != 240)
    assert mixed_avg.sum() < mixed.sum() < len(w["voxels"]) // 2


def test_constant_colour_gives_constant_voxels():
    p = synth.uniform_cloud(3000, 8)
    p["r"], p["g"], p["b"] = 7, 130, 251
    t = oracle.build(p, leaf_cap=30, max_level=12)
    v = t["voxels"]
    assert len(v) > 0 and np.all(v[:, 4] == 7) and np.all(v[:, 5] == 130) and np.all(v[:, 6] == 251)
    assert np.all(v[:, 7] == 255) and np.all(v[:, 3] == 0)


def test_voxels_in_morton_order_and_in_grid():
    p = synth.uniform_cloud(2000, 12)
    t = oracle.build(p, leaf_cap=25, max_level=12)
    for i in np.nonzero(t["is_leaf"] == 0)[0]:
        v = t["voxels"][t["offset"][i]:t["offset"][i] + t["count"][i]]
        assert np.all(v[:, :3] < 128)
        codes = brute.morton(v[:, :3].astype(np.uint32))
        assert np.all(np.diff(codes.astype(np.int64)) > 0)


def test_child_voxel_contribution_at_most_eight_per_cell():
    # a node whose children are all inner: each cell gathers at most 8 child voxels
    p = synth.uniform_cloud(4000, 21)
    t = oracle.build(p, leaf_cap=8, max_level=12)
    assert t["num_voxels"] > 0
    root = brute.tree_voxels(t, 0)
    # the root's voxels are at most the number of occupied level-7 cells
    q = brute.demorton(oracle.keys(p))
    assert len(root) == len({tuple(c) for c in (q >> np.uint32(14)).tolist()})


# --------------------------------------------------------------- builds in a given cube
#
# lod_oracle_build_in_cube / lod_oracle_keys_in_cube check every GPU build too
# large for the oracle to rebuild whole: the subtree of a node is rebuilt from
# the node's own points in the whole cloud's cube.  Below a node, everything
# depends on that node's points alone (Sec. 4.1: a node's split depends on its
# own count; Sec. 4.2: its voxels on its children's samples).

def _shifted_cube(p, grow: float, shift):
    """A cube that contains every point but is not the cloud's own: edge
    `grow` times the cloud's side, minimum corner moved down by `shift`
    (fractions of the side) -- a float32 corner, as the API takes it."""
    lo, _, side, _ = oracle.cube(p)
    lo2 = (lo.astype(np.float64) - np.asarray(shift) * side).astype(np.float32)
    side2 = side * grow + float(np.max(lo.astype(np.float64) - lo2.astype(np.float64)))
    return lo2, side2


def _teapot_in_stadium():
    a = synth.uniform_cloud(400, 1, lo=(0, 0, 0), hi=(100, 100, 100))
    b = synth.uniform_cloud(1600, 2, lo=(40, 40, 40), hi=(40.01, 40.01, 40.01))
    return np.concatenate([a, b])


IN_CUBE_CLOUDS = {
    "uniform": (lambda: synth.uniform_cloud(3000, 31, lo=(-3, 7, 1), hi=(5, 9, 2)), 25, 12),
    "teapot_in_stadium": (_teapot_in_stadium, 20, 14),
    "terrain": (lambda: synth.terrain(6000, seed=13), 60, 12),
    "aerial": (lambda: synth.aerial(6000, seed=14), 40, 12),
}


def test_keys_in_cube_with_the_cloud_cube_equal_keys():
    for make, _, _ in IN_CUBE_CLOUDS.values():
        p = make()
        lo, _, side, _ = oracle.cube(p)
        assert np.array_equal(oracle.keys_in_cube(p, lo, side), oracle.keys(p))


@pytest.mark.parametrize("grow,shift", [(1.0, (0.0, 0.0, 0.0)), (1.7, (0.1, 0.25, 0.0)), (3.0, (0.5, 0.5, 0.5))])
def test_keys_in_cube_match_vectorised_and_exact_quantization(grow, shift):
    p = synth.uniform_cloud(2000, 41, lo=(-50, 3, 1e3), hi=(80, 40, 1.02e3))
    lo, side = _shifted_cube(p, grow, shift)
    k = oracle.keys_in_cube(p, lo, side)
    q = brute.quantize_in_cube(p, lo, side)
    assert np.array_equal(k, brute.morton(q))
    # and within one cell of the exact rational value (rounding of the two
    # double operations), for a sample of the points
    for i in range(0, len(p), 37):
        for a, ax in enumerate("xyz"):
            exact = (Fraction(float(p[ax][i])) - Fraction(float(lo[a]))) * (1 << 21) / Fraction(side)
            assert abs(int(q[i, a]) - min(int(exact), (1 << 21) - 1)) <= 1


@pytest.mark.parametrize("sampling", [oracle.AVERAGE, oracle.FIRST, oracle.RANDOM, oracle.WEIGHTED])
def test_build_in_the_cloud_cube_equals_build(sampling):
    for make, T, ml in IN_CUBE_CLOUDS.values():
        p = make()
        lo, _, side, _ = oracle.cube(p)
        a = oracle.build(p, leaf_cap=T, max_level=ml, sampling=sampling, seed=5)
        b = oracle.build(p, leaf_cap=T, max_level=ml, sampling=sampling, seed=5, cube_lo=lo, cube_side=side)
        for f in ("level", "key", "is_leaf", "npoints", "child_mask", "first_child", "count", "offset",
                  "point_ids", "voxels", "aabb_min", "aabb_max"):
            assert np.array_equal(a[f], b[f]), f
        assert a["side"] == b["side"] and a["num_voxels"] == b["num_voxels"]


@pytest.mark.parametrize("grow,shift", [(1.5, (0.2, 0.0, 0.3)), (2.0, (0.0, 0.4, 0.1))])
def test_build_in_a_larger_cube_matches_merge_procedure_and_recursion(grow, shift):
    """In a cube that is not the cloud's own, the tree is the paper's merge
    procedure on the keys quantized in that cube, the voxels are the
    dict recursion and the closed forms on the same keys."""
    p = synth.uniform_cloud(1500, 43)
    lo, side = _shifted_cube(p, grow, shift)
    T, ml = 12, 12
    t = oracle.build(p, leaf_cap=T, max_level=ml, cube_lo=lo, cube_side=side)
    q = brute.quantize_in_cube(p, lo, side)
    k = brute.morton(q)
    assert t["side"] == side and np.array_equal(t["aabb_min"], lo)
    assert brute.tree_nodes(t) == brute.paper_merge_tree(k, T, ml)
    # membership by the in-cube keys
    seen = np.zeros(len(p), np.int64)
    for i in np.nonzero(t["is_leaf"])[0]:
        ids = t["point_ids"][t["offset"][i]:t["offset"][i] + t["count"][i]]
        seen[ids] += 1
        assert np.all(brute.prefix(k[ids], int(t["level"][i])) == t["key"][i])
    assert np.all(seen == 1)
    rec = brute.recursive_voxels(p, q, k, brute.tree_nodes(t), T, ml)
    for i in np.nonzero(t["is_leaf"] == 0)[0]:
        L, key = int(t["level"][i]), int(t["key"][i])
        got = brute.tree_voxels(t, i)
        assert got == rec[(L, key)]
        assert set(got) == brute.closed_form_cells(q, k, L, key)
    f = oracle.build(p, leaf_cap=T, max_level=ml, sampling=oracle.FIRST, cube_lo=lo, cube_side=side)
    for i in np.nonzero(f["is_leaf"] == 0)[0]:
        L, key = int(f["level"][i]), int(f["key"][i])
        got = {c: v[4] for c, v in brute.tree_voxels(f, i).items()}
        assert got == brute.closed_form_pick(p, q, k, L, key, oracle.FIRST, 0)


@pytest.mark.parametrize("sampling", [oracle.AVERAGE, oracle.FIRST, oracle.WEIGHTED])
@pytest.mark.parametrize("cloud", sorted(IN_CUBE_CLOUDS))
def test_subtree_rebuilt_from_its_points_equals_the_whole_build(cloud, sampling):
    """For every inner node X of the whole-cloud build, the build of X's points
    alone in the whole cloud's cube holds X (at the same level and key) with
    the same subtree: node fields, leaf members (mapped back to the cloud's
    indices), voxels, and the first-come picks (mapped back; the smallest
    local index is the smallest cloud index since the selection keeps input
    order).  RANDOM picks hash the point index, which a sub-build renumbers,
    so they are not compared here."""
    import canon

    make, T, ml = IN_CUBE_CLOUDS[cloud]
    p = make()
    lo, _, side, _ = oracle.cube(p)
    whole = oracle.build(p, leaf_cap=T, max_level=ml, sampling=sampling)
    keys = brute.morton(brute.quantize_in_cube(p, lo, side))
    inner = np.nonzero(whole["is_leaf"] == 0)[0]
    assert len(inner) >= 5
    for x in inner[1:]:
        L, kx = int(whole["level"][x]), np.uint64(int(whole["key"][x]))
        s = np.nonzero(brute.prefix(keys, L) == kx)[0]
        assert len(s) == whole["npoints"][x]
        o = oracle.build(np.ascontiguousarray(p[s]), leaf_cap=T, max_level=ml, sampling=sampling,
                         cube_lo=lo, cube_side=side)
        ox = np.nonzero((o["level"] == L) & (o["key"] == kx))[0]
        assert len(ox) == 1
        gi, oi = canon.subtree_indices(whole, int(x)), canon.subtree_indices(o, int(ox[0]))
        assert len(gi) == len(oi)
        for f in ("level", "key", "is_leaf", "npoints", "child_mask", "count"):
            assert np.array_equal(whole[f][gi], o[f][oi]), (cloud, int(x), f)
        for a, b in zip(gi, oi):
            ga, gc = int(whole["offset"][a]), int(whole["count"][a])
            ob, oc = int(o["offset"][b]), int(o["count"][b])
            if whole["is_leaf"][a]:
                assert np.array_equal(np.sort(whole["point_ids"][ga:ga + gc]),
                                      np.sort(s[o["point_ids"][ob:ob + oc]]))
            else:
                assert np.array_equal(whole["voxels"][ga:ga + gc], o["voxels"][ob:ob + oc]), (cloud, int(x), a)
                if sampling == oracle.FIRST:
                    assert np.array_equal(whole["voxel_ids"][ga:ga + gc], s[o["voxel_ids"][ob:ob + oc]])
