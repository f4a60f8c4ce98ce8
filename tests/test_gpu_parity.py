"""GPU parity: the HIP path (through the C ABI) against the CPU oracle,
element by element on the same seeded inputs.  Integer work is compared
bit-exactly; the only floating-point step (quantization) is part of it."""
from __future__ import annotations

import sys

import numpy as np
import pytest

import canon
import oracle
import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lod():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    import paper_2302_14801_amd as lod
    return lod


def to_dev(points):
    import torch
    raw = np.ascontiguousarray(points).view(np.uint8).reshape(-1)
    return torch.from_numpy(raw.copy()).to("cuda:0")


def gpu_tree(lod, points, **kw):
    t = lod.lod_build(to_dev(points), **kw)
    h = t.to_host()
    t.free()
    return h


def check(lod, points, T=50000, ml=12, sampling=0, seed=0, keep_ids=False, **extra):
    print(f"case n={len(points)} T={T} ml={ml} sampling={sampling}", flush=True)
    g = gpu_tree(lod, points, leaf_cap=T, max_level=ml, sampling=sampling, seed=seed, keep_ids=keep_ids, **extra)
    o = oracle.build(points, leaf_cap=T, max_level=ml, sampling=sampling, seed=seed)
    canon.compare_trees(g, o, points)
    return g, o


RANDOM_CASES = [(50, 1, 2), (300, 3, 4), (800, 7, 12), (2000, 50, 12), (1500, 1, 6), (2000, 100, 3),
                (20000, 200, 12), (60000, 1000, 14), (150000, 4000, 12)]


@pytest.mark.parametrize("sampling", [0, 1, 2, 3])
@pytest.mark.parametrize("n,T,ml", RANDOM_CASES)
def test_uniform_clouds(lod, n, T, ml, sampling):
    p = synth.uniform_cloud(n, 1000 + n, lo=(-3, 10, 100), hi=(5, 12, 101))
    check(lod, p, T, ml, sampling, seed=77)


@pytest.mark.parametrize("sampling", [0, 1, 2, 3])
def test_terrain_small(lod, sampling):
    p = synth.terrain(200_000, seed=5)
    check(lod, p, T=5000, ml=12, sampling=sampling, seed=3)


@pytest.mark.parametrize("sampling", [0, 3])
def test_aerial_small(lod, sampling):
    p = synth.aerial(400_000, seed=2)
    check(lod, p, T=10000, ml=12, sampling=sampling)


def test_scan_small(lod):
    p = synth.scan(300_000, seed=3)
    check(lod, p, T=2000, ml=14)


def test_terrain_1m_config(lod):
    """The 1M-point terrain plain build (T = 50 000, 128^3, colour-filtered), in full."""
    p = synth.terrain(1_000_000, seed=1)
    g, o = check(lod, p, T=50000, ml=12)
    assert g["num_voxels"] > 0


def test_keep_ids_average(lod):
    p = synth.uniform_cloud(5000, 4)
    g, _ = check(lod, p, T=40, ml=12, keep_ids=True)
    assert g["point_ids"] is not None


@pytest.mark.parametrize("sampling", [0, 1, 2, 3])
def test_empty(lod, sampling):
    for fp in (False, True):
        g = gpu_tree(lod, np.zeros(0, synth.POINT_DTYPE), sampling=sampling, full_precision=fp)
        assert g["num_nodes"] == 0 and g["num_voxels"] == 0


@pytest.mark.parametrize("sampling", [0, 3])
def test_shallow_depth_limits(lod, sampling):
    # depth limits 1 and 2: every inner node is a root or its child
    p = synth.terrain(30_000, seed=14)
    for ml in (1, 2):
        check(lod, p, T=100, ml=ml, sampling=sampling)


def test_single_point_and_small(lod):
    check(lod, synth.uniform_cloud(1, 3), T=1)
    check(lod, synth.uniform_cloud(49, 3), T=50)


def test_identical_points_chain_to_depth_limit(lod):
    p = np.zeros(1000, synth.POINT_DTYPE)
    p["x"], p["y"], p["z"] = 1.5, -2.0, 7.0
    p["r"] = np.arange(1000) % 256
    p[-1]["x"] = 9.0
    for s in (0, 1, 2, 3):
        g, _ = check(lod, p, T=10, ml=9, sampling=s)
        assert g["level"].max() == 9


def test_huge_micro_bucket_wide_path(lod):
    # 70 000 coincident points in one oversize leaf at the depth limit
    p = np.zeros(70_010, synth.POINT_DTYPE)
    p["x"], p["y"], p["z"] = 3.0, 3.0, 3.0
    rng = np.random.default_rng(1)
    p["r"] = rng.integers(0, 256, len(p))
    p["g"] = rng.integers(0, 256, len(p))
    p["b"] = rng.integers(0, 256, len(p))
    p["x"][-10:] = rng.uniform(0, 10, 10).astype(np.float32)
    check(lod, p, T=100, ml=5)
    check(lod, p, T=100, ml=5, sampling=3)


def test_lattice_and_max_face(lod):
    s = 8
    g1 = np.arange(s, dtype=np.float32)
    xs, ys, zs = np.meshgrid(g1, g1, g1, indexing="ij")
    p = np.zeros(s ** 3, synth.POINT_DTYPE)
    p["x"], p["y"], p["z"] = xs.ravel(), ys.ravel(), zs.ravel()
    p["g"] = np.arange(s ** 3) % 251
    for T in (1, 2, 7):
        check(lod, p, T=T, ml=12)


def test_teapot_in_stadium(lod):
    a = synth.uniform_cloud(20000, 1, lo=(0, 0, 0), hi=(1000, 1000, 1000))
    b = synth.uniform_cloud(80000, 2, lo=(400, 400, 400), hi=(400.05, 400.05, 400.05))
    p = np.concatenate([a, b])
    for s in (0, 2):
        g, _ = check(lod, p, T=500, ml=14, sampling=s, seed=5)
        assert g["level"].max() >= 12


def test_extreme_coordinates(lod):
    p = synth.uniform_cloud(3000, 9, lo=(-1e6, 1e-6, -3e5), hi=(1e6, 2e-6, 3e5))
    check(lod, p, T=20, ml=14)


def test_nonfinite_rejected(lod):
    p = synth.uniform_cloud(1000, 1)
    p["z"][500] = np.inf
    with pytest.raises(lod.LodError) as e:
        lod.lod_build(to_dev(p))
    assert e.value.status == -2


def test_invalid_params_rejected(lod):
    d = to_dev(synth.uniform_cloud(100, 1))
    for kw in ({"leaf_cap": 0}, {"max_level": 15}, {"sampling": 4}):
        with pytest.raises(lod.LodError) as e:
            lod.lod_build(d, **kw)
        assert e.value.status == -1


def test_tuning_and_repeat_do_not_change_results(lod):
    """Every plan (levels of the two partition passes, points per partition
    work item) gives the oracle's tree, and a repeated build the same one."""
    p = synth.terrain(300_000, seed=8)
    o = oracle.build(p, leaf_cap=3000, max_level=12)
    base = gpu_tree(lod, p, leaf_cap=3000, max_level=12)
    canon.compare_trees(base, o, p)
    again = gpu_tree(lod, p, leaf_cap=3000, max_level=12)
    for k in ("level", "key", "npoints", "count", "voxels"):
        assert np.array_equal(base[k], again[k])
    for t0, t1, ch in ((1, 1, 0), (2, 4, 1), (4, 2, 50_000), (3, 3, 7000), (4, 4, 0), (4, 4, 65_000)):
        print(f"plan {t0} {t1} {ch}", flush=True)
        params = lod.make_params(leaf_cap=3000, max_level=12, tune_levels0=t0, tune_levels1=t1, tune_chunk=ch)
        t = lod.lod_build(to_dev(p), params=params)
        h = t.to_host()
        t.free()
        canon.compare_trees(h, o, p)


def test_input_order_invariance(lod):
    p = synth.aerial(200_000, seed=12)
    perm = np.random.default_rng(0).permutation(len(p))
    a = gpu_tree(lod, p, leaf_cap=5000)
    b = gpu_tree(lod, p[perm], leaf_cap=5000)
    for k in ("level", "key", "npoints", "count", "voxels"):
        assert np.array_equal(a[k], b[k])
    # pick results follow the ids, so compare with the oracle on the permuted input
    check(lod, p[perm], T=5000, sampling=1)


@pytest.mark.parametrize("sampling", [0, 2, 3])
def test_batch_equals_single_builds(lod, sampling):
    sizes = [3000, 50, 120000, 0, 40000, 777]
    pts, offs = synth.batch_chunks(sizes, seed=4)
    trees = lod.lod_build_batch(to_dev(pts), offs, leaf_cap=2000, max_level=12, sampling=sampling, seed=11)
    assert len(trees) == len(sizes)
    for i, t in enumerate(trees):
        chunk = pts[offs[i]:offs[i + 1]]
        g = t.to_host()
        t.free()
        o = oracle.build(chunk, leaf_cap=2000, max_level=12, sampling=sampling, seed=11)
        canon.compare_trees(g, o, chunk)


def test_autotuned_batch_plan_gives_same_trees(lod):
    """The library's tuner (lod_tune_batch, and LOD_FLAG_AUTOTUNE) picks a plan
    whose trees are the oracle's; the second call of the class is cached."""
    from paper_2302_14801_amd import autotune
    sizes = [30_000, 200_000, 5_000, 90_000, 60_000, 1]
    pts, offs = synth.batch_chunks(sizes, seed=21)
    dev = to_dev(pts)
    base = lod.make_params(leaf_cap=4000, max_level=12)
    tuned, info = autotune.tune_batch(dev, offs, base)
    assert len(info["plan"]) == 3 and info["cached"] == 0 and info["sample_chunks"] == len(sizes)
    again, info2 = autotune.tune_batch(dev, offs, base)
    assert info2["cached"] == 1 and info2["plan"] == info["plan"]
    auto = lod.make_params(leaf_cap=4000, max_level=12)
    auto.flags |= lod.LOD_FLAG_AUTOTUNE
    for params in (tuned, auto):
        trees = lod.lod_build_batch(dev, offs, params=params)
        for i, t in enumerate(trees):
            chunk = pts[offs[i]:offs[i + 1]]
            g = t.to_host()
            t.free()
            canon.compare_trees(g, oracle.build(chunk, leaf_cap=4000, max_level=12), chunk)


def test_batch_many_uneven_chunks(lod):
    # 48 chunks of lognormal sizes (one launch sequence for all), every tree
    # checked against the oracle on its own chunk
    sizes = synth.chunk_sizes(48, seed=9, median=20_000, sigma=1.0, lo=1, hi=400_000)
    pts, offs = synth.batch_chunks(sizes, seed=9)
    trees = lod.lod_build_batch(to_dev(pts), offs, leaf_cap=3000, max_level=12)
    for i, t in enumerate(trees):
        chunk = pts[offs[i]:offs[i + 1]]
        g = t.to_host()
        t.free()
        canon.compare_trees(g, oracle.build(chunk, leaf_cap=3000, max_level=12), chunk)


def check_full(g, o, points):
    """Tree, accepted ids and full-precision records, node by node."""
    canon.compare_trees(g, o, points)
    assert g["voxel_points"] is not None and g["voxel_ids"] is not None
    for i in np.nonzero(g["is_leaf"] == 0)[0]:
        go, oo, c = int(g["offset"][i]), int(o["offset"][i]), int(g["count"][i])
        assert np.array_equal(g["voxel_points"][go:go + c], o["voxel_points"][oo:oo + c]), f"records of node {i}"


@pytest.mark.parametrize("sampling", [0, 1, 2, 3])
def test_full_precision_lower_levels(lod, sampling):
    p = synth.terrain(200_000, seed=5)
    print(f"full precision n={len(p)} sampling={sampling}", flush=True)
    g = gpu_tree(lod, p, leaf_cap=5000, max_level=12, sampling=sampling, seed=3, full_precision=True)
    o = oracle.build(p, leaf_cap=5000, max_level=12, sampling=sampling, seed=3, full_precision=True)
    check_full(g, o, p)


def test_full_precision_exact_rounds(lod):
    # a depth-limited cell of 999 samples (packed sums overflow: exact second
    # round) and a micro-bucket of 70 000 points (wide path)
    p = np.zeros(1000, synth.POINT_DTYPE)
    p["x"], p["y"], p["z"] = 1.5, -2.0, 7.0
    p["r"] = np.arange(1000) % 256
    p[-1]["x"] = 9.0
    q = np.zeros(70_010, synth.POINT_DTYPE)
    q["x"], q["y"], q["z"] = 3.0, 3.0, 3.0
    rng = np.random.default_rng(1)
    q["g"] = rng.integers(0, 256, len(q))
    q["x"][-10:] = rng.uniform(0, 10, 10).astype(np.float32)
    for pts, T, ml in ((p, 10, 9), (q[rng.permutation(len(q))], 100, 5)):
        print(f"full precision exact n={len(pts)}", flush=True)
        g = gpu_tree(lod, pts, leaf_cap=T, max_level=ml, full_precision=True)
        check_full(g, oracle.build(pts, leaf_cap=T, max_level=ml, full_precision=True), pts)


def test_full_precision_batch(lod):
    sizes = [3000, 50, 120000, 0, 40000, 777]
    pts, offs = synth.batch_chunks(sizes, seed=4)
    trees = lod.lod_build_batch(to_dev(pts), offs, leaf_cap=2000, max_level=12, full_precision=True)
    for i, t in enumerate(trees):
        chunk = pts[offs[i]:offs[i + 1]]
        g = t.to_host()
        t.free()
        if len(chunk) == 0:
            assert g["num_voxels"] == 0
            continue
        check_full(g, oracle.build(chunk, leaf_cap=2000, max_level=12, full_precision=True), chunk)


def test_server_results_equal_alone_and_in_mix(lod):
    sizes = [200_000, 5_000, 80_000, 1, 150_000, 30_000, 90_000, 10]
    pts, offs = synth.batch_chunks(sizes, seed=6)
    chunks = [np.ascontiguousarray(pts[offs[i]:offs[i + 1]]) for i in range(len(sizes))]
    srv = lod.lod_server_create(8 << 30, 3, leaf_cap=4000, max_level=12)
    tickets = [srv.submit(c) for c in chunks]
    import time
    done = {}
    t0 = time.time()
    while len(done) < len(tickets):
        for i, tk in enumerate(tickets):
            if i not in done:
                r = srv.poll(tk)
                if r is not None:
                    done[i] = r
        assert time.time() - t0 < 120
        time.sleep(0.001)
    for i, c in enumerate(chunks):
        g = done[i].to_host()
        alone = gpu_tree(lod, c, leaf_cap=4000, max_level=12)
        for k in ("level", "key", "npoints", "count", "first_child", "voxels"):
            assert np.array_equal(g[k], alone[k]), (i, k)
        canon.compare_trees(g, oracle.build(c, leaf_cap=4000, max_level=12), c)
        done[i].free()
    with pytest.raises(lod.LodError) as e:
        srv.poll(987654)
    assert e.value.status == -6
    srv.destroy()


def test_server_weighted_full_precision(lod):
    # requests with the weighted mode and full-precision records through the
    # server equal lod_build on the same points
    sizes = [60_000, 1_000, 120_000, 0]
    pts, offs = synth.batch_chunks(sizes, seed=17)
    chunks = [np.ascontiguousarray(pts[offs[i]:offs[i + 1]]) for i in range(len(sizes))]
    srv = lod.lod_server_create(8 << 30, 2, leaf_cap=3000, max_level=12, sampling=3, full_precision=True)
    tickets = [srv.submit(c) for c in chunks]
    import time
    t0 = time.time()
    for i, (tk, c) in enumerate(zip(tickets, chunks)):
        r = srv.poll(tk)
        while r is None:
            assert time.time() - t0 < 120
            time.sleep(0.001)
            r = srv.poll(tk)
        g = r.to_host()
        r.free()
        alone = gpu_tree(lod, c, leaf_cap=3000, max_level=12, sampling=3, full_precision=True)
        for k in ("level", "key", "count", "voxels", "voxel_ids", "voxel_points"):
            if alone[k] is None:
                assert g[k] is None or len(g[k]) == 0
            else:
                assert np.array_equal(g[k], alone[k]), (i, k)
        if len(c):
            check_full(g, oracle.build(c, leaf_cap=3000, max_level=12, sampling=3, full_precision=True), c)
    srv.destroy()


def test_server_rejects_too_large(lod):
    srv = lod.lod_server_create(1 << 20, 1, leaf_cap=1000)
    with pytest.raises(lod.LodError) as e:
        srv.submit(synth.uniform_cloud(100_000, 1))
    assert e.value.status == -5
    srv.destroy()


if __name__ == "__main__":
    sys.exit(pytest.main([__file__, "-x", "-v"]))


def lattice_cloud(side: int, seed: int) -> np.ndarray:
    """One point at the centre of every cell of a side^3 lattice in [0, 1)^3,
    in shuffled order, with random colours."""
    rng = np.random.default_rng(seed)
    g = ((np.arange(side, dtype=np.float64) + 0.5) / side).astype(np.float32)
    x, y, z = np.meshgrid(g, g, g, indexing="ij")
    a = np.empty(side ** 3, synth.POINT_DTYPE)
    a["x"], a["y"], a["z"] = x.ravel(), y.ravel(), z.ravel()
    for ax in "rgb":
        a[ax] = rng.integers(0, 256, a.size, dtype=np.uint8)
    a["a"] = 255
    return a[rng.permutation(a.size)]


def test_weighted_dense_blocks_windows(lod):
    # 64^3 lattice, T = 50 000: the root is inner and its 8 children are
    # leaves.  Each leaf work item brings 4096 points, each in a root cell of
    # its own, to one 32^3 block of the root's grid: more occupied cells than
    # one LDS window holds, and the cells around the block overflow the LDS
    # hash (their sums go through the global fallback).
    check(lod, lattice_cloud(64, 5), T=50000, ml=12, sampling=2, seed=3)


def test_weighted_dense_blocks_global_sums(lod):
    # 128^3 lattice, T = 5000: leaves at level 3, so the root's level uses
    # 16^3 blocks, and every such block of the root's grid is fully occupied
    # (4096 cells, more than its LDS sums hold): its own cells are summed
    # through the global atomics.
    check(lod, lattice_cloud(128, 6), T=5000, ml=12, sampling=2, seed=4)


@pytest.mark.parametrize("full_precision", [False, True])
@pytest.mark.parametrize("side,T", [(72, 50000), (80, 70000), (96, 120000)])
def test_leaf_items_at_the_sparse_kernel_limits(lod, side, T, full_precision):
    # Lattices whose 8 leaves (level 1) split into work items of side^3 / 64
    # points, each point in a leaf cell of its own: 5832 cells fit the sparse
    # leaf kernel's pool in the average mode but not with full-precision
    # records (4096 cells); 8000 points enter the sparse kernel and are handed
    # back for their cells in both; 13 824 points (over 8192) go straight to
    # the general leaf kernel.
    p = lattice_cloud(side, 7)
    print(f"leaf items side={side} T={T} full_precision={full_precision}", flush=True)
    if not full_precision:
        check(lod, p, T=T, ml=12, sampling=0, seed=3)
        return
    g = gpu_tree(lod, p, leaf_cap=T, max_level=12, sampling=0, seed=3, full_precision=True)
    check_full(g, oracle.build(p, leaf_cap=T, max_level=12, sampling=0, seed=3, full_precision=True), p)


def test_large_batch_second_count_from_cells(lod):
    # 68.9M points in 7 clouds (median 1M points, so 3 levels per partition):
    # the plan for the batch's total takes the second partition's counts from
    # the 2-byte cells the first insert stores; single builds of the clouds
    # (each under 64M points) count the records themselves.  Both must give
    # the same trees.
    sizes = [40_000_000, 1_000_000, 1_200_000, 0, 800_000, 25_000_000, 900_000]
    pts, offs = synth.batch_chunks(sizes, seed=8)
    print(f"large batch n={len(pts)}", flush=True)
    trees = lod.lod_build_batch(to_dev(pts), offs, leaf_cap=50000, max_level=12)
    for i, t in enumerate(trees):
        chunk = np.ascontiguousarray(pts[offs[i]:offs[i + 1]])
        g = t.to_host()
        t.free()
        if len(chunk) == 0:
            assert g["num_voxels"] == 0
            continue
        alone = gpu_tree(lod, chunk, leaf_cap=50000, max_level=12)
        for k in ("level", "key", "npoints", "count", "first_child", "voxels"):
            assert np.array_equal(g[k], alone[k]), (i, k)
