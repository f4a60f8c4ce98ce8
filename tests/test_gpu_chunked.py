"""GPU parity of the chunked (out-of-core) build: the tree of a host cloud,
built through cells of one level of the common cube and merged above them,
equals the oracle's in-core tree of the whole cloud, and has the layout of
the in-core GPU build (same node table, same voxel array, same leaf ranges),
in all four sampling modes.  Each case runs both forms of the build: the
cloud resident on the device (the default when it fits) and the streaming
form that keeps the sorted pieces in host memory (LOD_FLAG_LOW_MEMORY)."""
from __future__ import annotations

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


def host_tree(t):
    h = t.to_host()
    t.free()
    return h


def to_dev(points):
    import torch
    raw = np.ascontiguousarray(points).view(np.uint8).reshape(-1)
    return torch.from_numpy(raw.copy()).to("cuda:0")


def check_chunked(lod, points, chunk, T, ml=12, sampling=0, seed=0, keep_ids=False, full=False):
    print(f"case n={len(points)} chunk={chunk} T={T} ml={ml} sampling={sampling} full={full}", flush=True)
    kw = dict(leaf_cap=T, max_level=ml, sampling=sampling, seed=seed, keep_ids=keep_ids)
    params = lod.make_params(full_precision=full, **kw)
    o = oracle.build(points, leaf_cap=T, max_level=ml, sampling=sampling, seed=seed, full_precision=full)
    for low_memory in (True, False):  # the resident form last: it is returned
        pm = lod.make_params(full_precision=full, low_memory=low_memory, **kw)
        g = host_tree(lod.lod_build_chunked(np.ascontiguousarray(points), chunk, params=pm))
        canon.compare_trees(g, o, points)
        if full:
            assert g["voxel_points"] is not None and g["voxel_ids"] is not None
            for i in np.nonzero(g["is_leaf"] == 0)[0]:
                go, oo, c = int(g["offset"][i]), int(o["offset"][i]), int(g["count"][i])
                assert np.array_equal(g["voxel_points"][go:go + c], o["voxel_points"][oo:oo + c]), \
                    f"records of node {i} (low_memory={low_memory})"
    d = host_tree(lod.lod_build(to_dev(points), params=params))
    for f in canon.NODE_FIELDS + ("offset",):
        assert np.array_equal(g[f], d[f]), f"node field {f} differs from the in-core build"
    assert np.array_equal(g["voxels"], d["voxels"])
    if d["voxel_ids"] is not None:
        assert np.array_equal(g["voxel_ids"], d["voxel_ids"])
    if d["voxel_points"] is not None:
        assert np.array_equal(g["voxel_points"], d["voxel_points"])
    for i in np.nonzero(g["is_leaf"])[0]:
        a, c = int(g["offset"][i]), int(g["count"][i])
        assert np.array_equal(canon.rows_sorted(g["points"][a:a + c]), canon.rows_sorted(d["points"][a:a + c]))
        if d["point_ids"] is not None:
            assert np.array_equal(np.sort(g["point_ids"][a:a + c]), np.sort(d["point_ids"][a:a + c]))
    return g


@pytest.mark.parametrize("sampling", [0, 1, 2, 3])
def test_uniform(lod, sampling):
    p = synth.uniform_cloud(200_000, 31, lo=(-3, 10, 100), hi=(5, 12, 101))
    check_chunked(lod, p, 20_000, T=500, sampling=sampling, seed=5)


@pytest.mark.parametrize("sampling", [0, 1, 2, 3])
def test_terrain(lod, sampling):
    p = synth.terrain(300_000, seed=6)
    check_chunked(lod, p, 50_000, T=2000, sampling=sampling, seed=9)


@pytest.mark.parametrize("sampling", [0, 1, 3])
def test_aerial(lod, sampling):
    p = synth.aerial(400_000, seed=2)
    check_chunked(lod, p, 60_000, T=5000, sampling=sampling)


@pytest.mark.parametrize("sampling", [0, 1, 2, 3])
def test_full_precision(lod, sampling):
    p = synth.terrain(300_000, seed=12)
    check_chunked(lod, p, 40_000, T=2000, sampling=sampling, seed=4, full=True)


def test_full_precision_sparse_leaves(lod):
    blob = synth.uniform_cloud(60_000, 49, lo=(0.40, 0.40, 0.40), hi=(0.45, 0.43, 0.41))
    p = np.concatenate([synth.uniform_cloud(200, 50), blob])
    check_chunked(lod, p, 5_000, T=1000, sampling=3, full=True)


def test_scan_with_ids(lod):
    p = synth.scan(300_000, seed=3)
    check_chunked(lod, p, 40_000, T=2000, ml=14, keep_ids=True)


@pytest.mark.parametrize("sampling", [0, 2, 3])
def test_dense_blob_and_sparse_leaves(lod, sampling):
    """Small leaves above the split level next to chunk roots: a dense blob and
    a few hundred points spread over the cube."""
    blob = synth.uniform_cloud(100_000, 41, lo=(0.40, 0.40, 0.40), hi=(0.45, 0.43, 0.41))
    sparse = synth.uniform_cloud(300, 42)
    p = np.concatenate([sparse[:150], blob, sparse[150:]])
    check_chunked(lod, p, 5_000, T=1000, sampling=sampling, seed=3)


def test_chunk_of_one_point(lod):
    """No level has cells of at most one point: the split is at level 7, and
    every chunk root is a batch of its own."""
    blob = synth.uniform_cloud(30_000, 43, lo=(0.0, 0.0, 0.0), hi=(0.01, 0.01, 0.01))
    p = np.concatenate([blob, synth.uniform_cloud(2_000, 44)])
    check_chunked(lod, p, 1, T=300, sampling=1)


@pytest.mark.parametrize("sampling", [0, 3])
def test_everything_above_the_split(lod, sampling):
    p = synth.uniform_cloud(20_000, 45)
    check_chunked(lod, p, 1, T=300, sampling=sampling)


def test_identical_points_to_the_depth_limit(lod):
    p = synth.uniform_cloud(5_000, 46)
    p[:] = p[0]
    check_chunked(lod, p, 1_000, T=100, ml=6)


@pytest.mark.parametrize("ml", [1, 2, 3])
@pytest.mark.parametrize("sampling", [1, 3])
def test_shallow_depth_limits(lod, ml, sampling):
    p = synth.terrain(50_000, seed=7)
    check_chunked(lod, p, 4_000, T=500, ml=ml, sampling=sampling)


def test_one_chunk_is_the_in_core_build(lod):
    p = synth.terrain(30_000, seed=8)
    check_chunked(lod, p, 30_000, T=1000, sampling=2, seed=1)


def test_empty(lod):
    g = host_tree(lod.lod_build_chunked(synth.uniform_cloud(0, 1), 10))
    assert g["num_nodes"] == 0 and g["num_points"] == 0


def test_errors(lod):
    p = synth.uniform_cloud(1_000, 47)
    p["y"][500] = np.nan
    for low_memory in (False, True):
        with pytest.raises(lod.LodError) as e:
            lod.lod_build_chunked(p, 100, params=lod.make_params(low_memory=low_memory))
        assert e.value.status == -2
    with pytest.raises(lod.LodError) as e:
        lod.lod_build_chunked(synth.uniform_cloud(1_000, 48), 100, max_level=15)
    assert e.value.status == -1
