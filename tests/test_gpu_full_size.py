"""GPU parity at the benchmark's full size: the 100M-point aerial plain build
(T = 50 000, 128^3, colour-filtered), built exactly as bench.py builds it and
compared whole with the oracle's tree (node table, every leaf's point
multiset, every voxel), plus the properties and sampled oracle subtrees of
fullsize.py; and whole-tree parity at 5M points, where the build uses the
plan of large inputs (4 + 4 levels in the two partition passes)."""
from __future__ import annotations

import pytest

import canon
import fullsize
import oracle
import synth

pytestmark = pytest.mark.gpu

N = 100_000_000
T = 50_000
ML = 12


@pytest.mark.timeout(900)
def test_aerial_100m_bench_configuration():
    import torch

    import paper_2302_14801_amd as lod

    fullsize.log("generating")
    host = torch.empty(N * 16, dtype=torch.uint8, pin_memory=True)
    pts = host.numpy().view(synth.POINT_DTYPE)
    synth.aerial(N, seed=2, out=pts)
    dev = host.to("cuda:0")
    fullsize.log("building on the GPU")
    params = lod.make_params(leaf_cap=T, max_level=ML, timing=True)
    t = lod.lod_build(dev, params=params)
    g = t.to_host()
    t.free()
    del dev
    fullsize.log(f"{g['num_nodes']} nodes, {g['num_voxels']} voxels")
    fullsize.check_build(g, pts, T, ML)
    fullsize.log("oracle build of the whole cloud (one core)")
    o = oracle.build(pts, leaf_cap=T, max_level=ML)
    fullsize.log("comparing the whole tree")
    canon.compare_trees(g, o, pts)
    fullsize.log("the whole 100M tree equals the oracle's")


@pytest.mark.timeout(600)
@pytest.mark.parametrize("sampling,T", [(0, 50_000), (1, 50_000), (2, 50_000), (3, 50_000), (0, 2_000)])
def test_aerial_5m_whole_tree(sampling, T):
    """5M points take the large-input plan (4 + 4 levels, several chunks per
    root cell); T = 2 000 adds refinement partitions below level 8."""
    import numpy as np
    import torch

    import paper_2302_14801_amd as lod

    n = 5_000_000
    print(f"case aerial n={n} T={T} sampling={sampling}", flush=True)
    pts = synth.aerial(n, seed=17)
    dev = torch.from_numpy(pts.view(np.uint8).reshape(-1).copy()).to("cuda:0")
    t = lod.lod_build(dev, leaf_cap=T, max_level=ML, sampling=sampling, seed=31)
    g = t.to_host()
    t.free()
    o = oracle.build(pts, leaf_cap=T, max_level=ML, sampling=sampling, seed=31)
    canon.compare_trees(g, o, pts)


@pytest.mark.timeout(600)
def test_aerial_20m_weighted_and_full_precision():
    """The neighbourhood-weighted average on a 20M-point aerial cloud (T =
    50 000): same cells as the average build, colours checked on sampled
    subtrees rebuilt by the oracle; full-precision records of a pick build
    are input records of their voxels' cells."""
    import numpy as np
    import torch

    import paper_2302_14801_amd as lod

    n = 20_000_000
    fullsize.log("generating 20M")
    host = torch.empty(n * 16, dtype=torch.uint8, pin_memory=True)
    pts = host.numpy().view(synth.POINT_DTYPE)
    synth.aerial(n, seed=5, out=pts)
    dev = host.to("cuda:0")
    fullsize.log("building (weighted, average, first with full precision)")
    t = lod.lod_build(dev, leaf_cap=T, max_level=ML, sampling=3)
    g = t.to_host()
    t.free()
    t = lod.lod_build(dev, leaf_cap=T, max_level=ML)
    a = t.to_host()
    t.free()
    t = lod.lod_build(dev, leaf_cap=T, max_level=ML, sampling=1, full_precision=True)
    f = t.to_host()
    t.free()
    del dev
    for k in ("level", "key", "count", "offset"):
        assert np.array_equal(g[k], a[k]), k
    assert np.array_equal(g["voxels"][:, :4], a["voxels"][:, :4])
    assert not np.array_equal(g["voxels"][:, 4:], a["voxels"][:, 4:])
    raw = pts.view(np.uint8).reshape(-1, 16)
    assert np.array_equal(f["voxel_points"], raw[f["voxel_ids"].astype(np.int64)])
    fullsize.log("weighted cells equal the average's; full-precision records are input records")
    fullsize.check_build(g, pts, T, ML, subtree_picks=2, leaf_sample=2000, sampling=3)


@pytest.mark.timeout(900)
def test_aerial_100m_chunked_equals_in_core():
    """The 100M-point aerial cloud built from host memory in chunks of 10M
    points (bench.py's chunked run) equals the in-core build: the same node
    table, voxel array and leaf point sets; and passes the same checks."""
    import numpy as np
    import torch

    import paper_2302_14801_amd as lod

    fullsize.log("generating")
    host = torch.empty(N * 16, dtype=torch.uint8, pin_memory=True)
    pts = host.numpy().view(synth.POINT_DTYPE)
    synth.aerial(N, seed=2, out=pts)
    params = lod.make_params(leaf_cap=T, max_level=ML, keep_ids=True)
    fullsize.log("chunked build")
    t = lod.lod_build_chunked(pts, 10_000_000, params=params)
    g = t.to_host()
    t.free()
    fullsize.log("in-core build")
    dev = host.to("cuda:0")
    t = lod.lod_build(dev, params=params)
    d = t.to_host()
    t.free()
    del dev
    fullsize.log(f"{g['num_nodes']} nodes, {g['num_voxels']} voxels; comparing")
    for f in ("level", "key", "is_leaf", "npoints", "child_mask", "first_child", "count", "offset"):
        assert np.array_equal(g[f], d[f]), f
    assert np.array_equal(g["voxels"], d["voxels"])
    # leaf point sets: ids sorted inside the (identical) leaf ranges
    leaf = np.nonzero(g["is_leaf"])[0]
    order = np.argsort(g["offset"][leaf], kind="stable")
    owner = np.repeat(np.arange(len(leaf), dtype=np.uint64)[order], g["count"][leaf][order].astype(np.int64))
    for name in ("point_ids",):
        ka = np.sort((owner << np.uint64(32)) | g[name].astype(np.uint64))
        kb = np.sort((owner << np.uint64(32)) | d[name].astype(np.uint64))
        assert np.array_equal(ka, kb)
    raw = np.ascontiguousarray(pts).view(np.uint8).reshape(-1, 16)
    assert np.array_equal(g["points"], raw[g["point_ids"]])
    fullsize.check_build(g, pts, T, ML)
    fullsize.log("streaming chunked build (sorted pieces in host memory)")
    t = lod.lod_build_chunked(pts, 10_000_000, params=lod.make_params(leaf_cap=T, max_level=ML, keep_ids=True,
                                                                      low_memory=True))
    s = t.to_host()
    t.free()
    for f in ("level", "key", "is_leaf", "npoints", "child_mask", "first_child", "count", "offset"):
        assert np.array_equal(s[f], d[f]), f
    assert np.array_equal(s["voxels"], d["voxels"])
    ks = np.sort((owner << np.uint64(32)) | s["point_ids"].astype(np.uint64))
    assert np.array_equal(ks, kb)
    assert np.array_equal(s["points"], raw[s["point_ids"]])


@pytest.mark.timeout(600)
def test_aerial_20m_chunked_weighted_full_precision():
    """The weighted average with full-precision records on a 20M-point aerial
    cloud, built from host memory in 2M-point chunks, equals the in-core
    build: node table, voxels, accepted ids and records, leaf point sets."""
    import numpy as np
    import torch

    import paper_2302_14801_amd as lod

    n = 20_000_000
    fullsize.log("generating 20M")
    host = torch.empty(n * 16, dtype=torch.uint8, pin_memory=True)
    pts = host.numpy().view(synth.POINT_DTYPE)
    synth.aerial(n, seed=6, out=pts)
    params = lod.make_params(leaf_cap=T, max_level=ML, sampling=3, full_precision=True)
    fullsize.log("chunked build")
    t = lod.lod_build_chunked(pts, 2_000_000, params=params)
    g = t.to_host()
    t.free()
    fullsize.log("in-core build")
    dev = host.to("cuda:0")
    t = lod.lod_build(dev, params=params)
    d = t.to_host()
    t.free()
    del dev
    fullsize.log(f"{g['num_nodes']} nodes, {g['num_voxels']} voxels; comparing")
    for f in ("level", "key", "is_leaf", "npoints", "child_mask", "first_child", "count", "offset"):
        assert np.array_equal(g[f], d[f]), f
    for f in ("voxels", "voxel_ids", "voxel_points"):
        assert np.array_equal(g[f], d[f]), f
    leaf = np.nonzero(g["is_leaf"])[0]
    order = np.argsort(g["offset"][leaf], kind="stable")
    owner = np.repeat(np.arange(len(leaf), dtype=np.uint64)[order], g["count"][leaf][order].astype(np.int64))
    ka = np.sort((owner << np.uint64(32)) | g["point_ids"].astype(np.uint64))
    kb = np.sort((owner << np.uint64(32)) | d["point_ids"].astype(np.uint64))
    assert np.array_equal(ka, kb)
