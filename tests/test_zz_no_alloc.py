"""The allocation-free build (lod_build_noalloc) through the C ABI: its trees
equal lod_build's (node tables and voxel lists exactly, leaf point multisets)
on calls in a row that share the library's static scratch, the later ones
smaller; an output buffer too small for the voxels is reported with the size
it needs."""
from __future__ import annotations

import ctypes

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


def noalloc(lod, dev, n, p, out):
    """One call through the C ABI; (status, bytes, view)."""
    import torch
    from paper_2302_14801_amd import binding
    lib = binding.load_library()
    nbytes = ctypes.c_uint64(out.numel() if out is not None else 0)
    v = binding.lod_tree_view()
    st = lib.lod_build_noalloc(ctypes.c_void_p(dev.data_ptr()), n, ctypes.byref(p),
                               ctypes.c_void_p(torch.cuda.current_stream().cuda_stream),
                               ctypes.c_void_p(out.data_ptr()) if out is not None else None,
                               ctypes.byref(nbytes), ctypes.byref(v))
    return st, nbytes.value, v


def reference(lod, dev, **kw):
    t = lod.lod_build(dev, keep_ids=True, **kw)
    h = t.to_host()
    t.free()
    return h


def check_call(lod, pts, out, **kw):
    import torch
    from paper_2302_14801_amd import binding
    n = len(pts)
    print(f"noalloc case n={n} {kw}", flush=True)
    dev = to_dev(pts)
    p = lod.make_params(**kw)
    st, used, v = noalloc(lod, dev, n, p, out)
    assert st == 0, binding.load_library().lod_last_error()
    torch.cuda.synchronize()
    g = binding.view_to_host(v)
    assert used <= out.numel()
    ref = reference(lod, dev, **kw)
    canon.compare_trees(g, ref, pts)
    assert np.array_equal(g["offset"], ref["offset"])
    assert np.array_equal(g["voxels"], ref["voxels"])
    for k in ("voxel_ids", "voxel_points"):
        if ref.get(k) is not None:
            assert g.get(k) is not None and np.array_equal(g[k], ref[k]), k
    return g


def test_noalloc_equals_build_on_calls_in_a_row(lod):
    import torch
    out = torch.empty(160 << 20, dtype=torch.uint8, device="cuda:0")
    big = synth.terrain(1_000_000, seed=1)
    g1 = check_call(lod, big, out, leaf_cap=50000, max_level=12)
    small = synth.aerial(200_000, seed=3)
    g2 = check_call(lod, small, out, leaf_cap=5000, max_level=12)
    # the smaller call against the oracle as well
    canon.compare_trees(g2, oracle.build(small, leaf_cap=5000, max_level=12), small)
    # the first call's input again: the same tree as the first time
    g3 = check_call(lod, big, out, leaf_cap=50000, max_level=12)
    for k in canon.NODE_FIELDS:
        assert np.array_equal(g1[k], g3[k]), k
    assert np.array_equal(g1["voxels"], g3["voxels"])


@pytest.mark.parametrize("sampling", [1, 2])
def test_noalloc_pick_full_precision_in_a_row(lod, sampling):
    import torch
    out = torch.empty(64 << 20, dtype=torch.uint8, device="cuda:0")
    check_call(lod, synth.aerial(300_000, seed=11), out, leaf_cap=4000, max_level=12, sampling=sampling, seed=5,
               full_precision=True)
    check_call(lod, synth.terrain(40_000, seed=12), out, leaf_cap=1000, max_level=10, sampling=sampling, seed=5,
               full_precision=True)


def test_noalloc_reports_the_size_the_voxels_need(lod):
    import torch
    from paper_2302_14801_amd import binding
    pts = synth.aerial(120_000, seed=9)
    dev = to_dev(pts)
    p = lod.make_params(leaf_cap=3000, max_level=12)
    st, query, _ = noalloc(lod, dev, len(pts), p, None)
    assert st == 0 and query > 0
    # room for the points and nodes but only a few voxels
    ref = reference(lod, dev, leaf_cap=3000, max_level=12)
    fixed = query - 8 * (len(pts) + 64)
    small = torch.empty((fixed + 8 * 100 + 4095) // 4096 * 4096, dtype=torch.uint8, device="cuda:0")
    st, need, _ = noalloc(lod, dev, len(pts), p, small)
    assert st == binding.LOD_ERR_CAPACITY
    assert need >= fixed + 8 * ref["num_voxels"]
    exact = torch.empty(need, dtype=torch.uint8, device="cuda:0")
    st, used, v = noalloc(lod, dev, len(pts), p, exact)
    assert st == 0 and used <= need
    g = binding.view_to_host(v)
    assert g["num_voxels"] == ref["num_voxels"] and np.array_equal(g["voxels"], ref["voxels"])


def test_noalloc_empty_input(lod):
    import torch
    from paper_2302_14801_amd import binding
    out = torch.empty(1 << 20, dtype=torch.uint8, device="cuda:0")
    dev = torch.empty(16, dtype=torch.uint8, device="cuda:0")
    st, used, v = noalloc(lod, dev, 0, lod.make_params(), out)
    assert st == 0 and used == 0 and v.num_nodes == 0
    assert binding.view_to_host(v)["num_voxels"] == 0
