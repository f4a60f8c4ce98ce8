"""GPU parity at the benchmark's full size: the 100M-point aerial plain build
(T = 50 000, 128^3, colour-filtered), built exactly as bench.py builds it, and
checked by the properties and sampled oracle subtrees of fullsize.py."""
from __future__ import annotations

import pytest

import fullsize
import synth

pytestmark = pytest.mark.gpu

N = 100_000_000
T = 50_000
ML = 12


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
