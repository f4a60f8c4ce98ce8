"""Seeded synthetic point clouds (inputs only; none of the octree arithmetic).

Shared by the oracle side (tests, CPU baseline) and the GPU side (tests,
bench): one buffer is generated and handed to both.  The generators are
counter-based (SplitMix64 of (seed, stream, index)), so a slice of a cloud can
be produced without generating what precedes it, and output is identical for
any thread count.

Workloads (stand-ins for the paper's aerial and terrestrial scans, Sec. 6):
  * ``terrain``  -- heightfield of 4 sine octaves, uniform xy, colour from a
    height ramp plus noise (1M-point plain build on a 100 x 100 m box)
  * ``aerial``   -- 1 x 1 km scene: 70% terrain, 20% box buildings (roofs and
    walls), 10% Gaussian vegetation blobs (100M-point plain build)
  * ``scan``     -- 50 m box of spheres and rectangles with 1 mm surface noise
    (terrestrial-scan-like, 2B-point plain build)
  * ``batch_chunks`` -- many independent terrain+buildings tiles of lognormal
    size, each with its own bounding box (batched builds)
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

POINT_DTYPE = np.dtype([("x", "<f4"), ("y", "<f4"), ("z", "<f4"),
                        ("r", "u1"), ("g", "u1"), ("b", "u1"), ("a", "u1")])
assert POINT_DTYPE.itemsize == 16

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libsynth.so")
_SRC = os.path.join(_HERE, "synth.c")


def build_library() -> str:
    cmd = ["gcc", "-O2", "-std=c99", "-fopenmp", "-ffp-contract=off", "-shared", "-fPIC",
           "-o", _SO, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    return _SO


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
            build_library()
        lib = ctypes.CDLL(_SO)
        d, i, u64, vp = ctypes.c_double, ctypes.c_int, ctypes.c_uint64, ctypes.c_void_p
        lib.synth_tile.argtypes = [u64, d, d, d, d, d, d, i, d, i, u64, u64, vp]
        lib.synth_scan.argtypes = [u64, d, i, i, u64, u64, vp]
        lib.synth_uniform.argtypes = [u64, u64, u64, u64, vp]
        lib.synth_normal.argtypes = [u64, u64, u64, u64, vp]
        _lib = lib
    return _lib


def _out(n: int, out):
    if out is None:
        return np.empty(n, POINT_DTYPE)
    if out.dtype.itemsize != 16 or out.shape[0] < n or not out.flags.c_contiguous:
        raise ValueError("out must be a contiguous array of >= n 16-byte records")
    return out


def tile(n: int, seed: int, *, origin=(0.0, 0.0), side=100.0, amp=10.0, wavelength=100.0,
         f_building=0.0, n_buildings=0, f_veg=0.0, n_blobs=0, first: int = 0, out=None) -> np.ndarray:
    """Points [first, first + n) of a terrain/buildings/vegetation tile."""
    a = _out(n, out)
    if n:
        _load().synth_tile(seed, float(origin[0]), float(origin[1]), float(side), float(amp), float(wavelength),
                           float(f_building), int(n_buildings), float(f_veg), int(n_blobs), first, n,
                           a.ctypes.data)
    return a[:n]


def terrain(n: int = 1_000_000, seed: int = 1, out=None, first: int = 0) -> np.ndarray:
    """Heightfield on 100 x 100 m: A = 10 m, lambda = 100 m."""
    return tile(n, seed, side=100.0, amp=10.0, wavelength=100.0, first=first, out=out)


def aerial(n: int = 100_000_000, seed: int = 2, out=None, first: int = 0) -> np.ndarray:
    """1 x 1 km aerial scene: 70% terrain (A = 40 m, lambda = 1 km), 20% on 200
    box buildings, 10% in 2000 Gaussian vegetation blobs (sigma 2 m)."""
    return tile(n, seed, side=1000.0, amp=40.0, wavelength=1000.0, f_building=0.2, n_buildings=200,
                f_veg=0.1, n_blobs=2000, first=first, out=out)


def scan(n: int, seed: int = 3, out=None, first: int = 0) -> np.ndarray:
    """50 m box, 32 spheres + 32 rectangles, 1 mm Gaussian noise along the normal."""
    a = _out(n, out)
    if n:
        _load().synth_scan(seed, 50.0, 32, 32, first, n, a.ctypes.data)
    return a[:n]


def uniform(seed: int, stream: int, count: int, first: int = 0) -> np.ndarray:
    out = np.empty(count, np.float64)
    if count:
        _load().synth_uniform(seed, stream, first, count, out.ctypes.data)
    return out


def normal(seed: int, stream: int, count: int, first: int = 0) -> np.ndarray:
    out = np.empty(count, np.float64)
    if count:
        _load().synth_normal(seed, stream, first, count, out.ctypes.data)
    return out


def chunk_sizes(num_chunks: int = 512, seed: int = 4, median: float = 1e6, sigma: float = 0.5,
                lo: int = 10_000, hi: int = 20_000_000) -> np.ndarray:
    """Lognormal chunk sizes, clipped to [lo, hi]."""
    z = normal(seed, 900, num_chunks)
    s = np.rint(np.exp(math.log(median) + sigma * z))
    return np.clip(s, lo, hi).astype(np.int64)


def batch_chunks(sizes, seed: int = 4, out=None):
    """Concatenated independent tiles (terrain 7/9 + buildings 2/9), about
    100 points per square metre, tile i placed at (1000 (i mod 32), 1000 (i div 32)).
    Returns (points, offsets) with offsets of length len(sizes) + 1."""
    sizes = np.asarray(sizes, np.int64)
    offs = np.zeros(len(sizes) + 1, np.int64)
    offs[1:] = np.cumsum(sizes)
    a = _out(int(offs[-1]), out)
    for i, n in enumerate(sizes):
        n = int(n)
        side = 100.0 * math.sqrt(n / 1e6)
        nb = max(1, int(round(20 * n / 1e6)))
        tile(n, seed * 100003 + i, origin=(1000.0 * (i % 32), 1000.0 * (i // 32)), side=side, amp=10.0,
             wavelength=100.0, f_building=2.0 / 9.0, n_buildings=nb, out=a[offs[i]:offs[i + 1]])
    return a[:offs[-1]], offs


def serve_tile(n: int, seed: int, out=None) -> np.ndarray:
    """First n points of a 50M-point tile of the batch generator (terrain 7/9
    + buildings 2/9, 100 points per square metre, 707 m side).  Components
    interleave at random, so any prefix is a uniform subsample of the tile."""
    full = 50_000_000
    side = 100.0 * math.sqrt(full / 1e6)
    return tile(n, seed, side=side, amp=10.0, wavelength=100.0, f_building=2.0 / 9.0,
                n_buildings=int(round(20 * full / 1e6)), out=out)


def uniform_cloud(n: int, seed: int, lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0), colors: bool = True) -> np.ndarray:
    """Small uniform random cloud for tests (numpy only)."""
    rng = np.random.default_rng(seed)
    a = np.empty(n, POINT_DTYPE)
    for k, ax in enumerate("xyz"):
        a[ax] = rng.uniform(lo[k], hi[k], n).astype(np.float32)
    if colors:
        for ax in "rgb":
            a[ax] = rng.integers(0, 256, n, dtype=np.uint8)
    else:
        for ax in "rgb":
            a[ax] = 128
    a["a"] = rng.integers(0, 256, n, dtype=np.uint8) if colors else 255
    return a
