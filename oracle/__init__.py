"""CPU oracle for the hybrid voxel-point octree (arXiv 2302.14801, Sec. 3-4).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The GPU product
path (``paper_2302_14801_amd``) never imports it, and the two share no code.

The arithmetic lives in ``lod_oracle.c`` (plain single-threaded C, see its
header comment for the step-by-step citations); this module only marshals
numpy arrays through ctypes.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liblod_oracle.so")
_SRC = os.path.join(_HERE, "lod_oracle.c")

AVERAGE, FIRST, RANDOM, WEIGHTED = 0, 1, 2, 3
OK, ERR_INVALID, ERR_NONFINITE, ERR_OOM = 0, -1, -2, -3


class OracleError(RuntimeError):
    def __init__(self, status: int):
        super().__init__(f"oracle status {status}")
        self.status = status


def build_library() -> str:
    """Compile the oracle with the host C compiler (no GPU code involved)."""
    cmd = ["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-shared", "-fPIC",
           "-o", _SO, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    return _SO


class _Tree(ctypes.Structure):
    _fields_ = [
        ("aabb_min", ctypes.c_float * 3), ("aabb_max", ctypes.c_float * 3),
        ("side", ctypes.c_double), ("scale", ctypes.c_double),
        ("num_nodes", ctypes.c_uint32),
        ("level", ctypes.POINTER(ctypes.c_uint8)),
        ("is_leaf", ctypes.POINTER(ctypes.c_uint8)),
        ("child_mask", ctypes.POINTER(ctypes.c_uint8)),
        ("key", ctypes.POINTER(ctypes.c_uint64)),
        ("npoints", ctypes.POINTER(ctypes.c_uint32)),
        ("count", ctypes.POINTER(ctypes.c_uint32)),
        ("first_child", ctypes.POINTER(ctypes.c_uint32)),
        ("offset", ctypes.POINTER(ctypes.c_uint64)),
        ("num_points", ctypes.c_uint64),
        ("point_ids", ctypes.POINTER(ctypes.c_uint32)),
        ("num_voxels", ctypes.c_uint64),
        ("voxels", ctypes.POINTER(ctypes.c_uint8)),
        ("voxel_ids", ctypes.POINTER(ctypes.c_uint32)),
    ]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
            build_library()
        lib = ctypes.CDLL(_SO)
        vp, u64, u32 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32
        lib.lod_oracle_build.argtypes = [vp, u64, u32, u32, ctypes.c_int, u32, ctypes.POINTER(_Tree)]
        lib.lod_oracle_build.restype = ctypes.c_int
        lib.lod_oracle_free.argtypes = [ctypes.POINTER(_Tree)]
        lib.lod_oracle_cube.argtypes = [vp, u64, ctypes.c_float * 3, ctypes.c_float * 3,
                                        ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
        lib.lod_oracle_cube.restype = ctypes.c_int
        lib.lod_oracle_keys.argtypes = [vp, u64, vp]
        lib.lod_oracle_keys.restype = ctypes.c_int
        f3 = ctypes.c_float * 3
        lib.lod_oracle_build_in_cube.argtypes = [vp, u64, u32, u32, ctypes.c_int, u32, f3, ctypes.c_double,
                                                 ctypes.POINTER(_Tree)]
        lib.lod_oracle_build_in_cube.restype = ctypes.c_int
        lib.lod_oracle_keys_in_cube.argtypes = [vp, u64, f3, ctypes.c_double, vp]
        lib.lod_oracle_keys_in_cube.restype = ctypes.c_int
        lib.lod_oracle_hash.argtypes = [u32, u32]
        lib.lod_oracle_hash.restype = u32
        _lib = lib
    return _lib


def _as_records(points) -> np.ndarray:
    a = np.ascontiguousarray(points)
    if a.dtype.itemsize != 16 and not (a.ndim == 2 and a.shape[1] == 16 and a.dtype == np.uint8):
        raise ValueError("points must be 16-byte records (float32 x, y, z; uint8 r, g, b, a)")
    return a


def _arr(ptr, n, dtype):
    if n == 0 or not ptr:
        return np.zeros(0, dtype=dtype)
    return np.ctypeslib.as_array(ptr, shape=(n,)).copy().astype(dtype, copy=False)


def cube(points):
    """Steps 2-3: (aabb_min, aabb_max, side, scale)."""
    a = _as_records(points)
    n = a.shape[0]
    lo, hi = (ctypes.c_float * 3)(), (ctypes.c_float * 3)()
    side, scale = ctypes.c_double(), ctypes.c_double()
    st = _load().lod_oracle_cube(a.ctypes.data, n, lo, hi, ctypes.byref(side), ctypes.byref(scale))
    if st:
        raise OracleError(st)
    return np.array(lo[:], np.float32), np.array(hi[:], np.float32), side.value, scale.value


def keys(points) -> np.ndarray:
    """Steps 4-5: the 63-bit Morton key of every point."""
    a = _as_records(points)
    out = np.zeros(a.shape[0], np.uint64)
    st = _load().lod_oracle_keys(a.ctypes.data, a.shape[0], out.ctypes.data)
    if st:
        raise OracleError(st)
    return out


def keys_in_cube(points, lo, side: float) -> np.ndarray:
    """Morton keys of the points in a given cube (minimum corner lo, edge side)."""
    a = _as_records(points)
    out = np.zeros(a.shape[0], np.uint64)
    lo3 = (ctypes.c_float * 3)(*[float(v) for v in lo])
    st = _load().lod_oracle_keys_in_cube(a.ctypes.data, a.shape[0], lo3, float(side), out.ctypes.data)
    if st:
        raise OracleError(st)
    return out


def point_hash(ids, seed: int) -> np.ndarray:
    """32-bit hash used by the RANDOM pick (SplitMix64 output, high half)."""
    lib = _load()
    return np.array([lib.lod_oracle_hash(int(i), int(seed)) for i in np.asarray(ids).ravel()], np.uint32)


def build(points, leaf_cap: int = 50000, max_level: int = 12, sampling: int = AVERAGE, seed: int = 0,
          cube_lo=None, cube_side: float | None = None, full_precision: bool = False) -> dict:
    """Build the octree; returns numpy arrays (see lod_oracle.h for meaning).
    With cube_lo/cube_side the cube is given instead of computed from the points.
    full_precision adds "voxel_ids" and "voxel_points" (see full_precision_points)."""
    t = _build(points, leaf_cap, max_level, sampling, seed, cube_lo, cube_side)
    if full_precision:
        t = full_precision_points(points, t, leaf_cap, max_level, sampling, seed, cube_lo, cube_side)
    return t


def full_precision_points(points, tree: dict, leaf_cap: int, max_level: int, sampling: int, seed: int,
                          cube_lo=None, cube_side: float | None = None) -> dict:
    """Full-precision samples of the lower levels (Sec. 7, Discussion).

    The pick modes keep the picked point itself: its input coordinates, with
    quantization switched off.  For the (weighted) average, the cell's accepted sample
    is the one a first-come pass accepts (Sec. 4.2.1, made order-independent
    as the smallest input index), and the record takes its coordinates with
    the averaged colour.  The first-come voxel ids are those of the same tree
    built with FIRST sampling (same nodes, same occupied cells).  Returns the
    tree with "voxel_ids" and "voxel_points" ((num_voxels, 16) uint8 records
    x, y, z float32 and r, g, b, a of the voxel)."""
    raw = _as_records(points).view(np.uint8).reshape(-1, 16)
    out = dict(tree)
    if sampling in (AVERAGE, WEIGHTED):
        first = _build(points, leaf_cap, max_level, FIRST, seed, cube_lo, cube_side)
        assert first["num_voxels"] == tree["num_voxels"]
        ids = first["voxel_ids"]
    else:
        ids = tree["voxel_ids"]
    if ids is None:
        ids = np.zeros(0, np.uint32)
    rec = raw[ids.astype(np.int64)].copy() if len(ids) else np.zeros((0, 16), np.uint8)
    rec[:, 12:16] = tree["voxels"][:, 4:8]
    out["voxel_ids"] = ids
    out["voxel_points"] = rec
    return out


def _build(points, leaf_cap, max_level, sampling, seed, cube_lo, cube_side) -> dict:
    a = _as_records(points)
    n = a.shape[0]
    t = _Tree()
    if cube_lo is not None:
        lo3 = (ctypes.c_float * 3)(*[float(v) for v in cube_lo])
        st = _load().lod_oracle_build_in_cube(a.ctypes.data if n else None, n, leaf_cap, max_level, sampling,
                                              seed, lo3, float(cube_side), ctypes.byref(t))
    else:
        st = _load().lod_oracle_build(a.ctypes.data if n else None, n, leaf_cap, max_level, sampling, seed,
                                      ctypes.byref(t))
    if st:
        _load().lod_oracle_free(ctypes.byref(t))
        raise OracleError(st)
    try:
        nn = t.num_nodes
        res = {
            "aabb_min": np.array(t.aabb_min[:], np.float32),
            "aabb_max": np.array(t.aabb_max[:], np.float32),
            "side": t.side, "scale": t.scale,
            "num_nodes": nn,
            "level": _arr(t.level, nn, np.uint8),
            "is_leaf": _arr(t.is_leaf, nn, np.uint8),
            "child_mask": _arr(t.child_mask, nn, np.uint8),
            "key": _arr(t.key, nn, np.uint64),
            "npoints": _arr(t.npoints, nn, np.uint32),
            "count": _arr(t.count, nn, np.uint32),
            "first_child": _arr(t.first_child, nn, np.uint32),
            "offset": _arr(t.offset, nn, np.uint64),
            "num_points": t.num_points,
            "point_ids": _arr(t.point_ids, t.num_points, np.uint32),
            "num_voxels": t.num_voxels,
            "voxels": _arr(t.voxels, 8 * t.num_voxels, np.uint8).reshape(-1, 8),
            "voxel_ids": _arr(t.voxel_ids, t.num_voxels, np.uint32) if t.voxel_ids else None,
        }
    finally:
        _load().lod_oracle_free(ctypes.byref(t))
    return res
