"""ctypes binding of ``liblod.so`` (the C ABI in ``include/lod.h``).

Argument marshalling only: every step of the build runs in the library's HIP
kernels.  PyTorch supplies device memory and the current stream.  There is no
fallback: if the library is missing, importing the binding raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblod.so")

LOD_OK, LOD_PENDING = 0, 1
LOD_ERR_INVALID, LOD_ERR_NONFINITE, LOD_ERR_OOM, LOD_ERR_CAPACITY = -1, -2, -3, -4
LOD_ERR_TOO_LARGE, LOD_ERR_UNKNOWN_TICKET, LOD_ERR_HIP = -5, -6, -7
LOD_AVERAGE, LOD_PICK_FIRST, LOD_PICK_RANDOM, LOD_WEIGHTED = 0, 1, 2, 3
LOD_FLAG_POINT_IDS = 1
LOD_FLAG_TIMING = 2
LOD_FLAG_FULL_PRECISION = 4
LOD_FLAG_NO_GRAPH = 8
LOD_FLAG_AUTOTUNE = 16
LOD_FLAG_LOW_MEMORY = 32


class LodError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{status_str(status)}: {msg}")
        self.status = status


class lod_params(ctypes.Structure):
    _fields_ = [("leaf_cap", ctypes.c_uint32), ("max_level", ctypes.c_uint32), ("sampling", ctypes.c_uint32),
                ("seed", ctypes.c_uint32), ("flags", ctypes.c_uint32), ("tune_levels0", ctypes.c_uint32),
                ("tune_levels1", ctypes.c_uint32), ("tune_chunk", ctypes.c_uint32)]


class lod_tree_view(ctypes.Structure):
    _fields_ = [("aabb_min", ctypes.c_float * 3), ("aabb_max", ctypes.c_float * 3), ("cube_side", ctypes.c_double),
                ("num_nodes", ctypes.c_uint32), ("reserved", ctypes.c_uint32),
                ("num_points", ctypes.c_uint64), ("num_voxels", ctypes.c_uint64),
                ("node_level", ctypes.c_void_p), ("node_is_leaf", ctypes.c_void_p),
                ("node_child_mask", ctypes.c_void_p), ("node_key", ctypes.c_void_p),
                ("node_npoints", ctypes.c_void_p), ("node_count", ctypes.c_void_p),
                ("node_first_child", ctypes.c_void_p), ("node_offset", ctypes.c_void_p),
                ("points", ctypes.c_void_p), ("point_ids", ctypes.c_void_p),
                ("voxels", ctypes.c_void_p), ("voxel_ids", ctypes.c_void_p), ("voxel_points", ctypes.c_void_p)]


class lod_tune_info(ctypes.Structure):
    _fields_ = [("cached", ctypes.c_uint32), ("sample_chunks", ctypes.c_uint32), ("levels0", ctypes.c_uint32),
                ("levels1", ctypes.c_uint32), ("chunk", ctypes.c_uint32), ("best_ms", ctypes.c_float),
                ("default_ms", ctypes.c_float)]


class lod_timings(ctypes.Structure):
    _fields_ = [(name, ctypes.c_float) for name in
                ("bbox", "count0", "offsets0", "scatter0", "count1", "offsets1", "scatter1", "tree",
                 "leaf_voxels", "levels", "total")]


EXPORTED = ["lod_params_default", "lod_build", "lod_build_batch", "lod_build_noalloc", "lod_tune_batch",
            "lod_tree_view_get", "lod_tree_free",
            "lod_tree_timings",
            "lod_server_create", "lod_submit", "lod_poll", "lod_server_destroy", "lod_status_str",
            "lod_last_error"]

_lib = None
_hip = None


def load_library():
    """Load liblod.so (raises OSError if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise OSError(f"{LIB_PATH} is missing: build it with `python paper_2302_14801_amd/build.py` "
                      "(or __graft_entry__.build())")
    # PyTorch supplies the device memory and streams, so the library has to
    # run on the HIP runtime PyTorch loads: importing torch first makes the
    # library bind to that runtime instead of loading a second one, which
    # would not see the device once PyTorch's runtime holds it.
    import torch  # noqa: F401
    lib = ctypes.CDLL(LIB_PATH)
    P, vp, u32, u64 = ctypes.POINTER, ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64
    lib.lod_params_default.argtypes = [P(lod_params)]
    lib.lod_params_default.restype = None
    lib.lod_build.argtypes = [vp, u64, P(lod_params), vp, P(vp)]
    lib.lod_build.restype = ctypes.c_int
    lib.lod_build_batch.argtypes = [vp, P(u64), u32, P(lod_params), vp, P(vp)]
    lib.lod_build_batch.restype = ctypes.c_int
    lib.lod_tune_batch.argtypes = [vp, P(u64), u32, P(lod_params), vp, P(lod_params), P(lod_tune_info)]
    lib.lod_tune_batch.restype = ctypes.c_int
    lib.lod_build_noalloc.argtypes = [vp, u64, P(lod_params), vp, vp, P(u64), P(lod_tree_view)]
    lib.lod_build_noalloc.restype = ctypes.c_int
    lib.lod_build_chunked.argtypes = [vp, u64, P(lod_params), u64, vp, P(vp)]
    lib.lod_build_chunked.restype = ctypes.c_int
    lib.lod_tree_view_get.argtypes = [vp, P(lod_tree_view)]
    lib.lod_tree_view_get.restype = ctypes.c_int
    lib.lod_tree_timings.argtypes = [vp, P(lod_timings)]
    lib.lod_tree_timings.restype = ctypes.c_int
    lib.lod_tree_free.argtypes = [vp]
    lib.lod_tree_free.restype = None
    lib.lod_server_create.argtypes = [u64, u32, P(lod_params), P(vp)]
    lib.lod_server_create.restype = ctypes.c_int
    lib.lod_submit.argtypes = [vp, vp, u64, P(u64)]
    lib.lod_submit.restype = ctypes.c_int
    lib.lod_poll.argtypes = [vp, u64, P(vp)]
    lib.lod_poll.restype = ctypes.c_int
    lib.lod_server_destroy.argtypes = [vp]
    lib.lod_server_destroy.restype = None
    lib.lod_status_str.argtypes = [ctypes.c_int]
    lib.lod_status_str.restype = ctypes.c_char_p
    lib.lod_last_error.argtypes = []
    lib.lod_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def status_str(status: int) -> str:
    try:
        return load_library().lod_status_str(status).decode()
    except OSError:
        return str(status)


def _check(status: int):
    if status not in (LOD_OK, LOD_PENDING):
        raise LodError(status, load_library().lod_last_error().decode())
    return status


def make_params(leaf_cap=50000, max_level=12, sampling=LOD_AVERAGE, seed=0, keep_ids=False,
                tune_levels0=0, tune_levels1=0, timing=False, tune_chunk=0, full_precision=False,
                low_memory=False) -> lod_params:
    p = lod_params()
    load_library().lod_params_default(ctypes.byref(p))
    p.leaf_cap, p.max_level, p.sampling, p.seed = leaf_cap, max_level, sampling, seed
    p.flags = ((LOD_FLAG_POINT_IDS if keep_ids else 0) | (LOD_FLAG_TIMING if timing else 0)
               | (LOD_FLAG_FULL_PRECISION if full_precision else 0) | (LOD_FLAG_LOW_MEMORY if low_memory else 0))
    p.tune_levels0, p.tune_levels1, p.tune_chunk = tune_levels0, tune_levels1, tune_chunk
    return p


def _stream_handle(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _check_points(points):
    import torch
    if not isinstance(points, torch.Tensor) or not points.is_cuda:
        raise TypeError("points must be a device (cuda) torch tensor")
    if not points.is_contiguous() or points.numel() * points.element_size() % 16:
        raise ValueError("points must be a contiguous tensor of 16-byte records")
    return points.numel() * points.element_size() // 16


class Tree:
    """Owns an lod_tree handle; frees it with lod_tree_free."""

    def __init__(self, handle: int):
        self.handle = ctypes.c_void_p(handle)

    def view(self) -> lod_tree_view:
        v = lod_tree_view()
        _check(load_library().lod_tree_view_get(self.handle, ctypes.byref(v)))
        return v

    def timings(self) -> dict:
        t = lod_timings()
        _check(load_library().lod_tree_timings(self.handle, ctypes.byref(t)))
        return {name: float(getattr(t, name)) for name, _ in lod_timings._fields_}

    def free(self):
        if self.handle:
            load_library().lod_tree_free(self.handle)
            self.handle = ctypes.c_void_p(0)

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

    def to_host(self) -> dict:
        """Copy the tree to host numpy arrays (same keys as the oracle's result)."""
        return view_to_host(self.view())


def view_to_host(v: lod_tree_view) -> dict:
    """Copy the tree a view describes to host numpy arrays."""
    nn, nv, np_ = v.num_nodes, v.num_voxels, v.num_points
    out = {
        "aabb_min": np.array(v.aabb_min[:], np.float32), "aabb_max": np.array(v.aabb_max[:], np.float32),
        "side": v.cube_side, "num_nodes": nn, "num_points": np_, "num_voxels": nv,
        "level": _d2h(v.node_level, nn, np.uint8), "is_leaf": _d2h(v.node_is_leaf, nn, np.uint8),
        "child_mask": _d2h(v.node_child_mask, nn, np.uint8), "key": _d2h(v.node_key, nn, np.uint64),
        "npoints": _d2h(v.node_npoints, nn, np.uint32), "count": _d2h(v.node_count, nn, np.uint32),
        "first_child": _d2h(v.node_first_child, nn, np.uint32), "offset": _d2h(v.node_offset, nn, np.uint64),
        "points": _d2h(v.points, np_ * 16, np.uint8).reshape(-1, 16),
        "point_ids": _d2h(v.point_ids, np_, np.uint32) if v.point_ids else None,
        "voxels": _d2h(v.voxels, nv * 8, np.uint8).reshape(-1, 8),
        "voxel_ids": _d2h(v.voxel_ids, nv, np.uint32) if v.voxel_ids else None,
        "voxel_points": _d2h(v.voxel_points, nv * 16, np.uint8).reshape(-1, 16) if v.voxel_points else None,
    }
    return out


def _hip_lib():
    global _hip
    if _hip is None:
        for name in ("libamdhip64.so", "libamdhip64.so.7", "libamdhip64.so.6"):
            try:
                _hip = ctypes.CDLL(name)
                break
            except OSError:
                continue
        if _hip is None:
            _hip = ctypes.CDLL("/opt/rocm/lib/libamdhip64.so")
        _hip.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
        _hip.hipMemcpy.restype = ctypes.c_int
    return _hip


def _d2h(ptr, count, dtype):
    a = np.empty(int(count), dtype)
    if count and ptr:
        e = _hip_lib().hipMemcpy(a.ctypes.data, ptr, a.nbytes, 2)  # hipMemcpyDeviceToHost
        if e != 0:
            raise RuntimeError(f"hipMemcpy failed ({e})")
    return a


# ---------------------------------------------------------------- C names

def lod_build(points, leaf_cap=50000, max_level=12, sampling=LOD_AVERAGE, seed=0, keep_ids=False,
              stream=None, params: lod_params | None = None, full_precision=False) -> Tree:
    n = _check_points(points)
    p = params if params is not None else make_params(leaf_cap, max_level, sampling, seed, keep_ids,
                                                      full_precision=full_precision)
    out = ctypes.c_void_p()
    _check(load_library().lod_build(ctypes.c_void_p(points.data_ptr()), n, ctypes.byref(p),
                                    _stream_handle(stream), ctypes.byref(out)))
    return Tree(out.value)


def lod_build_noalloc(points, out, params: lod_params | None = None, stream=None, **kw):
    """Allocation-free build of `points` into the caller's device buffer `out`
    (a contiguous device tensor, 256-byte aligned; None = size query).
    Returns (view, bytes): the tree's view (device pointers into `out`) and
    the bytes of `out` it occupies (with out=None: (None, bytes needed))."""
    n = _check_points(points)
    p = params if params is not None else make_params(**kw)
    nbytes = ctypes.c_uint64(0)
    ptr = None
    if out is not None:
        if not out.is_cuda or not out.is_contiguous():
            raise ValueError("out must be a contiguous device tensor")
        nbytes.value = out.numel() * out.element_size()
        ptr = ctypes.c_void_p(out.data_ptr())
    v = lod_tree_view()
    _check(load_library().lod_build_noalloc(ctypes.c_void_p(points.data_ptr()), n, ctypes.byref(p),
                                            _stream_handle(stream), ptr, ctypes.byref(nbytes), ctypes.byref(v)))
    return (v if out is not None else None), nbytes.value


def lod_tune_batch(points, offsets, params: lod_params, stream=None):
    """(tuned lod_params, info dict) for batches like (points, offsets)."""
    _check_points(points)
    offs = np.ascontiguousarray(np.asarray(offsets, np.uint64))
    tuned, info = lod_params(), lod_tune_info()
    _check(load_library().lod_tune_batch(ctypes.c_void_p(points.data_ptr()),
                                         offs.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)), len(offs) - 1,
                                         ctypes.byref(params), _stream_handle(stream), ctypes.byref(tuned),
                                         ctypes.byref(info)))
    return tuned, {name: getattr(info, name) for name, _ in lod_tune_info._fields_}


def lod_build_batch(points, offsets, leaf_cap=50000, max_level=12, sampling=LOD_AVERAGE, seed=0,
                    keep_ids=False, stream=None, params: lod_params | None = None, full_precision=False) -> list:
    _check_points(points)
    offs = np.ascontiguousarray(np.asarray(offsets, np.uint64))
    k = len(offs) - 1
    p = params if params is not None else make_params(leaf_cap, max_level, sampling, seed, keep_ids,
                                                      full_precision=full_precision)
    outs = (ctypes.c_void_p * max(k, 1))()
    _check(load_library().lod_build_batch(ctypes.c_void_p(points.data_ptr()),
                                          offs.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)), k,
                                          ctypes.byref(p), _stream_handle(stream), outs))
    return [Tree(outs[i]) for i in range(k)]


def lod_build_chunked(host_points: np.ndarray, chunk_points: int, leaf_cap=50000, max_level=12,
                      sampling=LOD_AVERAGE, seed=0, keep_ids=False, stream=None,
                      params: lod_params | None = None, full_precision=False, low_memory=False) -> Tree:
    """The tree of a HOST array of 16-byte records, built chunk by chunk."""
    a = host_points
    if not a.flags.c_contiguous or a.nbytes % 16:
        raise ValueError("host_points must be a contiguous array of 16-byte records")
    n = a.nbytes // 16
    p = params if params is not None else make_params(leaf_cap, max_level, sampling, seed, keep_ids,
                                                      full_precision=full_precision, low_memory=low_memory)
    out = ctypes.c_void_p()
    _check(load_library().lod_build_chunked(ctypes.c_void_p(a.ctypes.data if n else 0), n, ctypes.byref(p),
                                            int(chunk_points), _stream_handle(stream), ctypes.byref(out)))
    return Tree(out.value)


def lod_tree_view_get(tree: Tree) -> lod_tree_view:
    return tree.view()


def lod_tree_free(tree: Tree):
    tree.free()


class Server:
    def __init__(self, hbm_budget_bytes: int, max_inflight: int = 4, params: lod_params | None = None, **kw):
        p = params if params is not None else make_params(**kw)
        self.handle = ctypes.c_void_p()
        _check(load_library().lod_server_create(hbm_budget_bytes, max_inflight, ctypes.byref(p),
                                                ctypes.byref(self.handle)))

    def submit(self, host_points: np.ndarray) -> int:
        a = host_points
        if not a.flags.c_contiguous or a.dtype.itemsize * (a.size // max(len(a), 1)) % 16:
            raise ValueError("host_points must be a contiguous array of 16-byte records")
        n = a.nbytes // 16
        t = ctypes.c_uint64()
        _check(load_library().lod_submit(self.handle, ctypes.c_void_p(a.ctypes.data), n, ctypes.byref(t)))
        return t.value

    def poll(self, ticket: int):
        out = ctypes.c_void_p()
        st = _check(load_library().lod_poll(self.handle, ticket, ctypes.byref(out)))
        if st == LOD_PENDING:
            return None
        return Tree(out.value)

    def destroy(self):
        if self.handle:
            load_library().lod_server_destroy(self.handle)
            self.handle = ctypes.c_void_p(0)

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def lod_server_create(hbm_budget_bytes: int, max_inflight: int = 4, **kw) -> Server:
    return Server(hbm_budget_bytes, max_inflight, **kw)


def lod_submit(server: Server, host_points: np.ndarray) -> int:
    return server.submit(host_points)


def lod_poll(server: Server, ticket: int):
    return server.poll(ticket)


def lod_server_destroy(server: Server):
    server.destroy()
