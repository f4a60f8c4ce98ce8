"""The C ABI library loads and exports every entry point that include/lod.h
declares; host-only argument checks (no GPU work) behave as documented."""
from __future__ import annotations

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lod.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lod_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_2302_14801_amd import binding
    return binding.load_library()


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert "lod_build" in names and "lod_build_batch" in names and "lod_submit" in names and "lod_poll" in names
    for name in names:
        assert hasattr(lib, name), f"{name} declared in lod.h but not exported"


def test_params_default_and_status_strings(lib):
    from paper_2302_14801_amd import binding
    p = binding.lod_params()
    lib.lod_params_default(ctypes.byref(p))
    assert (p.leaf_cap, p.max_level, p.sampling) == (50000, 12, 0)
    for st in range(-7, 2):
        assert lib.lod_status_str(st).decode().startswith("LOD_")


def test_argument_errors_before_any_device_work(lib):
    from paper_2302_14801_amd import binding
    p = binding.lod_params()
    lib.lod_params_default(ctypes.byref(p))
    out = ctypes.c_void_p()
    assert lib.lod_build(None, 10, ctypes.byref(p), None, ctypes.byref(out)) == binding.LOD_ERR_INVALID
    assert lib.lod_build(None, 0, ctypes.byref(p), None, None) == binding.LOD_ERR_INVALID
    p.leaf_cap = 0
    assert lib.lod_build(None, 0, ctypes.byref(p), None, ctypes.byref(out)) == binding.LOD_ERR_INVALID
    p.leaf_cap, p.max_level = 10, 15
    assert lib.lod_build(None, 0, ctypes.byref(p), None, ctypes.byref(out)) == binding.LOD_ERR_INVALID
    p.max_level = 12
    assert lib.lod_server_create(0, 1, ctypes.byref(p), ctypes.byref(out)) == binding.LOD_ERR_INVALID
    assert lib.lod_poll(None, 1, ctypes.byref(out)) == binding.LOD_ERR_INVALID
    assert b"invalid" in lib.lod_last_error()


def test_chunked_argument_errors_before_any_device_work(lib):
    from paper_2302_14801_amd import binding
    p = binding.lod_params()
    lib.lod_params_default(ctypes.byref(p))
    out = ctypes.c_void_p()
    assert lib.lod_build_chunked(None, 0, ctypes.byref(p), 10, None, None) == binding.LOD_ERR_INVALID
    assert lib.lod_build_chunked(None, 10, ctypes.byref(p), 10, None, ctypes.byref(out)) == binding.LOD_ERR_INVALID
    assert lib.lod_build_chunked(None, 0, ctypes.byref(p), 0, None, ctypes.byref(out)) == binding.LOD_ERR_INVALID
    p.sampling = 4
    assert lib.lod_build_chunked(None, 0, ctypes.byref(p), 10, None, ctypes.byref(out)) == binding.LOD_ERR_INVALID
    p.sampling, p.max_level = binding.LOD_AVERAGE, 15
    assert lib.lod_build_chunked(None, 0, ctypes.byref(p), 10, None, ctypes.byref(out)) == binding.LOD_ERR_INVALID
    assert out.value is None


def test_package_refuses_to_import_without_library(tmp_path, monkeypatch):
    from paper_2302_14801_amd import binding
    monkeypatch.setattr(binding, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(binding, "_lib", None)
    with pytest.raises(OSError):
        binding.load_library()


@pytest.mark.parametrize("name", ["lod_params", "lod_tree_view", "lod_timings"])
def test_struct_layouts_match_header(name, tmp_path):
    """The binding's ctypes mirrors have the C compiler's sizes and offsets."""
    import shutil
    import subprocess
    from paper_2302_14801_amd import binding
    if shutil.which("gcc") is None:
        pytest.skip("no C compiler")
    cls = getattr(binding, name)
    fields = [f for f, _ in cls._fields_]
    src = tmp_path / "layout.c"
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "lod.h"', "int main(void) {",
             f'  printf("%zu\\n", sizeof({name}));']
    lines += [f'  printf("%zu\\n", offsetof({name}, {f}));' for f in fields]
    lines += ["  return 0;", "}"]
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()]
    assert got[0] == ctypes.sizeof(cls)
    for f, off in zip(fields, got[1:]):
        assert getattr(cls, f).offset == off, f


def test_binding_constants_match_header():
    """Sampling modes, flags and status codes of the binding are the header's."""
    from paper_2302_14801_amd import binding
    text = open(HEADER).read()
    want = {name: int(val) for name, val in re.findall(r"\b(LOD_[A-Z_]+)\s*=\s*(-?\d+)", text)}
    for name in ("LOD_AVERAGE", "LOD_PICK_FIRST", "LOD_PICK_RANDOM", "LOD_WEIGHTED", "LOD_FLAG_POINT_IDS",
                 "LOD_FLAG_TIMING", "LOD_FLAG_FULL_PRECISION", "LOD_ERR_INVALID"):
        assert getattr(binding, name) == want[name], name


def test_one_hip_runtime_whatever_the_import_order():
    """The library must run on the HIP runtime that PyTorch loads (PyTorch
    supplies its device memory and streams): importing the package before
    torch must not bring in a second runtime, which would find no device."""
    import subprocess
    import sys
    code = ("import paper_2302_14801_amd, torch\n"
            "from paper_2302_14801_amd import binding\n"
            "binding._hip_lib()\n"
            "libs = {l.split()[-1] for l in open('/proc/self/maps') if 'libamdhip64' in l}\n"
            "print(len(libs))\n")
    out = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stderr
    assert out.stdout.strip().splitlines()[-1] == "1"


def test_build_entry_does_not_need_a_built_library():
    """build() reaches the build script without importing the package (which
    refuses to import before liblod.so exists), so a clean tree builds."""
    import subprocess
    import sys
    code = ("import sys, __graft_entry__ as g\n"
            "m = g._builder()\n"
            "assert callable(m.build) and m.LIB.endswith('liblod.so')\n"
            "assert 'paper_2302_14801_amd' not in sys.modules\n"
            "print('ok')\n")
    out = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stderr
    assert out.stdout.strip().endswith("ok")


def test_noalloc_host_checks_before_any_device_work(lib):
    """The allocation-free build refuses inputs its static scratch cannot
    hold, and the weighted average, before touching the device; a NULL
    output buffer is a size query."""
    from paper_2302_14801_amd import binding
    p = binding.lod_params()
    lib.lod_params_default(ctypes.byref(p))
    fake = ctypes.c_void_p(1 << 20)  # never dereferenced by these calls
    nbytes, v = ctypes.c_uint64(0), binding.lod_tree_view()
    assert lib.lod_build_noalloc(fake, 10_000_000, ctypes.byref(p), None, None, ctypes.byref(nbytes),
                                 ctypes.byref(v)) == binding.LOD_ERR_TOO_LARGE
    assert b"LOD_NOALLOC_SCRATCH_BYTES" in lib.lod_last_error()
    assert lib.lod_build_noalloc(fake, 1_000_000, ctypes.byref(p), None, None, ctypes.byref(nbytes),
                                 ctypes.byref(v)) == binding.LOD_OK
    # points (16 B), node tables and room for n + 64 voxels (8 B)
    assert nbytes.value >= 16 * 1_000_000 + 8 * 1_000_064
    assert lib.lod_build_noalloc(fake, 1_000_000, ctypes.byref(p), None, None, None,
                                 ctypes.byref(v)) == binding.LOD_ERR_INVALID
    p.sampling = binding.LOD_WEIGHTED
    assert lib.lod_build_noalloc(fake, 1000, ctypes.byref(p), None, None, ctypes.byref(nbytes),
                                 ctypes.byref(v)) == binding.LOD_ERR_INVALID
