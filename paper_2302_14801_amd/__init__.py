"""MI355X (gfx950) builder of the hybrid voxel-point layered-point-cloud octree
of Schuetz, Kerbl, Klaus, Wimmer, "GPU-Accelerated LOD Generation for Point
Clouds" (arXiv 2302.14801).

The work runs in ``liblod.so`` (hand-written HIP kernels behind the C ABI in
``include/lod.h``); this package is a thin ctypes binding with the same names.
Importing it loads the library and raises if it has not been built.
"""
from .binding import (LOD_AVERAGE, LOD_FLAG_AUTOTUNE, LOD_FLAG_FULL_PRECISION, LOD_FLAG_LOW_MEMORY,
                      LOD_FLAG_NO_GRAPH,  # noqa: F401
                      LOD_PICK_FIRST,
                      LOD_PICK_RANDOM, LOD_WEIGHTED,
                      LodError, Server, Tree,
                      load_library, lod_build, lod_build_batch, lod_build_chunked, lod_build_noalloc, lod_poll,
                      lod_server_create, lod_server_destroy, lod_submit, lod_tree_free, lod_tree_view_get,
                      lod_tune_batch, make_params, view_to_host)

load_library()
