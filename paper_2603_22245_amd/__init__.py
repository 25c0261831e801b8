"""RotorMap's hot path on AMD MI355X (gfx950).

The work runs in librotormap.so (hand-written HIP kernels behind a C ABI,
include/rotormap.h).  `_lib` binds its entry points with ctypes; `mapper`
allocates device buffers with torch and calls them in order.
"""
from . import _lib  # noqa: F401
from ._lib import RotorMapError, make_params  # noqa: F401
