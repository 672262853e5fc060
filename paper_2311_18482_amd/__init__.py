"""MI355X-native splatting and decoding for Language Embedded 3D Gaussians
(arXiv 2311.18482): HIP kernels for gfx950 behind the C ABI in include/legs.h,
with a thin ctypes binding.
"""
from . import _lib  # noqa: F401

__all__ = ["_lib", "raster"]
