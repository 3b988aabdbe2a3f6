"""MI355X-native exact mesh-to-mesh min/max distance (gDist hot path).

The compute path lives in libgdist.so (HIP for gfx950, C ABI in
include/gdist.h); ``gdist`` is its ctypes binding.  Importing the package does
not load the library; the first call does, and fails loudly if it is missing.
"""
from . import gdist  # noqa: F401
from .gdist import Context, GdistError  # noqa: F401

__all__ = ["gdist", "Context", "GdistError"]
