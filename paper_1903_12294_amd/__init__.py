"""mf4d: coupled point + field 4D region growing on AMD Instinct MI355X (gfx950).

The work runs in libmf4d.so (hand-written HIP kernels behind the C ABI of
include/mf4d.h); this package is its Python binding, its build script and the
seeded input generator.
"""
from ._lib import LibraryMissing, MF4DError, load_library  # noqa: F401
from .grower import Grower  # noqa: F401

__all__ = ["Grower", "MF4DError", "LibraryMissing", "load_library"]
