"""RA-FEAST on AMD MI355X (gfx950): randomized warmstart + FEAST with
matrix-free COCG shifted solves, behind the C ABI of include/rafeast.h.

``native`` is the ctypes binding of librafeast.so; the library is built by
``paper_2512_01257_amd.build.build()``.
"""

from . import native  # noqa: F401
from .native import Plan, RafeastError  # noqa: F401
