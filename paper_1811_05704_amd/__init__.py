"""MI355X (gfx950) smoothed-aggregation AMG: solve phase in HIP kernels.

The C ABI is declared in ``include/amg.h``; :mod:`paper_1811_05704_amd.amg`
binds it with ctypes.  Build the shared library with
``python -m paper_1811_05704_amd.build``.
"""

from . import amg  # noqa: F401
