"""MI355X-native staggered-grid P_N solver (StaRMAP scheme, arXiv 1211.2205).

The compute path is the gfx950 shared library libstarmap.so (HIP kernels
behind a C ABI, include/starmap.h); this package is its Python binding.
"""
from ._binding import LIB_PATH, StarmapError, lib  # noqa: F401
from .solver import (MLP, Batch, Solver, closure_pn, direction_moments, moment_info,  # noqa: F401
                     num_moments, spectral_radius, variant_count)
