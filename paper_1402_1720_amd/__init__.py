"""Proton-CT hull detection on AMD Instinct MI355X (gfx950).

The HIP library ``libhullmi.so`` (C ABI in ``include/hullmi.h``) runs the whole
hull path: classification, FP32 object-frame geometry, the exact integer voxel
walk, the SC/MSC/SM counts and rules, and the FDK hull. ``hullmi`` is its thin
ctypes binding; torch supplies device memory and streams.
"""
from . import hullmi  # noqa: F401
from .hullmi import (Histories, HullError, hull_abi_version, hull_all, hull_count_lines,  # noqa: F401
                     hull_fbp, hull_msc, hull_quantize, hull_sc, hull_sm, hull_strerror,
                     hull_workspace_bytes, make_fbp_params, make_grid, make_params)
