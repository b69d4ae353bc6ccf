"""GF2 on MI355X: the self-energy hot path of self-consistent second-order
Green's function theory (Phillips & Zgid, arXiv:1405.3273) as hand-written
HIP kernels for gfx950 behind a C ABI (include/gf2.h, libgf2.so).

``paper_1405_3273_amd.runtime.Gf2`` drives the library with torch device
tensors; ``paper_1405_3273_amd._lib`` holds the raw ctypes wrappers with the
C names.  Nothing here falls back to a CPU implementation: without the
built library every call raises.
"""
from . import _lib  # noqa: F401
from ._lib import (Gf2Error, gf2_dims, gf2_params, gf2_state, gf2_report, make_dims,
                   make_params, lib_path, load, EXPORTED)

__all__ = ["Gf2Error", "gf2_dims", "gf2_params", "gf2_state", "gf2_report", "make_dims",
           "make_params", "lib_path", "load", "EXPORTED"]
