"""Gravo MG (geometric multigrid on curved surfaces) for AMD MI355X.

A thin Python binding of the C ABI in include/gmg.h (libgmg.so, hand-written
HIP for gfx950).  Every step of the hierarchy construction and of the solve
runs in the library's kernels; this module only checks and marshals
arguments.  PyTorch provides device memory and streams.
"""
from .binding import (Hierarchy, Options, SolveInfo, GMGError, build_hierarchy, default_options,
                      library, EXPORTS, STATUS)

__all__ = ["Hierarchy", "Options", "SolveInfo", "GMGError", "build_hierarchy", "default_options",
           "library", "EXPORTS", "STATUS"]
