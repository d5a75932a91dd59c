"""MI355X-native hierarchical p-multigrid solver for finite cell systems.

The numerical work lives in libfcm.so (HIP kernels for gfx950, C-ABI in
include/fcm.h); :mod:`paper_2010_00881_amd.fcm` is its ctypes binding.
"""
from .fcm import Server, Solver, lib  # noqa: F401
