"""MI355X (gfx950) geometric-multigrid solver for node-based finite-difference
elasticity with spatially varying stiffness (Runnels, Agrawal, Zhang, Almgren,
arXiv 2001.04789).

The solver lives in the HIP library ``libemg.so`` (C ABI declared in
``include/emg.h``).  This package is a thin ctypes binding: argument
marshalling only, every step of a solve runs in the library's kernels.
Importing it fails loudly if the library has not been built.
"""
from ._abi import *  # noqa: F401,F403
from ._abi import Problem, Context, lib, EmgError  # noqa: F401
