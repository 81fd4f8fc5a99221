"""MI355X-native lattice-BGK solver of an oscillating body in a BGK gas.

Hand-written HIP kernels for gfx950 behind a C ABI (include/lbm.h,
liblbm.so); this package holds the sources (csrc/), the build step and the
ctypes binding.
"""
from .lbm import (  # noqa: F401
    Batch, LbmError, Params, Solver, default_params, lattice, lib, params_from_solve,
    required_bytes, strerror,
)
