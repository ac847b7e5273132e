"""MI355X-native Finite-Time Lyapunov Exponent (FTLE) library.

The compute path is libftle.so: hand-written HIP kernels for gfx950 behind the
C ABI in include/ftle.h.  This package only marshals arguments to it.
"""
from .api import (BatchedCall, FTLEError, FTLEFunction, Mesh, advect_rk4, advect_rk4_grid,  # noqa: F401
                  batched, batched_config, axis_ell, eig_threshold, force_wide_offsets, forward_ell, ftle,
                  pin_batched_config, ring1_csr, ring1_workspace_bytes, set_eig_threshold, cached_memory_bytes,
                  release_cached_memory)
from ._lib import LIB_PATH, load  # noqa: F401
