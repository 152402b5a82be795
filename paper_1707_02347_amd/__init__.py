"""MI355X-native time-blocked acoustic finite-difference sweeps.

The compute path is libfdwave.so (hand-written HIP for gfx950, C ABI in
include/fdwave.h); this package only binds it.  ``api`` holds torch-facing
wrappers, ``autograd`` the differentiable forward map v -> receiver traces.
"""
from ._lib import FdError, load  # noqa: F401

__all__ = ["FdError", "load"]
