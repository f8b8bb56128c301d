"""MI355X-native hierarchical low-rank view-factor matrices and radiosity solves.

The computation lives in librad.so (HIP for gfx950 behind the C-ABI of
include/rad.h); this package is its thin Python binding.
"""
from .rad import HMatrix, RadError, load  # noqa: F401
