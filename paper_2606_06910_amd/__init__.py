"""MI355X (gfx950) second-order acoustic FDTD + CPML.

Hot path: hand-written HIP kernels behind the C ABI of include/fdtd.h
(libfdtd.so).  This package holds the ctypes binding (argument marshalling
only), a Propagator handle, and a torch.autograd.Function for the model
gradient.  Importing the package never falls back to another implementation:
the library must be built (see build_lib.py).
"""
from ._lib import (BF16, F16, F32, FACE_DIRICHLET, FACE_GHOST, VARIANT_AUTO, VARIANT_NAIVE, VARIANT_TBLOCK,
                   VARIANT_ZMARCH, FDTDError, FDTDValueError, lib)
from .propagator import Propagator, Shot
from .pv import PVPropagator

__all__ = ["Propagator", "Shot", "PVPropagator", "lib", "FDTDError", "FDTDValueError", "F32", "F16", "BF16", "FACE_DIRICHLET",
           "FACE_GHOST", "VARIANT_AUTO", "VARIANT_NAIVE", "VARIANT_ZMARCH", "VARIANT_TBLOCK"]
