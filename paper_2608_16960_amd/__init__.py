"""MI355X-native spherical-grid tomographic projector (TomoSphero method).

The projector y = F rho and its adjoint run as hand-written HIP kernels for
gfx950 behind the C ABI declared in ``include/tsp.h``; this package is the thin
Python layer above it.  Submodules are imported on demand so that the input
generators (``workloads``) load without the native library.
"""
__all__ = ["workloads", "native", "projector", "solvers", "nn", "learned"]
