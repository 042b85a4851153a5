"""MI355X-native FP64 finite-volume compressible Navier-Stokes right-hand side.

Hand-written HIP kernels for gfx950 behind the C ABI declared in include/cfd.h;
this package holds the kernels' sources (csrc/), the ctypes binding and the
input generators. Importing the package does not load the native library; the
first call that needs it does, and fails loudly if it is missing.
"""
__all__ = ["workloads"]
