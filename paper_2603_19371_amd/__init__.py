"""Factored Levenberg-Marquardt registration step on AMD MI355X (gfx950).

The compute path is liblmreg.so (HIP kernels behind the C-ABI declared in
include/lmreg.h); ``_lib`` is its ctypes binding and ``phantoms`` builds the
seeded synthetic inputs.  Importing the binding raises if the library is not
built: there is no CPU fallback.
"""
__all__ = ["lib", "phantoms"]


def lib():
    from . import _lib
    return _lib
