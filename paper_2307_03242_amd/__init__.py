"""MI355X library for the LFA-tuned matrix-free elastic Helmholtz multigrid.

The numerical path lives in libelh.so (hand-written HIP for gfx950, C ABI
declared in include/elh.h); this package only marshals torch tensors to it.
Importing the package does not load the library; Problem() does, and
raises if it has not been built.
"""
from ._lib import (ELH_OK, ELH_NOT_CONVERGED, ELH_C64, ELH_C128, ELH_SHIFTED,
                   ELH_ADJOINT, ElhError, load as load_library)

__all__ = ["Problem", "Batch", "ElhError", "load_library", "ELH_OK", "ELH_NOT_CONVERGED",
           "ELH_C64", "ELH_C128", "ELH_SHIFTED", "ELH_ADJOINT"]


def __getattr__(name):
    if name == "Problem":
        from .api import Problem
        return Problem
    if name == "Batch":
        from .api import Batch
        return Batch
    if name == "ElasticFWI":
        from .autograd import ElasticFWI
        return ElasticFWI
    raise AttributeError(name)
