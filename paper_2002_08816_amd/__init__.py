"""MI355X (gfx950) implementation of the fifth-order hybrid Hermite WENO scheme with
artificial linear weights (Zhao & Qiu, arXiv 2002.08816).

The scheme runs entirely in the HIP library libhweno.so (C ABI: include/hweno.h); this
package only binds it.  Importing the package without the built library raises
ImportError: there is no CPU fallback.
"""
from . import capi  # noqa: F401  (loads libhweno.so or raises)
from .solver import BatchSolver, Solver, make_config  # noqa: F401
from .autograd import HWENOSolve, solve  # noqa: F401
