"""MI355X relativistic lattice Boltzmann (two-population D3Q19 RLB scheme of
arXiv:0912.2913) behind a C ABI (include/rlb.h).

Importing the package does not load the GPU library; ``Solver`` (and the
autograd functions) load ``librlb.so`` on first use and raise ImportError if it
has not been built.  There is no CPU path.
"""
from ._lib import (BC_INFLOW, BC_OUTFLOW, BC_PERIODIC, BF16DEV, F16DEV, F32, F32DEV, F64,
                   RLBError, UnphysicalState)

__all__ = ["Solver", "RLBError", "UnphysicalState", "F64", "F32", "F32DEV", "F16DEV", "BF16DEV",
           "BC_PERIODIC", "BC_OUTFLOW", "BC_INFLOW"]


def __getattr__(name):
    if name == "Solver":
        from .solver import Solver
        return Solver
    raise AttributeError(name)
