"""MI355X-native D2Q9 Onsager-regularized lattice Boltzmann step (arXiv 2602.21242).

The compute path is liblbm.so (hand-written HIP for gfx950, C ABI in include/lbm.h);
this package marshals arguments to it. Build with `python -m paper_2602_21242_amd.build`.
"""
from . import capi
from .capi import LBMError
from .simulation import LBMFunction, Simulation

__all__ = ["capi", "LBMError", "LBMFunction", "Simulation"]
