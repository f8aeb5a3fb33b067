"""mfhex: matrix-free high-order hexahedral operators on AMD MI355X (gfx950).

BP1 mass, BP3 / BP5 / BP6 diffusion by sum factorization in fused HIP
kernels, CG (FP64 and FP32-operator mixed precision with FP64 residual
replacement), the coefficient gradient behind a torch.autograd.Function,
multi-RHS batching and an elements-per-block autotuner; a tetrahedral P_p
diffusion operator whose non-tensor basis runs as matrix products on the FP64
matrix cores.  The C ABI is
include/mfhex.h; this package is its Python binding.
"""
from ._lib import (EXPORTS, MFHexError, load, mfhex_version,  # noqa: F401
                   MFHEX_OK, MFHEX_ERR_ARG, MFHEX_ERR_UNSUPPORTED, MFHEX_ERR_HIP, MFHEX_ERR_MESH,
                   MFHEX_ERR_NOCONV, MFHEX_ERR_BREAKDOWN, MFHEX_ERR_STATE)


def __getattr__(name):
    # torch-dependent pieces are imported lazily so that the ctypes binding
    # can be loaded (and its exports checked) without initialising a GPU
    if name == "Operator":
        from .operator import Operator
        return Operator
    if name == "TetOperator":
        from .tet import TetOperator
        return TetOperator
    if name == "CGResult":
        from .operator import CGResult
        return CGResult
    if name in ("MFHexDiffusion", "diffusion"):
        from . import autograd
        return getattr(autograd, name)
    raise AttributeError(name)
