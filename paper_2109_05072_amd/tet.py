"""Python face of the tetrahedral P_p diffusion operator (``mfhex_tet_*`` in include/mfhex.h).

Argument marshalling only: the set-up and the apply run in the HIP library
(the basis action as FP64 matrix-core products; Sec. 2.1 libCEED, Sec. 2.2 MAGMA).  Torch provides the
device memory and the stream.
"""
from __future__ import annotations

import ctypes as C
from typing import Optional

import numpy as np
import torch

from . import _lib as L


def _stream() -> int:
    return torch.cuda.current_stream().cuda_stream


class TetOperator:
    """y = A x for P_p Lagrange tetrahedra on the Kuhn split of a structured box mesh.

    vertices: [(nex+1)(ney+1)(nez+1), 3] float64 (x fastest), the hexahedral mesh's vertices;
    q: points per collapsed direction (p, the default, or p+1).
    """

    def __init__(self, nex: int, ney: int, nez: int, p: int, vertices: np.ndarray, q: Optional[int] = None,
                 dirichlet: bool = True, device: str = "cuda"):
        L.load()
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU: the tetrahedral operator runs only on the HIP device")
        self.device = torch.device(device)
        self._vert = np.ascontiguousarray(vertices, dtype=np.float64)
        self.p, self.q = p, q if q is not None else p
        self.desc = L.mfhex_tet_desc(nex, ney, nez, p, self.q, int(dirichlet),
                                     self._vert.ctypes.data_as(C.POINTER(C.c_double)))
        self.sizes = L.mfhex_tet_query(self.desc)
        self.n_nodes = int(self.sizes.n_nodes)
        self.n_elem = int(self.sizes.n_elem)
        self.n_basis = int(self.sizes.n_basis)
        self.n_points = int(self.sizes.n_points)
        with torch.cuda.device(self.device):
            self.workspace = torch.empty(int(self.sizes.workspace_bytes) + 256, dtype=torch.uint8, device=self.device)
            ptr = (self.workspace.data_ptr() + 255) & ~255
            self.handle = L.mfhex_tet_create(self.desc, ptr, int(self.sizes.workspace_bytes), _stream())

    def close(self):
        if getattr(self, "handle", None):
            L.mfhex_tet_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def apply(self, x: torch.Tensor, y: Optional[torch.Tensor] = None) -> torch.Tensor:
        if x.device.type != "cuda" or not x.is_contiguous() or x.dtype != torch.float64 or x.numel() != self.n_nodes:
            raise ValueError(f"x must be a contiguous float64 device tensor of {self.n_nodes} entries")
        y = torch.empty_like(x) if y is None else y
        if y.data_ptr() == x.data_ptr():
            raise ValueError("x and y must not alias")
        L.mfhex_tet_apply(self.handle, x.data_ptr(), y.data_ptr(), _stream())
        return y
