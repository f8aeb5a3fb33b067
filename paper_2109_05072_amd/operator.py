"""Torch-facing wrapper of one matrix-free operator.

PyTorch provides device memory and the stream; the operator itself (setup
of the geometric factors, every apply, the coefficient gradient, the load
vector and the CG solve) runs in libmfhex.so.  There is no fallback: if the
library or a GPU is missing, construction raises.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass
from typing import Optional

import numpy as np
import torch

from . import _lib as L

_KINDS = {"mass": L.MFHEX_MASS, "diffusion": L.MFHEX_DIFFUSION}
_QUADS = {"gauss": L.MFHEX_GAUSS, "gll": L.MFHEX_GLL}


def _stream() -> int:
    return torch.cuda.current_stream().cuda_stream


def _prec(dtype) -> int:
    if dtype == torch.float64:
        return L.MFHEX_F64
    if dtype == torch.float32:
        return L.MFHEX_F32
    raise TypeError(f"unsupported dtype {dtype}")


@dataclass
class CGResult:
    x: torch.Tensor
    status: int
    iters: int
    replacements: int
    fell_back_to_f64: bool
    rel_resid_true: float
    rel_resid_rec: float
    seconds: float
    history: np.ndarray


class Operator:
    """Mass or diffusion operator of order p on a structured hexahedral mesh.

    ``vertices``: host float64 array [(nex+1)(ney+1)(nez+1), 3], x fastest.
    ``quad``: "gauss" (q = p+2) or "gll" (q = p+1, collocated).
    ``otf``: diffusion in FP64 with the geometric factors evaluated in the kernel from the element
    vertices instead of stored (no factor array in the workspace).
    ``deterministic``: atomic-free scatter (element values stored, then summed per node in a fixed
    order), one right-hand side per apply.
    """

    def __init__(self, nex: int, ney: int, nez: int, p: int, vertices: np.ndarray, kind: str = "diffusion",
                 quad: str = "gauss", ncomp: int = 1, dirichlet: bool = True, variable_kappa: bool = False,
                 f32: bool = False, rhs: bool = False, otf: bool = False, deterministic: bool = False,
                 device: str = "cuda"):
        L.load()
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU: the matrix-free operators run only on the HIP device")
        self.device = torch.device(device)
        q = p + 2 if quad == "gauss" else p + 1
        self._vert = np.ascontiguousarray(vertices, dtype=np.float64)
        flags = ((L.MFHEX_FLAG_F32 if f32 else 0) | (L.MFHEX_FLAG_RHS if rhs else 0) | (L.MFHEX_FLAG_OTF if otf else 0)
                 | (L.MFHEX_FLAG_DETERMINISTIC if deterministic else 0))
        self.desc = L.mfhex_desc(nex, ney, nez, p, q, _QUADS[quad], _KINDS[kind], ncomp, int(dirichlet),
                                 int(variable_kappa), flags, self._vert.ctypes.data_as(C.POINTER(C.c_double)))
        self.sizes = L.mfhex_query(self.desc)
        self.p, self.q, self.ncomp = p, q, ncomp
        self.kind, self.quad = kind, quad
        self.n_nodes = int(self.sizes.n_nodes)
        self.n_elem = int(self.sizes.n_elem)
        with torch.cuda.device(self.device):
            self.workspace = torch.empty(int(self.sizes.workspace_bytes) + 256, dtype=torch.uint8, device=self.device)
            base = self.workspace.data_ptr()
            self._ws_ptr = (base + 255) & ~255
            self.handle = L.mfhex_create(self.desc, self._ws_ptr, int(self.sizes.workspace_bytes), _stream())
        self._cg_work = None

    # -- lifecycle ---------------------------------------------------------------------------
    def close(self):
        if getattr(self, "handle", None):
            L.mfhex_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- helpers -----------------------------------------------------------------------------
    def _check_vec(self, t: torch.Tensor, nrhs: int, dtype: Optional[torch.dtype] = None, name: str = "vector",
                   n: Optional[int] = None, device: bool = True):
        """Raise ValueError unless t has the expected dtype and length (and, with device=True, is a
        contiguous device tensor).

        The library sizes every read and write from the precision and the node count, so a wrong
        dtype or length would make it touch memory outside the tensor: checked before any call."""
        if dtype is not None and t.dtype != dtype:
            raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
        if t.dtype not in (torch.float64, torch.float32):
            raise ValueError(f"{name} must be float64 or float32, got {t.dtype}")
        n = self.n_nodes * nrhs * self.ncomp if n is None else n
        if t.numel() != n:
            raise ValueError(f"{name} has {t.numel()} entries, expected {n}")
        if device and (t.device.type != "cuda" or not t.is_contiguous()):
            raise ValueError(f"{name} must be a contiguous device tensor")

    def _check_pair(self, x: torch.Tensor, y: torch.Tensor, nrhs: int, dtype: Optional[torch.dtype] = None,
                    names=("x", "y"), n: Optional[int] = None):
        """Input and output of one call: same dtype and length, both on the device, not aliased."""
        self._check_vec(x, nrhs, dtype, names[0], n, device=False)
        self._check_vec(y, nrhs, x.dtype, names[1], n, device=False)
        self._check_vec(x, nrhs, dtype, names[0], n)
        self._check_vec(y, nrhs, x.dtype, names[1], n)
        self._check_distinct(x, y)

    @staticmethod
    def _check_distinct(x: torch.Tensor, y: torch.Tensor):
        if x.data_ptr() == y.data_ptr():
            raise ValueError("x and y must not alias")

    def _nrhs(self, x: torch.Tensor) -> int:
        per = self.n_nodes * self.ncomp
        if x.numel() % per:
            raise ValueError("vector length is not a multiple of n_nodes * ncomp")
        return x.numel() // per

    # -- operator actions --------------------------------------------------------------------
    def apply(self, x: torch.Tensor, y: Optional[torch.Tensor] = None) -> torch.Tensor:
        """y = A x (x: [N], [N, ncomp] or [N, nrhs, ncomp]; float64 or float32)."""
        nrhs = self._nrhs(x)
        y = torch.empty_like(x) if y is None else y
        self._check_pair(x, y, nrhs)
        L.mfhex_apply(self.handle, _prec(x.dtype), nrhs, x.data_ptr(), y.data_ptr(), _stream())
        return y

    def apply_add(self, x: torch.Tensor, y: torch.Tensor) -> torch.Tensor:
        nrhs = self._nrhs(x)
        self._check_pair(x, y, nrhs)
        L.mfhex_apply_add(self.handle, _prec(x.dtype), nrhs, x.data_ptr(), y.data_ptr(), _stream())
        return y

    def apply_adjoint(self, x: torch.Tensor, y: Optional[torch.Tensor] = None) -> torch.Tensor:
        nrhs = self._nrhs(x)
        y = torch.empty_like(x) if y is None else y
        self._check_pair(x, y, nrhs)
        L.mfhex_apply_adjoint(self.handle, _prec(x.dtype), nrhs, x.data_ptr(), y.data_ptr(), _stream())
        return y

    def apply_static(self, x: torch.Tensor, y: Optional[torch.Tensor] = None) -> torch.Tensor:
        """y = A x for one right-hand side in the deterministic summation order, with the element
        values in the library's own device buffer (mfhex_apply_static: no allocation in the call)."""
        nrhs = self._nrhs(x)
        if nrhs != 1:
            raise ValueError("apply_static takes one right-hand side")
        y = torch.empty_like(x) if y is None else y
        self._check_pair(x, y, 1)
        L.mfhex_apply_static(self.handle, _prec(x.dtype), x.data_ptr(), y.data_ptr(), _stream())
        return y

    def set_kappa(self, kappa: torch.Tensor) -> None:
        kappa = kappa.contiguous()
        self._check_vec(kappa, 1, dtype=torch.float64, name="kappa", n=self.n_elem * self.q ** 3)
        L.mfhex_set_kappa(self.handle, kappa.data_ptr(), _stream())

    def kappa_grad(self, u: torch.Tensor, r: torch.Tensor) -> torch.Tensor:
        """g[e, pt] = d(r^T A(kappa) u)/d kappa[e, pt]."""
        self._check_vec(u, 1, dtype=torch.float64, name="u", n=self.n_nodes, device=False)
        self._check_vec(r, 1, dtype=torch.float64, name="r", n=self.n_nodes, device=False)
        self._check_vec(u, 1, dtype=torch.float64, name="u", n=self.n_nodes)
        self._check_vec(r, 1, dtype=torch.float64, name="r", n=self.n_nodes)
        g = torch.empty(self.n_elem, self.q ** 3, dtype=torch.float64, device=u.device)
        L.mfhex_kappa_grad(self.handle, u.data_ptr(), r.data_ptr(), g.data_ptr(), _stream())
        return g

    def diagonal(self) -> torch.Tensor:
        """Diagonal of the assembled operator (FP64, [n_nodes], 0 at masked nodes)."""
        d = torch.empty(self.n_nodes, dtype=torch.float64, device=self.device)
        L.mfhex_diagonal(self.handle, d.data_ptr(), _stream())
        return d

    def qpoint_coords(self) -> torch.Tensor:
        xyz = torch.empty(self.n_elem, self.q ** 3, 3, dtype=torch.float64, device=self.device)
        L.mfhex_qpoint_coords(self.handle, xyz.data_ptr(), _stream())
        return xyz

    def node_coords(self) -> torch.Tensor:
        xyz = torch.empty(self.n_nodes, 3, dtype=torch.float64, device=self.device)
        L.mfhex_node_coords(self.handle, xyz.data_ptr(), _stream())
        return xyz

    def rhs(self, f_q: torch.Tensor) -> torch.Tensor:
        """Load vector of a per-point forcing f_q [n_elem, q^3] (masked when Dirichlet)."""
        f_q = f_q.contiguous()
        self._check_vec(f_q, 1, dtype=torch.float64, name="f_q", n=self.n_elem * self.q ** 3)
        b = torch.empty(self.n_nodes, dtype=torch.float64, device=f_q.device)
        L.mfhex_rhs(self.handle, f_q.data_ptr(), b.data_ptr(), _stream())
        return b

    # -- solver ------------------------------------------------------------------------------
    def cg(self, b: torch.Tensor, x: Optional[torch.Tensor] = None, maxit: int = 1000, rtol: float = 1e-10,
           mode: str = "f64", check_every: int = 1, replace_every: int = 100, replace_delta: float = 0.1,
           exact_iters: bool = False, precond: str = "none") -> CGResult:
        """Solve A x = b by CG: mode "f64" or "mixed" (reliable updates), precond "none", "jacobi" or "mg"
        (one p-multigrid V-cycle per iteration; mg_setup first, FP64 mode)."""
        if x is not None:
            self._check_pair(b, x, 1, dtype=torch.float64, names=("b", "x"), n=self.n_nodes)
        self._check_vec(b, 1, dtype=torch.float64, name="b", n=self.n_nodes)
        if self._cg_work is None:
            self._cg_work = torch.empty(int(self.sizes.cg_work_bytes) + 256, dtype=torch.uint8, device=self.device)
        work = (self._cg_work.data_ptr() + 255) & ~255
        x0_zero = x is None
        x = torch.zeros_like(b) if x is None else x
        if precond not in ("none", "jacobi", "mg"):
            raise ValueError(f"unknown preconditioner {precond!r}")
        opts = L.mfhex_cg_opts(maxit=maxit, check_every=check_every,
                               mode=L.MFHEX_CG_MIXED if mode == "mixed" else L.MFHEX_CG_F64,
                               replace_every=replace_every, x0_is_zero=int(x0_zero), max_iters_exact=int(exact_iters),
                               precond={"none": L.MFHEX_PRECOND_NONE, "jacobi": L.MFHEX_PRECOND_JACOBI,
                                        "mg": L.MFHEX_PRECOND_MG}[precond],
                               rtol=rtol, replace_delta=replace_delta)
        hist = np.zeros(min(maxit, 8191) + 1)
        code, st = L.mfhex_cg(self.handle, b.data_ptr(), x.data_ptr(), work, opts,
                              hist.ctypes.data_as(C.POINTER(C.c_double)), _stream())
        return CGResult(x, code, st.iters, st.replacements, bool(st.fell_back_to_f64), st.rel_resid_true,
                        st.rel_resid_rec, st.seconds, hist[: min(st.iters, 8191) + 1])

    # -- p-multigrid -------------------------------------------------------------------------
    def mg_setup(self, degree: int = 0, coarse_degree: int = 0, power_iters: int = 0, max_levels: int = 0,
                 lo: float = 0.0, hi: float = 0.0, dtype: torch.dtype = torch.float64) -> int:
        """Build the p-multigrid hierarchy (levels p, p/2, ..., 1); 0 keeps a default.  dtype: arithmetic of
        the V-cycle (float32 needs an operator built with f32=True).  Returns the level count."""
        opts = L.mfhex_mg_opts(degree, coarse_degree, power_iters, max_levels, _prec(dtype), 0, lo, hi)
        nbytes, nl = L.mfhex_mg_query(self.desc, opts)
        self._mg_work = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        ptr = (self._mg_work.data_ptr() + 255) & ~255
        L.mfhex_mg_setup(self.handle, self.desc, opts, ptr, nbytes, _stream())
        return nl

    def mg_apply(self, r: torch.Tensor, z: Optional[torch.Tensor] = None) -> torch.Tensor:
        """z = M^-1 r, one V-cycle."""
        z = torch.empty_like(r) if z is None else z
        self._check_pair(r, z, 1, dtype=torch.float64, names=("r", "z"), n=self.n_nodes)
        L.mfhex_mg_apply(self.handle, r.data_ptr(), z.data_ptr(), _stream())
        return z

    def mg_levels(self):
        """[(order, nodes, lambda_max estimate)] from the finest level down."""
        out, lvl = [], 0
        while True:
            try:
                out.append(L.mfhex_mg_level(self.handle, lvl))
            except L.MFHexError:
                return out
            lvl += 1

    # -- tuning ------------------------------------------------------------------------------
    def tune(self, dtype=torch.float64, nrhs: int = 1, cache_path: Optional[str] = None):
        n = self.n_nodes * nrhs * self.ncomp
        scratch = torch.empty(L.tune_scratch_bytes(n) + 256, dtype=torch.uint8, device=self.device)
        ptr = (scratch.data_ptr() + 255) & ~255
        L.mfhex_tune(self.handle, _prec(dtype), nrhs, ptr, cache_path, _stream())
        return self.get_config(dtype, nrhs)

    def get_config(self, dtype=torch.float64, nrhs: int = 1):
        """(variant, elements per group, threads per group, pipeline depth) of the apply launch."""
        return L.mfhex_get_config(self.handle, _prec(dtype), nrhs)

    def set_config(self, variant: int, dtype=torch.float64, nrhs: int = 1, groups_per_block: int = 0) -> None:
        """Force the launch variant and (mass only) the pipeline depth; 0 keeps the default depth."""
        L.mfhex_set_config(self.handle, _prec(dtype), nrhs, variant, groups_per_block)
