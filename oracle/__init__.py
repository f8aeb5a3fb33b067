"""FP64 CPU oracle for the matrix-free hexahedral operators -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product path (the HIP library and
its Python binding) never imports it, and it imports nothing from the
product.  The arithmetic lives in ``oracle.c`` (plain C, no sum
factorization: dense tabulations of the tensor basis, straight from the
element-operator definition A^e = D^T G^e D of Sec. 2); this module only
marshals arrays and assembles sparse matrices for brute-force checks.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

from . import build as _build

GAUSS, GLL = 0, 1
MASS, DIFFUSION = 1, 2

OK, ERR_ARG, ERR_MEM, ERR_BREAKDOWN, ERR_NOCONV = 0, -1, -2, -3, -4


class _Prob(C.Structure):
    _fields_ = [("nex", C.c_int32), ("ney", C.c_int32), ("nez", C.c_int32), ("p", C.c_int32),
                ("q", C.c_int32), ("quad", C.c_int32), ("kind", C.c_int32), ("dirichlet", C.c_int32),
                ("vert", C.POINTER(C.c_double)), ("kappa", C.POINTER(C.c_double))]


_lib = None


def lib():
    global _lib
    if _lib is None:
        path = _build.ensure_built()
        L = C.CDLL(path)
        dp = C.POINTER(C.c_double)
        pp = C.POINTER(_Prob)
        L.orc_gauss.argtypes = [C.c_int, dp, dp]
        L.orc_gll.argtypes = [C.c_int, dp, dp]
        L.orc_lagrange.argtypes = [C.c_int, dp, C.c_int, dp, dp, dp]
        L.orc_lagrange.restype = None
        L.orc_num_nodes.argtypes = [pp]
        L.orc_num_nodes.restype = C.c_int64
        L.orc_element_matrix.argtypes = [pp, C.c_int64, dp]
        L.orc_element_nodes.argtypes = [pp, C.c_int64, C.POINTER(C.c_int64)]
        L.orc_apply.argtypes = [pp, C.c_int, dp, dp, C.c_int]
        L.orc_qpoint_geometry.argtypes = [pp, dp, dp]
        L.orc_node_coords.argtypes = [pp, dp]
        L.orc_rhs.argtypes = [pp, dp, dp]
        L.orc_kappa_grad.argtypes = [pp, dp, dp, dp]
        L.orc_cg.argtypes = [pp, dp, dp, C.c_int, C.c_double, dp, C.POINTER(C.c_int), C.c_int]
        L.orc_diagonal.argtypes = [pp, dp]
        L.orc_pcg.argtypes = [pp, dp, dp, dp, C.c_int, C.c_double, dp, C.POINTER(C.c_int), C.c_int]
        _lib = L
    return _lib


def _dp(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _check(code: int, what: str):
    if code != OK:
        raise RuntimeError(f"oracle {what} failed with code {code}")


def gauss(q: int):
    """Gauss-Legendre points and weights on [-1, 1] (ascending)."""
    x, w = np.zeros(q), np.zeros(q)
    _check(lib().orc_gauss(q, _dp(x), _dp(w)), "gauss")
    return x, w


def gll(p: int):
    """The p+1 Gauss-Lobatto-Legendre points and weights on [-1, 1]."""
    x, w = np.zeros(p + 1), np.zeros(p + 1)
    _check(lib().orc_gll(p, _dp(x), _dp(w)), "gll")
    return x, w


def lagrange(nodes: np.ndarray, xq: np.ndarray):
    """B[k, j] = l_j(xq_k), G[k, j] = l_j'(xq_k) for the Lagrange basis on ``nodes``."""
    nodes = np.ascontiguousarray(nodes, dtype=np.float64)
    xq = np.ascontiguousarray(xq, dtype=np.float64)
    B = np.zeros((len(xq), len(nodes)))
    G = np.zeros_like(B)
    lib().orc_lagrange(len(nodes), _dp(nodes), len(xq), _dp(xq), _dp(B), _dp(G))
    return B, G


@dataclass
class Problem:
    """One operator on a structured hexahedral mesh of the unit cube.

    ``vert`` holds the (nex+1)(ney+1)(nez+1) vertex coordinates, x fastest;
    ``kappa`` (optional) the per-quadrature-point coefficient, [E][q^3].
    """
    nex: int
    ney: int
    nez: int
    p: int
    q: int
    quad: int
    kind: int
    dirichlet: int
    vert: np.ndarray
    kappa: Optional[np.ndarray] = None
    _c: _Prob = field(default=None, repr=False)

    def __post_init__(self):
        self.vert = np.ascontiguousarray(self.vert, dtype=np.float64).reshape(-1, 3)
        assert self.vert.shape[0] == (self.nex + 1) * (self.ney + 1) * (self.nez + 1)
        if self.kappa is not None:
            self.kappa = np.ascontiguousarray(self.kappa, dtype=np.float64).reshape(self.n_elem, self.q ** 3)

    @property
    def n_elem(self) -> int:
        return self.nex * self.ney * self.nez

    @property
    def n_nodes(self) -> int:
        return (self.p * self.nex + 1) * (self.p * self.ney + 1) * (self.p * self.nez + 1)

    def cstruct(self) -> _Prob:
        kap = _dp(self.kappa) if self.kappa is not None else C.POINTER(C.c_double)()
        self._c = _Prob(self.nex, self.ney, self.nez, self.p, self.q, self.quad, self.kind,
                        self.dirichlet, _dp(self.vert), kap)
        return self._c

    def with_(self, **kw) -> "Problem":
        d = dict(nex=self.nex, ney=self.ney, nez=self.nez, p=self.p, q=self.q, quad=self.quad,
                 kind=self.kind, dirichlet=self.dirichlet, vert=self.vert, kappa=self.kappa)
        d.update(kw)
        return Problem(**d)


def apply(pr: Problem, x: np.ndarray, nthreads: int = 0) -> np.ndarray:
    """y = M (sum_e R_e^T A^e R_e) M x on each column of x ([N] or [N][nvec])."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    nvec = 1 if x.ndim == 1 else x.shape[1]
    assert x.shape[0] == pr.n_nodes
    y = np.zeros_like(x)
    c = pr.cstruct()
    _check(lib().orc_apply(C.byref(c), nvec, _dp(x), _dp(y), nthreads), "apply")
    return y


def element_matrix(pr: Problem, e: int) -> np.ndarray:
    P3 = (pr.p + 1) ** 3
    A = np.zeros((P3, P3))
    c = pr.cstruct()
    _check(lib().orc_element_matrix(C.byref(c), e, _dp(A)), "element_matrix")
    return A


def element_nodes(pr: Problem, e: int) -> np.ndarray:
    P3 = (pr.p + 1) ** 3
    g = np.zeros(P3, dtype=np.int64)
    c = pr.cstruct()
    _check(lib().orc_element_nodes(C.byref(c), e, g.ctypes.data_as(C.POINTER(C.c_int64))), "element_nodes")
    return g


def assemble(pr: Problem):
    """Global sparse matrix M (sum_e R_e^T A^e R_e) M as scipy CSR (brute force)."""
    import scipy.sparse as sp
    rows, cols, vals = [], [], []
    for e in range(pr.n_elem):
        A = element_matrix(pr, e)
        g = element_nodes(pr, e)
        keep = g >= 0
        gi = g[keep]
        Ak = A[np.ix_(keep, keep)]
        rows.append(np.repeat(gi, len(gi)))
        cols.append(np.tile(gi, len(gi)))
        vals.append(Ak.ravel())
    N = pr.n_nodes
    return sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(N, N)).tocsr()


def qpoint_geometry(pr: Problem):
    """Physical coordinates [E, q^3, 3] and detJ [E, q^3] of the quadrature points."""
    Q3 = pr.q ** 3
    xyz = np.zeros((pr.n_elem, Q3, 3))
    det = np.zeros((pr.n_elem, Q3))
    c = pr.cstruct()
    _check(lib().orc_qpoint_geometry(C.byref(c), _dp(xyz), _dp(det)), "qpoint_geometry")
    return xyz, det


def node_coords(pr: Problem) -> np.ndarray:
    xyz = np.zeros((pr.n_nodes, 3))
    c = pr.cstruct()
    _check(lib().orc_node_coords(C.byref(c), _dp(xyz)), "node_coords")
    return xyz


def rhs(pr: Problem, fq: np.ndarray) -> np.ndarray:
    """b_n = sum over points of w detJ f phi_n (masked for Dirichlet problems)."""
    fq = np.ascontiguousarray(fq, dtype=np.float64).reshape(pr.n_elem, pr.q ** 3)
    b = np.zeros(pr.n_nodes)
    c = pr.cstruct()
    _check(lib().orc_rhs(C.byref(c), _dp(fq), _dp(b)), "rhs")
    return b


def kappa_grad(pr: Problem, u: np.ndarray, r: np.ndarray) -> np.ndarray:
    """d(r^T M A(kappa) M u)/d kappa per quadrature point, [E, q^3]."""
    u = np.ascontiguousarray(u, dtype=np.float64)
    r = np.ascontiguousarray(r, dtype=np.float64)
    g = np.zeros((pr.n_elem, pr.q ** 3))
    c = pr.cstruct()
    _check(lib().orc_kappa_grad(C.byref(c), _dp(u), _dp(r), _dp(g)), "kappa_grad")
    return g


def cg(pr: Problem, b: np.ndarray, maxit: int, rtol: float, nthreads: int = 0):
    """Unpreconditioned CG from x0 = 0.  Returns (x, residual-norm history, iters, code)."""
    b = np.ascontiguousarray(b, dtype=np.float64)
    x = np.zeros_like(b)
    hist = np.zeros(maxit + 1)
    it = C.c_int(0)
    c = pr.cstruct()
    code = lib().orc_cg(C.byref(c), _dp(b), _dp(x), maxit, rtol, _dp(hist), C.byref(it), nthreads)
    if code not in (OK, ERR_NOCONV):
        raise RuntimeError(f"oracle cg failed with code {code}")
    return x, hist[: it.value + 1], it.value, code


def diagonal(pr: Problem) -> np.ndarray:
    """Diagonal of the assembled operator M (sum_e R_e^T A^e R_e) M (0 at masked nodes)."""
    d = np.zeros(pr.n_nodes)
    c = pr.cstruct()
    code = lib().orc_diagonal(C.byref(c), _dp(d))
    if code != OK:
        raise RuntimeError(f"oracle diagonal failed with code {code}")
    return d


def jacobi_inverse(d: np.ndarray) -> np.ndarray:
    """Inverse diagonal for Jacobi preconditioning: 1/d where d > 0, 0 at masked nodes."""
    out = np.zeros_like(d)
    pos = d > 0
    out[pos] = 1.0 / d[pos]
    return out


def pcg(pr: Problem, b: np.ndarray, dinv: np.ndarray, maxit: int, rtol: float, nthreads: int = 0):
    """Jacobi-preconditioned CG from x0 = 0.  Returns (x, residual-norm history, iters, code)."""
    b = np.ascontiguousarray(b, dtype=np.float64)
    dinv = np.ascontiguousarray(dinv, dtype=np.float64)
    x = np.zeros_like(b)
    hist = np.zeros(maxit + 1)
    it = C.c_int(0)
    c = pr.cstruct()
    code = lib().orc_pcg(C.byref(c), _dp(b), _dp(dinv), _dp(x), maxit, rtol, _dp(hist), C.byref(it), nthreads)
    if code not in (OK, ERR_NOCONV):
        raise RuntimeError(f"oracle pcg failed with code {code}")
    return x, hist[: it.value + 1], it.value, code


def num_threads() -> int:
    return int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
