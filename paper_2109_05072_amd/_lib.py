"""ctypes binding of libmfhex.so: the C ABI of include/mfhex.h, same names.

Argument marshalling only -- every step of the operator runs in the HIP
library.  Device pointers are passed as integers (e.g. ``tensor.data_ptr()``),
streams as ``torch.cuda.current_stream().cuda_stream``.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmfhex.so")

MFHEX_OK = 0
MFHEX_ERR_ARG = -1
MFHEX_ERR_UNSUPPORTED = -2
MFHEX_ERR_HIP = -3
MFHEX_ERR_MESH = -4
MFHEX_ERR_NOCONV = -5
MFHEX_ERR_BREAKDOWN = -6
MFHEX_ERR_STATE = -7

MFHEX_MASS, MFHEX_DIFFUSION = 1, 2
MFHEX_GAUSS, MFHEX_GLL = 0, 1
MFHEX_F64, MFHEX_F32 = 0, 1
MFHEX_CG_F64, MFHEX_CG_MIXED = 0, 1
MFHEX_PRECOND_NONE, MFHEX_PRECOND_JACOBI, MFHEX_PRECOND_MG = 0, 1, 2
MFHEX_FLAG_F32, MFHEX_FLAG_RHS, MFHEX_FLAG_OTF, MFHEX_FLAG_DETERMINISTIC = 1, 2, 4, 8

# every symbol include/mfhex.h declares
EXPORTS = (
    "mfhex_query", "mfhex_create", "mfhex_destroy", "mfhex_set_kappa", "mfhex_apply", "mfhex_apply_add",
    "mfhex_apply_adjoint", "mfhex_apply_static", "mfhex_apply_static_max_bytes", "mfhex_kappa_grad", "mfhex_qpoint_coords", "mfhex_node_coords", "mfhex_rhs",
    "mfhex_cg", "mfhex_tune", "mfhex_get_config", "mfhex_set_config", "mfhex_diagonal", "mfhex_mg_query", "mfhex_mg_setup",
    "mfhex_mg_apply", "mfhex_mg_level", "mfhex_strerror", "mfhex_last_error",
    "mfhex_basis_1d", "mfhex_version",
    "mfhex_tet_query", "mfhex_tet_create", "mfhex_tet_apply", "mfhex_tet_destroy", "mfhex_tet_basis",
)


def tune_scratch_bytes(length: int) -> int:
    """MFHEX_TUNE_SCRATCH(len) of the header."""
    return 3 * ((length * 8 + 255) & ~255) + 32768


class mfhex_desc(C.Structure):
    _fields_ = [("nex", C.c_int32), ("ney", C.c_int32), ("nez", C.c_int32), ("p", C.c_int32),
                ("q", C.c_int32), ("quad", C.c_int32), ("kind", C.c_int32), ("ncomp", C.c_int32),
                ("dirichlet", C.c_int32), ("variable_kappa", C.c_int32), ("flags", C.c_uint32),
                ("vertex_xyz", C.POINTER(C.c_double))]


class mfhex_sizes(C.Structure):
    _fields_ = [("n_nodes", C.c_int64), ("n_elem", C.c_int64), ("n_qpts", C.c_int64),
                ("workspace_bytes", C.c_size_t), ("cg_work_bytes", C.c_size_t)]


class mfhex_cg_opts(C.Structure):
    _fields_ = [("maxit", C.c_int32), ("check_every", C.c_int32), ("mode", C.c_int32),
                ("replace_every", C.c_int32), ("x0_is_zero", C.c_int32), ("max_iters_exact", C.c_int32),
                ("precond", C.c_int32), ("pad_", C.c_int32), ("rtol", C.c_double), ("replace_delta", C.c_double)]


class mfhex_mg_opts(C.Structure):
    _fields_ = [("degree", C.c_int32), ("coarse_degree", C.c_int32), ("power_iters", C.c_int32),
                ("max_levels", C.c_int32), ("precision", C.c_int32), ("pad_", C.c_int32), ("lo", C.c_double),
                ("hi", C.c_double)]


class mfhex_tet_desc(C.Structure):
    _fields_ = [("nex", C.c_int32), ("ney", C.c_int32), ("nez", C.c_int32), ("p", C.c_int32), ("q", C.c_int32),
                ("dirichlet", C.c_int32), ("vertex_xyz", C.POINTER(C.c_double))]


class mfhex_tet_sizes(C.Structure):
    _fields_ = [("n_nodes", C.c_int64), ("n_elem", C.c_int64), ("n_qpts", C.c_int64),
                ("workspace_bytes", C.c_size_t), ("n_basis", C.c_int32), ("n_points", C.c_int32)]


class mfhex_cg_stats(C.Structure):
    _fields_ = [("iters", C.c_int32), ("replacements", C.c_int32), ("fell_back_to_f64", C.c_int32),
                ("pad_", C.c_int32), ("rel_resid_true", C.c_double), ("rel_resid_rec", C.c_double),
                ("seconds", C.c_double)]


class MFHexError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"mfhex error {code}: {msg}")
        self.code = code


_lib = None


def load(path: str = LIB_PATH):
    """Load the HIP library (building it in-tree first if no build exists); raises if unavailable."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        from . import build as _build
        _build.build()
    if not os.path.exists(path):
        raise ImportError(f"libmfhex.so not found at {path}; run python -m paper_2109_05072_amd.build")
    L = C.CDLL(path)
    vp, i32, sz = C.c_void_p, C.c_int, C.c_size_t
    sig = {
        "mfhex_query": ([C.POINTER(mfhex_desc), C.POINTER(mfhex_sizes)], i32),
        "mfhex_create": ([C.POINTER(mfhex_desc), vp, sz, vp, C.POINTER(vp)], i32),
        "mfhex_destroy": ([vp], i32),
        "mfhex_set_kappa": ([vp, vp, vp], i32),
        "mfhex_apply": ([vp, i32, i32, vp, vp, vp], i32),
        "mfhex_apply_add": ([vp, i32, i32, vp, vp, vp], i32),
        "mfhex_apply_adjoint": ([vp, i32, i32, vp, vp, vp], i32),
        "mfhex_apply_static": ([vp, i32, vp, vp, vp], i32),
        "mfhex_apply_static_max_bytes": ([], sz),
        "mfhex_kappa_grad": ([vp, vp, vp, vp, vp], i32),
        "mfhex_qpoint_coords": ([vp, vp, vp], i32),
        "mfhex_node_coords": ([vp, vp, vp], i32),
        "mfhex_rhs": ([vp, vp, vp, vp], i32),
        "mfhex_cg": ([vp, vp, vp, vp, C.POINTER(mfhex_cg_opts), C.POINTER(mfhex_cg_stats),
                      C.POINTER(C.c_double), vp], i32),
        "mfhex_tune": ([vp, i32, i32, vp, C.c_char_p, vp], i32),
        "mfhex_get_config": ([vp, i32, i32, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                              C.POINTER(C.c_int32), C.POINTER(C.c_int32)], i32),
        "mfhex_mg_query": ([C.POINTER(mfhex_desc), C.POINTER(mfhex_mg_opts), C.POINTER(sz), C.POINTER(C.c_int32)], i32),
        "mfhex_mg_setup": ([vp, C.POINTER(mfhex_desc), C.POINTER(mfhex_mg_opts), vp, sz, vp], i32),
        "mfhex_mg_apply": ([vp, vp, vp, vp], i32),
        "mfhex_mg_level": ([vp, i32, C.POINTER(C.c_int32), C.POINTER(C.c_int64), C.POINTER(C.c_double)], i32),
        "mfhex_diagonal": ([vp, vp, vp], i32),
        "mfhex_set_config": ([vp, i32, i32, C.c_int32, C.c_int32], i32),
        "mfhex_strerror": ([i32], C.c_char_p),
        "mfhex_last_error": ([vp], C.c_char_p),
        "mfhex_basis_1d": ([i32, i32, i32] + [C.POINTER(C.c_double)] * 5, i32),
        "mfhex_version": ([], C.c_char_p),
        "mfhex_tet_query": ([C.POINTER(mfhex_tet_desc), C.POINTER(mfhex_tet_sizes)], i32),
        "mfhex_tet_create": ([C.POINTER(mfhex_tet_desc), vp, sz, vp, C.POINTER(vp)], i32),
        "mfhex_tet_apply": ([vp, vp, vp, vp], i32),
        "mfhex_tet_destroy": ([vp], i32),
        "mfhex_tet_basis": ([i32, i32] + [C.POINTER(C.c_double)] * 4, i32),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    _lib = L
    return L


def check(code: int, op=None):
    if code != MFHEX_OK:
        L = load()
        msg = L.mfhex_last_error(op).decode() or L.mfhex_strerror(code).decode()
        raise MFHexError(code, msg)
    return code


# thin wrappers with the C names ------------------------------------------------------------

def mfhex_query(desc: mfhex_desc) -> mfhex_sizes:
    s = mfhex_sizes()
    check(load().mfhex_query(C.byref(desc), C.byref(s)))
    return s


def mfhex_create(desc: mfhex_desc, workspace: int, workspace_bytes: int, stream: int) -> int:
    h = C.c_void_p()
    check(load().mfhex_create(C.byref(desc), workspace, workspace_bytes, stream, C.byref(h)))
    return h.value


def mfhex_destroy(op: int) -> None:
    check(load().mfhex_destroy(op))


def mfhex_set_kappa(op: int, kappa: int, stream: int) -> None:
    check(load().mfhex_set_kappa(op, kappa, stream), op)


def mfhex_apply(op: int, prec: int, nrhs: int, x: int, y: int, stream: int) -> None:
    check(load().mfhex_apply(op, prec, nrhs, x, y, stream), op)


def mfhex_apply_add(op: int, prec: int, nrhs: int, x: int, y: int, stream: int) -> None:
    check(load().mfhex_apply_add(op, prec, nrhs, x, y, stream), op)


def mfhex_apply_adjoint(op: int, prec: int, nrhs: int, x: int, y: int, stream: int) -> None:
    check(load().mfhex_apply_adjoint(op, prec, nrhs, x, y, stream), op)


def mfhex_apply_static(op: int, prec: int, x: int, y: int, stream: int) -> None:
    check(load().mfhex_apply_static(op, prec, x, y, stream), op)


def mfhex_apply_static_max_bytes() -> int:
    return int(load().mfhex_apply_static_max_bytes())


def mfhex_kappa_grad(op: int, u: int, r: int, g: int, stream: int) -> None:
    check(load().mfhex_kappa_grad(op, u, r, g, stream), op)


def mfhex_qpoint_coords(op: int, xyz: int, stream: int) -> None:
    check(load().mfhex_qpoint_coords(op, xyz, stream), op)


def mfhex_node_coords(op: int, xyz: int, stream: int) -> None:
    check(load().mfhex_node_coords(op, xyz, stream), op)


def mfhex_rhs(op: int, f: int, b: int, stream: int) -> None:
    check(load().mfhex_rhs(op, f, b, stream), op)


def mfhex_cg(op: int, b: int, x: int, work: int, opts: mfhex_cg_opts, rhist, stream: int):
    """Returns (status, stats); NOCONV is returned, not raised."""
    st = mfhex_cg_stats()
    code = load().mfhex_cg(op, b, x, work, C.byref(opts), C.byref(st), rhist, stream)
    if code not in (MFHEX_OK, MFHEX_ERR_NOCONV):
        check(code, op)
    return code, st


def mfhex_tune(op: int, prec: int, nrhs: int, scratch: int, cache_path, stream: int) -> None:
    cp = cache_path.encode() if cache_path else None
    check(load().mfhex_tune(op, prec, nrhs, scratch, cp, stream), op)


def mfhex_get_config(op: int, prec: int, nrhs: int):
    """(variant, elements per group, threads per group, pipeline depth)."""
    v, g, t, d = C.c_int32(), C.c_int32(), C.c_int32(), C.c_int32()
    check(load().mfhex_get_config(op, prec, nrhs, C.byref(v), C.byref(g), C.byref(t), C.byref(d)), op)
    return v.value, g.value, t.value, d.value


def mfhex_set_config(op: int, prec: int, nrhs: int, variant: int, groups_per_block: int = 0) -> None:
    check(load().mfhex_set_config(op, prec, nrhs, variant, groups_per_block), op)


def mfhex_diagonal(op: int, d: int, stream: int) -> None:
    check(load().mfhex_diagonal(op, d, stream), op)


def mfhex_mg_query(d: mfhex_desc, opts: mfhex_mg_opts):
    """(work bytes, number of levels) of a p-multigrid hierarchy."""
    nb, nl = C.c_size_t(), C.c_int32()
    check(load().mfhex_mg_query(C.byref(d), C.byref(opts), C.byref(nb), C.byref(nl)), None)
    return nb.value, nl.value


def mfhex_mg_setup(op: int, d: mfhex_desc, opts: mfhex_mg_opts, work: int, nbytes: int, stream: int) -> None:
    check(load().mfhex_mg_setup(op, C.byref(d), C.byref(opts), work, nbytes, stream), op)


def mfhex_mg_apply(op: int, r: int, z: int, stream: int) -> None:
    check(load().mfhex_mg_apply(op, r, z, stream), op)


def mfhex_mg_level(op: int, level: int):
    """(order, nodes, lambda_max estimate) of a level (0 = finest)."""
    p, n, lam = C.c_int32(), C.c_int64(), C.c_double()
    check(load().mfhex_mg_level(op, level, C.byref(p), C.byref(n), C.byref(lam)), op)
    return p.value, n.value, lam.value


def mfhex_strerror(code: int) -> str:
    return load().mfhex_strerror(code).decode()


def mfhex_basis_1d(p: int, q: int, quad: int):
    """(nodes, xq, wq, B, D) as numpy arrays, from the library's host setup code."""
    import numpy as np
    P = p + 1
    out = [np.zeros(P), np.zeros(q), np.zeros(q), np.zeros((q, P)), np.zeros((q, q))]
    ptrs = [a.ctypes.data_as(C.POINTER(C.c_double)) for a in out]
    check(load().mfhex_basis_1d(p, q, quad, *ptrs))
    return tuple(out)


def mfhex_tet_query(desc: mfhex_tet_desc) -> mfhex_tet_sizes:
    s = mfhex_tet_sizes()
    check(load().mfhex_tet_query(C.byref(desc), C.byref(s)))
    return s


def mfhex_tet_create(desc: mfhex_tet_desc, work: int, nbytes: int, stream: int) -> int:
    h = C.c_void_p()
    check(load().mfhex_tet_create(C.byref(desc), work, nbytes, stream, C.byref(h)))
    return h.value


def mfhex_tet_apply(op: int, x: int, y: int, stream: int) -> None:
    check(load().mfhex_tet_apply(op, x, y, stream))


def mfhex_tet_destroy(op: int) -> None:
    check(load().mfhex_tet_destroy(op))


def mfhex_tet_basis(p: int, q: int):
    """(xi [Q,3], w [Q], B [Q,P], G [3,Q,P]) from the library's host set-up code."""
    import numpy as np
    Q, P = q ** 3, (p + 1) * (p + 2) * (p + 3) // 6
    out = [np.zeros((Q, 3)), np.zeros(Q), np.zeros((Q, P)), np.zeros((3, Q, P))]
    ptrs = [a.ctypes.data_as(C.POINTER(C.c_double)) for a in out]
    check(load().mfhex_tet_basis(p, q, *ptrs))
    return tuple(out)


def mfhex_version() -> str:
    return load().mfhex_version().decode()
