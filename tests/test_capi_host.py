"""Host-side checks of the C ABI (no GPU): the library loads, exports every
declared symbol, validates descriptions, and its 1D setup matches the
mathematics (independently of the oracle's own construction)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import synth
from paper_2109_05072_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "mfhex.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(mfhex_[a-z0-9_]+)\s*\(", src)))


def test_every_declared_symbol_is_exported():
    lib = L.load()
    names = _declared()
    assert len(names) >= 18
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(L.EXPORTS) == names


def _desc(nex=2, ney=2, nez=2, p=3, q=None, quad=L.MFHEX_GAUSS, kind=L.MFHEX_DIFFUSION, ncomp=1, dirichlet=1,
          vark=0, flags=0, vert=None):
    if q is None:
        q = p + 2 if quad == L.MFHEX_GAUSS else p + 1
    if vert is None:
        vert = synth.mesh_vertices(max(nex, 1), max(ney, 1), max(nez, 1))
    d = L.mfhex_desc(nex, ney, nez, p, q, quad, kind, ncomp, dirichlet, vark, flags,
                     vert.ctypes.data_as(C.POINTER(C.c_double)) if vert is not False else C.POINTER(C.c_double)())
    d._keep = vert
    return d


def test_query_sizes():
    d = _desc(3, 2, 4, p=2, flags=L.MFHEX_FLAG_F32)
    s = L.mfhex_query(d)
    assert s.n_nodes == 7 * 5 * 9
    assert s.n_elem == 24
    assert s.n_qpts == 24 * 64
    # vertices + offsets + FP64 and FP32 factors + 1D basis block (B, B^T, D, D^T in FP64
    # and FP32) + flag, each 256-aligned
    al = lambda x: (x + 255) // 256 * 256  # noqa: E731
    P, Q = 3, 4
    h = lambda n: (n + 1) // 2  # noqa: E731
    # plain B, B^T, D, D^T and their folded (even-odd) half-row forms
    nb = 2 * Q * P + 2 * Q * Q + h(Q) * P + h(P) * Q + 2 * h(Q) * Q + 2 * Q  # ... and the 1D rule (x, w)
    nb += h(Q) * P + h(P) * Q  # folded basis derivative at the points and its transpose
    expect = (al(4 * 3 * 5 * 3 * 8) + al(24 * 27 * 4) + al(24 * 6 * 64 * 8) + al(24 * 6 * 64 * 4)
              + al(nb * 12 + 256) + 256)
    assert s.workspace_bytes == expect
    assert s.cg_work_bytes >= s.n_nodes * (3 * 8 + 3 * 4)
    # in-kernel geometric factors: the same layout without either factor array
    d2 = _desc(3, 2, 4, p=2, flags=L.MFHEX_FLAG_OTF)
    assert L.mfhex_query(d2).workspace_bytes == expect - al(24 * 6 * 64 * 8) - al(24 * 6 * 64 * 4)
    # deterministic scatter: the same layout plus the element-value buffer [E][P^3][ncomp] in FP64
    d3 = _desc(3, 2, 4, p=2, ncomp=3, flags=L.MFHEX_FLAG_F32 | L.MFHEX_FLAG_DETERMINISTIC)
    assert L.mfhex_query(d3).workspace_bytes == expect + al(24 * 27 * 3 * 8)


@pytest.mark.parametrize("kw,code", [
    (dict(p=0), L.MFHEX_ERR_UNSUPPORTED),
    (dict(p=9), L.MFHEX_ERR_UNSUPPORTED),
    (dict(nex=0), L.MFHEX_ERR_ARG),
    (dict(ncomp=2), L.MFHEX_ERR_ARG),
    (dict(quad=L.MFHEX_GLL, q=5, p=3), L.MFHEX_ERR_ARG),
    (dict(quad=L.MFHEX_GAUSS, q=4, p=3), L.MFHEX_ERR_UNSUPPORTED),
    (dict(kind=3), L.MFHEX_ERR_ARG),
    (dict(kind=L.MFHEX_MASS, vark=1), L.MFHEX_ERR_ARG),
    (dict(flags=16), L.MFHEX_ERR_ARG),
    (dict(flags=L.MFHEX_FLAG_OTF, kind=L.MFHEX_MASS, dirichlet=0), L.MFHEX_ERR_UNSUPPORTED),
    (dict(flags=L.MFHEX_FLAG_OTF | L.MFHEX_FLAG_F32), L.MFHEX_ERR_UNSUPPORTED),
    (dict(flags=L.MFHEX_FLAG_OTF, vark=1), L.MFHEX_ERR_UNSUPPORTED),
    (dict(dirichlet=2), L.MFHEX_ERR_ARG),
    (dict(vert=False), L.MFHEX_ERR_ARG),
])
def test_query_rejects_bad_descriptions(kw, code):
    with pytest.raises(L.MFHexError) as ei:
        L.mfhex_query(_desc(**kw))
    assert ei.value.code == code
    assert L.mfhex_strerror(code) != "unknown status"


def test_strerror_and_version():
    for c in range(0, -8, -1):
        assert L.mfhex_strerror(c)
    assert "gfx950" in L.mfhex_version()


@pytest.mark.parametrize("p", range(1, 9))
@pytest.mark.parametrize("quad", [L.MFHEX_GAUSS, L.MFHEX_GLL])
def test_library_bases_match_the_mathematics(p, quad):
    q = p + 2 if quad == L.MFHEX_GAUSS else p + 1
    nodes, xq, wq, B, D = L.mfhex_basis_1d(p, q, quad)
    # nodes: -1, roots of P_p', +1
    c = np.zeros(p + 1)
    c[p] = 1.0
    inner = np.sort(np.polynomial.legendre.legroots(np.polynomial.legendre.legder(c))) if p > 1 else []
    np.testing.assert_allclose(nodes, np.concatenate([[-1.0], inner, [1.0]]), atol=4e-15)
    if quad == L.MFHEX_GAUSS:
        xr, wr = np.polynomial.legendre.leggauss(q)
        np.testing.assert_allclose(xq, xr, atol=4e-15)
        np.testing.assert_allclose(wq, wr, atol=4e-15)
        # B interpolates every polynomial of degree <= p exactly
        for k in range(p + 1):
            np.testing.assert_allclose(B @ nodes ** k, xq ** k, atol=2e-14)
    else:
        np.testing.assert_allclose(xq, nodes, atol=0)
        np.testing.assert_allclose(B, np.eye(p + 1), atol=0)
        assert abs(wq.sum() - 2.0) < 1e-14
    # nodes and points are symmetric about 0, so B is centro-symmetric and D
    # anti-centro-symmetric (the kernels evaluate contractions in even-odd form)
    np.testing.assert_allclose(B[::-1, ::-1], B, atol=1e-14)
    np.testing.assert_allclose(D[::-1, ::-1], -D, atol=1e-13)
    # D differentiates every polynomial of degree < q on the points exactly
    for k in range(q):
        dk = k * xq ** (k - 1) if k else np.zeros(q)
        np.testing.assert_allclose(D @ xq ** k, dk, atol=5e-12 * max(1, k))


def test_cg_option_struct_layout():
    # int32 maxit, check_every, mode, replace_every, x0_is_zero, max_iters_exact, precond, pad_;
    # double rtol, replace_delta -- the binding must agree with the header byte for byte
    assert C.sizeof(L.mfhex_cg_opts) == 48
    assert L.mfhex_cg_opts.rtol.offset == 32 and L.mfhex_cg_opts.precond.offset == 24
    src = open(os.path.join(ROOT, "include", "mfhex.h")).read()
    assert "max_iters_exact, precond, pad_;" in src


def test_mg_option_struct_layout():
    # int32 degree, coarse_degree, power_iters, max_levels, precision, pad_; double lo, hi
    assert C.sizeof(L.mfhex_mg_opts) == 40
    assert L.mfhex_mg_opts.precision.offset == 16 and L.mfhex_mg_opts.lo.offset == 24
    src = open(os.path.join(ROOT, "include", "mfhex.h")).read()
    assert "int32_t precision, pad_;" in src
