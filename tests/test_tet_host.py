"""Host-side checks of the tetrahedral C ABI (no GPU): sizes, rejects, struct layouts, and the
library's reference rule and basis against the oracle's independent construction (scipy
Gauss-Jacobi roots, numpy Silvester products)."""
import ctypes as C
import os

import numpy as np
import pytest

import synth
from oracle import tet as otet
from paper_2109_05072_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _desc(nex=2, ney=2, nez=2, p=2, q=None, dirichlet=1):
    vert = synth.mesh_vertices(max(nex, 1), max(ney, 1), max(nez, 1))
    d = L.mfhex_tet_desc(nex, ney, nez, p, p if q is None else q, dirichlet,
                         vert.ctypes.data_as(C.POINTER(C.c_double)))
    d._keep = vert
    return d


def test_struct_layouts_match_the_header():
    assert C.sizeof(L.mfhex_tet_desc) == 32 and L.mfhex_tet_desc.vertex_xyz.offset == 24
    assert C.sizeof(L.mfhex_tet_sizes) == 40 and L.mfhex_tet_sizes.n_basis.offset == 32
    src = open(os.path.join(ROOT, "include", "mfhex.h")).read()
    assert "int32_t nex, ney, nez, p, q, dirichlet;" in src and "int32_t n_basis, n_points;" in src


@pytest.mark.parametrize("p,q", [(1, 1), (2, 3), (4, 4), (6, 6)])
def test_query_sizes(p, q):
    s = L.mfhex_tet_query(_desc(3, 2, 4, p, q))
    assert s.n_elem == 6 * 24 and s.n_nodes == (3 * p + 1) * (2 * p + 1) * (4 * p + 1)
    assert s.n_basis == (p + 1) * (p + 2) * (p + 3) // 6 and s.n_points == q ** 3
    assert s.n_qpts == s.n_elem * q ** 3
    groups = -(-s.n_elem // 16)
    # at least the per-point factors and the element restriction of every 16-element group
    assert s.workspace_bytes >= groups * 16 * (6 * 8 * q ** 3 + 4 * s.n_basis)


@pytest.mark.parametrize("kw,code", [(dict(p=7), L.MFHEX_ERR_UNSUPPORTED), (dict(p=0), L.MFHEX_ERR_UNSUPPORTED),
                                     (dict(p=3, q=5), L.MFHEX_ERR_UNSUPPORTED),
                                     (dict(p=3, q=2), L.MFHEX_ERR_UNSUPPORTED),
                                     (dict(nex=0), L.MFHEX_ERR_ARG)])
def test_query_rejects(kw, code):
    with pytest.raises(L.MFHexError) as ei:
        L.mfhex_tet_query(_desc(**kw))
    assert ei.value.code == code


@pytest.mark.parametrize("p,q", [(1, 1), (2, 2), (3, 4), (4, 4), (5, 6), (6, 6), (6, 7)])
def test_library_rule_and_basis_match_the_oracle(p, q):
    xi, w, B, G = L.mfhex_tet_basis(p, q)
    oxi, ow = otet.tet_rule(q)
    np.testing.assert_allclose(xi, oxi, rtol=0, atol=2e-15)
    np.testing.assert_allclose(w, ow, rtol=1e-13, atol=0)
    ob, og = otet.basis(p, oxi)
    scale = max(1.0, np.abs(og).max())
    np.testing.assert_allclose(B, ob, rtol=0, atol=1e-13)
    np.testing.assert_allclose(G, np.transpose(og, (1, 0, 2)), rtol=0, atol=1e-13 * scale)
