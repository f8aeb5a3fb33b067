"""GPU parity of the tetrahedral P_p operator (matrix-core basis products) against the oracle.

Tolerance: max-norm relative 1e-12, as for the hexahedral FP64 apply.  Both sides compute the
same sums of FP64 products of length ~3(P + Q) in different orders (the oracle forms K_e first),
so the difference is a few hundred unit roundoffs of the largest term; 1e-12 leaves margin.
"""
import numpy as np
import pytest
import torch

import synth
from oracle import tet as otet

pytestmark = pytest.mark.gpu

TOL64 = 1e-12


def _say(*a):
    print("[case]", *a, flush=True)


def relerr(a, b):
    return float(np.abs(np.asarray(a) - np.asarray(b)).max() / max(np.abs(np.asarray(b)).max(), 1e-300))


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda", torch.float64)


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def build(mf, ne, p, q=None, dirichlet=True, perturb=0.1):
    vert = synth.mesh_vertices(*ne, perturb)
    op = mf.TetOperator(*ne, p, vert, q=q, dirichlet=dirichlet)
    pr = otet.TetProblem(*ne, p, q or p, int(dirichlet), vert)
    return op, pr


@pytest.mark.parametrize("p", range(1, 7))
@pytest.mark.parametrize("dq", [0, 1])
@pytest.mark.parametrize("dirichlet", [True, False])
def test_tet_apply_matches_oracle(gpu_lib, p, dq, dirichlet):
    # 3 x 2 x 2 cubes = 72 tetrahedra: four full groups of 16 and a ragged fifth of 8
    _say("tet apply", p, p + dq, dirichlet)
    op, pr = build(gpu_lib, (3, 2, 2), p, p + dq, dirichlet)
    assert op.n_elem == 72 and op.n_nodes == pr.n_nodes
    x = synth.uniform_vector(pr.n_nodes)
    y = host(op.apply(dev(x)))
    yo = otet.apply(pr, x)
    print("tet rel err", p, p + dq, dirichlet, relerr(y, yo))
    assert relerr(y, yo) <= TOL64
    # twice in a row on the same output: y is overwritten, not accumulated
    y2 = host(op.apply(dev(x), dev(np.full(pr.n_nodes, 7.0))))
    assert np.array_equal(y2, y) or relerr(y2, y) <= 1e-15


@pytest.mark.parametrize("p", [2, 4, 6])
def test_tet_kills_constants_and_linears_on_a_larger_mesh(gpu_lib, p):
    # unmasked: A 1 = 0; (A u)_i = 0 at interior nodes for u linear in x; u^T A u = |a|^2 |Omega|
    ne = (6, 5, 4)
    op, pr = build(gpu_lib, ne, p, dirichlet=False)
    pos = otet.node_coords(pr)
    y1 = host(op.apply(dev(np.ones(pr.n_nodes))))
    a = np.array([0.3, -1.2, 0.7])
    u = pos @ a + 0.4
    yu = host(op.apply(dev(u)))
    scale = np.abs(host(op.apply(dev(synth.uniform_vector(pr.n_nodes))))).max()
    nx, ny, nz = p * ne[0] + 1, p * ne[1] + 1, p * ne[2] + 1
    n = np.arange(pr.n_nodes)
    I, J, K = n % nx, (n // nx) % ny, n // (nx * ny)
    inner = (I > 0) & (I < nx - 1) & (J > 0) & (J < ny - 1) & (K > 0) & (K < nz - 1)
    assert np.abs(y1).max() <= 1e-12 * scale
    assert np.abs(yu[inner]).max() <= 1e-12 * scale * np.abs(u).max()
    assert abs(u @ yu - a @ a) <= 1e-11


def _sampled_oracle(pr, x, nodes):
    """y at the given lattice nodes from the oracle's element matrices of the elements holding them."""
    p = pr.p
    nx, ny = p * pr.nex + 1, p * pr.ney + 1
    out = []
    for g in nodes:
        I, J, K = g % nx, (g // nx) % ny, g // (nx * ny)
        acc = 0.0
        cubes = set()
        for ex in {min(I // p, pr.nex - 1), max((I - 1) // p, 0)}:
            for ey in {min(J // p, pr.ney - 1), max((J - 1) // p, 0)}:
                for ez in {min(K // p, pr.nez - 1), max((K - 1) // p, 0)}:
                    cubes.add(ex + pr.nex * (ey + pr.ney * ez))
        for c in sorted(cubes):
            for t in range(6):
                e = 6 * c + t
                en = otet.element_nodes(pr, e)
                hit = np.nonzero(en == g)[0]
                if len(hit):
                    m = en >= 0
                    xe = np.where(m, x[np.maximum(en, 0)], 0.0)
                    acc += (otet.element_stiffness(pr, e) @ xe)[hit[0]]
        out.append(acc)
    return np.array(out)


@pytest.mark.parametrize("p", [2, 4, 6])
def test_tet_full_size_sampled(gpu_lib, p):
    # the benchmark's size (about 1e7 nodes), sampled nodes against the oracle's element sums
    ne = synth.elems_for_dofs(1e7, p)
    _say("tet full size", p, ne)
    op, pr = build(gpu_lib, (ne, ne, ne), p)
    x = synth.uniform_vector(pr.n_nodes)
    y = host(op.apply(dev(x)))
    rng = np.random.default_rng(5)
    nx = p * ne + 1
    # interior, near-boundary and cube-corner nodes
    picks = list(rng.integers(0, pr.n_nodes, 24)) + [nx * nx + nx + 1, (nx * nx + nx + 1) * p,
                                                     pr.n_nodes // 2, pr.n_nodes - nx * nx - nx - 2]
    ys = _sampled_oracle(pr, x, picks)
    scale = np.abs(y).max()
    err = np.abs(y[picks] - ys).max() / scale
    print("tet sampled rel err", p, err)
    assert err <= TOL64


def test_tet_rejects_aliasing_and_bad_sizes(gpu_lib):
    from paper_2109_05072_amd import _lib as L
    op, pr = build(gpu_lib, (2, 2, 2), 2)
    x = dev(synth.uniform_vector(pr.n_nodes))
    with pytest.raises(L.MFHexError) as ei:
        L.mfhex_tet_apply(op.handle, x.data_ptr(), x.data_ptr(), torch.cuda.current_stream().cuda_stream)
    assert ei.value.code == L.MFHEX_ERR_ARG
    # partial overlap: y starts inside x
    big = dev(np.zeros(2 * pr.n_nodes))
    with pytest.raises(L.MFHexError) as ei:
        L.mfhex_tet_apply(op.handle, big.data_ptr(), big.data_ptr() + 8 * (pr.n_nodes - 1),
                          torch.cuda.current_stream().cuda_stream)
    assert ei.value.code == L.MFHEX_ERR_ARG
    with pytest.raises(ValueError):
        op.apply(x[:-1].contiguous())
    with pytest.raises(L.MFHexError) as ei:
        gpu_lib.TetOperator(2, 2, 2, 7, synth.mesh_vertices(2, 2, 2))
    assert ei.value.code == L.MFHEX_ERR_UNSUPPORTED


def test_tet_degenerate_element_is_reported(gpu_lib):
    # two neighbouring interior vertices moved onto each other: every tetrahedron holding the edge
    # between them has two equal corners, det J = 0
    from paper_2109_05072_amd import _lib as L
    vert = synth.mesh_vertices(4, 3, 3)
    v = lambda i, j, k: i + 5 * (j + 4 * k)
    vert[v(2, 1, 1)] = vert[v(1, 1, 1)]
    with pytest.raises(L.MFHexError) as ei:
        gpu_lib.TetOperator(4, 3, 3, 2, vert)
    assert ei.value.code == L.MFHEX_ERR_MESH


def test_tet_fully_masked_mesh_gives_zero(gpu_lib):
    # one cube, p = 1: all 8 nodes lie on the box boundary
    op, pr = build(gpu_lib, (1, 1, 1), 1)
    assert op.n_elem == 6 and op.n_nodes == 8
    y = host(op.apply(dev(synth.uniform_vector(8)), dev(np.full(8, 3.0))))
    assert np.all(y == 0.0)
