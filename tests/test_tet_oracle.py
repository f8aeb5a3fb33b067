"""Pins of the tetrahedral oracle (CPU): closed forms, invariants and brute force, chosen so that a
wrong index, sign or weight anywhere in the basis, rule, mesh or element matrix fails one of them."""
import itertools

import numpy as np
import pytest

import synth
from oracle import tet


@pytest.mark.parametrize("q", range(1, 8))
def test_rule_integrates_monomials_exactly(q):
    # collapsed Gauss-Jacobi rule: exact to degree 2q-1 on the reference tetrahedron
    x, w = tet.tet_rule(q)
    assert np.all(w > 0) and np.all(x >= 0) and np.all(x.sum(axis=1) <= 1)
    for a, b, c in itertools.product(range(2 * q), repeat=3):
        if a + b + c <= 2 * q - 1:
            got = np.sum(w * x[:, 0] ** a * x[:, 1] ** b * x[:, 2] ** c)
            assert abs(got - tet.monomial_integral(a, b, c)) <= 1e-14, (q, a, b, c)


def test_rule_is_not_exact_beyond_its_degree():
    # the one-point rule must miss a quadratic: guards against a rule that is secretly richer or a
    # test that checks nothing
    x, w = tet.tet_rule(1)
    assert abs(np.sum(w * x[:, 0] ** 2) - tet.monomial_integral(2, 0, 0)) > 1e-3


@pytest.mark.parametrize("p", range(1, 7))
def test_basis_is_nodal_and_reproduces_linears(p):
    idx = tet.simplex_indices(p)
    assert len(idx) == tet.n_basis(p) and np.all(idx.sum(axis=1) == p) and np.all(idx >= 0)
    nodes = idx[:, 1:] / p
    val, grad = tet.basis(p, nodes)
    assert np.allclose(val, np.eye(len(idx)), atol=1e-13)
    pts = synth.splitmix_uniform(60, 11).reshape(20, 3) * 0.5 + 0.5
    pts = pts / np.maximum(1.0, pts.sum(axis=1, keepdims=True)) * 0.999
    val, grad = tet.basis(p, pts)
    assert np.allclose(val.sum(axis=1), 1.0, atol=1e-13)          # partition of unity
    assert np.allclose(grad.sum(axis=2), 0.0, atol=1e-11)         # its gradient vanishes
    assert np.allclose(val @ nodes, pts, atol=1e-13)              # reproduces xi
    assert np.allclose(grad @ nodes, np.broadcast_to(np.eye(3), (len(pts), 3, 3)), atol=1e-11)


@pytest.mark.parametrize("p", [2, 4, 6])
def test_basis_gradient_matches_finite_differences(p):
    pts = np.array([[0.1, 0.2, 0.3], [0.25, 0.05, 0.4], [0.3, 0.3, 0.1]])
    _, grad = tet.basis(p, pts)
    h = 1e-6
    for d in range(3):
        e = np.zeros(3)
        e[d] = h
        fd = (tet.basis(p, pts + e)[0] - tet.basis(p, pts - e)[0]) / (2 * h)
        assert np.allclose(grad[:, d, :], fd, atol=1e-6 * p ** 2)


def test_kuhn_tetrahedra_tile_the_cube():
    # six tetrahedra of volume 1/6 each, all sharing the main diagonal, disjoint interiors: a point
    # of the cube with distinct coordinates lies in exactly one of them (x_pi0 > x_pi1 > x_pi2)
    vols = []
    for t in range(6):
        c = tet.kuhn_corners(t).astype(float)
        vols.append(abs(np.linalg.det(c[1:] - c[0])) / 6)
        assert list(c[0]) == [0, 0, 0] and list(c[3]) == [1, 1, 1]
    assert np.allclose(vols, 1 / 6)
    pt = np.array([0.7, 0.2, 0.5])
    inside = 0
    for t in range(6):
        c = tet.kuhn_corners(t).astype(float)
        lam = np.linalg.solve(np.vstack([np.ones(4), c.T]), np.concatenate([[1.0], pt]))
        inside += bool(np.all(lam > 0))
    assert inside == 1


def problem(ne=(2, 2, 1), p=2, q=None, dirichlet=1, perturb=0.1):
    vert = synth.mesh_vertices(*ne, perturb)
    return tet.TetProblem(*ne, p, q or p, dirichlet, vert)


@pytest.mark.parametrize("p", [1, 2, 3])
def test_mesh_is_conforming_and_fills_the_box(p):
    pr = problem((2, 2, 2), p, dirichlet=0)
    vol = sum(tet.element_volume(pr, e) for e in range(pr.n_elem))
    assert abs(vol - 1.0) <= 1e-14  # box boundary vertices are not perturbed
    # every lattice node is reached, and every element that holds a node puts it in the same place
    pos = tet.node_coords(pr)
    assert not np.isnan(pos).any()
    ref = tet.simplex_indices(p)[:, 1:] / p
    for e in range(pr.n_elem):
        X = tet.element_vertices(pr, e)
        x = X[0] + ref @ np.stack([X[1] - X[0], X[2] - X[0], X[3] - X[0]])
        assert np.allclose(pos[tet.element_nodes(pr, e)], x, atol=1e-14)


def test_linear_element_matches_textbook_formula():
    # P1: K_e = vol * grad(lambda_i) . grad(lambda_j), grad(lambda) from the inverse vertex matrix
    pr = problem((1, 1, 1), 1, q=1, dirichlet=0, perturb=0.0)
    pr.vert = pr.vert + 0.05 * synth.splitmix_uniform(pr.vert.size, 3).reshape(pr.vert.shape)
    for e in range(6):
        X = tet.element_vertices(pr, e)
        M = np.vstack([np.ones(4), X.T])  # lambda = M^-1 [1; x]
        gl = np.linalg.inv(M)[:, 1:]       # [4, 3] grad lambda_i
        K = tet.element_volume(pr, e) * gl @ gl.T
        assert np.allclose(tet.element_stiffness(pr, e), K, atol=1e-13)


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_operator_kills_constants_and_linears_inside(p):
    # unmasked: A 1 = 0; for a linear u, (A u)_i = 0 at every node whose basis function vanishes on
    # the boundary, and u^T A u = |grad u|^2 |Omega| (quadrature q = p is exact for affine elements)
    pr = problem((2, 2, 2), p, dirichlet=0)
    pos = tet.node_coords(pr)
    ones = np.ones(pr.n_nodes)
    assert np.abs(tet.apply(pr, ones)).max() <= 1e-12
    a = np.array([0.3, -1.2, 0.7])
    u = pos @ a + 0.4
    y = tet.apply(pr, u)
    nx, ny, nz = p * pr.nex + 1, p * pr.ney + 1, p * pr.nez + 1
    I, J, K = np.arange(pr.n_nodes) % nx, (np.arange(pr.n_nodes) // nx) % ny, np.arange(pr.n_nodes) // (nx * ny)
    interior = (I > 0) & (I < nx - 1) & (J > 0) & (J < ny - 1) & (K > 0) & (K < nz - 1)
    assert np.abs(y[interior]).max() <= 1e-12
    assert abs(u @ y - a @ a) <= 1e-12


@pytest.mark.parametrize("p", [2, 3])
def test_masked_operator_is_spd_and_apply_equals_assembled(p):
    pr = problem((2, 1, 2), p)
    A = tet.assemble(pr)
    assert np.allclose(A, A.T, atol=1e-13)
    x = synth.uniform_vector(pr.n_nodes)
    assert np.allclose(tet.apply(pr, x), A @ x, atol=1e-12)
    nx, ny, nz = p * pr.nex + 1, p * pr.ney + 1, p * pr.nez + 1
    n = np.arange(pr.n_nodes)
    I, J, K = n % nx, (n // nx) % ny, n // (nx * ny)
    inner = (I > 0) & (I < nx - 1) & (J > 0) & (J < ny - 1) & (K > 0) & (K < nz - 1)
    Ai = A[np.ix_(inner, inner)]
    assert np.linalg.eigvalsh(Ai).min() > 0
    assert np.all(A[~inner] == 0) and np.all(A[:, ~inner] == 0)


def test_mutation_a_wrong_jacobian_transpose_is_caught():
    # planting J^-T in place of J^-1 in the gradient map must break the linear-field identity
    pr = problem((1, 1, 1), 2, dirichlet=0)
    e = 1
    X = tet.element_vertices(pr, e)
    J = np.stack([X[1] - X[0], X[2] - X[0], X[3] - X[0]], axis=1)
    xq, wq = tet.tet_rule(2)
    _, grad = tet.basis(2, xq)
    wrong = np.einsum("cd,kdp->kcp", np.linalg.inv(J), grad)
    Kw = np.einsum("k,kcp,kcq->pq", wq * abs(np.linalg.det(J)), wrong, wrong)
    ref = tet.simplex_indices(2)[:, 1:] / 2
    x = X[0] + ref @ np.stack([X[1] - X[0], X[2] - X[0], X[3] - X[0]])
    a = np.array([0.3, -1.2, 0.7])
    u = x @ a
    vol = tet.element_volume(pr, e)
    assert abs(u @ tet.element_stiffness(pr, e) @ u - (a @ a) * vol) <= 1e-13
    assert abs(u @ Kw @ u - (a @ a) * vol) > 1e-6
