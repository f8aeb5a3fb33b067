"""Pins for the FP64 CPU oracle: it is checked against what the mathematics fixes,
never against itself or the GPU path.

Each test names the fact it relies on.  Together they are chosen so that a
plausible slip in the oracle (a wrong node, a transposed adjugate, a dropped
gradient term, a wrong restriction index, a misplaced coefficient) breaks at
least one of them.
"""
import math
import os

import numpy as np
import pytest
import scipy.sparse.linalg as spla

import oracle
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _expr(s):
    return float(eval(s.strip(), {"sqrt": math.sqrt, "__builtins__": {}}))


def _golden_rows(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append([c.strip() for c in line.split("|")])
    return rows


def _interior(pr):
    nx, ny, nz = pr.p * pr.nex + 1, pr.p * pr.ney + 1, pr.p * pr.nez + 1
    I = np.arange(pr.n_nodes)
    ix, iy, iz = I % nx, (I // nx) % ny, I // (nx * ny)
    return (ix > 0) & (ix < nx - 1) & (iy > 0) & (iy < ny - 1) & (iz > 0) & (iz < nz - 1)


def _prob(ne, p, kind, quad=oracle.GAUSS, q=None, dirichlet=0, perturb=0.1, kappa=None):
    if q is None:
        q = p + 2 if quad == oracle.GAUSS else p + 1
    v = synth.mesh_vertices(ne, ne, ne, perturb)
    return oracle.Problem(ne, ne, ne, p, q, quad, kind, dirichlet, v, kappa)


# --- 1D rules and bases --------------------------------------------------------------------

def test_quadrature_closed_forms():
    for row in _golden_rows("quadrature_closed_forms.txt"):
        head, nodes, weights = row
        rule, n = head.split()
        n = int(n)
        x, w = oracle.gll(n) if rule == "gll" else oracle.gauss(n)
        xe = np.array([_expr(s) for s in nodes.split(",")])
        we = np.array([_expr(s) for s in weights.split(",")])
        np.testing.assert_allclose(x, xe, atol=1e-15)
        np.testing.assert_allclose(w, we, atol=1e-15)


@pytest.mark.parametrize("q", range(1, 13))
def test_gauss_matches_library(q):
    x, w = oracle.gauss(q)
    xl, wl = np.polynomial.legendre.leggauss(q)
    np.testing.assert_allclose(x, xl, atol=2e-15)
    np.testing.assert_allclose(w, wl, atol=2e-15)


@pytest.mark.parametrize("p", range(2, 12))
def test_gll_interior_roots_of_dPp(p):
    x, w = oracle.gll(p)
    c = np.zeros(p + 1)
    c[p] = 1.0
    r = np.sort(np.polynomial.legendre.legroots(np.polynomial.legendre.legder(c)))
    np.testing.assert_allclose(x[1:-1], r, atol=5e-15)
    assert x[0] == -1.0 and x[-1] == 1.0
    assert abs(w.sum() - 2.0) < 1e-14


@pytest.mark.parametrize("n", range(1, 10))
def test_quadrature_exactness_degree(n):
    # Gauss with n points is exact to degree 2n-1, Gauss-Lobatto with n points to 2n-3.
    xg, wg = oracle.gauss(n)
    for k in range(2 * n):
        exact = 0.0 if k % 2 else 2.0 / (k + 1)
        assert abs(wg @ xg ** k - exact) < 1e-14
    if n >= 2:
        xl, wl = oracle.gll(n - 1)
        for k in range(2 * n - 2):
            exact = 0.0 if k % 2 else 2.0 / (k + 1)
            assert abs(wl @ xl ** k - exact) < 1e-14


@pytest.mark.parametrize("p", range(1, 9))
def test_lagrange_reproduces_monomials(p):
    xi, _ = oracle.gll(p)
    xq, _ = oracle.gauss(p + 2)
    B, G = oracle.lagrange(xi, xq)
    np.testing.assert_allclose(B.sum(axis=1), 1.0, atol=1e-13)
    np.testing.assert_allclose(G.sum(axis=1), 0.0, atol=1e-12)
    for k in range(p + 1):
        np.testing.assert_allclose(B @ xi ** k, xq ** k, atol=1e-13)
        dk = k * xq ** (k - 1) if k > 0 else np.zeros_like(xq)
        np.testing.assert_allclose(G @ xi ** k, dk, atol=1e-11)
    # collocated case: B is the identity, G the Lagrange derivative matrix at the nodes
    Bc, Gc = oracle.lagrange(xi, xi)
    np.testing.assert_allclose(Bc, np.eye(p + 1), atol=1e-14)


# --- p = 1 textbook element matrices and stencils -----------------------------------------

@pytest.mark.parametrize("h_ne", [1, 2])
def test_p1_element_rows_textbook(h_ne):
    h = 1.0 / h_ne
    for name, rule, scale, row in _golden_rows("p1_element_rows.txt"):
        qr, qn = rule.split()
        kind = oracle.MASS if name.startswith("mass") else oracle.DIFFUSION
        quad = oracle.GAUSS if qr == "gauss" else oracle.GLL
        pr = _prob(h_ne, 1, kind, quad=quad, q=int(qn), perturb=0.0)
        A = oracle.element_matrix(pr, 0)
        s = {"12/h": 12 / h, "216/h^3": 216 / h ** 3, "4/h": 4 / h}[scale]
        expect = np.array([float(v) for v in row.split(",")])
        np.testing.assert_allclose(A[0] * s, expect, atol=1e-12)
        # every vertex row is the same stencil up to the symmetry of the cube
        np.testing.assert_allclose(np.sort(A[5] * s), np.sort(expect), atol=1e-12)


def test_p1_global_stencils():
    ne = 4
    h = 1.0 / ne
    n = ne + 1
    c = 2 + n * (2 + n * 2)  # the centre node
    # BP3, Gauss q=3: 27-point stencil 8h/3 | faces 0 | edges -h/6 | corners -h/12
    A = oracle.assemble(_prob(ne, 1, oracle.DIFFUSION, q=3, perturb=0.0)).toarray()
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                m = abs(dx) + abs(dy) + abs(dz)
                expect = {0: 8 * h / 3, 1: 0.0, 2: -h / 6, 3: -h / 12}[m]
                assert abs(A[c, c + dx + n * (dy + n * dz)] - expect) < 1e-14
    # BP5, Lobatto q=2: h * 7-point stencil (6, -1)
    A = oracle.assemble(_prob(ne, 1, oracle.DIFFUSION, quad=oracle.GLL, q=2, perturb=0.0)).toarray()
    row = A[c]
    assert abs(row[c] - 6 * h) < 1e-14
    for off in (1, -1, n, -n, n * n, -n * n):
        assert abs(row[c + off] + h) < 1e-14
    assert np.count_nonzero(np.abs(row) > 1e-14) == 7


# --- mass (BP1) -------------------------------------------------------------------------

@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_mass_volume_is_one(p):
    pr = _prob(3, p, oracle.MASS)
    one = np.ones(pr.n_nodes)
    Mone = oracle.apply(pr, one)
    assert abs(one @ Mone - 1.0) < 1e-13
    assert abs(Mone.sum() - 1.0) < 1e-13


@pytest.mark.parametrize("p", [1, 2, 3])
def test_mass_gauss_p_plus_2_is_exact(p):
    # On trilinear elements the mass integrand has degree <= 2p+2 per variable, so q = p+2
    # Gauss points integrate it exactly: a much finer rule must give the same operator.
    pr = _prob(2, p, oracle.MASS)
    x = synth.uniform_vector(pr.n_nodes)
    y1 = oracle.apply(pr, x)
    y2 = oracle.apply(pr.with_(q=p + 6), x)
    assert np.abs(y1 - y2).max() <= 1e-14 * np.abs(y1).max() * 10


@pytest.mark.parametrize("p", [2, 3])
def test_mass_monomial_integrals(p):
    # Unperturbed (affine) mesh: nodal interpolants of x^a y^b z^c (a,b,c <= p) are exact and
    # u^T M v is the exact integral of u v over the unit cube.
    pr = _prob(2, p, oracle.MASS, perturb=0.0)
    X = oracle.node_coords(pr)
    rng = np.random.default_rng(3)
    for _ in range(6):
        e1 = rng.integers(0, p + 1, size=3)
        e2 = rng.integers(0, p + 1, size=3)
        u = np.prod(X ** e1, axis=1)
        v = np.prod(X ** e2, axis=1)
        exact = np.prod(1.0 / (e1 + e2 + 1.0))
        assert abs(u @ oracle.apply(pr, v) - exact) < 1e-14


# --- diffusion (BP3 / BP5) ----------------------------------------------------------------

@pytest.mark.parametrize("p,quad", [(1, oracle.GAUSS), (2, oracle.GAUSS), (3, oracle.GAUSS),
                                    (5, oracle.GAUSS), (2, oracle.GLL), (3, oracle.GLL), (4, oracle.GLL)])
def test_diffusion_annihilates_affine_fields(p, quad):
    # u = a + b.x lies in the space on trilinear meshes; its weak Laplacian vanishes at every
    # interior node, and the quadrature integrates w grad(phi)^T adj(J) b exactly.
    pr = _prob(3, p, oracle.DIFFUSION, quad=quad)
    X = oracle.node_coords(pr)
    u = 0.7 + X @ np.array([1.3, -0.4, 2.1])
    y = oracle.apply(pr, u)
    inner = _interior(pr)
    assert np.abs(y[inner]).max() < 1e-13 * np.abs(y).max() + 1e-14
    assert np.abs(y[~inner]).max() > 1e-3  # boundary flux is not zero


@pytest.mark.parametrize("kind,quad,dirichlet", [(oracle.DIFFUSION, oracle.GAUSS, 1),
                                                 (oracle.DIFFUSION, oracle.GLL, 0),
                                                 (oracle.MASS, oracle.GAUSS, 0)])
def test_symmetry(kind, quad, dirichlet):
    pr = _prob(3, 3, kind, quad=quad, dirichlet=dirichlet)
    u = synth.uniform_vector(pr.n_nodes, seed=1)
    v = synth.uniform_vector(pr.n_nodes, seed=2)
    Au, Av = oracle.apply(pr, u), oracle.apply(pr, v)
    assert abs(u @ Av - v @ Au) <= 1e-14 * np.linalg.norm(u) * np.linalg.norm(Av)


@pytest.mark.parametrize("quad", [oracle.GAUSS, oracle.GLL])
def test_spd_on_interior(quad):
    pr = _prob(2, 2, oracle.DIFFUSION, quad=quad, dirichlet=1)
    A = oracle.assemble(pr).toarray()
    inner = _interior(pr)
    ev = np.linalg.eigvalsh(A[np.ix_(inner, inner)])
    assert ev.min() > 0
    np.testing.assert_allclose(A, A.T, atol=1e-15)
    assert np.abs(A[~inner]).max() == 0.0


@pytest.mark.parametrize("kind,quad,dirichlet,kap", [(oracle.DIFFUSION, oracle.GAUSS, 1, False),
                                                     (oracle.DIFFUSION, oracle.GAUSS, 0, True),
                                                     (oracle.DIFFUSION, oracle.GLL, 1, False),
                                                     (oracle.MASS, oracle.GAUSS, 0, False)])
def test_matrix_free_equals_sparse_assembly(kind, quad, dirichlet, kap):
    pr = _prob(3, 2, kind, quad=quad, dirichlet=dirichlet)
    if kap:
        xq, _ = oracle.qpoint_geometry(pr)
        pr = pr.with_(kappa=synth.kappa_field(xq))
    A = oracle.assemble(pr)
    x = synth.uniform_vector(pr.n_nodes, nvec=3)
    y = oracle.apply(pr, x)
    assert np.abs(y - A @ x).max() < 1e-14 * np.abs(y).max() * 10


def test_kappa_sits_at_its_quadrature_point():
    # For affine u = b.x the reference gradient is exact at every point, so
    # u^T A(kappa) u = |b|^2 sum_q w_q detJ_q kappa_q, and by the partition of unity that sum
    # equals the total of the load vector of f = kappa (an independent code path).
    pr = _prob(2, 3, oracle.DIFFUSION)
    xq, _ = oracle.qpoint_geometry(pr)
    kap = synth.kappa_field(xq)
    X = oracle.node_coords(pr)
    b = np.array([0.3, -1.1, 0.8])
    u = X @ b
    lhs = u @ oracle.apply(pr.with_(kappa=kap), u)
    rhs = (b @ b) * oracle.rhs(pr, kap).sum()
    assert abs(lhs - rhs) < 1e-13 * abs(rhs)


def test_thread_count_does_not_change_result():
    pr = _prob(4, 2, oracle.DIFFUSION, dirichlet=1)
    x = synth.uniform_vector(pr.n_nodes)
    y1 = oracle.apply(pr, x, nthreads=1)
    y4 = oracle.apply(pr, x, nthreads=4)
    assert np.array_equal(y1, y4)


# --- CG and end-to-end solutions ---------------------------------------------------------

@pytest.mark.parametrize("p", [2, 3])
def test_galerkin_exactness(p):
    # Unperturbed mesh, u = x(1-x)y(1-y)z(1-z) lies in Q_p (p >= 2) and vanishes on the boundary;
    # with q = p+2 Gauss every integral is exact, so the discrete solution IS the nodal u.
    pr = _prob(3, p, oracle.DIFFUSION, dirichlet=1, perturb=0.0)
    xq, _ = oracle.qpoint_geometry(pr)
    b = oracle.rhs(pr, synth.poly_forcing(xq))
    x, hist, it, code = oracle.cg(pr, b, maxit=2000, rtol=1e-14)
    u = synth.poly_solution(oracle.node_coords(pr))
    assert np.abs(x - u).max() < 1e-12
    xs = spla.spsolve(oracle.assemble(pr)[_interior(pr)][:, _interior(pr)], b[_interior(pr)])
    assert np.abs(xs - u[_interior(pr)]).max() < 1e-12


def test_cg_matches_direct_solve_on_perturbed_mesh():
    pr = _prob(3, 2, oracle.DIFFUSION, dirichlet=1)
    inner = _interior(pr)
    b = synth.uniform_vector(pr.n_nodes) * inner
    x, hist, it, code = oracle.cg(pr, b, maxit=1000, rtol=1e-13)
    assert code == oracle.OK
    A = oracle.assemble(pr)
    xs = spla.spsolve(A[inner][:, inner], b[inner])
    assert np.abs(x[inner] - xs).max() < 1e-10 * np.abs(xs).max()
    assert np.all(x[~inner] == 0.0)
    # the logged residual norms are the true ones up to rounding drift
    assert hist[0] == pytest.approx(np.linalg.norm(b), rel=1e-15)


@pytest.mark.parametrize("p", [1, 2])
def test_manufactured_solution_converges_at_rate(p):
    # a-priori estimate: the L2 / nodal error falls like h^(p+1) (the paper quotes O(h^p) for
    # the energy norm, Sec. 1); check the observed order on two refinements.
    errs = []
    for ne in (2, 4, 8):
        pr = _prob(ne, p, oracle.DIFFUSION, dirichlet=1, perturb=0.0)
        inner = _interior(pr)
        xq, _ = oracle.qpoint_geometry(pr)
        b = oracle.rhs(pr, synth.sin_forcing(xq))
        A = oracle.assemble(pr)
        x = np.zeros(pr.n_nodes)
        x[inner] = spla.spsolve(A[inner][:, inner], b[inner])
        errs.append(np.abs(x - synth.sin_solution(oracle.node_coords(pr))).max())
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert rates[-1] > p + 1 - 0.3, (errs, rates)


# --- gradient with respect to the coefficient --------------------------------------------

def test_kappa_gradient_central_differences_are_exact():
    # L(kappa) = 0.5 ||A(kappa) u - f||^2 is exactly quadratic in kappa, so a central difference
    # equals the directional derivative up to rounding, for any step.
    pr = _prob(2, 2, oracle.DIFFUSION, dirichlet=1)
    xq, _ = oracle.qpoint_geometry(pr)
    kap = synth.kappa_field(xq)
    inner = _interior(pr)
    u = synth.uniform_vector(pr.n_nodes, seed=1) * inner
    f = synth.uniform_vector(pr.n_nodes, seed=2) * inner

    def loss(k):
        r = oracle.apply(pr.with_(kappa=k), u) - f
        return 0.5 * r @ r

    r = oracle.apply(pr.with_(kappa=kap), u) - f
    g = oracle.kappa_grad(pr.with_(kappa=kap), u, r)
    rng = np.random.default_rng(synth.SEED_DIR)
    for _ in range(4):
        d = rng.standard_normal(kap.shape)
        eps = 1e-2 * np.linalg.norm(kap) / np.linalg.norm(d)
        fd = (loss(kap + eps * d) - loss(kap - eps * d)) / (2 * eps)
        an = (g * d).sum()
        assert abs(fd - an) <= 1e-9 * abs(an)
    # single components, including one on an element touching the boundary
    for (e, q) in [(0, 0), (3, 17), (7, 63)]:
        d = np.zeros_like(kap)
        d[e, q] = 1.0
        fd = (loss(kap + 0.5 * d) - loss(kap - 0.5 * d)) / 1.0
        assert abs(fd - g[e, q]) <= 1e-9 * max(1.0, abs(g[e, q]))


# --- operator diagonal and Jacobi-preconditioned CG ---------------------------------------

@pytest.mark.parametrize("kind,quad,dirichlet,with_kappa", [
    (oracle.DIFFUSION, oracle.GAUSS, 1, False), (oracle.DIFFUSION, oracle.GAUSS, 0, True),
    (oracle.DIFFUSION, oracle.GLL, 1, False), (oracle.MASS, oracle.GAUSS, 0, False)])
def test_diagonal_is_the_diagonal_of_the_applied_identity(kind, quad, dirichlet, with_kappa):
    # A e_i for every unit vector e_i (the apply on the identity, one column per node) gives
    # the dense matrix; its diagonal must be what orc_diagonal accumulates element by element
    kappa = None
    if with_kappa:
        pr0 = _prob(2, 2, kind, quad, dirichlet=dirichlet)
        xq, _ = oracle.qpoint_geometry(pr0)
        kappa = synth.kappa_field(xq.reshape(-1, 3)).reshape(pr0.n_elem, -1)
    pr = _prob(2, 2, kind, quad, dirichlet=dirichlet, kappa=kappa)
    A = oracle.apply(pr, np.eye(pr.n_nodes))
    d = oracle.diagonal(pr)
    np.testing.assert_allclose(d, np.diag(A), rtol=1e-13, atol=1e-15 * np.abs(d).max())
    if dirichlet:
        assert np.all(d[~_interior(pr)] == 0.0) and np.all(d[_interior(pr)] > 0.0)


def test_pcg_matches_direct_solve():
    pr = _prob(3, 2, oracle.DIFFUSION, dirichlet=1)
    inner = _interior(pr)
    b = synth.uniform_vector(pr.n_nodes) * inner
    dinv = oracle.jacobi_inverse(oracle.diagonal(pr))
    x, hist, it, code = oracle.pcg(pr, b, dinv, maxit=1000, rtol=1e-13)
    assert code == oracle.OK
    xs = spla.spsolve(oracle.assemble(pr)[inner][:, inner], b[inner])
    assert np.abs(x[inner] - xs).max() < 1e-10 * np.abs(xs).max()
    assert np.all(x[~inner] == 0.0)


def test_pcg_with_identity_scaling_is_cg():
    # Dinv = 1 on the unmasked nodes (0 on masked ones, where r is 0 anyway) makes z = r, so
    # r.z = r.r and every iterate equals plain CG's: the histories agree to the last bit
    pr = _prob(3, 3, oracle.DIFFUSION, dirichlet=1)
    inner = _interior(pr)
    b = synth.uniform_vector(pr.n_nodes) * inner
    _, h_cg, it_cg, _ = oracle.cg(pr, b, maxit=60, rtol=0.0)
    _, h_pcg, it_pcg, _ = oracle.pcg(pr, b, inner.astype(np.float64), maxit=60, rtol=0.0)
    assert it_cg == it_pcg == 60
    assert np.array_equal(h_cg, h_pcg)


def test_jacobi_cuts_iterations_for_a_high_contrast_coefficient():
    # kappa varying over four orders of magnitude across the mesh: diagonal scaling removes the
    # coefficient scale from the spectrum, so PCG needs far fewer iterations than CG
    pr0 = _prob(4, 2, oracle.DIFFUSION, dirichlet=1)
    xq, _ = oracle.qpoint_geometry(pr0)
    xyz = xq.reshape(pr0.n_elem, -1, 3)
    kappa = 10.0 ** (4.0 * xyz[:, :, 0])
    pr = _prob(4, 2, oracle.DIFFUSION, dirichlet=1, kappa=kappa)
    b = synth.uniform_vector(pr.n_nodes) * _interior(pr)
    _, _, it_cg, c1 = oracle.cg(pr, b, maxit=5000, rtol=1e-10)
    _, _, it_pcg, c2 = oracle.pcg(pr, b, oracle.jacobi_inverse(oracle.diagonal(pr)), maxit=5000, rtol=1e-10)
    assert c1 == oracle.OK and c2 == oracle.OK
    assert it_pcg < 0.5 * it_cg


# --- p-multigrid (oracle) -------------------------------------------------------------------

def test_splitmix_uniform_follows_the_published_definition():
    # SplitMix64 (Steele, Lea, Flood 2014): from state 1234567 the first output is
    # 6457827717110365317; the vectorized generator must agree with plain integer arithmetic
    M = (1 << 64) - 1

    def mix(z):
        z = (z + 0x9E3779B97F4A7C15) & M
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M
        return z ^ (z >> 31)

    assert mix(1234567) == 6457827717110365317
    seed = 99
    v = synth.splitmix_uniform(7, seed)
    for i in range(7):
        z = mix((seed * 0x632BE59BD9B4E019 + i) & M)
        assert v[i] == 2.0 * ((z >> 11) / 9007199254740992.0) - 1.0


def test_prolongation_reproduces_coarse_polynomials_on_affine_meshes():
    # unperturbed mesh: a polynomial of degree <= p_c in each variable lies in the coarse space,
    # so its coarse nodal values prolong to its values at the fine nodes (interpolation exactness)
    from oracle import multigrid as mg
    for pc, pf in [(1, 2), (1, 3), (2, 4), (2, 5), (3, 6), (4, 8)]:
        prf = _prob(2, pf, oracle.DIFFUSION, perturb=0.0)
        prc = mg.level_problem(prf, pc)
        P = mg.prolongation(prc, prf)
        f = lambda X: X[:, 0] ** pc * (1 + X[:, 1]) + X[:, 2] ** pc - 2 * X[:, 0] * X[:, 1] * X[:, 2] ** (pc - 1)
        xc = f(oracle.node_coords(prc))
        np.testing.assert_allclose(P @ xc, f(oracle.node_coords(prf)), atol=1e-13)
        # partition of unity on the perturbed mesh too (no mask)
        prf2 = _prob(2, pf, oracle.DIFFUSION)
        P2 = mg.prolongation(mg.level_problem(prf2, pc), prf2)
        np.testing.assert_allclose(P2 @ np.ones(P2.shape[1]), 1.0, atol=1e-13)


def test_chebyshev_meets_its_error_bound():
    # with the exact extreme eigenvalues of D^-1 A (dense generalized eigenproblem on a tiny
    # mesh), k Chebyshev steps reduce the A-norm error by at most 2 c^k / (1 + c^2k),
    # c = (sqrt(kappa) - 1) / (sqrt(kappa) + 1) -- the textbook minimax bound
    import scipy.linalg as sla
    from oracle import multigrid as mg
    pr = _prob(2, 2, oracle.DIFFUSION, dirichlet=1)
    inner = _interior(pr)
    A = oracle.apply(pr, np.eye(pr.n_nodes))[np.ix_(inner, inner)]
    d = oracle.diagonal(pr)
    dinv = oracle.jacobi_inverse(d)
    ev = sla.eigh(A, np.diag(d[inner]), eigvals_only=True)
    lo, hi = ev[0], ev[-1]
    b = synth.uniform_vector(pr.n_nodes) * inner
    xs = np.zeros(pr.n_nodes)
    xs[inner] = np.linalg.solve(A, b[inner])
    kap = hi / lo
    c = (np.sqrt(kap) - 1) / (np.sqrt(kap) + 1)
    e0 = np.sqrt(xs[inner] @ A @ xs[inner])
    for k in (1, 2, 4, 8, 16):
        x = mg.chebyshev(pr, dinv, lo, hi, b, np.zeros(pr.n_nodes), k)
        e = xs[inner] - x[inner]
        assert np.sqrt(e @ A @ e) <= 2 * c ** k / (1 + c ** (2 * k)) * e0 * (1 + 1e-10)


def test_power_method_brackets_the_top_eigenvalue():
    import scipy.linalg as sla
    from oracle import multigrid as mg
    pr = _prob(2, 3, oracle.DIFFUSION, dirichlet=1)
    inner = _interior(pr)
    A = oracle.apply(pr, np.eye(pr.n_nodes))[np.ix_(inner, inner)]
    d = oracle.diagonal(pr)
    top = sla.eigh(A, np.diag(d[inner]), eigvals_only=True)[-1]
    lam = mg.lambda_max(pr, oracle.jacobi_inverse(d), 15, 2024)
    assert 0.85 * top <= lam <= top * (1 + 1e-12)


def test_vcycle_is_a_symmetric_positive_preconditioner_and_mg_pcg_solves():
    from oracle import multigrid as mg
    pr = _prob(3, 4, oracle.DIFFUSION, dirichlet=1)
    h = mg.Hierarchy(pr)
    assert [L["pr"].p for L in h.levels] == [4, 2, 1]
    inner = _interior(pr)
    u = synth.uniform_vector(pr.n_nodes, seed=1) * inner
    v = synth.uniform_vector(pr.n_nodes, seed=2) * inner
    Mu, Mv = h.vcycle(u), h.vcycle(v)
    # symmetric (R = P^T, equal pre- and post-smoothers) and positive definite
    assert abs(u @ Mv - v @ Mu) <= 1e-12 * abs(u @ Mv)
    assert u @ Mu > 0 and v @ Mv > 0
    b = synth.uniform_vector(pr.n_nodes, seed=3) * inner
    x, hist, it = mg.mg_pcg(h, b, maxit=200, rtol=1e-10)
    xs = spla.spsolve(oracle.assemble(pr)[inner][:, inner], b[inner])
    assert np.abs(x[inner] - xs).max() < 1e-8 * np.abs(xs).max()
    _, _, it_j, _ = oracle.pcg(pr, b, oracle.jacobi_inverse(oracle.diagonal(pr)), maxit=2000, rtol=1e-10)
    assert it < 0.3 * it_j
