"""Tetrahedral P_p diffusion operator -- oracle, TEST INFRASTRUCTURE ONLY.

Plain numpy / scipy; it shares no code with the GPU library.  Only the tests
and the benchmark's CPU leg use it.

The paper (Sec. 2.1 libCEED and Sec. 2.2 MAGMA) treats non-tensor elements
through the caller's full basis arrays: the interpolation / gradient matrix
of one element (all quadrature points by all basis functions) is applied to
every element, which for all elements at once is one matrix product.  This
oracle evaluates the same operator the slow, direct way: one dense element
stiffness matrix per element, from its definition, then the global sum.

Readings taken here (the paper gives no tetrahedral mesh, basis or rule):

* mesh: every hexahedron of the perturbed structured box mesh is split into
  the 6 Kuhn tetrahedra sharing its main diagonal (corner 0 to corner 7);
  tetrahedron pi (a permutation of the axes) has the cube-corner vertices
  0, e_pi0, e_pi0 + e_pi1, (1,1,1), and is affine between the physical
  positions of those corners;
* basis: Lagrange P_p on the equispaced nodes of each tetrahedron
  (barycentric multi-indices n with |n| = p), in Silvester's product form;
  the nodes of all tetrahedra are exactly the points of the hexahedral
  lattice of spacing h/p, numbered as in the hexahedral operator;
* quadrature: the collapsed (conical product) rule, Gauss-Legendre in the
  first collapsed coordinate and Gauss-Jacobi with weights (1-s) and
  (1-s)^2 in the other two, q points each (exact to degree 2q-1; q = p
  integrates the stiffness of an affine element exactly);
* operator: y = sum_e P_e^T K_e P_e x with K_e[i][j] = sum_k w_k |det J|
  grad(phi_i)^T J^-1 J^-T grad(phi_j) at the points, and the Dirichlet mask
  of the hexahedral operator (box-boundary nodes held at zero).
"""
from __future__ import annotations

import itertools
import math
from dataclasses import dataclass

import numpy as np
from scipy.special import roots_jacobi

# Kuhn tetrahedra: axis permutations; vertex k of tetrahedron t is the cube corner
# sum_{m < k} e_{pi[m]} (vertex 0 the origin, vertex 3 the opposite corner).
KUHN = list(itertools.permutations(range(3)))


def kuhn_corners(t: int) -> np.ndarray:
    """[4, 3] int cube-corner coordinates of tetrahedron t's vertices."""
    pi = KUHN[t]
    v = np.zeros((4, 3), dtype=np.int64)
    for k in range(1, 4):
        v[k] = v[k - 1]
        v[k, pi[k - 1]] = 1
    return v


def simplex_indices(p: int) -> np.ndarray:
    """[P, 4] barycentric multi-indices (n0, n1, n2, n3), sum p."""
    out = []
    for n3 in range(p + 1):
        for n2 in range(p + 1 - n3):
            for n1 in range(p + 1 - n3 - n2):
                out.append((p - n1 - n2 - n3, n1, n2, n3))
    return np.array(out, dtype=np.int64)


def n_basis(p: int) -> int:
    return (p + 1) * (p + 2) * (p + 3) // 6


def _silvester(k: int, z: np.ndarray):
    """R_k(z) = prod_{j<k} (z - j) / (k - j) and its derivative in z."""
    r = np.ones_like(z)
    dr = np.zeros_like(z)
    for j in range(k):
        f = (z - j) / (k - j)
        dr = dr * f + r / (k - j)
        r = r * f
    return r, dr


def basis(p: int, xi: np.ndarray):
    """Values [M, P] and reference gradients [M, 3, P] of the P_p Lagrange basis at points xi [M, 3]."""
    xi = np.atleast_2d(np.asarray(xi, dtype=np.float64))
    lam = np.concatenate([1.0 - xi.sum(axis=1, keepdims=True), xi], axis=1)  # [M, 4]
    idx = simplex_indices(p)
    M, P = xi.shape[0], idx.shape[0]
    val = np.empty((M, P))
    dlam = np.empty((M, 4, P))  # d phi / d lambda_i
    for m in range(P):
        R = [_silvester(int(idx[m, i]), p * lam[:, i]) for i in range(4)]
        val[:, m] = R[0][0] * R[1][0] * R[2][0] * R[3][0]
        for i in range(4):
            prod = p * R[i][1]
            for k in range(4):
                if k != i:
                    prod = prod * R[k][0]
            dlam[:, i, m] = prod
    # lambda_0 = 1 - xi_1 - xi_2 - xi_3, lambda_d = xi_d
    grad = dlam[:, 1:, :] - dlam[:, :1, :]
    return val, grad


def gauss_jacobi_01(n: int, alpha: int):
    """n-point rule for int_0^1 f(s) (1-s)^alpha ds."""
    t, w = roots_jacobi(n, alpha, 0)
    return (1.0 + t) / 2.0, w / 2.0 ** (alpha + 1)


def tet_rule(q: int):
    """Collapsed rule on the reference tetrahedron {xi >= 0, sum xi <= 1}: points [q^3, 3], weights [q^3]."""
    a, wa = gauss_jacobi_01(q, 0)
    b, wb = gauss_jacobi_01(q, 1)
    c, wc = gauss_jacobi_01(q, 2)
    pts, wts = [], []
    for k in range(q):
        for j in range(q):
            for i in range(q):
                pts.append((a[i] * (1 - b[j]) * (1 - c[k]), b[j] * (1 - c[k]), c[k]))
                wts.append(wa[i] * wb[j] * wc[k])
    return np.array(pts), np.array(wts)


@dataclass
class TetProblem:
    nex: int
    ney: int
    nez: int
    p: int
    q: int
    dirichlet: int
    vert: np.ndarray  # [(nex+1)(ney+1)(nez+1), 3]

    @property
    def n_elem(self) -> int:
        return 6 * self.nex * self.ney * self.nez

    @property
    def n_nodes(self) -> int:
        return (self.p * self.nex + 1) * (self.p * self.ney + 1) * (self.p * self.nez + 1)


def element_vertices(pr: TetProblem, e: int) -> np.ndarray:
    """[4, 3] physical vertex coordinates of element e = 6 * cube + t."""
    cube, t = divmod(e, 6)
    ex = cube % pr.nex
    ey = (cube // pr.nex) % pr.ney
    ez = cube // (pr.nex * pr.ney)
    c = kuhn_corners(t)
    vid = (ex + c[:, 0]) + (pr.nex + 1) * ((ey + c[:, 1]) + (pr.ney + 1) * (ez + c[:, 2]))
    return pr.vert[vid]


def element_nodes(pr: TetProblem, e: int) -> np.ndarray:
    """[P] global lattice node of each local node (order of simplex_indices), -1 where masked."""
    cube, t = divmod(e, 6)
    ex = cube % pr.nex
    ey = (cube // pr.nex) % pr.ney
    ez = cube // (pr.nex * pr.ney)
    c = kuhn_corners(t)
    idx = simplex_indices(pr.p)
    a = idx[:, 1:] @ c[1:]  # lattice offset n1 v1 + n2 v2 + n3 v3 inside the cube, [P, 3]
    nx, ny, nz = pr.p * pr.nex + 1, pr.p * pr.ney + 1, pr.p * pr.nez + 1
    I = pr.p * ex + a[:, 0]
    J = pr.p * ey + a[:, 1]
    K = pr.p * ez + a[:, 2]
    g = I + nx * (J + ny * K)
    if pr.dirichlet:
        bnd = (I == 0) | (I == nx - 1) | (J == 0) | (J == ny - 1) | (K == 0) | (K == nz - 1)
        g = np.where(bnd, -1, g)
    return g


def element_stiffness(pr: TetProblem, e: int) -> np.ndarray:
    """[P, P] K_e from its definition, by the collapsed rule."""
    X = element_vertices(pr, e)
    J = np.stack([X[1] - X[0], X[2] - X[0], X[3] - X[0]], axis=1)  # columns dx/dxi_d
    detJ = np.linalg.det(J)
    Jinv = np.linalg.inv(J)
    xq, wq = tet_rule(pr.q)
    _, grad = basis(pr.p, xq)  # [Q, 3, P]
    gphys = np.einsum("dc,kdp->kcp", Jinv, grad)  # d phi / dx_c = sum_d dxi_d/dx_c dphi/dxi_d
    return np.einsum("k,kcp,kcq->pq", wq * abs(detJ), gphys, gphys)


def element_volume(pr: TetProblem, e: int) -> float:
    X = element_vertices(pr, e)
    return abs(np.linalg.det(np.stack([X[1] - X[0], X[2] - X[0], X[3] - X[0]], axis=1))) / 6.0


def node_coords(pr: TetProblem) -> np.ndarray:
    """[N, 3] physical node positions (each element's affine image of its reference nodes)."""
    out = np.full((pr.n_nodes, 3), np.nan)
    ref = simplex_indices(pr.p)[:, 1:] / pr.p
    unmasked = TetProblem(pr.nex, pr.ney, pr.nez, pr.p, pr.q, 0, pr.vert)
    for e in range(pr.n_elem):
        X = element_vertices(pr, e)
        x = X[0] + ref @ np.stack([X[1] - X[0], X[2] - X[0], X[3] - X[0]])
        out[element_nodes(unmasked, e)] = x
    return out


def apply(pr: TetProblem, x: np.ndarray) -> np.ndarray:
    """y = A x: element stiffness matrices summed into the lattice vector (masked rows/columns zero)."""
    y = np.zeros(pr.n_nodes)
    for e in range(pr.n_elem):
        g = element_nodes(pr, e)
        m = g >= 0
        xe = np.where(m, x[np.maximum(g, 0)], 0.0)
        ye = element_stiffness(pr, e) @ xe
        np.add.at(y, g[m], ye[m])
    return y


def assemble(pr: TetProblem) -> np.ndarray:
    """Dense global matrix (tiny meshes only)."""
    A = np.zeros((pr.n_nodes, pr.n_nodes))
    for e in range(pr.n_elem):
        g = element_nodes(pr, e)
        K = element_stiffness(pr, e)
        m = np.nonzero(g >= 0)[0]
        A[np.ix_(g[m], g[m])] += K[np.ix_(m, m)]
    return A


def monomial_integral(a: int, b: int, c: int) -> float:
    """int over the reference tetrahedron of xi1^a xi2^b xi3^c = a! b! c! / (a+b+c+3)!."""
    return math.factorial(a) * math.factorial(b) * math.factorial(c) / math.factorial(a + b + c + 3)
