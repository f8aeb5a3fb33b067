"""p-multigrid V-cycle with Chebyshev-Jacobi smoothing -- oracle, TEST INFRASTRUCTURE ONLY.

Plain numpy / scipy on top of the oracle's own matrix-free apply and
diagonal (``oracle.apply``, ``oracle.diagonal``); it shares no code with the
GPU library.  Only the tests and the benchmark's CPU leg use it.

The paper (Sec. 1) notes that high-order codes replace low-order
preconditioners by p-multigrid, and the Nek5000/RS solvers of Sec. 2
smooth with Chebyshev-accelerated Jacobi.  The details are not given there;
the readings taken here (also listed in the design notes) are:

* levels p, floor(p/2), ..., 1 on the same mesh, same quadrature family
  (Gauss q = p_l + 2, or Gauss-Lobatto q = p_l + 1) and Dirichlet mask;
* prolongation P: the coarse finite-element field evaluated at the fine
  nodes (tensor Lagrange interpolation from the coarse to the fine
  Gauss-Lobatto nodes in every element; exact since Q_pc is in Q_pf);
  restriction R = P^T;
* smoother: Chebyshev iteration on D^-1 A (D the operator diagonal) over
  [lo lambda, hi lambda], lambda from ``power_iters`` steps of the power
  method on D^-1 A started from the counter-based vector
  ``synth.splitmix_uniform(n, seed)`` (masked), with the generalized Rayleigh
  quotient v^T A v / v^T D v of the last iterate;
* V-cycle: pre-smooth (degree k from x = 0), restrict the residual, recurse,
  prolong and add, post-smooth (degree k); the coarsest level is smoothed
  only (degree k_coarse) -- no exact coarse solve.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

import synth

from . import GAUSS, Problem, apply, diagonal, element_nodes, gll, jacobi_inverse, lagrange

DEFAULTS = dict(degree=3, coarse_degree=8, lo=0.25, hi=1.1, power_iters=15, seed=2024)


def level_orders(p: int):
    """p, floor(p/2), ..., 1."""
    out = [p]
    while out[-1] > 1:
        out.append(max(1, out[-1] // 2))
    return out


def level_problem(pr: Problem, p: int) -> Problem:
    return pr.with_(p=p, q=p + 2 if pr.quad == GAUSS else p + 1)


def interpolation_1d(pc: int, pf: int) -> np.ndarray:
    """[pf+1, pc+1]: coarse Gauss-Lobatto Lagrange basis at the fine Gauss-Lobatto nodes."""
    xc, _ = gll(pc)
    xf, _ = gll(pf)
    return lagrange(xc, xf)[0]


def prolongation(prc: Problem, prf: Problem) -> sp.csr_matrix:
    """P [N_f, N_c]: P[i, j] = coarse basis function j at fine node i (masked nodes dropped)."""
    I1 = interpolation_1d(prc.p, prf.p)
    I3 = np.kron(np.kron(I1, I1), I1)  # local index i + P (j + P k) on both sides
    rows, cols, vals = [], [], []
    done = np.zeros(prf.n_nodes, dtype=bool)
    for e in range(prf.n_elem):
        gf = element_nodes(prf, e)
        gc = element_nodes(prc, e)
        for r in np.nonzero((gf >= 0) & ~done[np.maximum(gf, 0)])[0]:
            done[gf[r]] = True
            for c in np.nonzero(gc >= 0)[0]:
                if I3[r, c] != 0.0:
                    rows.append(gf[r])
                    cols.append(gc[c])
                    vals.append(I3[r, c])
    return sp.csr_matrix((vals, (rows, cols)), shape=(prf.n_nodes, prc.n_nodes))


def lambda_max(pr: Problem, dinv: np.ndarray, iters: int, seed: int) -> float:
    """Power method on D^-1 A; returns v^T A v / v^T D v of the last iterate."""
    mask = dinv > 0
    v = synth.splitmix_uniform(pr.n_nodes, seed) * mask
    v = v / np.linalg.norm(v)
    d = np.where(mask, 1.0 / np.where(mask, dinv, 1.0), 0.0)
    lam = 0.0
    for _ in range(iters):
        Av = apply(pr, v)
        lam = (v @ Av) / (v @ (d * v))
        w = dinv * Av
        v = w / np.linalg.norm(w)
    return float(lam)


def chebyshev(pr: Problem, dinv: np.ndarray, lo: float, hi: float, b: np.ndarray, x: np.ndarray,
              degree: int) -> np.ndarray:
    """``degree`` steps of the Chebyshev iteration for A x = b preconditioned by D^-1, for
    eigenvalues of D^-1 A in [lo, hi] (three-term form: theta, delta, sigma, rho)."""
    theta, delta = 0.5 * (hi + lo), 0.5 * (hi - lo)
    sigma = theta / delta
    r = dinv * (b - apply(pr, x))
    rho = 1.0 / sigma
    d = r / theta
    for k in range(degree):
        x = x + d
        if k == degree - 1:
            break
        r = r - dinv * apply(pr, d)
        rho_new = 1.0 / (2.0 * sigma - rho)
        d = (rho_new * rho) * d + (2.0 * rho_new / delta) * r
        rho = rho_new
    return x


class Hierarchy:
    """Levels of the p-multigrid preconditioner for one (fine) problem."""

    def __init__(self, pr: Problem, **kw):
        self.opts = dict(DEFAULTS, **kw)
        self.levels = []
        for p in level_orders(pr.p):
            prl = level_problem(pr, p)
            dinv = jacobi_inverse(diagonal(prl))
            lam = lambda_max(prl, dinv, self.opts["power_iters"], self.opts["seed"])
            self.levels.append(dict(pr=prl, dinv=dinv, lam=lam))
        for l in range(len(self.levels) - 1):
            self.levels[l]["P"] = prolongation(self.levels[l + 1]["pr"], self.levels[l]["pr"])

    def vcycle(self, b: np.ndarray, l: int = 0) -> np.ndarray:
        """z = M^-1 b (one V-cycle from x = 0 on level l)."""
        L, o = self.levels[l], self.opts
        lo, hi = o["lo"] * L["lam"], o["hi"] * L["lam"]
        x = np.zeros_like(b)
        if l == len(self.levels) - 1:
            return chebyshev(L["pr"], L["dinv"], lo, hi, b, x, o["coarse_degree"])
        x = chebyshev(L["pr"], L["dinv"], lo, hi, b, x, o["degree"])
        r = b - apply(L["pr"], x)
        xc = self.vcycle(L["P"].T @ r, l + 1)
        x = x + L["P"] @ xc
        return chebyshev(L["pr"], L["dinv"], lo, hi, b, x, o["degree"])


def mg_pcg(h: Hierarchy, b: np.ndarray, maxit: int, rtol: float):
    """CG preconditioned by one V-cycle per iteration, x0 = 0, stopping on ||r|| <= rtol ||b||.
    Returns (x, residual-norm history, iterations)."""
    pr = h.levels[0]["pr"]
    x = np.zeros_like(b)
    r = b.copy()
    z = h.vcycle(r)
    p = z.copy()
    rz = r @ z
    bn = np.linalg.norm(b)
    hist = [bn]
    for k in range(1, maxit + 1):
        Ap = apply(pr, p)
        alpha = rz / (p @ Ap)
        x += alpha * p
        r -= alpha * Ap
        hist.append(np.linalg.norm(r))
        if hist[-1] <= rtol * bn:
            return x, np.array(hist), k
        z = h.vcycle(r)
        rz_new = r @ z
        p = z + (rz_new / rz) * p
        rz = rz_new
    return x, np.array(hist), maxit
