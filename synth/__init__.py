"""Seeded synthetic inputs shared by the GPU library's callers and the oracle.

This module holds input generation only -- random draws and closed-form
fields -- and none of the discretization's arithmetic (no basis, no
quadrature, no geometry, no operator).  Each side pushes these inputs
through its own code.

Recipes (the paper defers the benchmark definitions to the CEED bake-off
paper; these stand in for that suite's structured box meshes):

* mesh: unit cube, ``nex x ney x nez`` hexahedra, vertices on a uniform
  grid; every *interior* vertex coordinate shifted by i.i.d.
  U(-a h_d, a h_d) with h_d = 1/ne_d (a = 0.1 by default); boundary vertices
  fixed, so the domain stays exactly [0,1]^3.  Draws in lexicographic vertex
  order (x fastest), then (dx, dy, dz).
* vectors: i.i.d. U[-1, 1] in FP64.
* counter-based U[-1, 1] (``splitmix_uniform``): element i of stream ``seed``
  is 2 u - 1 with u the top 53 bits of SplitMix64 (Steele, Lea, Flood 2014)
  applied to seed * 0x632be59bd9b4e019 + i, divided by 2^53.  A draw that a
  solver makes internally (the start vector of a power iteration) is
  reproduced exactly from this definition on every side.
* coefficient: kappa = exp(g), g(x) = sigma sqrt(2/M) sum_k cos(2 pi w_k.x + phi_k),
  w_k ~ N(0, s^2 I_3), phi_k ~ U[0, 2 pi), M = 32, sigma = 0.5, s = 2.
* manufactured solutions: u = sin(pi x) sin(pi y) sin(pi z) with
  f = 3 pi^2 u, and the polynomial u = x(1-x) y(1-y) z(1-z) with f = -lap u.
"""
from __future__ import annotations

import math

import numpy as np

SEED_MESH = 2109
SEED_VEC = 5072
SEED_KAPPA = 7
SEED_DIR = 11


def mesh_vertices(nex: int, ney: int, nez: int, perturb: float = 0.1, seed: int = SEED_MESH) -> np.ndarray:
    """[(nex+1)(ney+1)(nez+1), 3] float64 vertex coordinates, x fastest."""
    gx = np.linspace(0.0, 1.0, nex + 1)
    gy = np.linspace(0.0, 1.0, ney + 1)
    gz = np.linspace(0.0, 1.0, nez + 1)
    Z, Y, X = np.meshgrid(gz, gy, gx, indexing="ij")
    v = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
    if perturb != 0.0:
        rng = np.random.default_rng(seed)
        d = rng.uniform(-1.0, 1.0, size=v.shape) * perturb * np.array([1.0 / nex, 1.0 / ney, 1.0 / nez])
        ix = np.tile(np.arange(nex + 1), (nez + 1) * (ney + 1))
        iy = np.tile(np.repeat(np.arange(ney + 1), nex + 1), nez + 1)
        iz = np.repeat(np.arange(nez + 1), (ney + 1) * (nex + 1))
        interior = (ix > 0) & (ix < nex) & (iy > 0) & (iy < ney) & (iz > 0) & (iz < nez)
        v[interior] += d[interior]
    return np.ascontiguousarray(v)


def uniform_vector(n: int, nvec: int = 1, seed: int = SEED_VEC) -> np.ndarray:
    """i.i.d. U[-1, 1] float64, shape [n] (nvec == 1) or [n, nvec]."""
    rng = np.random.default_rng(seed)
    x = rng.uniform(-1.0, 1.0, size=(n, nvec))
    return np.ascontiguousarray(x[:, 0] if nvec == 1 else x)


_MASK64 = (1 << 64) - 1


def splitmix_uniform(n: int, seed: int) -> np.ndarray:
    """Counter-based U[-1, 1] float64 [n]: element i from SplitMix64 of seed*0x632be59bd9b4e019 + i."""
    with np.errstate(over="ignore"):
        z = (np.uint64((seed * 0x632BE59BD9B4E019) & _MASK64) + np.arange(n, dtype=np.uint64))
        z = z + np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    return 2.0 * ((z >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)) - 1.0


def kappa_modes(nmodes: int = 32, sigma: float = 0.5, scale: float = 2.0, seed: int = SEED_KAPPA):
    """Random Fourier modes of the log-coefficient: (omega [M,3], phi [M], sigma)."""
    rng = np.random.default_rng(seed)
    omega = rng.normal(0.0, scale, size=(nmodes, 3))
    phi = rng.uniform(0.0, 2.0 * math.pi, size=nmodes)
    return omega, phi, sigma


def kappa_field(xyz: np.ndarray, modes=None) -> np.ndarray:
    """kappa = exp(g(x)) at the given physical points ([..., 3] -> [...])."""
    omega, phi, sigma = modes if modes is not None else kappa_modes()
    xyz = np.asarray(xyz, dtype=np.float64)
    arg = 2.0 * math.pi * (xyz @ omega.T) + phi
    g = sigma * math.sqrt(2.0 / len(phi)) * np.cos(arg).sum(axis=-1)
    return np.exp(g)


def sin_solution(xyz: np.ndarray) -> np.ndarray:
    x, y, z = xyz[..., 0], xyz[..., 1], xyz[..., 2]
    return np.sin(math.pi * x) * np.sin(math.pi * y) * np.sin(math.pi * z)


def sin_forcing(xyz: np.ndarray) -> np.ndarray:
    """-lap of sin_solution."""
    return 3.0 * math.pi ** 2 * sin_solution(xyz)


def poly_solution(xyz: np.ndarray) -> np.ndarray:
    x, y, z = xyz[..., 0], xyz[..., 1], xyz[..., 2]
    return x * (1 - x) * y * (1 - y) * z * (1 - z)


def poly_forcing(xyz: np.ndarray) -> np.ndarray:
    """-lap of poly_solution."""
    x, y, z = xyz[..., 0], xyz[..., 1], xyz[..., 2]
    a, b, c = x * (1 - x), y * (1 - y), z * (1 - z)
    return 2.0 * (b * c + a * c + a * b)


def elems_for_dofs(ndofs: float, p: int) -> int:
    """Elements per direction of a cubic mesh with about ``ndofs`` nodes: round((N^(1/3) - 1)/p)."""
    return max(1, int(round((ndofs ** (1.0 / 3.0) - 1.0) / p)))
