"""Seeded synthetic inputs shared by the GPU path, the CPU oracle and the benchmark.

This module draws random numbers and lays them out; it holds none of the solver's
arithmetic (no basis functions, quadrature, operators or transfers), so both
implementations can take their inputs from it without sharing any of the method.

Conventions used by every array returned here:
  * node grid of a degree-p problem on n^d cells: (p*n+1)^d nodes, lexicographic with
    x fastest; node (i, j, k) has index i + m*(j + m*k), m = p*n+1;
  * vertex grid: (n+1)^d vertices, same ordering, coordinates in [0, 1]^d.
"""
from __future__ import annotations

import numpy as np


def node_count(dim: int, n: int, p: int) -> int:
    return (p * n + 1) ** dim


def boundary_mask(dim: int, m: int) -> np.ndarray:
    """Boolean mask over an m^dim lexicographic grid, True on the outer faces."""
    idx = np.arange(m)
    on_face = (idx == 0) | (idx == m - 1)
    mask = np.zeros((m,) * dim, dtype=bool)
    for axis in range(dim):
        shape = [1] * dim
        shape[dim - 1 - axis] = m  # C order: last array axis is x
        mask |= on_face.reshape(shape)
    return mask.reshape(-1)


def rhs_vector(dim: int, n: int, p: int, seed: int) -> np.ndarray:
    """Right-hand side b: seeded uniform[-1, 1] entries on interior nodes, 0 on the
    homogeneous Dirichlet boundary (float64, length (p*n+1)^dim)."""
    rng = np.random.default_rng(seed)
    m = p * n + 1
    b = rng.uniform(-1.0, 1.0, size=m ** dim)
    b[boundary_mask(dim, m)] = 0.0
    return b


def cartesian_vertices(dim: int, n: int) -> np.ndarray:
    """Vertices of the uniform n^dim grid of the unit box, shape ((n+1)^dim, dim)."""
    t = np.arange(n + 1, dtype=np.float64) / n
    grids = np.meshgrid(*([t] * dim), indexing="ij")  # grids[a][i, j, (k)] = t[index a]
    # lexicographic with x fastest: flatten in Fortran order over (x, y, z)
    return np.stack([g.reshape(-1, order="F") for g in grids], axis=1)


def jittered_vertices(dim: int, n: int, delta: float, seed: int) -> np.ndarray:
    """Distorted mesh: each interior vertex moves by delta*h_v in a uniformly random
    direction, h_v = shortest edge attached to it on the undistorted grid (= 1/n);
    boundary vertices stay.  Returns ((n+1)^dim, dim) float64."""
    rng = np.random.default_rng(seed)
    v = cartesian_vertices(dim, n)
    nv = (n + 1) ** dim
    direction = rng.standard_normal((nv, dim))
    direction /= np.linalg.norm(direction, axis=1, keepdims=True)
    h_v = 1.0 / n
    interior = ~boundary_mask(dim, n + 1)
    v[interior] += delta * h_v * direction[interior]
    return v


class CoefficientField:
    """a(x) = exp(ln(10) * g(x)), g = sum_m c_m cos(2 pi k_m.x + phi_m) / sum_m |c_m|,
    so that a lies in [0.1, 10].  Parameters are drawn from the seed."""

    def __init__(self, dim: int, seed: int, n_modes: int = 8):
        rng = np.random.default_rng(seed)
        self.dim = dim
        self.c = rng.uniform(-1.0, 1.0, size=n_modes)
        self.k = rng.integers(0, 4, size=(n_modes, dim)).astype(np.float64)
        self.phi = rng.uniform(0.0, 2.0 * np.pi, size=n_modes)

    def __call__(self, x: np.ndarray) -> np.ndarray:
        x = np.asarray(x, dtype=np.float64)
        arg = 2.0 * np.pi * (x @ self.k.T) + self.phi  # (..., n_modes)
        g = (np.cos(arg) @ self.c) / np.sum(np.abs(self.c))
        return np.exp(np.log(10.0) * g)
