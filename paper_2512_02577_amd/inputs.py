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


# ---------------------------------------------------------------------------------------
# General hexahedral (quadrilateral) meshes as cell lists with stored DoF maps
# ---------------------------------------------------------------------------------------
def _cube_symmetries(dim: int) -> list[tuple[tuple[int, ...], tuple[int, ...]]]:
    """Axis permutations with reflections: (perm, flip), 48 in 3D, 8 in 2D."""
    import itertools
    out = []
    for perm in itertools.permutations(range(dim)):
        for flip in itertools.product((0, 1), repeat=dim):
            out.append((perm, flip))
    return out


def hex_mesh(dim: int, n: int, p: int, seed: int, shape: str = "L", distortion: float = 0.0,
             permute: bool = True, orient: bool = True, renumber_nodes: bool = True) -> dict:
    """A general hex (2D: quad) mesh of degree-p nodes given as cell lists.

    The cells are the unit voxels of an n^dim lattice that belong to the domain:
    "box" keeps all, "L" drops those with x >= n/2 and y >= n/2, "hole" drops an inner
    block [n/4, 3n/4)^dim (a cavity with its own boundary).  Each vertex moves by
    distortion * (uniform[-1/2, 1/2]^dim) / n.  With `permute`, vertices, cells and (unless
    renumber_nodes is False, which keeps the lattice order of the nodes, as a numbering with
    locality) nodes are numbered in a random order; with `orient`, every cell lists its corners and nodes
    in the lexicographic order (x fastest) of a randomly rotated and reflected local
    frame.  Returns a dict with
      vertices       (n_vertices, dim) float64
      cell_vertices  (n_cells, 2^dim) int32, corners in the cell's local order
      cell_dofs      (n_cells, (p+1)^dim) int32, nodes in the cell's local order
      n_dofs         number of distinct nodes
      dof_lattice    (n_dofs, dim) int64 lattice position of each node (p*n+1 per axis)
      cell_lattice   (n_cells, dim) int64 lattice position of each cell
    The lattice fields only describe how the mesh was laid out."""
    rng = np.random.default_rng(seed)
    import itertools
    cells = []
    for c in itertools.product(range(n), repeat=dim):
        c = c[::-1]  # x fastest
        if shape == "L" and c[0] >= n // 2 and c[1] >= n // 2:
            continue
        if shape == "hole" and all(n // 4 <= c[a] < n - n // 4 for a in range(dim)):
            continue
        if shape not in ("box", "L", "hole"):
            raise ValueError(shape)
        cells.append(c)
    cells = np.array(cells, dtype=np.int64)
    nc = len(cells)
    m, mv = p * n + 1, n + 1
    loc1 = np.array([c[::-1] for c in itertools.product((0, 1), repeat=dim)], dtype=np.int64)
    locp = np.array([c[::-1] for c in itertools.product(range(p + 1), repeat=dim)], dtype=np.int64)

    def lin(x, mm):
        return sum(x[..., a] * mm ** a for a in range(dim))

    vkeys = lin(cells[:, None, :] + loc1[None, :, :], mv)            # (nc, 2^d)
    nkeys = lin(p * cells[:, None, :] + locp[None, :, :], m)         # (nc, (p+1)^d)
    vu = np.unique(vkeys)
    nu = np.unique(nkeys)
    jitter = distortion * rng.uniform(-0.5, 0.5, (len(vu), dim)) / n  # drawn first: same geometry either way
    vperm = rng.permutation(len(vu)) if permute else np.arange(len(vu))
    nperm = rng.permutation(len(nu)) if permute and renumber_nodes else np.arange(len(nu))
    cell_vertices = vperm[np.searchsorted(vu, vkeys)].astype(np.int32)
    cell_dofs = nperm[np.searchsorted(nu, nkeys)].astype(np.int32)
    # vertex coordinates on the lattice, then jitter
    vlat = np.stack([(vu // mv ** a) % mv for a in range(dim)], axis=1)
    vertices = np.empty((len(vu), dim))
    vertices[vperm] = vlat / n + jitter
    dof_lattice = np.empty((len(nu), dim), dtype=np.int64)
    dof_lattice[nperm] = np.stack([(nu // m ** a) % m for a in range(dim)], axis=1)
    if orient:
        syms = _cube_symmetries(dim)
        for c in range(nc):
            perm, flip = syms[rng.integers(len(syms))]
            for k, loc, arr in ((1, loc1, cell_vertices), (p, locp, cell_dofs)):
                # local index in the new frame -> lattice offset in the old one
                src = np.empty_like(loc)
                for a in range(dim):
                    src[:, perm[a]] = np.where(flip[a], k - loc[:, a], loc[:, a])
                arr[c] = arr[c][lin(src, k + 1)]
    corder = rng.permutation(nc) if permute else np.arange(nc)
    return {
        "vertices": vertices,
        "cell_vertices": np.ascontiguousarray(cell_vertices[corder]),
        "cell_dofs": np.ascontiguousarray(cell_dofs[corder]),
        "n_dofs": int(len(nu)),
        "dof_lattice": dof_lattice,
        "cell_lattice": cells[corder],
    }
