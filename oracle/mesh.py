"""Structured meshes of the unit box, DoF numbering and vertex-patch index sets
(test infrastructure only).

Follows Sec. 2 (nested mesh hierarchy, vertex patches built from the cells around an
interior vertex) and Sec. 4 (mesh built by global refinement, distorted variant).
All integer maps here are derived by brute-force set membership on the nodes'
logical coordinates, not by index arithmetic, so that they pin the library's
arithmetic maps.

Numbering (the contract both sides keep):
  node (i, j, k), 0 <= i, j, k <= p*n          -> i + m*(j + m*k), m = p*n + 1
  cell (cx, cy, cz)                            -> cx + n*(cy + n*cz)
  cell-local node (a, b, e)                    -> a + (p+1)*(b + (p+1)*e)
  patch of interior vertex (vx, vy, vz), 1..n-1 -> (vx-1) + (n-1)*((vy-1) + (n-1)*(vz-1))
  closure / interior of a patch                -> lexicographic, x fastest
(2D drops the third index.)
"""
from __future__ import annotations

import itertools

import numpy as np

from .basis import gauss_lobatto

_TOL = 1e-12


def hlevel_sizes(n: int, n_levels: int = 0) -> list[int]:
    """Cells per direction on each mesh level, coarsest first.  The mesh hierarchy is
    nested by bisection (Sec. 2); by default it coarsens while the count is even and
    above 3, so the coarsest mesh has 2 or 3 cells per direction (or n if odd)."""
    sizes = [n]
    while sizes[-1] % 2 == 0 and sizes[-1] > 3 and (n_levels == 0 or len(sizes) < n_levels):
        sizes.append(sizes[-1] // 2)
    if n_levels and len(sizes) != n_levels:
        raise ValueError(f"cannot build {n_levels} nested levels from n={n}")
    return sizes[::-1]


def p_hierarchy(p: int) -> list[int]:
    """Degrees of the local p-multigrid levels, coarsest first (Sec. 2.2): the geometric
    sequence 1, 3, 7, ... below p, then p itself."""
    if p < 1:
        raise ValueError("degree must be >= 1")
    levels = []
    q = 1
    while q < p:
        levels.append(q)
        q = 2 * q + 1
    levels.append(p)
    return levels


class StructuredMesh:
    """n^dim cells of a (possibly distorted) unit box with multilinear cell maps."""

    def __init__(self, dim: int, n: int, vertices: np.ndarray | None = None):
        if dim not in (2, 3):
            raise ValueError("dim must be 2 or 3")
        self.dim, self.n = dim, n
        if vertices is None:
            t = np.arange(n + 1, dtype=np.float64) / n
            grids = np.meshgrid(*([t] * dim), indexing="ij")
            vertices = np.stack([g.reshape(-1, order="F") for g in grids], axis=1)
        vertices = np.asarray(vertices, dtype=np.float64)
        if vertices.shape != ((n + 1) ** dim, dim):
            raise ValueError("vertices must have shape ((n+1)^dim, dim)")
        self.vertices = vertices

    # --- topology -----------------------------------------------------------------
    def n_cells(self) -> int:
        return self.n ** self.dim

    def cell_index_tuple(self, c: int) -> tuple[int, ...]:
        out = []
        for _ in range(self.dim):
            out.append(c % self.n)
            c //= self.n
        return tuple(out)

    def cell_corners(self, c: int) -> np.ndarray:
        """(2^dim, dim) corner coordinates, corner (a, b, e) in lexicographic order."""
        ci = self.cell_index_tuple(c)
        m = self.n + 1
        corners = []
        for offs in itertools.product((0, 1), repeat=self.dim):
            offs = offs[::-1]  # x fastest
            idx = 0
            stride = 1
            for a in range(self.dim):
                idx += (ci[a] + offs[a]) * stride
                stride *= m
            corners.append(self.vertices[idx])
        return np.array(corners)

    def coarsened(self, n_coarse: int) -> "StructuredMesh":
        """The coarser mesh whose vertices are a subset of this mesh's vertices
        (topological nesting, Sec. 2)."""
        r = self.n // n_coarse
        if r * n_coarse != self.n:
            raise ValueError("not nested")
        m = self.n + 1
        sel = []
        for kk in itertools.product(range(n_coarse + 1), repeat=self.dim):
            kk = kk[::-1]
            idx = 0
            stride = 1
            for a in range(self.dim):
                idx += kk[a] * r * stride
                stride *= m
            sel.append(idx)
        return StructuredMesh(self.dim, n_coarse, self.vertices[np.array(sel)])


def multilinear_map(corners: np.ndarray, xi: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    """Image x(xi) and Jacobian J[i, j] = dx_i/dxi_j of the multilinear cell map.
    xi: (nq, dim) reference points.  Returns (nq, dim) and (nq, dim, dim)."""
    dim = corners.shape[1]
    xi = np.atleast_2d(xi)
    nq = xi.shape[0]
    x = np.zeros((nq, dim))
    J = np.zeros((nq, dim, dim))
    for ci, offs in enumerate(itertools.product((0, 1), repeat=dim)):
        offs = offs[::-1]
        lam = np.ones(nq)
        dlam = np.ones((nq, dim))
        for a in range(dim):
            val = xi[:, a] if offs[a] else 1.0 - xi[:, a]
            der = 1.0 if offs[a] else -1.0
            lam = lam * val
            for b in range(dim):
                dlam[:, b] *= der if a == b else val
        x += lam[:, None] * corners[ci][None, :]
        J += corners[ci][None, :, None] * dlam[:, None, :]
    return x, J


def node_logical_coords(dim: int, n: int, p: int) -> np.ndarray:
    """Logical coordinates in [0,1]^dim of every node, in global index order.  A node
    sits at the Gauss-Lobatto point xi_a of cell c in each direction: (c + xi_a)/n."""
    gll = gauss_lobatto(p)
    m = p * n + 1
    t = np.empty(m)
    for i in range(m):
        c = min(i // p, n - 1)
        a = i - p * c
        t[i] = (c + gll[a]) / n
    grids = np.meshgrid(*([t] * dim), indexing="ij")
    return np.stack([g.reshape(-1, order="F") for g in grids], axis=1)


def node_physical_coords(mesh: StructuredMesh, p: int) -> np.ndarray:
    """Physical coordinates of every node: the cell map applied to its reference point."""
    L = node_logical_coords(mesh.dim, mesh.n, p)
    n = mesh.n
    out = np.empty_like(L)
    cell_of = np.minimum((L * n + _TOL).astype(int), n - 1)
    # reference coordinate inside the chosen cell
    xi = L * n - cell_of
    strides = n ** np.arange(mesh.dim)
    cidx = cell_of @ strides
    for c in np.unique(cidx):
        sel = cidx == c
        out[sel], _ = multilinear_map(mesh.cell_corners(int(c)), xi[sel])
    return out


def _sorted_members(L: np.ndarray, inside: np.ndarray) -> np.ndarray:
    idx = np.nonzero(inside)[0]
    keys = tuple(L[idx, a] for a in range(L.shape[1]))  # lexsort: last key is primary
    return idx[np.lexsort(keys)].astype(np.int32)


def cell_dofs(dim: int, n: int, p: int) -> np.ndarray:
    """(n^dim, (p+1)^dim): nodes inside each closed cell box, x fastest."""
    L = node_logical_coords(dim, n, p)
    out = np.empty((n ** dim, (p + 1) ** dim), dtype=np.int32)
    for c in range(n ** dim):
        ci = [(c // n ** a) % n for a in range(dim)]
        inside = np.ones(len(L), dtype=bool)
        for a in range(dim):
            lo, hi = ci[a] / n, (ci[a] + 1) / n
            inside &= (L[:, a] >= lo - _TOL) & (L[:, a] <= hi + _TOL)
        out[c] = _sorted_members(L, inside)
    return out


def patch_vertices(dim: int, n: int) -> np.ndarray:
    """(n_patches, dim) interior vertex of each patch, patch index order."""
    rng = range(1, n)
    out = [v[::-1] for v in itertools.product(rng, repeat=dim)]
    return np.array(out, dtype=np.int64).reshape(-1, dim)


def patch_index_sets(dim: int, n: int, p: int) -> tuple[np.ndarray, np.ndarray]:
    """Closure (nodes in the closed box of the 2^dim cells around the vertex) and
    interior (nodes strictly inside) of every vertex patch (Sec. 2.1), x fastest."""
    L = node_logical_coords(dim, n, p)
    verts = patch_vertices(dim, n)
    closure = np.empty((len(verts), (2 * p + 1) ** dim), dtype=np.int32)
    interior = np.empty((len(verts), (2 * p - 1) ** dim), dtype=np.int32)
    for j, v in enumerate(verts):
        inc = np.ones(len(L), dtype=bool)
        ins = np.ones(len(L), dtype=bool)
        for a in range(dim):
            lo, hi = (v[a] - 1) / n, (v[a] + 1) / n
            inc &= (L[:, a] >= lo - _TOL) & (L[:, a] <= hi + _TOL)
            ins &= (L[:, a] > lo + _TOL) & (L[:, a] < hi - _TOL)
        closure[j] = _sorted_members(L, inc)
        interior[j] = _sorted_members(L, ins)
    return closure, interior


def patch_colors(dim: int, n: int) -> np.ndarray:
    """Parity coloring of the vertex patches: sum_k (v_k mod 2) 2^k."""
    verts = patch_vertices(dim, n)
    return sum((verts[:, a] % 2) << a for a in range(dim)).astype(np.uint8)


def boundary_nodes(dim: int, n: int, p: int) -> np.ndarray:
    """Boolean mask of nodes on the boundary of the unit box."""
    L = node_logical_coords(dim, n, p)
    return np.any((L < _TOL) | (L > 1 - _TOL), axis=1)
