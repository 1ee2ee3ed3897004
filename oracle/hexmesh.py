"""General hexahedral (2D: quadrilateral) meshes given as cell lists with stored DoF
maps, DSATUR coloring of the vertex patches, and the multiplicative patch smoother on
them (test infrastructure only).

Sec. 3 (implementation of the patch smoother): at setup the cells forming each vertex
patch are identified, and the patch works on the cells' own DoF indices (gather from
the global vectors, cell-wise evaluation, masked scatter-add).  Sec. 4.4: the patches
are colored with DSATUR (Brelaz 1979) so that no two patches of one color share a DoF
whose update would race, and the smoother runs color by color.

Readings:
  * A mesh is a list of cells, each given by its 2^d corner vertices and its (p+1)^d
    nodes in the cell's own lexicographic order (x fastest).  Cells may be numbered,
    rotated and reflected arbitrarily; every quantity here is computed in each cell's
    own frame, so no orientation is assumed.
  * The homogeneous Dirichlet boundary is the set of nodes on faces that belong to one
    cell only.
  * A vertex patch exists at every vertex that lies on no boundary face; its cells are
    the cells containing the vertex (2^d of them on the meshes used here).
  * Two patches conflict when one's interior meets the other's closure; on these
    meshes that is exactly when they share a cell.  DSATUR: repeatedly color the
    uncolored patch with the most distinct colors among its neighbours (saturation),
    ties to the most uncolored neighbours, then to the lowest patch index, with the
    smallest color no neighbour has.  Patches are indexed by ascending vertex index.
  * The patch operators of the local p-levels are assembled from the patch's cells
    (element matrices in each cell's frame); nodes of one degree shared by several
    cells are identified by their physical position.  The p-embedding evaluates the
    coarser Lagrange basis at the finer Gauss-Lobatto nodes cell by cell, as on
    structured meshes (Sec. 2.2).
"""
from __future__ import annotations

import itertools
from functools import reduce

import numpy as np
import scipy.sparse as sp
from scipy.spatial import cKDTree

from .assembly import apply_dirichlet, element_stiffness
from .basis import gauss_lobatto, lagrange_values
from .mesh import multilinear_map
from .smoother import LevelSmoother, PatchData, VmultCounter, default_omega


def _lex(dim: int, k: int) -> np.ndarray:
    """(k^dim, dim) local index tuples in lexicographic order, x fastest."""
    return np.array([c[::-1] for c in itertools.product(range(k), repeat=dim)], dtype=np.int64)


def dsatur(adj: list[set[int]]) -> np.ndarray:
    """Brelaz's DSATUR coloring with the tie-breaks stated in the module docstring."""
    nv = len(adj)
    color = np.full(nv, -1, dtype=np.int64)
    sat = [set() for _ in range(nv)]
    udeg = np.array([len(a) for a in adj], dtype=np.int64)
    for _ in range(nv):
        best = -1
        for v in range(nv):
            if color[v] >= 0:
                continue
            if best < 0 or (len(sat[v]), udeg[v]) > (len(sat[best]), udeg[best]):
                best = v
        c = 0
        while c in sat[best]:
            c += 1
        color[best] = c
        for w in adj[best]:
            sat[w].add(c)
            if color[w] < 0:
                udeg[w] -= 1
    return color


class HexMesh:
    """Cells with corner vertices and stored DoF maps of one degree p."""

    def __init__(self, dim: int, vertices: np.ndarray, cell_vertices: np.ndarray, p: int,
                 cell_dofs: np.ndarray, n_dofs: int):
        self.dim, self.p, self.n_dofs = dim, p, int(n_dofs)
        self.vertices = np.asarray(vertices, dtype=np.float64)
        self.cell_vertices = np.asarray(cell_vertices, dtype=np.int64)
        self.cell_dofs = np.asarray(cell_dofs, dtype=np.int64)
        self.n_cells = len(self.cell_vertices)
        if self.cell_vertices.shape != (self.n_cells, 2 ** dim):
            raise ValueError("cell_vertices must have 2^dim columns")
        if self.cell_dofs.shape != (self.n_cells, (p + 1) ** dim):
            raise ValueError("cell_dofs must have (p+1)^dim columns")
        self._faces()

    # --- topology ---------------------------------------------------------------------
    def corners(self, c: int) -> np.ndarray:
        return self.vertices[self.cell_vertices[c]]

    def _face_key(self, c: int, axis: int, side: int) -> tuple:
        loc = _lex(self.dim, 2)
        sel = loc[:, axis] == side
        return tuple(sorted(self.cell_vertices[c][sel].tolist()))

    def _faces(self):
        count: dict[tuple, int] = {}
        for c in range(self.n_cells):
            for a in range(self.dim):
                for s in (0, 1):
                    k = self._face_key(c, a, s)
                    count[k] = count.get(k, 0) + 1
        self.boundary_faces = {k for k, v in count.items() if v == 1}

    def boundary_dofs(self) -> np.ndarray:
        """Mask of nodes on a face that belongs to one cell only."""
        mask = np.zeros(self.n_dofs, dtype=bool)
        loc = _lex(self.dim, self.p + 1)
        for c in range(self.n_cells):
            for a in range(self.dim):
                for s in (0, 1):
                    if self._face_key(c, a, s) in self.boundary_faces:
                        mask[self.cell_dofs[c][loc[:, a] == s * self.p]] = True
        return mask

    def patch_vertices(self) -> np.ndarray:
        on_bnd = np.zeros(len(self.vertices), dtype=bool)
        for k in self.boundary_faces:
            on_bnd[list(k)] = True
        used = np.zeros(len(self.vertices), dtype=bool)
        used[self.cell_vertices.reshape(-1)] = True
        return np.nonzero(used & ~on_bnd)[0]

    def patch_cells(self) -> list[np.ndarray]:
        """Cells of every patch (ascending cell index), patches by ascending vertex."""
        verts = self.patch_vertices()
        pos = {int(v): i for i, v in enumerate(verts)}
        out = [[] for _ in verts]
        for c in range(self.n_cells):
            for v in self.cell_vertices[c]:
                if int(v) in pos:
                    out[pos[int(v)]].append(c)
        return [np.array(sorted(x), dtype=np.int64) for x in out]

    def patch_colors(self) -> np.ndarray:
        cells = self.patch_cells()
        by_cell = [[] for _ in range(self.n_cells)]
        for j, cs in enumerate(cells):
            for c in cs:
                by_cell[c].append(j)
        adj = [set() for _ in cells]
        for js in by_cell:
            for a in js:
                adj[a].update(js)
        for j in range(len(cells)):
            adj[j].discard(j)
        return dsatur(adj)

    # --- operators --------------------------------------------------------------------
    def stiffness(self, q: int | None = None, dirichlet: bool = True) -> sp.csr_matrix:
        """Global Q_p Laplacian assembled cell by cell, each cell in its own frame."""
        p = self.p
        rows, cols, vals = [], [], []
        for c in range(self.n_cells):
            Ae = element_stiffness(p, self.corners(c))
            d = self.cell_dofs[c]
            rows.append(np.repeat(d, len(d)))
            cols.append(np.tile(d, len(d)))
            vals.append(Ae.reshape(-1))
        N = self.n_dofs
        A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                          shape=(N, N)).tocsr()
        if dirichlet:
            A = apply_dirichlet(A, self.boundary_dofs())
        return A

    def node_positions(self, c: int, q: int) -> np.ndarray:
        """Physical positions of the degree-q Gauss-Lobatto nodes of cell c (local order)."""
        xi = gauss_lobatto(q)[_lex(self.dim, q + 1)]
        x, _ = multilinear_map(self.corners(c), xi)
        return x


def _merge(points: np.ndarray, tol: float) -> np.ndarray:
    """Group ids of points that coincide within tol (first occurrence order)."""
    tree = cKDTree(points)
    parent = np.arange(len(points))
    for i, j in tree.query_pairs(tol):
        a, b = min(i, j), max(i, j)
        while parent[a] != a:
            a = parent[a]
        while parent[b] != b:
            b = parent[b]
        if a != b:
            parent[max(a, b)] = min(a, b)
    root = np.array([_find(parent, i) for i in range(len(points))])
    _, gid = np.unique(root, return_inverse=True)
    return gid


def _find(parent, i):
    while parent[i] != i:
        i = parent[i]
    return i


class PatchSpace:
    """Degree-q nodes of one patch: group ids per (cell, local node) and the interior."""

    def __init__(self, mesh: HexMesh, cells: np.ndarray, q: int):
        dim = mesh.dim
        self.q, self.cells = q, cells
        k = q + 1
        loc = _lex(dim, k)
        pts = np.concatenate([mesh.node_positions(int(c), q) for c in cells])
        h = min(np.linalg.norm(mesh.corners(int(c))[1] - mesh.corners(int(c))[0]) for c in cells)
        self.gid = _merge(pts, 1e-7 * h).reshape(len(cells), k ** dim)
        ng = int(self.gid.max()) + 1
        # patch boundary: faces of patch cells not shared by two patch cells
        keys = {}
        for c in cells:
            for a in range(dim):
                for s in (0, 1):
                    kk = mesh._face_key(int(c), a, s)
                    keys[kk] = keys.get(kk, 0) + 1
        on_bnd = np.zeros(ng, dtype=bool)
        for ci, c in enumerate(cells):
            for a in range(dim):
                for s in (0, 1):
                    if keys[mesh._face_key(int(c), a, s)] == 1:
                        on_bnd[self.gid[ci][loc[:, a] == s * q]] = True
        self.n_groups = ng
        self.interior_groups = np.nonzero(~on_bnd)[0]

    def assemble(self, mesh: HexMesh) -> np.ndarray:
        ng = self.n_groups
        A = np.zeros((ng, ng))
        for ci, c in enumerate(self.cells):
            g = self.gid[ci]
            A[np.ix_(g, g)] += element_stiffness(self.q, mesh.corners(int(c)))
        I = self.interior_groups
        return A[np.ix_(I, I)]


def _embedding_1d(qc: int, qf: int) -> np.ndarray:
    return lagrange_values(gauss_lobatto(qc), gauss_lobatto(qf))  # (qf+1, qc+1)


class HexLevelSmoother(LevelSmoother):
    """The patch smoother of oracle.smoother on a HexMesh: Alg. 1 over the DSATUR colors
    (patches of one color in ascending index), Alg. 2 / Alg. 3 on each patch.  Jacobi
    smoothing of the local p-levels only."""

    def __init__(self, mesh: HexMesh, degrees: list[int], omega: list[float] | None = None,
                 local: str = "half", n_local_iter: int = 1):
        if degrees[-1] != mesh.p:
            raise ValueError("the finest p-level must be the mesh's degree")
        if local not in ("half", "full", "direct"):
            raise ValueError(local)
        self.mesh = mesh
        self.degrees = list(degrees)
        dim = mesh.dim
        self.smoother, self.AC = "jacobi", None
        self.A = [None] * (len(degrees) - 1) + [mesh.stiffness()]
        self.cells = mesh.patch_cells()
        self.colors = mesh.patch_colors()
        self.n_colors = int(self.colors.max()) + 1 if len(self.colors) else 0
        self.omega = list(omega) if omega is not None else [default_omega(dim, q) for q in degrees]
        self.local = local
        self.n_local_iter = n_local_iter
        self.counter = VmultCounter(len(degrees))
        self._cache: dict[int, PatchData] = {}
        top = []
        for cs in self.cells:
            sp_top = PatchSpace(mesh, cs, mesh.p)
            top.append(self._global_ids(sp_top))
        self.interior = [None] * (len(degrees) - 1) + [top]

    def _global_ids(self, space: PatchSpace) -> np.ndarray:
        """Global DoF of each interior group of the top degree, in ascending DoF order."""
        g2d = np.full(space.n_groups, -1, dtype=np.int64)
        for ci, c in enumerate(space.cells):
            g2d[space.gid[ci]] = self.mesh.cell_dofs[int(c)]
        return np.sort(g2d[space.interior_groups])

    def patch(self, j: int) -> PatchData:
        if j in self._cache:
            return self._cache[j]
        mesh, dim = self.mesh, self.mesh.dim
        spaces = [PatchSpace(mesh, self.cells[j], q) for q in self.degrees]
        # order the top level's interior by global DoF so that it matches interior[-1]
        top = spaces[-1]
        g2d = np.full(top.n_groups, -1, dtype=np.int64)
        for ci, c in enumerate(top.cells):
            g2d[top.gid[ci]] = mesh.cell_dofs[int(c)]
        top.interior_groups = top.interior_groups[np.argsort(g2d[top.interior_groups])]
        A, D, P = [], [], [None]
        for l, sp_l in enumerate(spaces):
            Al = sp_l.assemble(mesh)
            A.append(Al)
            D.append(np.diag(Al).copy())
            if l > 0:
                spc = spaces[l - 1]
                E1 = _embedding_1d(spc.q, sp_l.q)
                E = reduce(np.kron, [E1] * dim)  # x fastest in rows and columns
                Pg = np.zeros((sp_l.n_groups, spc.n_groups))
                for ci in range(len(sp_l.cells)):
                    Pg[np.ix_(sp_l.gid[ci], spc.gid[ci])] = E
                P.append(Pg[np.ix_(sp_l.interior_groups, spc.interior_groups)])
        pd = PatchData(A, D, P)
        self._cache[j] = pd
        return pd
