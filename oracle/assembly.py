"""Element matrices by brute-force quadrature and assembled global operators
(test infrastructure only).

Follows Sec. 2: the discrete operator A_l is obtained by applying the bilinear form
a(u, v) = int grad u . grad v (eq. bilinear-form; with a coefficient mu at quadrature
points as in Sec. 3) to the basis of V_l (eq. matrix).  Every level, in h and in p,
is rediscretized with its own quadrature.  Homogeneous Dirichlet conditions on the
whole boundary: boundary rows and columns carry no coupling and the boundary rows are
identity rows.  No sum factorization: full (p+1)^d x nq^d tables per element.
"""
from __future__ import annotations

from functools import reduce

import numpy as np
import scipy.sparse as sp

from .basis import gauss_legendre, gauss_lobatto, lagrange_derivatives, lagrange_values
from .mesh import StructuredMesh, boundary_nodes, cell_dofs, multilinear_map


def _kron_list(mats):
    # kron(A_z, kron(A_y, A_x)) so that the x index runs fastest in rows and columns
    return reduce(np.kron, mats[::-1])


def reference_tables(dim: int, p: int, nq: int):
    """Tensor quadrature points/weights (x fastest) and the reference values Phi[q, i]
    and gradients Grad[q, i, k] of the (p+1)^dim tensor-product Lagrange basis."""
    xq, wq = gauss_legendre(nq)
    nodes = gauss_lobatto(p)
    V = lagrange_values(nodes, xq)
    D = lagrange_derivatives(nodes, xq)
    grids = np.meshgrid(*([xq] * dim), indexing="ij")
    pts = np.stack([g.reshape(-1, order="F") for g in grids], axis=1)
    w = _kron_list([wq[:, None]] * dim)[:, 0]
    Phi = _kron_list([V] * dim)
    Grad = np.stack([_kron_list([D if a == k else V for a in range(dim)]) for k in range(dim)], axis=2)
    return pts, w, Phi, Grad


def element_stiffness(p: int, corners: np.ndarray, coef=None, nq: int | None = None) -> np.ndarray:
    """A_K[i, j] = sum_q w_q a(x_q) gradref_i^T |det J| J^{-1} J^{-T} gradref_j."""
    dim = corners.shape[1]
    pts, w, _, Grad = reference_tables(dim, p, nq or p + 1)
    x, J = multilinear_map(corners, pts)
    detJ = np.linalg.det(J)
    Jinv = np.linalg.inv(J)
    a = np.ones(len(w)) if coef is None else np.asarray(coef(x), dtype=np.float64)
    G = (w * a * np.abs(detJ))[:, None, None] * np.einsum("qik,qjk->qij", Jinv, Jinv)
    return np.einsum("qik,qkl,qjl->ij", Grad, G, Grad)


def element_mass(p: int, corners: np.ndarray, nq: int | None = None) -> np.ndarray:
    dim = corners.shape[1]
    pts, w, Phi, _ = reference_tables(dim, p, nq or p + 1)
    _, J = multilinear_map(corners, pts)
    s = w * np.abs(np.linalg.det(J))
    return np.einsum("qi,q,qj->ij", Phi, s, Phi)


def _assemble(mesh: StructuredMesh, p: int, elem) -> sp.csr_matrix:
    dofs = cell_dofs(mesh.dim, mesh.n, p)
    N = (p * mesh.n + 1) ** mesh.dim
    rows, cols, vals = [], [], []
    for c in range(mesh.n_cells()):
        Ae = elem(c)
        d = dofs[c]
        rows.append(np.repeat(d, len(d)))
        cols.append(np.tile(d, len(d)))
        vals.append(Ae.reshape(-1))
    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(N, N))
    return A.tocsr()  # duplicates summed


def apply_dirichlet(A: sp.csr_matrix, bnd: np.ndarray) -> sp.csr_matrix:
    """Zero boundary rows and columns, unit diagonal on boundary rows."""
    keep = sp.diags((~bnd).astype(np.float64))
    return (keep @ A @ keep + sp.diags(bnd.astype(np.float64))).tocsr()


def stiffness_matrix(mesh: StructuredMesh, p: int, coef=None, dirichlet: bool = True) -> sp.csr_matrix:
    """Global Q_p Laplacian (variable coefficient optional) on the mesh."""
    cache = {}

    def elem(c):
        corners = mesh.cell_corners(c)
        if coef is not None:
            return element_stiffness(p, corners, coef)
        key = np.round(corners - corners[0], 13).tobytes()
        if key not in cache:
            cache[key] = element_stiffness(p, corners)
        return cache[key]

    A = _assemble(mesh, p, elem)
    if dirichlet:
        A = apply_dirichlet(A, boundary_nodes(mesh.dim, mesh.n, p))
    return A


def mass_matrix(mesh: StructuredMesh, p: int, nq: int | None = None) -> sp.csr_matrix:
    return _assemble(mesh, p, lambda c: element_mass(p, mesh.cell_corners(c), nq))


def load_vector(mesh: StructuredMesh, p: int, f, nq: int | None = None) -> np.ndarray:
    """b_i = int f phi_i (boundary entries set to zero, homogeneous Dirichlet)."""
    dim = mesh.dim
    nq = nq or p + 3
    pts, w, Phi, _ = reference_tables(dim, p, nq)
    dofs = cell_dofs(dim, mesh.n, p)
    b = np.zeros((p * mesh.n + 1) ** dim)
    for c in range(mesh.n_cells()):
        x, J = multilinear_map(mesh.cell_corners(c), pts)
        s = w * np.abs(np.linalg.det(J)) * f(x)
        np.add.at(b, dofs[c], Phi.T @ s)
    b[boundary_nodes(dim, mesh.n, p)] = 0.0
    return b


def l2_error(mesh: StructuredMesh, p: int, u: np.ndarray, exact, nq: int | None = None) -> float:
    dim = mesh.dim
    nq = nq or p + 3
    pts, w, Phi, _ = reference_tables(dim, p, nq)
    dofs = cell_dofs(dim, mesh.n, p)
    err2 = 0.0
    for c in range(mesh.n_cells()):
        x, J = multilinear_map(mesh.cell_corners(c), pts)
        uh = Phi @ u[dofs[c]]
        err2 += np.sum(w * np.abs(np.linalg.det(J)) * (uh - exact(x)) ** 2)
    return float(np.sqrt(err2))


def quadrature_points(mesh: StructuredMesh, p: int, nq: int | None = None) -> np.ndarray:
    """Physical Gauss points of every cell, (n_cells, nq^dim, dim), x fastest."""
    pts, _, _, _ = reference_tables(mesh.dim, p, nq or p + 1)
    return np.stack([multilinear_map(mesh.cell_corners(c), pts)[0] for c in range(mesh.n_cells())])


def cells_of_node_1d(i: int, n: int, p: int) -> list[int]:
    """Cells (per direction) whose closed interval holds node i of the degree-p line of
    n cells: cell i // p, and also cell i // p - 1 when the node is a shared cell end."""
    cs = {min(i // p, n - 1)}
    if i % p == 0 and i > 0:
        cs.add(i // p - 1)
    return sorted(x for x in cs if 0 <= x < n)


def apply_rows(mesh: StructuredMesh, p: int, u: np.ndarray, rows: np.ndarray, coef=None) -> np.ndarray:
    """(A u)_i for selected global rows i without assembling A: the sum over the cells
    that contain node i of (element matrix row) . (element values of u), with the
    Dirichlet convention (identity rows on the boundary, boundary values of u ignored)."""
    dim, n = mesh.dim, mesh.n
    m = p * n + 1
    bnd = boundary_nodes(dim, n, p)
    out = np.zeros(len(rows))
    cache = {}
    for r_i, g in enumerate(np.asarray(rows)):
        if bnd[g]:
            out[r_i] = u[g]
            continue
        idx = [(g // m**a) % m for a in range(dim)]
        cands = [cells_of_node_1d(idx[a], n, p) for a in range(dim)]
        total = 0.0
        for cell in np.array(np.meshgrid(*cands, indexing="ij")).reshape(dim, -1).T:
            c = int(sum(cell[a] * n**a for a in range(dim)))
            loc = [idx[a] - p * cell[a] for a in range(dim)]
            if any(l < 0 or l > p for l in loc):
                continue
            li = int(sum(loc[a] * (p + 1) ** a for a in range(dim)))
            corners = mesh.cell_corners(c)
            if coef is None:
                key = np.round(corners - corners[0], 13).tobytes()
                if key not in cache:
                    cache[key] = element_stiffness(p, corners)
                Ae = cache[key]
            else:
                Ae = element_stiffness(p, corners, coef)
            dofs = np.array([sum((p * cell[a] + ((e // (p + 1) ** a) % (p + 1))) * m**a for a in range(dim))
                             for e in range((p + 1) ** dim)])
            ue = np.where(bnd[dofs], 0.0, u[dofs])
            total += Ae[li] @ ue
        out[r_i] = total
    return out
