"""Transfers between levels by embedding (test infrastructure only).

Sec. 2: the h-prolongation between nested meshes is the embedding of V_l into V_{l+1}
and the restriction is its l2-adjoint (transpose).  Sec. 2.2: the p-prolongation from
degree p_{l-1} to p_l on the same cells is the natural embedding, restriction its
adjoint.  The embedding is evaluated in reference coordinates of the coarse cell
(topological nesting, Sec. 2), which is exact on Cartesian meshes.  Homogeneous
Dirichlet: rows of fine boundary nodes and columns of coarse boundary nodes vanish.
"""
from __future__ import annotations

from functools import reduce

import numpy as np
import scipy.sparse as sp

from .basis import gauss_lobatto, lagrange_values
from .mesh import boundary_nodes, cell_dofs, node_logical_coords

_TOL = 1e-12


def embedding(dim: int, n_coarse: int, p_coarse: int, n_fine: int, p_fine: int) -> sp.csr_matrix:
    """P[i, k] = coarse basis function k evaluated at fine node i."""
    if n_fine % n_coarse:
        raise ValueError("meshes are not nested")
    Lf = node_logical_coords(dim, n_fine, p_fine)
    dofs_c = cell_dofs(dim, n_coarse, p_coarse)
    nodes_c = gauss_lobatto(p_coarse)
    cell = np.minimum((Lf * n_coarse + _TOL).astype(int), n_coarse - 1)
    xi = Lf * n_coarse - cell
    cidx = cell @ (n_coarse ** np.arange(dim))
    rows, cols, vals = [], [], []
    for i in range(len(Lf)):
        vals1d = [lagrange_values(nodes_c, xi[i, a])[0] for a in range(dim)]
        phi = reduce(np.kron, vals1d[::-1])  # x fastest
        nz = np.abs(phi) > 1e-15
        rows.append(np.full(nz.sum(), i))
        cols.append(dofs_c[cidx[i]][nz])
        vals.append(phi[nz])
    Nf = len(Lf)
    Nc = (p_coarse * n_coarse + 1) ** dim
    P = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(Nf, Nc))
    keep_f = sp.diags((~boundary_nodes(dim, n_fine, p_fine)).astype(np.float64))
    keep_c = sp.diags((~boundary_nodes(dim, n_coarse, p_coarse)).astype(np.float64))
    return (keep_f @ P @ keep_c).tocsr()


def h_prolongation(dim: int, n_coarse: int, p: int) -> sp.csr_matrix:
    """Embedding of the degree-p space on n_coarse^dim cells into the one on 2x finer cells."""
    return embedding(dim, n_coarse, p, 2 * n_coarse, p)


def p_prolongation(dim: int, n: int, p_coarse: int, p_fine: int) -> sp.csr_matrix:
    """Embedding of the degree-p_coarse space into the degree-p_fine space on one mesh."""
    return embedding(dim, n, p_coarse, n, p_fine)
