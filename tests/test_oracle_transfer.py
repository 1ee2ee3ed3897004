"""Pins of the oracle's h- and p-embeddings (Sec. 2 transfers, Sec. 2.2 p-transfers)."""
import numpy as np
import pytest

from oracle.assembly import stiffness_matrix
from oracle.mesh import StructuredMesh, boundary_nodes, node_logical_coords
from oracle.transfer import h_prolongation, p_prolongation


def _bubble(x):
    # vanishes on the boundary, degree 2 in each variable
    return np.prod(x * (1 - x), axis=1)


@pytest.mark.parametrize("dim,nc,p", [(2, 2, 2), (2, 3, 3), (3, 2, 2), (3, 2, 3)])
def test_h_embedding_reproduces_coarse_functions(dim, nc, p):
    P = h_prolongation(dim, nc, p)
    uc = _bubble(node_logical_coords(dim, nc, p))
    uf = _bubble(node_logical_coords(dim, 2 * nc, p))
    np.testing.assert_allclose(P @ uc, uf, atol=1e-14)


@pytest.mark.parametrize("dim,n,pc,pf", [(2, 2, 1, 2), (2, 3, 2, 3), (3, 2, 1, 3), (3, 2, 3, 4), (2, 2, 3, 7)])
def test_p_embedding_reproduces_coarse_functions(dim, n, pc, pf):
    P = p_prolongation(dim, n, pc, pf)
    rng = np.random.default_rng(0)
    # any function of the coarse space: random nodal values (zero on the boundary)
    Lc = node_logical_coords(dim, n, pc)
    uc = rng.uniform(-1, 1, len(Lc))
    uc[boundary_nodes(dim, n, pc)] = 0
    uf = P @ uc
    # evaluate the coarse function at fine nodes independently via cellwise 1D
    # interpolation is what P is; check instead that re-embedding the coarse space into
    # an even finer degree commutes: P(pc->pf2) == P(pf->pf2) P(pc->pf) when pf2 > pf
    P2 = p_prolongation(dim, n, pf, pf + 1)
    P12 = p_prolongation(dim, n, pc, pf + 1)
    np.testing.assert_allclose(P2 @ uf, P12 @ uc, atol=1e-13)
    if pc >= 2:
        ub = _bubble(Lc)
        np.testing.assert_allclose(P @ ub, _bubble(node_logical_coords(dim, n, pf)), atol=1e-14)


@pytest.mark.parametrize("dim,nc,p", [(2, 2, 2), (2, 2, 4), (3, 2, 2)])
def test_galerkin_identity_h(dim, nc, p):
    # On Cartesian meshes the coarse space is a subspace and the Gauss rule is exact,
    # so rediscretization equals the Galerkin product R A_f P
    P = h_prolongation(dim, nc, p)
    Af = stiffness_matrix(StructuredMesh(dim, 2 * nc), p)
    Ac = stiffness_matrix(StructuredMesh(dim, nc), p)
    inner = ~boundary_nodes(dim, nc, p)
    G = (P.T @ Af @ P).toarray()[np.ix_(inner, inner)]
    np.testing.assert_allclose(G, Ac.toarray()[np.ix_(inner, inner)], atol=1e-13 * abs(G).max())


@pytest.mark.parametrize("dim,n,pc,pf", [(2, 2, 1, 3), (2, 3, 3, 4), (3, 2, 1, 2), (3, 2, 3, 4)])
def test_galerkin_identity_p(dim, n, pc, pf):
    P = p_prolongation(dim, n, pc, pf)
    Af = stiffness_matrix(StructuredMesh(dim, n), pf)
    Ac = stiffness_matrix(StructuredMesh(dim, n), pc)
    inner = ~boundary_nodes(dim, n, pc)
    G = (P.T @ Af @ P).toarray()[np.ix_(inner, inner)]
    np.testing.assert_allclose(G, Ac.toarray()[np.ix_(inner, inner)], atol=1e-13 * abs(G).max())


def test_boundary_rows_and_columns_vanish():
    P = h_prolongation(3, 2, 2).toarray()
    assert not P[boundary_nodes(3, 4, 2)].any()
    assert not P[:, boundary_nodes(3, 2, 2)].any()
