"""Pins of the oracle pieces that serve as references at full size, where the assembled
operator is out of reach: row-wise products (A u)_i without assembly, physical Gauss
points, and the exact coarse solve.

`apply_rows` is compared on every row (or, for the largest 3D degrees, on every row that
couples several cells plus a seeded sample) with the assembled operator of eq. matrix,
which is pinned independently in test_oracle_operator.py (closed forms, exactness,
symmetry); a planted mistake in its candidate-cell set must make the comparison fail.
`quadrature_points` is compared with Gauss-Legendre points written in closed form.  The
consistent mass matrix (the right-hand side b = M f of the benchmark, and the reference of the
GPU's mass apply) is pinned by its row sums (the integrals of the basis functions: products of
Gauss-Lobatto weights, computed here from their closed form), symmetry and definiteness, and
the textbook Q1 matrix.
"""
import itertools

import numpy as np
import pytest

import oracle.assembly as asm
from oracle.assembly import apply_rows, quadrature_points, stiffness_matrix
from oracle.mesh import StructuredMesh, boundary_nodes
from oracle.solver import MultigridProblem
from paper_2512_02577_amd.inputs import CoefficientField, jittered_vertices


def _mesh(dim, n, jit):
    return StructuredMesh(dim, n, jittered_vertices(dim, n, jit, 17) if jit else None)


def _rows_all(dim, n, p):
    return np.arange((p * n + 1) ** dim)


def _rows_shared_plus_sample(dim, n, p, k=120):
    # rows whose node lies on a cell face, edge or corner in some direction (the rows that
    # sum over several cells), boundary rows, and a seeded sample of the others
    m = p * n + 1
    g = np.arange(m ** dim)
    idx = np.stack([(g // m ** a) % m for a in range(dim)], axis=1)
    shared = np.any(idx % p == 0, axis=1)
    rest = np.nonzero(~shared)[0]
    pick = np.random.default_rng(5).choice(rest, min(k, len(rest)), replace=False)
    return np.union1d(np.nonzero(shared)[0], pick)


CASES = ([(2, 3, p, 0.0, False, "all") for p in range(1, 9)] +
         [(2, 3, p, 0.15, True, "all") for p in (1, 2, 3, 4)] +
         [(3, 2, p, 0.0, False, "all") for p in (1, 2, 3, 4)] +
         [(3, 3, 2, 0.0, False, "all"), (3, 2, 1, 0.1, True, "all"), (3, 2, 2, 0.1, True, "all")] +
         [(3, 2, p, 0.0, False, "shared") for p in (5, 6, 7, 8)])


@pytest.mark.parametrize("dim,n,p,jit,use_coef,rows", CASES)
def test_apply_rows_equals_assembled_operator(dim, n, p, jit, use_coef, rows):
    mesh = _mesh(dim, n, jit)
    coef = CoefficientField(dim, 23) if use_coef else None
    A = stiffness_matrix(mesh, p, coef)
    u = np.random.default_rng(p).uniform(-1, 1, A.shape[0])
    sel = _rows_all(dim, n, p) if rows == "all" else _rows_shared_plus_sample(dim, n, p)
    ref = (A @ u)[sel]
    got = apply_rows(mesh, p, u, sel, coef)
    assert abs(got - ref).max() <= 1e-14 * max(1.0, abs(ref).max())
    # boundary rows are identity rows
    bnd = boundary_nodes(dim, n, p)[sel]
    assert np.array_equal(got[bnd], u[sel][bnd])


@pytest.mark.parametrize("plant", ["drop_lower", "drop_upper"])
def test_planted_candidate_cell_mistake_is_caught(monkeypatch, plant):
    # a node on a shared cell end belongs to two cells per direction; dropping either one
    # from the candidate set must change some rows of the product
    right = asm.cells_of_node_1d

    def wrong(i, n, p):
        cs = right(i, n, p)
        if len(cs) == 2:
            cs = cs[1:] if plant == "drop_lower" else cs[:1]
        return cs

    dim, n, p = 2, 3, 2
    mesh = _mesh(dim, n, 0.0)
    A = stiffness_matrix(mesh, p)
    u = np.random.default_rng(0).uniform(-1, 1, A.shape[0])
    sel = _rows_all(dim, n, p)
    monkeypatch.setattr(asm, "cells_of_node_1d", wrong)
    got = asm.apply_rows(mesh, p, u, sel)
    assert abs(got - A @ u).max() > 1e-3


def _gl_closed_form(nq):
    # Gauss-Legendre nodes on [-1, 1] in closed form (roots of P_nq), mapped to [0, 1]
    s = {1: [0.0],
         2: [-1 / np.sqrt(3), 1 / np.sqrt(3)],
         3: [-np.sqrt(3 / 5), 0.0, np.sqrt(3 / 5)],
         4: sorted([sg * np.sqrt(3 / 7 + t * 2 / 7 * np.sqrt(6 / 5)) for sg in (-1, 1) for t in (-1, 1)]),
         5: sorted([0.0] + [sg * np.sqrt(5 + t * 2 * np.sqrt(10 / 7)) / 3 for sg in (-1, 1) for t in (-1, 1)])}[nq]
    return (np.array(s) + 1) / 2


@pytest.mark.parametrize("dim,n,p", [(2, 3, 1), (2, 2, 2), (2, 2, 4), (3, 2, 1), (3, 2, 2), (3, 1, 3)])
def test_quadrature_points_affine_closed_form(dim, n, p):
    # a global affine map x = B xi + t of the unit box makes every cell a parallelepiped;
    # the Gauss points of cell c are B (c + g) / n + t with g the tensor of closed-form
    # Gauss-Legendre nodes (x fastest), for the (p+1)-point rule of the degree-p level
    rng = np.random.default_rng(4)
    B = np.eye(dim) + 0.3 * rng.uniform(-1, 1, (dim, dim))
    t0 = rng.uniform(-0.5, 0.5, dim)
    tt = np.arange(n + 1) / n
    g = np.meshgrid(*([tt] * dim), indexing="ij")
    X = np.stack([a.reshape(-1, order="F") for a in g], axis=1) @ B.T + t0
    mesh = StructuredMesh(dim, n, X)
    got = quadrature_points(mesh, p)
    x1 = _gl_closed_form(p + 1)
    ref = np.empty_like(got)
    for c in range(n ** dim):
        ci = np.array([(c // n ** a) % n for a in range(dim)])
        for k, pt in enumerate(itertools.product(*([x1] * dim))):
            xi = (ci + np.array(pt[::-1])) / n  # itertools varies the last factor fastest
            ref[c, k] = B @ xi + t0
    np.testing.assert_allclose(got, ref, atol=1e-14, rtol=0)


@pytest.mark.parametrize("dim,n,p,jit", [(2, 4, 3, 0.0), (3, 4, 2, 0.0), (2, 6, 2, 0.1)])
def test_coarse_solve_inverts_the_coarse_operator(dim, n, p, jit):
    # z = coarse_solve(r): A_0 z = r on every row (interior rows by the solve, boundary
    # rows because they are identity rows and z keeps r there)
    verts = jittered_vertices(dim, n, jit, 3) if jit else None
    pb = MultigridProblem(dim, n, p, vertices=verts)
    r = np.random.default_rng(8).uniform(-1, 1, (p * pb.sizes[0] + 1) ** dim)
    z = pb.coarse_solve(r)
    A0 = stiffness_matrix(pb.meshes[0], p)
    assert abs(A0 @ z - r).max() <= 1e-12 * abs(r).max()


def _gll_weights_unit(p):
    """Gauss-Lobatto weights on [0, 1] in closed form: nodes -1, 1 and the roots of P_p',
    weights 2 / (p (p + 1) P_p(x)^2) on [-1, 1] (independent of the oracle's quadrature)."""
    from numpy.polynomial import legendre as L

    c = np.zeros(p + 1)
    c[p] = 1.0
    x = np.concatenate([[-1.0], np.sort(np.real(L.legroots(L.legder(c)))), [1.0]]) if p > 1 else np.array([-1.0, 1.0])
    w = 2.0 / (p * (p + 1) * L.legval(x, c) ** 2)
    return w / 2.0


@pytest.mark.parametrize("dim,n,p", [(2, 3, 1), (2, 2, 3), (2, 3, 5), (3, 2, 2), (3, 2, 4), (2, 2, 8)])
def test_mass_matrix_row_sums_are_integrals_of_the_basis(dim, n, p):
    # the nodal basis sums to one, so a row sum of the consistent mass matrix is the integral
    # of that basis function: on the uniform mesh the product over the directions of h times
    # the Gauss-Lobatto weights of the (one or two) cells containing the node's coordinate
    # (the Lobatto rule with p+1 points integrates the degree-p basis exactly)
    M = asm.mass_matrix(StructuredMesh(dim, n), p)
    m = p * n + 1
    w = _gll_weights_unit(p) / n
    w1 = np.zeros(m)
    for c in range(n):
        w1[p * c:p * c + p + 1] += w
    ref = w1
    for _ in range(dim - 1):
        ref = np.multiply.outer(w1, ref).reshape(-1)  # x fastest: the last factor varies fastest
    assert abs(M.sum(axis=1).A1 - ref).max() <= 1e-14
    assert abs(M.sum() - 1.0) <= 1e-13  # the unit box's volume


@pytest.mark.parametrize("dim,n,p,jit", [(2, 3, 3, 0.0), (3, 2, 2, 0.0), (2, 3, 2, 0.2)])
def test_mass_matrix_is_symmetric_positive_definite(dim, n, p, jit):
    M = asm.mass_matrix(_mesh(dim, n, jit), p).toarray()
    assert abs(M - M.T).max() <= 1e-15 * abs(M).max()
    assert np.linalg.eigvalsh(M).min() > 0


def test_mass_matrix_of_q1_is_the_textbook_kronecker_product():
    # Q1 on a uniform 1D mesh of n cells: h/6 tridiag(1, 4, 1) (2 h/6 at the ends); the 2D
    # matrix is the Kronecker product of two 1D ones
    n = 4
    h = 1.0 / n
    M1 = np.diag(np.full(n + 1, 4.0)) + np.diag(np.ones(n), 1) + np.diag(np.ones(n), -1)
    M1[0, 0] = M1[n, n] = 2.0
    M1 *= h / 6
    M = asm.mass_matrix(StructuredMesh(2, n), 1).toarray()
    assert abs(M - np.kron(M1, M1)).max() <= 1e-15
