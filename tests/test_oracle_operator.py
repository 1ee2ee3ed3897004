"""Pins of the oracle's element and global operators (eq. bilinear-form, eq. matrix)."""
import itertools

import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle.assembly import (element_stiffness, l2_error, load_vector, mass_matrix, stiffness_matrix)
from oracle.mesh import StructuredMesh, node_physical_coords, patch_index_sets
from paper_2512_02577_amd.inputs import jittered_vertices


def _box_corners(dim, h):
    return np.array([np.array(o[::-1], dtype=float) * h for o in itertools.product((0, 1), repeat=dim)])


@pytest.mark.parametrize("dim", [2, 3])
def test_q1_element_matches_textbook(dim):
    # 1D linear elements on a cell of size h: K = [[1,-1],[-1,1]]/h, M = h/6 [[2,1],[1,2]];
    # the Q1 Laplacian on a box is the sum over directions of K in that direction and M
    # in the others (x index fastest)
    h = 0.37
    K = np.array([[1.0, -1.0], [-1.0, 1.0]]) / h
    M = h / 6 * np.array([[2.0, 1.0], [1.0, 2.0]])
    exp = 0
    for k in range(dim):
        mats = [K if a == k else M for a in range(dim)]
        t = mats[-1]
        for m_ in mats[-2::-1]:
            t = np.kron(t, m_)
        exp = exp + t
    np.testing.assert_allclose(element_stiffness(1, _box_corners(dim, h)), exp, rtol=1e-13, atol=1e-14)


@pytest.mark.parametrize("dim,n", [(2, 4), (3, 4), (3, 2)])
def test_q1_patch_diagonal(dim, n):
    # Q1 vertex patch: A_{j,1} = 8/3 in 2D and 8h/3 in 3D (h = 1/n)
    A = stiffness_matrix(StructuredMesh(dim, n), 1)
    _, inn = patch_index_sets(dim, n, 1)
    exp = 8.0 / 3.0 if dim == 2 else 8.0 / (3.0 * n)
    np.testing.assert_allclose(A.diagonal()[inn[:, 0]], exp, rtol=1e-14)


@pytest.mark.parametrize("dim,n,p,jit", [(2, 3, 3, 0.0), (2, 3, 2, 0.2), (3, 2, 2, 0.15), (3, 2, 3, 0.0)])
def test_symmetric_positive_definite_and_constant_kernel(dim, n, p, jit):
    verts = jittered_vertices(dim, n, jit, 7) if jit else None
    mesh = StructuredMesh(dim, n, verts)
    coef = (lambda x: 1.0 + x[:, 0] ** 2 + 0.5 * x[:, -1]) if jit else None
    A = stiffness_matrix(mesh, p, coef)
    Ad = A.toarray()
    np.testing.assert_allclose(Ad, Ad.T, atol=1e-13 * abs(Ad).max())
    assert np.linalg.eigvalsh(Ad).min() > 0
    An = stiffness_matrix(mesh, p, coef, dirichlet=False)
    assert abs(An @ np.ones(An.shape[0])).max() < 1e-12 * abs(An).max()


def _affine_mesh(dim, n):
    # global affine map of the unit box: every cell is a parallelepiped
    rng = np.random.default_rng(3)
    Mm = np.eye(dim) + 0.3 * rng.uniform(-1, 1, (dim, dim))
    t = np.arange(n + 1) / n
    g = np.meshgrid(*([t] * dim), indexing="ij")
    X = np.stack([a.reshape(-1, order="F") for a in g], axis=1)
    return StructuredMesh(dim, n, X @ Mm.T + 0.1), Mm


@pytest.mark.parametrize("dim,n,p", [(2, 2, 2), (2, 3, 3), (3, 2, 2), (3, 1, 3)])
def test_polynomial_exactness_on_affine_mesh(dim, n, p):
    # for u, v polynomials of total degree <= p in physical coordinates, u^T A v equals
    # the exact integral of grad u . grad v (the space contains them on affine cells and
    # the (p+1)-point Gauss rule integrates the integrand exactly)
    mesh, Mm = _affine_mesh(dim, n)
    A = stiffness_matrix(mesh, p, dirichlet=False)
    X = node_physical_coords(mesh, p)
    rng = np.random.default_rng(11)
    exps = [e for e in itertools.product(range(p + 1), repeat=dim) if sum(e) <= p]
    cu, cv = rng.uniform(-1, 1, len(exps)), rng.uniform(-1, 1, len(exps))

    def val(c, x):
        return sum(ci * np.prod([x[:, a] ** e[a] for a in range(dim)], axis=0) for ci, e in zip(c, exps))

    def grad(c, x):
        out = np.zeros((len(x), dim))
        for ci, e in zip(c, exps):
            for k in range(dim):
                if e[k] == 0:
                    continue
                term = ci * e[k] * np.ones(len(x))
                for a in range(dim):
                    term = term * x[:, a] ** (e[a] - (a == k))
                out[:, k] += term
        return out

    u, v = val(cu, X), val(cv, X)
    # exact integral by a high-order tensor Gauss rule on the unit box pulled through x = M xi + 0.1
    xg, wg = np.polynomial.legendre.leggauss(p + 2)
    xg, wg = (xg + 1) / 2, wg / 2
    pts = np.array(list(itertools.product(xg, repeat=dim)))
    wts = np.prod(np.array(list(itertools.product(wg, repeat=dim))), axis=1)
    x = pts @ Mm.T + 0.1
    exact = abs(np.linalg.det(Mm)) * np.sum(wts * np.sum(grad(cu, x) * grad(cv, x), axis=1))
    assert abs(u @ (A @ v) - exact) < 1e-11 * max(1.0, abs(exact))


def test_coefficient_scales_and_linear_coefficient_is_exact():
    mesh = StructuredMesh(2, 3, jittered_vertices(2, 3, 0.2, 5))
    A1 = stiffness_matrix(mesh, 2, dirichlet=False)
    A3 = stiffness_matrix(mesh, 2, coef=lambda x: 3.0 * np.ones(len(x)), dirichlet=False)
    np.testing.assert_allclose(A3.toarray(), 3.0 * A1.toarray(), atol=1e-13)
    # linear a, linear u and v on the unit square: int a grad u . grad v exactly
    m2 = StructuredMesh(2, 2)
    A = stiffness_matrix(m2, 1, coef=lambda x: 1.0 + x[:, 0], dirichlet=False)
    X = node_physical_coords(m2, 1)
    u, v = X[:, 0] + 2 * X[:, 1], X[:, 1]
    # grad u . grad v = 2, int_0^1 int_0^1 2 (1 + x) = 3
    assert abs(u @ (A @ v) - 3.0) < 1e-13


@pytest.mark.slow
@pytest.mark.parametrize("dim,p", [(2, 1), (2, 2), (2, 3), (3, 2)])
def test_manufactured_solution_rates(dim, p):
    # u* = prod sin(pi x_k), f = dim pi^2 u*: L2 error decays like h^(p+1)
    exact = lambda x: np.prod(np.sin(np.pi * x), axis=1)
    f = lambda x: dim * np.pi**2 * exact(x)
    errs = []
    ns = (4, 8) if dim == 2 else (2, 4)
    for n in ns:
        mesh = StructuredMesh(dim, n)
        A = stiffness_matrix(mesh, p)
        b = load_vector(mesh, p, f)
        u = spla.spsolve(A.tocsc(), b)
        errs.append(l2_error(mesh, p, u, exact))
    rate = np.log2(errs[0] / errs[1])
    assert rate > p + 1 - 0.35, (errs, rate)


def test_mass_matrix_integrates_one():
    mesh = StructuredMesh(3, 2, jittered_vertices(3, 2, 0.1, 2))
    M = mass_matrix(mesh, 3)
    one = np.ones(M.shape[0])
    # only interior vertices move, so the cells still tile the unit cube exactly
    assert abs(one @ (M @ one) - 1.0) < 1e-13
