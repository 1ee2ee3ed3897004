"""Pins of the oracle's local p-multigrid (Alg. 2, Alg. 3) and patch smoother (Alg. 1)."""
import os

import numpy as np
import pytest

from oracle.mesh import StructuredMesh, patch_index_sets
from oracle.smoother import LevelSmoother, default_omega
from paper_2512_02577_amd.inputs import jittered_vertices, rhs_vector

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _local_matrix(ls, j, full):
    """Columns: the local solve applied to unit vectors."""
    n = ls.interior[-1].shape[1]
    return np.stack([ls.local_solve(j, e) for e in np.eye(n)], axis=1)


@pytest.mark.parametrize("dim,p", [(2, 2), (3, 2), (2, 3)])
def test_half_vcycle_two_level_closed_form(dim, p):
    # Two p-levels {1, p}: the half V-cycle from zero is
    # B = S + P A_c^{-1} P^T (I - A S), S = omega D^{-1}
    ls = LevelSmoother(StructuredMesh(dim, 2), [1, p], omega=[1.0, 0.6], local="half")
    pd = ls.patch(0)
    A, D, P, Ac = pd.A[1], pd.D[1], pd.P[1], pd.A[0]
    S = 0.6 * np.diag(1 / D)
    B = S + P @ np.linalg.inv(Ac) @ P.T @ (np.eye(len(D)) - A @ S)
    np.testing.assert_allclose(_local_matrix(ls, 0, False), B, atol=1e-13 * abs(B).max())


@pytest.mark.parametrize("dim,levels", [(2, [1, 3]), (2, [1, 2, 3]), (3, [1, 2])])
def test_full_vcycle_is_symmetric_half_is_not(dim, levels):
    mesh = StructuredMesh(dim, 2, jittered_vertices(dim, 2, 0.2, 1))
    full = LevelSmoother(mesh, levels, local="full")
    Bf = _local_matrix(full, 0, True)
    np.testing.assert_allclose(Bf, Bf.T, atol=1e-12 * abs(Bf).max())
    half = LevelSmoother(mesh, levels, local="half")
    Bh = _local_matrix(half, 0, False)
    assert abs(Bh - Bh.T).max() > 1e-6 * abs(Bh).max()


@pytest.mark.parametrize("local", ["half", "full"])
def test_many_vcycles_approach_direct_solve(local):
    # Table 1 uses 25 V-cycles as a nearly exact local solve
    ls = LevelSmoother(StructuredMesh(3, 2), [1, 3, 4], local=local, n_local_iter=60)
    r = np.random.default_rng(2).uniform(-1, 1, ls.interior[-1].shape[1])
    pd = ls.patch(0)
    exact = np.linalg.solve(pd.A[-1], r)
    np.testing.assert_allclose(ls.local_solve(0, r), exact, rtol=0, atol=1e-9 * abs(exact).max())


def test_vmult_counts_match_paper():
    with open(os.path.join(GOLDEN, "paper_vmult_counts.txt")) as f:
        rows = [l.split() for l in f if l.strip() and not l.startswith("#")]
    for local, n_iter, vm in rows:
        ls = LevelSmoother(StructuredMesh(2, 2), [1, 3, 7], local=local, n_local_iter=int(n_iter))
        ls.local_solve(0, np.ones(ls.interior[-1].shape[1]))
        assert ls.counter.count[-1] == int(vm), (local, n_iter, ls.counter.count)


def test_coarse_level_is_exact_scalar_solve():
    ls = LevelSmoother(StructuredMesh(3, 2), [1, 2], local="half")
    pd = ls.patch(0)
    assert pd.A[0].shape == (1, 1)
    np.testing.assert_allclose(pd.A[0][0, 0], 8.0 / 6.0, rtol=1e-14)  # 8h/3 with h = 1/2


@pytest.mark.parametrize("dim,n,p", [(2, 4, 2), (3, 3, 2)])
def test_direct_local_solve_zeroes_patch_residual_and_decreases_energy(dim, n, p):
    mesh = StructuredMesh(dim, n, jittered_vertices(dim, n, 0.1, 4))
    ls = LevelSmoother(mesh, [1, p], local="direct")
    A = ls.A[-1]
    b = rhs_vector(dim, n, p, 9)
    x_star = np.linalg.solve(A.toarray(), b)
    u = np.zeros_like(b)
    energy = lambda v: (v - x_star) @ (A @ (v - x_star))
    e_prev = energy(u)
    for j in ls.patch_order():
        u = ls.smooth(u, b, order=[j])
        I = ls.interior[-1][j]
        assert abs((b - A @ u)[I]).max() < 1e-12 * abs(b).max()
        e = energy(u)
        assert e <= e_prev * (1 + 1e-12)
        e_prev = e


@pytest.mark.parametrize("local", ["half", "full"])
def test_order_independence_within_color(local):
    dim, n, p = 3, 4, 2
    ls = LevelSmoother(StructuredMesh(dim, n), [1, p], local=local)
    b = rhs_vector(dim, n, p, 1)
    u0 = np.random.default_rng(5).uniform(-1, 1, len(b))
    ref = ls.smooth(u0, b)
    rng = np.random.default_rng(6)
    perm = ls.patch_order(permute_within_color=lambda js: rng.permutation(js))
    np.testing.assert_allclose(ls.smooth(u0, b, order=perm), ref, rtol=0, atol=1e-14)
    # a different color order gives a different (also valid) result
    assert abs(ls.smooth(u0, b, descending=True) - ref).max() > 1e-6


def test_exact_solution_is_fixed_point():
    dim, n, p = 2, 4, 3
    ls = LevelSmoother(StructuredMesh(dim, n), [1, 2, 3], local="half")
    b = rhs_vector(dim, n, p, 2)
    x = np.linalg.solve(ls.A[-1].toarray(), b)
    np.testing.assert_allclose(ls.smooth(x, b), x, atol=1e-13)


@pytest.mark.parametrize("dim,q", [(2, 3), (3, 2), (3, 4)])
def test_default_omega_in_stable_range(dim, q):
    # damped Jacobi needs 0 < omega < 2 / lambda_max(D^{-1} A)
    w = default_omega(dim, q)
    mesh = StructuredMesh(dim, 2)
    ls = LevelSmoother(mesh, [1, q], omega=[1.0, w])
    pd = ls.patch(0)
    lam = np.linalg.eigvals(np.diag(1 / pd.D[1]) @ pd.A[1]).real.max()
    assert 0 < w * lam < 2
    np.testing.assert_allclose(w * lam, 4 / 3, rtol=1e-10)


# ---- Cartesian-reinforced p-level smoother (Sec. 2.2: fast-diagonalization inverse of the
# Cartesian patch operator with diagonal scaling) and the exact local solve --------------

@pytest.mark.parametrize("dim,levels", [(2, [1, 3]), (3, [1, 2]), (2, [1, 3, 7])])
def test_reinforced_half_vcycle_is_exact_on_cartesian_patches(dim, levels):
    # on a Cartesian mesh the reinforced preconditioner inverts the patch operator, so with
    # its default damping 1 the first pre-smoothing step already solves the patch problem
    # and the coarse correction vanishes: one half V-cycle equals the direct solve
    ls = LevelSmoother(StructuredMesh(dim, 3), levels, local="half", smoother="reinforced")
    assert ls.omega[1:] == [1.0] * (len(levels) - 1)
    direct = LevelSmoother(StructuredMesh(dim, 3), levels, local="direct")
    r = np.random.default_rng(2).uniform(-1, 1, ls.interior[-1].shape[1])
    for j in (0, 3):
        A = ls.patch(j).A[-1]
        d = ls.local_solve(j, r)
        np.testing.assert_allclose(d, direct.local_solve(j, r), atol=1e-12 * abs(d).max())
        assert abs(A @ d - r).max() <= 1e-12 * abs(r).max()


@pytest.mark.parametrize("dim,p,w", [(2, 3, 0.7), (3, 2, 0.8)])
def test_reinforced_two_level_closed_form(dim, p, w):
    # two p-levels {1, p}, damping w, Cartesian: B = w A^{-1} + P A_c^{-1} P^T (I - w I)
    ls = LevelSmoother(StructuredMesh(dim, 2), [1, p], omega=[1.0, w], local="half", smoother="reinforced")
    pd = ls.patch(0)
    A, P, Ac = pd.A[1], pd.P[1], pd.A[0]
    n = A.shape[0]
    B = w * np.linalg.inv(A) + (1 - w) * P @ np.linalg.inv(Ac) @ P.T
    np.testing.assert_allclose(_local_matrix(ls, 0, False), B, atol=1e-12 * abs(B).max())


def test_reinforced_preconditioner_on_a_distorted_patch():
    # the preconditioner matrix P = S^-1 A_C S^-1 (S = D^-1/2 D_C^1/2) keeps the coupling of
    # the Cartesian patch operator and takes the diagonal of the actual one; it is symmetric
    # positive definite
    mesh = StructuredMesh(2, 3, jittered_vertices(2, 3, 0.2, 4))
    ls = LevelSmoother(mesh, [1, 3], local="half", smoother="reinforced")
    pd = ls.patch(2)
    n = pd.A[1].shape[0]
    Pinv = np.stack([ls.precondition(pd, 1, e) for e in np.eye(n)], axis=1)
    np.testing.assert_allclose(Pinv, Pinv.T, atol=1e-12 * abs(Pinv).max())
    Pm = np.linalg.inv(Pinv)
    np.testing.assert_allclose(np.diag(Pm), pd.D[1], rtol=1e-10)
    assert np.linalg.eigvalsh(Pm).min() > 0
    # the Cartesian coupling: P_ij / sqrt(P_ii P_jj) equals that of the Cartesian matrix
    C = pd.AC[1]
    np.testing.assert_allclose(Pm / np.sqrt(np.outer(np.diag(Pm), np.diag(Pm))),
                               C / np.sqrt(np.outer(np.diag(C), np.diag(C))), atol=1e-10)
