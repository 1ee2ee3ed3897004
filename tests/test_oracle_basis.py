"""Pins of the oracle's 1D building blocks against closed forms and invariants."""
import numpy as np
import pytest

from oracle.basis import gauss_legendre, gauss_lobatto, lagrange_derivatives, lagrange_values

GLL_CLOSED = {
    1: [0.0, 1.0],
    2: [0.0, 0.5, 1.0],
    3: [0.0, (1 - 1 / np.sqrt(5)) / 2, (1 + 1 / np.sqrt(5)) / 2, 1.0],
    4: [0.0, (1 - np.sqrt(3 / 7)) / 2, 0.5, (1 + np.sqrt(3 / 7)) / 2, 1.0],
}


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_gll_closed_forms(p):
    np.testing.assert_allclose(gauss_lobatto(p), GLL_CLOSED[p], rtol=0, atol=1e-15)


@pytest.mark.parametrize("p", range(1, 9))
def test_gll_symmetric_and_lobatto_exact(p):
    x = gauss_lobatto(p)
    np.testing.assert_allclose(x + x[::-1], 1.0, atol=1e-15)
    # Lobatto quadrature with these nodes is exact to degree 2p-1: recover weights from
    # the moment system and check the next moments
    V = np.vander(x, p + 1, increasing=True).T
    w = np.linalg.solve(V, 1.0 / np.arange(1, p + 2))
    for k in range(2 * p):
        assert abs(w @ x**k - 1.0 / (k + 1)) < 1e-12


@pytest.mark.parametrize("nq", range(1, 10))
def test_gauss_exactness(nq):
    x, w = gauss_legendre(nq)
    for k in range(2 * nq):
        assert abs(w @ x**k - 1.0 / (k + 1)) < 1e-14
    assert abs(w @ x ** (2 * nq) - 1.0 / (2 * nq + 1)) > 1e-12  # first inexact degree


@pytest.mark.parametrize("p", range(1, 9))
def test_lagrange_cardinal_and_partition(p):
    nodes = gauss_lobatto(p)
    np.testing.assert_allclose(lagrange_values(nodes, nodes), np.eye(p + 1), atol=1e-14)
    x = np.linspace(0, 1, 37)
    np.testing.assert_allclose(lagrange_values(nodes, x).sum(1), 1.0, atol=1e-12)
    np.testing.assert_allclose(lagrange_derivatives(nodes, x).sum(1), 0.0, atol=1e-10)


@pytest.mark.parametrize("p", range(1, 9))
def test_lagrange_reproduces_polynomials_and_derivatives(p):
    nodes = gauss_lobatto(p)
    x = np.linspace(0, 1, 23)
    V = lagrange_values(nodes, x)
    D = lagrange_derivatives(nodes, x)
    for k in range(p + 1):
        np.testing.assert_allclose(V @ nodes**k, x**k, atol=1e-12)
        dk = k * x ** (k - 1) if k else np.zeros_like(x)
        np.testing.assert_allclose(D @ nodes**k, dk, atol=1e-9)


def test_lagrange_derivative_matches_finite_difference():
    nodes = gauss_lobatto(5)
    x = np.linspace(0.05, 0.95, 11)
    h = 1e-6
    fd = (lagrange_values(nodes, x + h) - lagrange_values(nodes, x - h)) / (2 * h)
    np.testing.assert_allclose(lagrange_derivatives(nodes, x), fd, atol=1e-6)
