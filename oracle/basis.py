"""1D building blocks on the reference interval [0, 1] (test infrastructure only).

The paper builds its operators from tensor-product shape functions on hexahedra with
sum factorization (Sec. 3, Sec. 3.2); it does not print the 1D rule.  Reading used here:
Lagrange polynomials on the p+1 Gauss-Lobatto points, integrated with the (p+1)-point
Gauss-Legendre rule (exact for the Laplacian on affine cells).
"""
from __future__ import annotations

import numpy as np
from numpy.polynomial import legendre as npleg


def gauss_legendre(nq: int) -> tuple[np.ndarray, np.ndarray]:
    """nq-point Gauss-Legendre rule mapped to [0, 1]: exact for degree 2*nq-1."""
    x, w = npleg.leggauss(nq)
    return 0.5 * (x + 1.0), 0.5 * w


def gauss_lobatto(p: int) -> np.ndarray:
    """The p+1 Gauss-Lobatto points on [0, 1]: both end points and the roots of P_p'."""
    if p < 1:
        raise ValueError("degree must be >= 1")
    interior = np.array([])
    if p >= 2:
        coeffs = np.zeros(p + 1)
        coeffs[p] = 1.0
        dP = npleg.legder(coeffs)
        r = np.sort(npleg.legroots(dP).real)
        # one Newton polish step per root on P_p' (companion-matrix roots carry ~1e-15 error)
        d2P = npleg.legder(dP)
        for _ in range(2):
            r = r - npleg.legval(r, dP) / npleg.legval(r, d2P)
        interior = r
    x = np.concatenate([[-1.0], interior, [1.0]])
    return 0.5 * (x + 1.0)


def lagrange_values(nodes: np.ndarray, x: np.ndarray) -> np.ndarray:
    """V[q, i] = l_i(x_q), l_i the Lagrange polynomial with l_i(nodes[m]) = delta_im."""
    nodes = np.asarray(nodes, dtype=np.float64)
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    k = len(nodes)
    V = np.ones((len(x), k))
    for i in range(k):
        for m in range(k):
            if m != i:
                V[:, i] *= (x - nodes[m]) / (nodes[i] - nodes[m])
    return V


def lagrange_derivatives(nodes: np.ndarray, x: np.ndarray) -> np.ndarray:
    """D[q, i] = l_i'(x_q) by the product rule: sum over the dropped factor."""
    nodes = np.asarray(nodes, dtype=np.float64)
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    k = len(nodes)
    D = np.zeros((len(x), k))
    for i in range(k):
        for s in range(k):
            if s == i:
                continue
            term = np.full(len(x), 1.0 / (nodes[i] - nodes[s]))
            for m in range(k):
                if m != i and m != s:
                    term *= (x - nodes[m]) / (nodes[i] - nodes[m])
            D[:, i] += term
    return D
