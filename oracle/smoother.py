"""Local p-multigrid patch solver and the multiplicative vertex-patch smoother
(test infrastructure only).

Sec. 2.1, Alg. 1: for each patch j, gather, evaluate the local residual
r_j = Pi_j b - Pi_j Abar_j ubar_j, solve approximately, scatter u += Pi_j^T d_j.
Here r_j is taken as the rows I_j of b - A u with the assembled global matrix, which is
the same vector because interior basis functions of a patch are supported inside it.
The sweep visits colors in ascending order (descending for post-smoothing) and patches
of one color by ascending index; the parity coloring makes the result independent of
the order inside a color.

Sec. 2.2, Alg. 2 (LocalSolve, preconditioned Richardson, first step from zero) and
Alg. 3 (p-V-cycle: damped Richardson pre-smoothing from zero, residual, restriction by
the transposed embedding, recursion, prolongation, optional post-smoothing; exact solve
on the coarsest level, a 1x1 system when its degree is 1).  Patch matrices A_{j,l} are
the dense extraction of the assembled degree-p_l matrix at the patch interior indices.

The Richardson preconditioner P_{j,l} of a p-level (Sec. 2.2) is either the diagonal
(damped Jacobi, the default) or the Cartesian-reinforced one: the inverse of the patch
operator of the undistorted (Cartesian) mesh, which fast diagonalization applies cheaply,
combined with diagonal scaling for the actual geometry.  The paper names the
combination without writing it out; the reading taken here is
    P^{-1} = D^{-1/2} D_C^{1/2} A_C^{-1} D_C^{1/2} D^{-1/2},
D = diag(A_{j,l}), A_C the same patch's matrix on the Cartesian mesh with the same cells,
D_C its diagonal; on a Cartesian mesh P^{-1} = A_{j,l}^{-1}.  Its default damping is 1.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from .assembly import stiffness_matrix
from .mesh import StructuredMesh, patch_colors, patch_index_sets
from .transfer import p_prolongation


class VmultCounter:
    """Counts local matrix-vector products per p-level (Sec. 2.2.1 counts them)."""

    def __init__(self, n_levels: int):
        self.count = [0] * n_levels

    def reset(self):
        self.count = [0] * len(self.count)


class PatchData:
    """Dense operators of one patch on every p-level."""

    def __init__(self, A, D, P, AC=None):
        self.A = A  # list over p-levels of dense (n_l, n_l)
        self.D = D  # list of diagonals
        self.P = P  # P[l]: (n_l, n_{l-1}) embedding, P[0] is None
        self.AC = AC  # Cartesian-reinforced smoother: the patch matrices on the Cartesian mesh


class LevelSmoother:
    """Everything the patch smoother needs on one mesh level."""

    def __init__(self, mesh: StructuredMesh, degrees: list[int], omega: list[float] | None = None,
                 coef=None, local: str = "half", n_local_iter: int = 1, smoother: str = "jacobi"):
        self.mesh = mesh
        self.degrees = list(degrees)
        dim, n = mesh.dim, mesh.n
        self.A = [stiffness_matrix(mesh, q, coef) for q in degrees]
        if smoother not in ("jacobi", "reinforced"):
            raise ValueError(smoother)
        self.smoother = smoother
        # the reinforced preconditioner's Cartesian patch operators (unit coefficient)
        self.AC = [stiffness_matrix(StructuredMesh(dim, n), q) for q in degrees] if smoother == "reinforced" else None
        self.interior = [patch_index_sets(dim, n, q)[1] for q in degrees]
        self.closure = patch_index_sets(dim, n, degrees[-1])[0]
        self.P = [None] + [p_prolongation(dim, n, degrees[l - 1], degrees[l]) for l in range(1, len(degrees))]
        self.colors = patch_colors(dim, n)
        self.n_colors = 2 ** dim
        if omega is None:
            omega = [default_omega(dim, q) if smoother == "jacobi" else 1.0 for q in degrees]
        self.omega = list(omega)
        if local not in ("half", "full", "direct"):
            raise ValueError(local)
        self.local = local
        self.n_local_iter = n_local_iter
        self.counter = VmultCounter(len(degrees))
        self._cache: dict[int, PatchData] = {}

    # ------------------------------------------------------------------ patch data
    def patch(self, j: int) -> PatchData:
        if j in self._cache:
            return self._cache[j]
        A, D, P, AC = [], [], [None], []
        for l in range(len(self.degrees)):
            I = self.interior[l][j]
            Al = self.A[l][I][:, I].toarray()
            A.append(Al)
            D.append(np.diag(Al).copy())
            if self.AC is not None:
                AC.append(self.AC[l][I][:, I].toarray())
            if l > 0:
                P.append(self.P[l][I][:, self.interior[l - 1][j]].toarray())
        pd = PatchData(A, D, P, AC if self.AC is not None else None)
        per_patch = sum(a.nbytes for a in A) + sum(x.nbytes for x in P[1:])
        if (len(self._cache) + 1) * per_patch < 2e9:
            self._cache[j] = pd
        return pd

    # ------------------------------------------- Richardson preconditioner P_{j,l}^{-1}
    def precondition(self, pd: PatchData, l: int, r: np.ndarray) -> np.ndarray:
        if self.smoother == "jacobi":
            return r / pd.D[l]
        s = np.sqrt(np.diag(pd.AC[l]) / pd.D[l])  # D^{-1/2} D_C^{1/2}
        return s * np.linalg.solve(pd.AC[l], s * r)

    # ------------------------------------------------------- Alg. 3: p-V-cycle
    def vcycle(self, pd: PatchData, l: int, r: np.ndarray, full: bool) -> np.ndarray:
        if l == 0:
            return np.linalg.solve(pd.A[0], r)  # 1x1 when the coarsest degree is 1
        d = self.omega[l] * self.precondition(pd, l, r)  # pre-smoothing from a zero guess
        res = r - pd.A[l] @ d
        self.counter.count[l] += 1
        rc = pd.P[l].T @ res
        ec = self.vcycle(pd, l - 1, rc, full)
        d = d + pd.P[l] @ ec
        if full:
            res = r - pd.A[l] @ d
            self.counter.count[l] += 1
            d = d + self.omega[l] * self.precondition(pd, l, res)
        return d

    # ------------------------------------------------------- Alg. 2: LocalSolve
    def local_solve(self, j: int, r: np.ndarray) -> np.ndarray:
        pd = self.patch(j)
        top = len(self.degrees) - 1
        if self.local == "direct":
            return sla.solve(pd.A[top], r, assume_a="pos")
        full = self.local == "full"
        d = self.vcycle(pd, top, r, full)
        for _ in range(1, self.n_local_iter):
            res = r - pd.A[top] @ d
            self.counter.count[top] += 1
            d = d + self.vcycle(pd, top, res, full)
        return d

    # ------------------------------------------------------- Alg. 1, colored order
    def patch_order(self, descending: bool = False, permute_within_color=None) -> list[int]:
        order = []
        cols = range(self.n_colors - 1, -1, -1) if descending else range(self.n_colors)
        for c in cols:
            js = np.nonzero(self.colors == c)[0]
            if permute_within_color is not None:
                js = permute_within_color(js)
            order.extend(int(j) for j in js)
        return order

    def smooth(self, u: np.ndarray, b: np.ndarray, descending: bool = False, order=None) -> np.ndarray:
        u = np.array(u, dtype=np.float64, copy=True)
        A = self.A[-1]
        I_top = self.interior[-1]
        for j in (order if order is not None else self.patch_order(descending)):
            I = I_top[j]
            r = b[I] - A[I] @ u
            u[I] += self.local_solve(j, r)
        return u


def default_omega(dim: int, q: int) -> float:
    """Jacobi damping of a p-level (the paper does not give it): 4 / (3 lambda_max) of
    D^{-1} A on the interior of one Cartesian vertex patch of degree q (h-independent)."""
    if q == 1:
        return 1.0
    mesh = StructuredMesh(dim, 2)
    A = stiffness_matrix(mesh, q)
    I = patch_index_sets(dim, 2, q)[1][0]
    Ap = A[I][:, I].toarray()
    lam = sla.eigh(Ap, np.diag(np.diag(Ap)), eigvals_only=True)
    return 4.0 / (3.0 * lam[-1])
