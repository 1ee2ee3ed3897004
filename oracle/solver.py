"""h-multigrid V-cycle with the patch smoother and the outer flexible CG
(test infrastructure only).

Sec. 2: mesh hierarchy M_0 ... M_L, operators rediscretized on every level,
prolongation = embedding, restriction = its transpose, the vertex-patch smoother of
Sec. 2.1 on every level but the coarsest.  The paper leaves the cycle shape and the
coarse solver open; the reading taken here is V(1,1) from a zero guess, pre-smoothing
in ascending color order, post-smoothing in descending order, and an exact dense
Cholesky solve on M_0.  The paper wraps the preconditioner in GMRES because the
half V-cycle and the multiplicative sweep are not symmetric; the reading here is the
flexible CG of Notay (FCG(1), Polak-Ribiere beta), which tolerates a nonsymmetric,
varying preconditioner.  Dirichlet rows are identity rows on every level.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse.linalg as spla

from .mesh import StructuredMesh, boundary_nodes, hlevel_sizes, p_hierarchy
from .smoother import LevelSmoother
from .transfer import h_prolongation


class MultigridProblem:
    """All levels of the h-multigrid preconditioner for one problem (FP64)."""

    def __init__(self, dim: int, n: int, p: int, p_levels: list[int] | None = None,
                 vertices: np.ndarray | None = None, coef=None, n_hlevels: int = 0,
                 omega: list[float] | None = None, local: str = "half", n_local_iter: int = 1,
                 n_pre: int = 1, n_post: int = 1, smoother: str = "jacobi"):
        self.dim, self.n, self.p = dim, n, p
        self.degrees = list(p_levels) if p_levels is not None else p_hierarchy(p)
        if self.degrees[-1] != p:
            raise ValueError("the last p-level must be the degree")
        self.sizes = hlevel_sizes(n, n_hlevels)
        fine = StructuredMesh(dim, n, vertices)
        self.meshes = [fine.coarsened(s) for s in self.sizes]
        self.coef = coef
        self.n_pre, self.n_post = n_pre, n_post
        self.levels = []
        for li, m in enumerate(self.meshes):
            if li == 0:
                self.levels.append(None)
            else:
                self.levels.append(LevelSmoother(m, self.degrees, omega, coef, local, n_local_iter, smoother))
        from .assembly import stiffness_matrix

        self.A = [lv.A[-1] if lv is not None else stiffness_matrix(self.meshes[0], p, coef) for lv in self.levels]
        self.P = [None] + [h_prolongation(dim, self.sizes[l - 1], p) for l in range(1, len(self.sizes))]
        self.bnd = [boundary_nodes(dim, s, p) for s in self.sizes]
        inner = ~self.bnd[0]
        A0 = self.A[0][inner][:, inner].toarray()
        self._coarse = (sla.cho_factor(A0), inner)

    @property
    def N(self) -> int:
        return (self.p * self.n + 1) ** self.dim

    def coarse_solve(self, r: np.ndarray) -> np.ndarray:
        fac, inner = self._coarse
        z = r.copy()
        z[inner] = sla.cho_solve(fac, r[inner])
        return z

    def smooth(self, level: int, u: np.ndarray, b: np.ndarray, descending: bool = False) -> np.ndarray:
        return self.levels[level].smooth(u, b, descending)

    def vcycle(self, r: np.ndarray, level: int | None = None) -> np.ndarray:
        """z = V(r) on mesh level `level` (default finest), zero initial guess."""
        if level is None:
            level = len(self.sizes) - 1
        if level == 0:
            return self.coarse_solve(r)
        bnd = self.bnd[level]
        z = np.zeros_like(r)
        z[bnd] = r[bnd]
        for _ in range(self.n_pre):
            z = self.smooth(level, z, r, descending=False)
        res = r - self.A[level] @ z
        zc = self.vcycle(self.P[level].T @ res, level - 1)
        z = z + self.P[level] @ zc
        for _ in range(self.n_post):
            z = self.smooth(level, z, r, descending=True)
        return z

    def apply(self, u: np.ndarray, level: int | None = None) -> np.ndarray:
        return self.A[len(self.sizes) - 1 if level is None else level] @ u

    def direct_solve(self, b: np.ndarray) -> np.ndarray:
        return spla.splu(self.A[-1].tocsc()).solve(b)


def fcg(A, b: np.ndarray, precond, rtol: float = 1e-8, max_iter: int = 200, x0: np.ndarray | None = None):
    """Flexible CG, FCG(1) with the Polak-Ribiere beta:
    q = A p; alpha = (r,z)/(p,q); x += alpha p; r' = r - alpha q;
    stop when |r'| <= rtol |b|; z' = B r'; beta = (z', r' - r)/(z, r); p = z' + beta p.
    Returns (x, iterations, relative residual history)."""
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64, copy=True)
    r = b - A(x)
    nb = np.linalg.norm(b)
    hist = [np.linalg.norm(r) / nb]
    if hist[-1] <= rtol:
        return x, 0, hist
    z = precond(r)
    p = z.copy()
    rz = r @ z
    for it in range(1, max_iter + 1):
        q = A(p)
        alpha = rz / (p @ q)
        x = x + alpha * p
        r_new = r - alpha * q
        hist.append(np.linalg.norm(r_new) / nb)
        if hist[-1] <= rtol:
            return x, it, hist
        z_new = precond(r_new)
        beta = (z_new @ (r_new - r)) / rz
        p = z_new + beta * p
        r, z = r_new, z_new
        rz = r @ z
    return x, max_iter, hist


def solve(problem: MultigridProblem, b: np.ndarray, rtol: float = 1e-8, max_iter: int = 200):
    return fcg(problem.apply, b, problem.vcycle, rtol, max_iter)


def gmres(A, b: np.ndarray, precond, rtol: float = 1e-8, restart: int = 30, max_iter: int = 500):
    """Restarted GMRES(restart) with right preconditioning, the outer solver the paper uses
    (Sec. 2.2.1, Table 1): x = x0 + B y, y minimizing |b - A x0 - A B y| over the Krylov
    space of A B built by Arnoldi with modified Gram-Schmidt; stops when the true residual
    |b - A x| <= rtol |b| (with right preconditioning the least-squares residual is the true
    one).  Returns (x, iterations, relative residual history)."""
    n = len(b)
    x = np.zeros(n)
    nb = np.linalg.norm(b)
    r = b.copy()
    beta = np.linalg.norm(r)
    hist = [beta / nb]
    it = 0
    while hist[-1] > rtol and it < max_iter:
        m = min(restart, max_iter - it)
        V = np.zeros((m + 1, n))
        Z = np.zeros((m, n))
        H = np.zeros((m + 1, m))
        V[0] = r / beta
        k_done = 0
        for k in range(m):
            Z[k] = precond(V[k])
            w = A(Z[k])
            for i in range(k + 1):
                H[i, k] = w @ V[i]
                w = w - H[i, k] * V[i]
            H[k + 1, k] = np.linalg.norm(w)
            if H[k + 1, k] > 0:
                V[k + 1] = w / H[k + 1, k]
            k_done = k + 1
            it += 1
            e1 = np.zeros(k + 2)
            e1[0] = beta
            y, *_ = np.linalg.lstsq(H[:k + 2, :k + 1], e1, rcond=None)
            res = np.linalg.norm(e1 - H[:k + 2, :k + 1] @ y)
            hist.append(res / nb)
            if hist[-1] <= rtol or H[k + 1, k] == 0:
                break
        x = x + y @ Z[:k_done]
        r = b - A(x)
        beta = np.linalg.norm(r)
        hist[-1] = beta / nb
        if H[k_done, k_done - 1] == 0:
            break
    return x, it, hist


def gmres_solve(problem: MultigridProblem, b: np.ndarray, rtol: float = 1e-8, restart: int = 30,
                max_iter: int = 500):
    return gmres(problem.apply, b, problem.vcycle, rtol, restart, max_iter)
