"""Algorithmic flop and byte counts of the kernels, for roofline reporting.

Flops count the multiply-adds the sum-factorized formulation performs (2 flops each,
skipping the structural zeros of the 1D matrices, as the kernels do) plus the scaling
and Jacobi multiplies.  Bytes are the minimum data a launch must move: every vector
entry it reads or writes once (index maps are computed, not loaded; the 1D tables are a
few KB and ignored).
"""
from __future__ import annotations


def _nnz_interior(q: int) -> int:  # square interior patch matrix of degree q
    n = 2 * q - 1
    return sum(((q if o + 1 < q else 2 * q - 1) - (q - 1 if o + 1 > q else 0)) for o in range(n))


def _nnz_residual(p: int) -> int:  # (2p-1) x (2p+1)
    n = 2 * p - 1
    return sum(((p + 1 if o + 1 < p else 2 * p + 1) - (p if o + 1 > p else 0)) for o in range(n))


def _nnz_prolong(qf: int, qc: int) -> int:
    return sum(((qc if o + 1 <= qf else 2 * qc - 1) - (qc - 1 if o + 1 >= qf else 0)) for o in range(2 * qf - 1))


def _nnz_restrict(qf: int, qc: int) -> int:
    return sum(((qf if o + 1 < qc else 2 * qf - 1) - (qf - 1 if o + 1 > qc else 0)) for o in range(2 * qc - 1))


def laplace_flops(dim: int, nin: int, nout: int, nnz: int) -> int:
    if dim == 3:
        fma = 2 * nnz * nin * nin + 3 * nnz * nout * nin + 2 * nnz * nout * nout
        return 2 * fma + 2 * nout**3
    fma = 2 * nnz * nin + 2 * nnz * nout
    return 2 * fma + 2 * nout**2


def kron_flops(dim: int, nin: int, nout: int, nnz: int) -> int:
    if dim == 3:
        return 2 * nnz * (nin * nin + nout * nin + nout * nout)
    return 2 * nnz * (nin + nout)


def fdm_flops(dim: int, n: int) -> int:
    """Fast diagonalization on an n^dim patch tensor: 2 dim dense n x n contractions (each
    n^(dim+1) multiply-adds) and the eigenvalue scaling."""
    return 2 * dim * 2 * n ** (dim + 1) + 2 * n**dim


def local_solve_flops(dim: int, degrees: list[int], full: bool = False, n_iter: int = 1,
                      smoother: str = "jacobi", direct: bool = False) -> int:
    top = len(degrees) - 1
    if direct:
        return fdm_flops(dim, 2 * degrees[top] - 1)

    def precond(n):  # one Richardson preconditioner application on an n^dim tensor
        return 2 * n**dim if smoother == "jacobi" else fdm_flops(dim, n) + n**dim

    def cycle(l: int) -> int:
        if l == 0:
            return 2
        q, qc = degrees[l], degrees[l - 1]
        n, nc = 2 * q - 1, 2 * qc - 1
        nd = n**dim
        f = precond(n) + laplace_flops(dim, n, n, _nnz_interior(q))
        f += kron_flops(dim, n, nc, _nnz_restrict(q, qc)) + kron_flops(dim, nc, n, _nnz_prolong(q, qc))
        f += cycle(l - 1)
        if full:
            f += laplace_flops(dim, n, n, _nnz_interior(q)) + precond(n) + nd
        return f

    n = 2 * degrees[top] - 1
    one = cycle(top)
    extra = laplace_flops(dim, n, n, _nnz_interior(degrees[top])) + one + n**dim
    return one + (n_iter - 1) * extra


def patch_flops(dim: int, p: int, degrees: list[int], full: bool = False, n_iter: int = 1) -> int:
    """One patch of the smoother kernel: residual, LocalSolve, scatter-add."""
    n = 2 * p - 1
    return laplace_flops(dim, 2 * p + 1, n, _nnz_residual(p)) + local_solve_flops(dim, degrees, full, n_iter) + n**dim


def color_counts(dim: int, n: int, color: int) -> list[int]:
    out = []
    for a in range(dim):
        first = 1 if (color >> a) & 1 else 2
        out.append((n - 1 - first) // 2 + 1 if first <= n - 1 else 0)
    return out


def smooth_launch_bytes(dim: int, n: int, p: int, color: int, word: int = 8) -> int:
    """Unique vector bytes of one color launch: u on the union of the patch closures,
    b on the patch interiors, u written on the patch interiors."""
    cnt = color_counts(dim, n, color)
    closure, interior = 1, 1
    for c in cnt:
        closure *= 2 * p * c + 1 if c else 0
        interior *= c * (2 * p - 1)
    return word * (closure + 2 * interior)


def smooth_launch_patches(dim: int, n: int, color: int) -> int:
    out = 1
    for c in color_counts(dim, n, color):
        out *= c
    return out


def apply_bytes(dim: int, n: int, p: int, word: int = 8) -> int:
    return 2 * word * (p * n + 1) ** dim


def hex_smooth_bytes(dim: int, p: int, degrees: list[int], n_patches: int, word: int = 8, index: int = 4) -> int:
    """Bytes one application of the stored-map smoother moves, summed over its patches
    (patches of one color share no cell, so nothing a launch reads is read twice by it):
    the patch's closure map and cell list, u on the closure, b and u on the interior, u
    written on the interior, and on every p-level the metric of the patch's 2^d cells at
    their Gauss points and the patch's inverse diagonal."""
    comp = 6 if dim == 3 else 3
    N, n = 2 * p + 1, 2 * p - 1
    per = index * (N ** dim + 2 ** dim) + word * (N ** dim + 3 * n ** dim)
    for q in degrees:
        per += word * (2 ** dim * comp * (q + 1) ** dim + (2 * q - 1) ** dim)
    return per * n_patches


def hex_apply_bytes(dim: int, p: int, n_cells: int, n_dofs: int, word: int = 8, index: int = 4) -> int:
    """Bytes of the stored-map apply: the init pass (u read, out written, boundary flag per
    node) and per cell its node map, u on its nodes, out read and written on its nodes
    and the metric at its Gauss points."""
    comp = 6 if dim == 3 else 3
    kd = (p + 1) ** dim
    return n_dofs * (2 * word + 1) + n_cells * (index * kd + 3 * word * kd + word * comp * kd)
