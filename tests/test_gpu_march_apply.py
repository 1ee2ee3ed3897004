"""GPU parity of the 3D operator apply that marches in z (degrees 1-8), and of the mass
matrix apply (b = M f), against the oracle.

Element by element against the assembled oracle matrix on meshes that leave partial xy
tiles, tiles ending exactly at the upper face (the extra boundary row and column), several z
segments and a last segment shorter than the others; at the full benchmark sizes, sampled
rows against the oracle's row-by-row apply (apply_rows), with rows picked on the planes,
rows and columns where z segments and xy tiles meet.  Tolerances as in test_gpu_parity.py:
FP64 1e-12, FP32 2e-5 (max-norm, relative to the reference)."""
import numpy as np
import pytest
import scipy.sparse as sp

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle.assembly import apply_rows, mass_matrix, stiffness_matrix  # noqa: E402
from oracle.mesh import StructuredMesh, boundary_nodes  # noqa: E402
from paper_2512_02577_amd import pmg  # noqa: E402
from paper_2512_02577_amd.inputs import jittered_vertices, rhs_vector  # noqa: E402

DEV = "cuda:0"
TILE = {1: (16, 16), 2: (8, 8), 3: (5, 5), 4: (4, 3), 5: (3, 3), 6: (2, 2), 7: (2, 2), 8: (2, 2)}  # xy tile cells
BLOCKS = 4096                            # workgroups it aims for


def dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device=DEV)


def host(t):
    torch.cuda.synchronize()
    return t.detach().to("cpu", torch.float64).numpy()


def relerr(x, ref):
    return float(abs(x - ref).max() / max(abs(ref).max(), 1e-300))


def segments(n, p):
    """Cell layers per z segment of the library's launch (to aim sampled rows at seams)."""
    mxy = -(-n // TILE[p][0]) * -(-n // TILE[p][1])
    s = min(max(-(-BLOCKS // mxy), 1), n)
    return -(-n // s)


@pytest.mark.parametrize("n,p", [(17, 1), (33, 1), (9, 2), (16, 2), (11, 3), (10, 3), (5, 4), (9, 4), (8, 4),
                                 (4, 5), (7, 5), (6, 5), (5, 6), (4, 6), (3, 7), (4, 7), (3, 8), (4, 8)])
def test_apply_residual_elementwise(n, p):
    print(f"case march apply n {n} p {p}", flush=True)
    pr = pmg.make_problem(3, n, p)
    A = stiffness_matrix(StructuredMesh(3, n), p)
    u = np.random.default_rng(21).uniform(-1, 1, A.shape[0])
    b = rhs_vector(3, n, p, 22)
    ref = A @ u
    ud, bd = dev(u), dev(b)
    v, r = torch.empty_like(ud), torch.empty_like(ud)
    pmg.apply_operator(pr, pr.finest, ud, v)
    pmg.residual(pr, pr.finest, bd, ud, r)
    assert relerr(host(v), ref) <= 1e-12
    assert relerr(host(r), b - ref) <= 1e-12
    v32, r32 = torch.empty(len(u), dtype=torch.float32, device=DEV), torch.empty(len(u), dtype=torch.float32, device=DEV)
    pmg.apply_operator(pr, pr.finest, dev(u, torch.float32), v32)
    pmg.residual(pr, pr.finest, dev(b, torch.float32), dev(u, torch.float32), r32)
    assert relerr(host(v32), ref) <= 2e-5
    assert relerr(host(r32), b - ref) <= 2e-5


def seam_rows(n, p, rng, count):
    m = p * n + 1
    zc = segments(n, p)
    planes = sorted({min(max(p * zc * k + d, 0), m - 1) for k in range(n // zc + 1) for d in (-1, 0, 1)})
    lines = [sorted({min(max(p * t * k + d, 0), m - 1) for k in range(n // t + 1) for d in (-1, 0, 1)}) for t in TILE[p]]
    z = rng.choice(planes, count)
    y = np.where(rng.random(count) < 0.5, rng.choice(lines[1], count), rng.integers(0, m, count))
    x = np.where(rng.random(count) < 0.5, rng.choice(lines[0], count), rng.integers(0, m, count))
    return np.unique(x + m * (y + m * z))


@pytest.mark.parametrize("n,p", [(64, 4), (128, 2), (48, 5), (40, 6), (33, 7), (32, 8)])
def test_full_size_sampled_rows(n, p):
    # 64^3 Q4 is the benchmark's workload; the library's own launch geometry (z segments of
    # a few layers) is exercised at its real size
    print(f"case march apply full size n {n} p {p}", flush=True)
    N = (p * n + 1) ** 3
    rng = np.random.default_rng(n + p)
    u = rng.uniform(-1, 1, N)
    b = rng.uniform(-1, 1, N)
    rows = np.concatenate([seam_rows(n, p, rng, 250), rng.choice(N, 150, replace=False)])
    mesh = StructuredMesh(3, n)
    ref = apply_rows(mesh, p, u, rows)
    pr = pmg.make_problem(3, n, p)
    ud = dev(u)
    v = torch.empty_like(ud)
    pmg.apply_operator(pr, pr.finest, ud, v)
    assert relerr(host(v)[rows], ref) <= 1e-12
    pmg.residual(pr, pr.finest, dev(b), ud, v)
    assert relerr(host(v)[rows], b[rows] - ref) <= 1e-12
    u32 = ud.float()
    v32 = torch.empty_like(u32)
    pmg.apply_operator(pr, pr.finest, u32, v32)
    assert relerr(host(v32)[rows], ref) <= 2e-5


@pytest.mark.parametrize("dim,n,p", [(3, 5, 4), (3, 9, 2), (3, 4, 6), (3, 3, 8), (2, 7, 3), (2, 4, 7)])
def test_mass_operator(dim, n, p):
    # b = M f for a nodal source f (zero on the boundary): the consistent mass matrix of the
    # oracle's quadrature with the Dirichlet rows and columns removed
    print(f"case mass operator dim {dim} n {n} p {p}", flush=True)
    mesh = StructuredMesh(dim, n)
    keep = sp.diags((~boundary_nodes(dim, n, p)).astype(np.float64))
    Mm = (keep @ mass_matrix(mesh, p) @ keep).tocsr()
    u = np.random.default_rng(31).uniform(-1, 1, Mm.shape[0])
    ref = Mm @ u
    pr = pmg.make_problem(dim, n, p)
    v = torch.empty(len(u), dtype=torch.float64, device=DEV)
    pmg.mass_operator(pr, pr.finest, dev(u), v)
    assert relerr(host(v), ref) <= 1e-12
    v32 = torch.empty(len(u), dtype=torch.float32, device=DEV)
    pmg.mass_operator(pr, pr.finest, dev(u, torch.float32), v32)
    assert relerr(host(v32), ref) <= 2e-5
    f = rhs_vector(dim, n, p, 32)
    pmg.mass_operator(pr, pr.finest, dev(f), v)
    assert relerr(host(v), Mm @ f) <= 1e-12


def test_mass_operator_rejects_the_general_path():
    pr = pmg.make_problem(3, 4, 3, vertices=jittered_vertices(3, 4, 0.1, 1))
    u = torch.zeros(pr.n_nodes[-1], dtype=torch.float64, device=DEV)
    with pytest.raises(pmg.PmgError) as e:
        pmg.mass_operator(pr, pr.finest, u, torch.empty_like(u))
    assert e.value.status == pmg.ERR_UNSUPPORTED
