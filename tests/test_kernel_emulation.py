"""The HIP kernels' bodies executed on the CPU against the oracle, with an exactly sized
arena, either on one thread per workgroup or on one host thread per lane at the lane
counts of the library's launches (a barrier for every workgroup barrier, the workgroup
sum over the lanes).  This pins the index arithmetic, LDS layouts, 1D tables and the
lane-count dependent paths (split stages, strided per-lane reads and read-ahead registers)
of every kernel family before any GPU run; the GPU parity tests then check the same
bodies on gfx950.

Lane codes: 0 one lane, 1 the library's lane count of that body, 2 the 256-lane latency
variant of the patch smoother."""
import ctypes
import os

import numpy as np
import pytest

import scipy.sparse as sp

from oracle.assembly import mass_matrix, stiffness_matrix
from oracle.mesh import StructuredMesh, boundary_nodes, p_hierarchy
from oracle.smoother import LevelSmoother
from oracle.solver import MultigridProblem
from oracle.transfer import h_prolongation
from paper_2512_02577_amd.inputs import rhs_vector

EMU = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2512_02577_amd",
                   "libpmg_hostemu.so")
DP = ctypes.POINTER(ctypes.c_double)


@pytest.fixture(scope="module")
def emu():
    if not os.path.exists(EMU):
        pytest.fail("libpmg_hostemu.so is not built (python -m paper_2512_02577_amd.build)")
    return ctypes.CDLL(EMU)


def P(a):
    return a.ctypes.data_as(DP)


def ci(a):
    return (ctypes.c_int * len(a))(*a)


def cd(a):
    return (ctypes.c_double * len(a))(*a)


@pytest.mark.parametrize("lanes", [0, 1])
@pytest.mark.parametrize("dim,n,p", [(2, 4, 1), (2, 5, 2), (2, 5, 3), (2, 3, 7), (2, 3, 8), (3, 3, 1), (3, 5, 2),
                                     (3, 4, 3), (3, 3, 4), (3, 5, 4), (3, 6, 4), (3, 3, 5), (3, 4, 5), (3, 2, 6), (3, 2, 7),
                                     (3, 2, 8), (3, 17, 1), (3, 9, 2)])
def test_apply_residual_and_mass(emu, dim, n, p, lanes):
    if p == 8 and lanes == 0:
        pytest.skip("degree 8 runs at the library's lane count only (the one-lane emulation takes seconds)")
    # the 3D degrees 1-5 run the marching apply; n = 17 (p = 1) and 9 (p = 2) leave a partial
    # xy tile, n = 5 (p = 4) one at the upper end with the extra boundary row; zsplit 1 walks
    # every layer in one workgroup, 0 takes the library's z segments
    mesh = StructuredMesh(dim, n)
    A = stiffness_matrix(mesh, p)
    bnd = boundary_nodes(dim, n, p)
    keep = sp.diags((~bnd).astype(np.float64))
    Mm = (keep @ mass_matrix(mesh, p) @ keep).tocsr()
    u = np.random.default_rng(1).uniform(-1, 1, A.shape[0])
    b = rhs_vector(dim, n, p, 2)
    ref = A @ u
    s = abs(ref).max()
    for zsplit in (0, 1):
        v, r, w = np.zeros_like(u), np.zeros_like(u), np.zeros_like(u)
        assert emu.pmgemu_apply(dim, n, p, 0, P(u), P(b), P(v), lanes, zsplit) == 0
        assert emu.pmgemu_apply(dim, n, p, 1, P(u), P(b), P(r), lanes, zsplit) == 0
        assert emu.pmgemu_apply(dim, n, p, 2, P(u), P(b), P(w), lanes, zsplit) == 0
        assert abs(v - ref).max() <= 1e-13 * s
        assert abs(r - (b - ref)).max() <= 1e-13 * s
        mref = Mm @ u
        assert abs(w - mref).max() <= 1e-13 * abs(mref).max()


CASES = [(2, 4, 2, None, "half"), (2, 5, 3, [1, 2, 3], "half"), (2, 4, 3, None, "full"), (3, 3, 2, None, "half"),
         (3, 4, 4, None, "half"), (3, 3, 4, None, "full"), (3, 3, 4, [1, 2, 3, 4], "half"), (2, 4, 7, None, "half"),
         (2, 3, 8, None, "full"), (3, 2, 1, None, "half"), (3, 2, 5, None, "half")]


@pytest.mark.parametrize("dim,n,p,lv,local", CASES)
def test_smoother(emu, dim, n, p, lv, local):
    deg = lv or p_hierarchy(p)
    om = [1.0] + [0.5 + 0.05 * l for l in range(1, len(deg))]
    ls = LevelSmoother(StructuredMesh(dim, n), deg, omega=om, local=local)
    b = rhs_vector(dim, n, p, 3)
    u0 = np.random.default_rng(4).uniform(-1, 1, len(b))
    for it in (1, 2):
        ls.n_local_iter = it
        for direction in (1, -1):
            ref = ls.smooth(u0, b, descending=direction < 0)
            u = u0.copy()
            assert emu.pmgemu_smooth(dim, n, p, ci(deg), len(deg), cd(om), int(local == "full"), 0, it,
                                     direction, P(u), P(b), 0, 0, 0) == 0
            assert abs(u - ref).max() <= 1e-12 * abs(ref).max()


# (dim, n, p, levels): the library's lane counts for every degree; n chosen so that each
# color has several patches
LANE_CASES = [(2, 4, 2, None), (2, 3, 3, [1, 2, 3]), (2, 3, 7, None), (3, 3, 1, None), (3, 4, 2, None),
              (3, 3, 3, None), (3, 3, 4, None), (3, 3, 4, [1, 2, 3, 4]), (3, 2, 5, None), (3, 2, 6, None),
              (3, 2, 7, None), (3, 2, 8, None)]


@pytest.mark.parametrize("dim,n,p,lv", LANE_CASES)
def test_smoother_lane_teams(emu, dim, n, p, lv):
    # the default local solver in its own compiled variant (one = 1) and the general variant,
    # at the library's narrow lane count and at 256 lanes, on both table layouts
    deg = lv or p_hierarchy(p)
    om = [1.0] + [0.5 + 0.05 * l for l in range(1, len(deg))]
    ls = LevelSmoother(StructuredMesh(dim, n), deg, omega=om, local="half")
    b = rhs_vector(dim, n, p, 3)
    u0 = np.random.default_rng(4).uniform(-1, 1, len(b))
    for direction in (1, -1):
        ref = ls.smooth(u0, b, descending=direction < 0)
        # 3D degrees 4 and 5 also on half the lanes (the kernel of large launches, default solver)
        wave = ((3, 1, 1),) if dim == 3 and p in (4, 5) else ()
        for lanes, one, tabmode in ((1, 1, 1), (2, 1, 0), (1, 0, 0), (2, 0, 1)) + wave:
            u = u0.copy()
            assert emu.pmgemu_smooth(dim, n, p, ci(deg), len(deg), cd(om), 0, 0, 1, direction, P(u), P(b), lanes,
                                     one, tabmode) == 0
            assert abs(u - ref).max() <= 1e-12 * abs(ref).max(), (lanes, one, tabmode, direction)


@pytest.mark.parametrize("dim,n,p", [(3, 3, 4), (2, 4, 3), (3, 2, 5)])
def test_smoother_lane_teams_full_and_richardson(emu, dim, n, p):
    deg = p_hierarchy(p)
    om = [1.0] + [0.5 + 0.05 * l for l in range(1, len(deg))]
    b = rhs_vector(dim, n, p, 5)
    u0 = np.random.default_rng(6).uniform(-1, 1, len(b))
    for local, it in (("full", 1), ("half", 2), ("full", 2)):
        ls = LevelSmoother(StructuredMesh(dim, n), deg, omega=om, local=local, n_local_iter=it)
        ref = ls.smooth(u0, b)
        for lanes in (1, 2):
            u = u0.copy()
            assert emu.pmgemu_smooth(dim, n, p, ci(deg), len(deg), cd(om), int(local == "full"), 0, it, 1, P(u),
                                     P(b), lanes, 0, 1) == 0
            assert abs(u - ref).max() <= 1e-12 * abs(ref).max(), (local, it, lanes)


def test_one_variant_rejects_other_solvers(emu):
    deg = p_hierarchy(4)
    om = [1.0, 0.6, 0.6]
    b = rhs_vector(3, 2, 4, 1)
    u = np.zeros_like(b)
    assert emu.pmgemu_smooth(3, 2, 4, ci(deg), 3, cd(om), 1, 0, 1, 1, P(u), P(b), 1, 1, 0) == -3
    assert emu.pmgemu_smooth(3, 2, 4, ci(deg), 3, cd(om), 0, 1, 1, 1, P(u), P(b), 1, 1, 0) == -3


# exact patch solve (fast diagonalization) and the Cartesian-reinforced p-level smoother
FDM_CASES = [(2, 4, 3, None), (2, 3, 7, None), (3, 3, 2, None), (3, 3, 4, None), (3, 3, 4, [1, 2, 3, 4]),
             (3, 2, 5, None), (3, 2, 8, None)]


@pytest.mark.parametrize("dim,n,p,lv", FDM_CASES)
def test_direct_and_reinforced_smoother(emu, dim, n, p, lv):
    deg = lv or p_hierarchy(p)
    b = rhs_vector(dim, n, p, 7)
    u0 = np.random.default_rng(8).uniform(-1, 1, len(b))
    om_r = [1.0] + [0.8 + 0.05 * l for l in range(1, len(deg))]
    cases = [("direct", "jacobi", [1.0] * len(deg), 2, 0, 1),
             ("half", "reinforced", om_r, 0, 1, 1), ("full", "reinforced", om_r, 1, 1, 1),
             ("half", "reinforced", om_r, 0, 1, 2)]
    for local, sm, om, code, reinf, it in cases if p < 8 else cases[:2]:  # degree 8: the oracle takes ~20 s a case
        ls = LevelSmoother(StructuredMesh(dim, n), deg, omega=om, local=local, smoother=sm, n_local_iter=it)
        # degree 8: the library's lane count only (each oracle sweep there takes seconds)
        for direction, lanes in ((1, 1), (-1, 2), (1, 0)) if p < 8 else ((1, 1),):
            ref = ls.smooth(u0, b, descending=direction < 0)
            u = u0.copy()
            assert emu.pmgemu_smooth(dim, n, p, ci(deg), len(deg), cd(om), code, reinf, it, direction, P(u), P(b),
                                     lanes, 0, lanes % 2) == 0
            assert abs(u - ref).max() <= 1e-12 * abs(ref).max(), (local, sm, it, lanes)


@pytest.mark.parametrize("dim,p", [(3, 4), (2, 7)])
def test_direct_and_reinforced_local_solve(emu, dim, p):
    deg = p_hierarchy(p)
    om = [1.0] + [0.9] * (len(deg) - 1)
    r = None
    for local, sm, code, reinf in (("direct", "jacobi", 2, 0), ("half", "reinforced", 0, 1),
                                   ("full", "reinforced", 1, 1)):
        ls = LevelSmoother(StructuredMesh(dim, 3), deg, omega=om, local=local, smoother=sm)
        nb, nd = ls.interior[-1].shape
        if r is None:
            r = np.random.default_rng(1).uniform(-1, 1, nb * nd)
        d = np.zeros_like(r)
        assert emu.pmgemu_local_solve(dim, 3, p, ci(deg), len(deg), cd(om), code, reinf, 1, nb, P(r), P(d), 1,
                                      1) == 0
        for j in range(nb):
            ref = ls.local_solve(j, r[j * nd:(j + 1) * nd])
            assert abs(d[j * nd:(j + 1) * nd] - ref).max() <= 1e-12 * abs(ref).max(), (local, sm)


@pytest.mark.parametrize("dim,p", [(2, 3), (3, 4), (3, 2)])
def test_local_solve(emu, dim, p):
    deg = p_hierarchy(p)
    om = [1.0] + [0.6] * (len(deg) - 1)
    ls = LevelSmoother(StructuredMesh(dim, 3), deg, omega=om, local="half")
    nb = ls.interior[-1].shape[0]
    nd = ls.interior[-1].shape[1]
    r = np.random.default_rng(0).uniform(-1, 1, nb * nd)
    d = np.zeros_like(r)
    for lanes in (0, 1):
        d[:] = 0
        assert emu.pmgemu_local_solve(dim, 3, p, ci(deg), len(deg), cd(om), 0, 0, 1, nb, P(r), P(d), lanes,
                                      lanes) == 0
        for j in range(nb):
            ref = ls.local_solve(j, r[j * nd:(j + 1) * nd])
            assert abs(d[j * nd:(j + 1) * nd] - ref).max() <= 1e-13 * abs(ref).max()


@pytest.mark.parametrize("dim,nc,p", [(2, 2, 1), (2, 3, 3), (3, 2, 2), (3, 2, 4), (2, 2, 8), (3, 3, 1), (3, 2, 7)])
def test_h_transfers(emu, dim, nc, p):
    Ph = h_prolongation(dim, nc, p)
    rng = np.random.default_rng(5)
    fine = rng.uniform(-1, 1, Ph.shape[0])
    coarse = rng.uniform(-1, 1, Ph.shape[1])
    outc = np.zeros(Ph.shape[1])
    assert emu.pmgemu_transfer(dim, nc, p, 1, P(fine), P(outc)) == 0
    outf = fine.copy()
    assert emu.pmgemu_transfer(dim, nc, p, 0, P(coarse), P(outf)) == 0
    assert abs(outc - Ph.T @ fine).max() <= 1e-13 * abs(outc).max()
    assert abs(outf - (fine + Ph @ coarse)).max() <= 1e-13 * abs(outf).max()


@pytest.mark.parametrize("dim,n0,p", [(2, 2, 3), (3, 2, 4), (3, 3, 2), (2, 3, 8), (3, 2, 1)])
def test_coarse_solve(emu, dim, n0, p):
    pb = MultigridProblem(dim, n0, p)
    r = np.random.default_rng(7).uniform(-1, 1, pb.N)
    ref = pb.coarse_solve(r)
    for lanes in (0, 1):
        z = np.zeros_like(r)
        assert emu.pmgemu_coarse_solve(dim, n0, p, P(r), P(z), lanes) == 0
        assert abs(z - ref).max() <= 1e-12 * abs(ref).max()


# ---- general path: distorted cells and a variable coefficient -------------------------
from oracle.assembly import quadrature_points  # noqa: E402
from paper_2512_02577_amd.inputs import CoefficientField, jittered_vertices  # noqa: E402

GENERAL = [(2, 3, 2, 0.15, True), (2, 4, 4, 0.2, True), (2, 3, 7, 0.1, False), (3, 2, 2, 0.1, False),
           (3, 3, 3, 0.1, True), (3, 2, 4, 0.1, True), (3, 2, 6, 0.1, True)]


def _general_setup(dim, n, p, jit, use_coef):
    verts = jittered_vertices(dim, n, jit, 3) if jit else None
    field = CoefficientField(dim, 5) if use_coef else None
    mesh = StructuredMesh(dim, n, verts)
    V = np.ascontiguousarray(verts) if verts is not None else None
    return mesh, field, V


def _coef(mesh, field, q):
    if field is None:
        return None
    return np.ascontiguousarray(field(quadrature_points(mesh, q).reshape(-1, mesh.dim)))


@pytest.mark.parametrize("dim,n,p,jit,use_coef", GENERAL)
def test_general_apply(emu, dim, n, p, jit, use_coef):
    mesh, field, V = _general_setup(dim, n, p, jit, use_coef)
    A = stiffness_matrix(mesh, p, field)
    u = np.random.default_rng(1).uniform(-1, 1, A.shape[0])
    b = rhs_vector(dim, n, p, 2)
    c = _coef(mesh, field, p)
    for resid, lanes in ((0, 0), (1, 0), (0, 1), (1, 1)):
        out = np.zeros_like(u)
        assert emu.pmgemu_metric_apply(dim, n, p, P(V) if V is not None else None, P(c) if c is not None else None,
                                       resid, P(u), P(b), P(out), lanes) == 0
        ref = b - A @ u if resid else A @ u
        assert abs(out - ref).max() <= 1e-13 * abs(ref).max()


@pytest.mark.parametrize("dim,n,p,jit,use_coef", GENERAL)
def test_general_smoother_and_local_solve(emu, dim, n, p, jit, use_coef):
    mesh, field, V = _general_setup(dim, n, p, jit, use_coef)
    deg = p_hierarchy(p)
    om = [1.0] + [0.62] * (len(deg) - 1)
    coefs = [_coef(mesh, field, q) for q in deg]
    carr = (DP * len(deg))(*[P(x) if x is not None else None for x in coefs])
    b = rhs_vector(dim, n, p, 3)
    u0 = np.random.default_rng(4).uniform(-1, 1, len(b))
    for local, it, direction, lanes, one in (("half", 1, 1, 0, 0), ("full", 2, -1, 0, 0), ("half", 1, -1, 1, 1),
                                             ("full", 2, 1, 1, 0)):
        ls = LevelSmoother(mesh, deg, omega=om, coef=field, local=local, n_local_iter=it)
        u = u0.copy()
        assert emu.pmgemu_metric_smooth(dim, n, p, ci(deg), len(deg), cd(om), int(local == "full"), it, direction,
                                        P(V) if V is not None else None, carr, P(u), P(b), 0, None, None, lanes,
                                        one) == 0
        ref = ls.smooth(u0, b, descending=direction < 0)
        assert abs(u - ref).max() <= 1e-12 * abs(ref).max(), (local, lanes, one)
    ls = LevelSmoother(mesh, deg, omega=om, coef=field, local="half")
    nb, nd = ls.interior[-1].shape
    r = np.random.default_rng(0).uniform(-1, 1, nb * nd)
    d = np.zeros_like(r)
    assert emu.pmgemu_metric_smooth(dim, n, p, ci(deg), len(deg), cd(om), 0, 1, 1, P(V) if V is not None else None,
                                    carr, None, None, nb, P(r), P(d), 1, 0) == 0
    for j in range(nb):
        ref = ls.local_solve(j, r[j * nd:(j + 1) * nd])
        assert abs(d[j * nd:(j + 1) * nd] - ref).max() <= 1e-12 * abs(ref).max()


# ---- general hex meshes: the stored-map bodies against the hex-mesh oracle ----
I32 = ctypes.POINTER(ctypes.c_int32)


def _hex_args(h):
    v = np.ascontiguousarray(h["vertices"], dtype=np.float64)
    cv = np.ascontiguousarray(h["cell_vertices"], dtype=np.int32)
    cdofs = np.ascontiguousarray(h["cell_dofs"], dtype=np.int32)
    return v, cv, cdofs


@pytest.mark.parametrize("lanes", [0, 1])
@pytest.mark.parametrize("dim,n,p,shape", [(2, 6, 3, "L"), (2, 8, 2, "hole"), (2, 4, 7, "L"), (3, 4, 2, "L"),
                                           (3, 4, 3, "box"), (3, 4, 4, "L"), (3, 2, 6, "box")])
def test_hex_apply_and_smoother(emu, dim, n, p, shape, lanes):
    if p == 6 and lanes == 0:
        pytest.skip("degree 6 runs at the library's lane count only (the oracle sweep takes seconds)")
    from oracle.hexmesh import HexLevelSmoother, HexMesh
    from paper_2512_02577_amd.inputs import hex_mesh

    emu.pmgemu_hex_apply.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_long, DP, ctypes.c_long, I32, ctypes.c_long,
                                     I32, ctypes.c_int, DP, DP, DP, ctypes.c_int]
    emu.pmgemu_hex_smooth.argtypes = [ctypes.c_int, ctypes.c_int, DP, ctypes.c_long, DP, ctypes.c_long, I32,
                                      ctypes.c_long, I32, ctypes.c_int, ctypes.c_int, ctypes.c_int, DP, DP,
                                      ctypes.c_int, ctypes.c_int]
    h = hex_mesh(dim, n, p, 3, shape=shape, distortion=0.3)
    v, cv, cdofs = _hex_args(h)
    nd = h["n_dofs"]
    hm = HexMesh(dim, v, cv, p, cdofs, nd)
    rng = np.random.default_rng(2)
    u, b = rng.uniform(-1, 1, nd), rng.uniform(-1, 1, nd)
    ref = b - hm.stiffness() @ u
    out = np.zeros(nd)
    assert emu.pmgemu_hex_apply(dim, p, len(v), P(v), len(cv), cv.ctypes.data_as(I32), nd,
                                cdofs.ctypes.data_as(I32), 1, P(u), P(b), P(out), lanes) == 0
    assert abs(out - ref).max() <= 1e-13 * abs(ref).max()
    if p == 8:
        return  # the oracle's degree-8 patch smoother is minutes of CPU time
    hs = HexLevelSmoother(hm, p_hierarchy(p))
    om = np.ascontiguousarray(hs.omega, dtype=np.float64)
    for direction, one in ((1, 1), (-1, 0)):
        ue = u.copy()
        assert emu.pmgemu_hex_smooth(dim, p, P(om), len(v), P(v), len(cv), cv.ctypes.data_as(I32), nd,
                                     cdofs.ctypes.data_as(I32), 0, 1, direction, P(ue), P(b), lanes, one) == 0
        uo = hs.smooth(u, b, descending=direction < 0)
        assert abs(ue - uo).max() <= 1e-13 * abs(uo).max()
