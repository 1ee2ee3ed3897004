"""CPU checks of libpmg.so: it loads, exports every declared symbol, and its host-only
entry points (setup, sizes, index maps, damping, argument checks) agree with the
oracle.  No compute kernel runs here."""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle.mesh import cell_dofs, p_hierarchy, patch_colors, patch_index_sets
from oracle.smoother import default_omega
from paper_2512_02577_amd import pmg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
GOLDEN = os.path.join(ROOT, "tests", "golden")


def _declared(header):
    text = open(os.path.join(ROOT, "include", header)).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pmg_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(pmg.LIB_PATH)
    names = _declared("pmg.h")
    assert len(names) >= 18
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.parametrize("dim,n,p,levels", [(2, 8, 3, [1, 2, 3]), (3, 4, 4, None), (3, 5, 2, None), (2, 6, 7, None),
                                            (3, 3, 8, None)])
def test_maps_bit_exact_against_brute_force(dim, n, p, levels):
    pr = pmg.setup_dofmap(pmg.setup_mesh(dim, n), p, levels)
    for hl in range(pr.n_hlevels):
        nl = pr.cells[hl]
        for pl, q in enumerate(pr.degrees):
            if nl ** dim * (q + 1) ** dim > 3e5:
                continue
            mp = pmg.export_maps(pr, hl, pl)
            np.testing.assert_array_equal(mp["cell_dofs"], cell_dofs(dim, nl, q))
            clo, inn = patch_index_sets(dim, nl, q)
            np.testing.assert_array_equal(mp["patch_interior"], inn)
            np.testing.assert_array_equal(mp["patch_closure"], clo)
            np.testing.assert_array_equal(mp["patch_color"], patch_colors(dim, nl))


def test_sizes_match_paper_tables():
    with open(os.path.join(GOLDEN, "paper_problem_sizes.txt")) as f:
        rows = [list(map(int, l.split())) for l in f if l.strip() and not l.startswith("#")]
    for r, patches, *dofs in rows:
        n = 2 ** (r + 1)
        for p, nd in zip((2, 3, 4, 7), dofs):
            pr = pmg.setup_dofmap(pmg.setup_mesh(3, n), p)
            assert pr.n_nodes[-1] == nd and pr.n_patches[-1] == patches


@pytest.mark.parametrize("p", range(1, 9))
def test_default_hierarchy_and_damping(p):
    for dim in (2, 3):
        if dim == 3 and p > 6:
            continue  # the oracle's dense eigensolve gets slow; p <= 6 covers every level degree
        pr = pmg.setup_dofmap(pmg.setup_mesh(dim, 4), p)
        assert pr.degrees == p_hierarchy(p)
        for q, w in zip(pr.degrees[1:], pr.omega[1:]):
            assert abs(w - default_omega(dim, q)) < 1e-6 * w, (dim, q)


def test_explicit_omega_is_used():
    cfg = pmg.default_config()
    cfg.n_omega = 3
    cfg.omega[1], cfg.omega[2] = 0.61, 0.55
    pr = pmg.setup_dofmap(pmg.setup_mesh(3, 4), 4, None, cfg)
    assert pr.omega[1:] == [0.61, 0.55]


def test_levels_and_errors():
    assert pmg.setup_mesh(3, 48).levels() == [3, 6, 12, 24, 48]
    assert pmg.setup_mesh(2, 8, 2).levels() == [4, 8]
    bad = [lambda: pmg.setup_mesh(4, 8), lambda: pmg.setup_mesh(3, 1), lambda: pmg.setup_mesh(3, 8, 5),
           lambda: pmg.setup_dofmap(pmg.setup_mesh(3, 8), 9),
           lambda: pmg.setup_dofmap(pmg.setup_mesh(3, 8), 4, [1, 4, 3]),
           lambda: pmg.setup_dofmap(pmg.setup_mesh(3, 8), 4, [2, 4])]
    for f in bad:
        with pytest.raises(pmg.PmgError) as e:
            f()
        assert e.value.status == pmg.ERR_INVALID_ARG
    with pytest.raises(pmg.PmgError) as e:
        pmg.setup_dofmap(pmg.setup_mesh(3, 8), 5, [1, 2, 5])  # valid list, not compiled in
    assert e.value.status == pmg.ERR_UNSUPPORTED
    verts = np.zeros((729, 3))
    pmg.setup_mesh(3, 8, 0, verts)  # distorted meshes are accepted (general path)
    verts[5, 1] = np.nan
    with pytest.raises(pmg.PmgError) as e:
        pmg.setup_mesh(3, 8, 0, verts)
    assert e.value.status == pmg.ERR_INVALID_ARG
    cfg = pmg.default_config()
    cfg.rtol = 0.0
    with pytest.raises(pmg.PmgError):
        pmg.setup_dofmap(pmg.setup_mesh(3, 8), 4, None, cfg)


def test_device_calls_before_init_fail_cleanly():
    pr = pmg.setup_dofmap(pmg.setup_mesh(3, 4), 2)
    L = pmg.lib()
    null = ctypes.c_void_p(0)
    assert L.pmg_apply_operator(pr.handle, 0, 0, null, null, null) == pmg.ERR_STATE
    assert L.pmg_smooth(pr.handle, 1, 0, 1, null, null, null) == pmg.ERR_STATE
    assert L.pmg_vcycle(pr.handle, 0, null, null, null) == pmg.ERR_STATE
    info = pmg.SolveInfo()
    assert L.pmg_solve(pr.handle, 0, null, null, 0, ctypes.byref(info), null) == pmg.ERR_STATE
    assert "pmg_device_init" in pmg.last_error()


def test_batch_rejects_problems_without_device_state():
    L = pmg.lib()
    pr = pmg.setup_dofmap(pmg.setup_mesh(3, 4), 2)
    out = ctypes.c_void_p()
    arr = (ctypes.c_void_p * 1)(pr.handle.value)
    assert L.pmg_batch_create(arr, 1, None, ctypes.byref(out)) == pmg.ERR_INVALID_ARG
    assert "pmg_device_init" in pmg.last_error()
    assert L.pmg_batch_create(arr, 0, None, ctypes.byref(out)) == pmg.ERR_INVALID_ARG
    arr17 = (ctypes.c_void_p * 17)(*([pr.handle.value] * 17))
    assert L.pmg_batch_create(arr17, 17, None, ctypes.byref(out)) == pmg.ERR_INVALID_ARG
    assert L.pmg_batch_create(None, 1, None, ctypes.byref(out)) == pmg.ERR_INVALID_ARG
    assert L.pmg_batch_solve(None, pmg.FP32, None, None, None, None) == pmg.ERR_INVALID_ARG
    assert L.pmg_batch_vcycle(None, pmg.FP32, None, None, None) == pmg.ERR_INVALID_ARG
    assert L.pmg_batch_stats(None, pmg.FP32, None, None) == pmg.ERR_INVALID_ARG
    L.pmg_destroy_batch(None)


def test_cell_counts_per_direction_and_lane_option():
    assert pmg.setup_mesh(3, (8, 8, 8)).levels() == [2, 4, 8]
    assert pmg.setup_mesh(2, (6, 6)).levels() == [3, 6]
    with pytest.raises(pmg.PmgError) as e:
        pmg.setup_mesh(3, (8, 8, 4))  # the kernels index cubic node grids only
    assert e.value.status == pmg.ERR_UNSUPPORTED
    with pytest.raises(pmg.PmgError) as e:
        pmg.setup_mesh(3, (8, 1, 8))
    assert e.value.status == pmg.ERR_INVALID_ARG
    assert pmg.lib().pmg_setup_mesh(3, None, 0, None, ctypes.byref(ctypes.c_void_p())) == pmg.ERR_INVALID_ARG
    for lanes in (pmg.LANES_AUTO, pmg.LANES_NARROW, pmg.LANES_WIDE, pmg.LANES_HALF):
        cfg = pmg.default_config()
        cfg.patch_lanes = lanes
        pmg.setup_dofmap(pmg.setup_mesh(3, 4), 4, None, cfg)
    cfg.patch_lanes = 4
    with pytest.raises(pmg.PmgError) as e:
        pmg.setup_dofmap(pmg.setup_mesh(3, 4), 4, None, cfg)
    assert e.value.status == pmg.ERR_INVALID_ARG
