"""GPU parity of the batched entry points (pmg_batch_*): a batch of problems of mixed mesh
size and degree against the single-problem entry points on the same problems (which
test_gpu_parity.py holds to the oracle) and, for the small members, against the FP64
oracle directly.

Tolerances: the batch runs the same kernel bodies with the same tables as the single
problem calls, so its FP64 V-cycle agrees with pmg_vcycle to rounding (1e-12) and with
the oracle as the single-problem V-cycle does (1e-11); FP32 V-cycles agree with
pmg_vcycle in FP32 to 1e-5 and with the oracle to 2e-4.  Solves: relative residual
<= rtol, the true residual within 2x of it, iteration counts within one of the single
problem solve (the dot-product reduction trees differ)."""
import json
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle.mesh import p_hierarchy  # noqa: E402
from oracle.solver import MultigridProblem  # noqa: E402
from paper_2512_02577_amd import pmg  # noqa: E402
from paper_2512_02577_amd.inputs import jittered_vertices, rhs_vector  # noqa: E402

DEV = "cuda:0"

# (n, p): every register class of degrees, h-depths 0 to 2, coarse meshes of 2 and 3 cells
SMALL = [(4, 2), (6, 3), (4, 4), (4, 5), (4, 6), (4, 7), (8, 1), (3, 2)]
ORACLE_CHECKED = {(4, 2), (6, 3), (4, 4), (8, 1), (3, 2)}

# the 16-problem batched workload: 3D, Cartesian, seeds 500 + k
C5 = [(16, 2), (24, 3), (32, 4), (48, 5), (16, 6), (24, 7), (32, 2), (48, 3), (16, 4), (24, 5), (32, 6), (48, 7),
      (16, 7), (24, 6), (32, 5), (48, 4)]


def dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device=DEV)


def host(t):
    torch.cuda.synchronize()
    return t.detach().to("cpu", torch.float64).numpy()


def relerr(x, ref):
    return float(abs(x - ref).max() / max(abs(ref).max(), 1e-300))


def fixed_omega(L):
    return [1.0] + [0.55 + 0.05 * l for l in range(1, L)]


def make(n, p, rtol=1e-8, fixed=True):
    cfg = pmg.default_config()
    cfg.rtol = rtol
    if fixed:
        om = fixed_omega(len(p_hierarchy(p)))
        cfg.n_omega = len(om)
        for i, w in enumerate(om):
            cfg.omega[i] = w
    return pmg.make_problem(3, n, p, config=cfg)


@pytest.fixture(scope="module")
def small():
    probs = [make(n, p) for n, p in SMALL]
    return probs, pmg.batch_create(probs)


def test_batch_vcycle_matches_single_problem_and_oracle(small):
    probs, bt = small
    rs = [dev(rhs_vector(3, n, p, 40 + k)) for k, (n, p) in enumerate(SMALL)]
    for prec, tol_single, tol_oracle in ((pmg.FP64, 1e-12, 1e-11), (pmg.FP32, 1e-5, 2e-4)):
        zs = [torch.empty_like(r) for r in rs]
        pmg.batch_vcycle(bt, rs, zs, prec)
        for k, ((n, p), pr) in enumerate(zip(SMALL, probs)):
            zref = torch.empty_like(rs[k])
            pmg.vcycle(pr, rs[k], zref, prec)
            zb = host(zs[k])
            assert relerr(zb, host(zref)) <= tol_single, (prec, n, p)
            if (n, p) in ORACLE_CHECKED:
                pb = MultigridProblem(3, n, p, omega=fixed_omega(len(p_hierarchy(p))))
                assert relerr(zb, pb.vcycle(host(rs[k]))) <= tol_oracle, (prec, n, p)


def test_batch_vcycle_deterministic(small):
    probs, bt = small
    rs = [dev(rhs_vector(3, n, p, 7 + k)) for k, (n, p) in enumerate(SMALL)]
    z1 = [torch.empty_like(r) for r in rs]
    z2 = [torch.empty_like(r) for r in rs]
    pmg.batch_vcycle(bt, rs, z1, pmg.FP32)
    pmg.batch_vcycle(bt, rs, z2, pmg.FP32)
    torch.cuda.synchronize()
    assert all(torch.equal(a, b) for a, b in zip(z1, z2))


def test_batch_solve_matches_single_problem(small):
    probs, bt = small
    bs = [dev(rhs_vector(3, n, p, 60 + k)) for k, (n, p) in enumerate(SMALL)]
    for prec in (pmg.FP64, pmg.FP32):
        xs = [torch.empty_like(b) for b in bs]
        infos = pmg.batch_solve(bt, bs, xs, prec)
        for k, ((n, p), pr) in enumerate(zip(SMALL, probs)):
            x1 = torch.empty_like(bs[k])
            ref = pmg.solve(pr, bs[k], x1, prec)
            assert infos[k].status == pmg.OK and infos[k].rel_residual <= 1e-8, (prec, n, p)
            assert abs(infos[k].iterations - ref.iterations) <= 1, (prec, n, p, infos[k].iterations, ref.iterations)
            r = torch.empty_like(bs[k])
            pmg.residual(pr, pr.finest, bs[k], xs[k], r)
            true_rel = float(torch.linalg.norm(r) / torch.linalg.norm(bs[k]))
            assert true_rel <= 2e-8, (prec, n, p, true_rel)
            xb, xr = host(xs[k]), host(x1)
            assert np.linalg.norm(xb - xr) / np.linalg.norm(xr) <= 1e-6
            if (n, p) in ORACLE_CHECKED and prec == pmg.FP64:
                pb = MultigridProblem(3, n, p, omega=fixed_omega(len(p_hierarchy(p))))
                bh = host(bs[k])
                assert np.linalg.norm(bh - pb.A[-1] @ xb) / np.linalg.norm(bh) <= 2e-8


def test_batch_per_problem_tolerances_and_zero_rhs():
    spec = [(4, 3, 1e-4), (4, 3, 1e-8), (6, 2, 1e-11), (4, 4, 1e-8)]
    probs = [make(n, p, rtol) for n, p, rtol in spec]
    bt = pmg.batch_create(probs)
    bs = [dev(rhs_vector(3, n, p, 80 + k)) for k, (n, p, _) in enumerate(spec)]
    bs[3].zero_()
    xs = [torch.full_like(b, 7.0) for b in bs]
    infos = pmg.batch_solve(bt, bs, xs, pmg.FP32)
    for k, ((n, p, rtol), pr) in enumerate(zip(spec, probs)):
        x1 = torch.empty_like(bs[k])
        ref = pmg.solve(pr, bs[k], x1, pmg.FP32)
        assert infos[k].rel_residual <= rtol and abs(infos[k].iterations - ref.iterations) <= 1
    assert infos[3].iterations == 0 and not torch.any(xs[3] != 0)
    assert infos[0].iterations < infos[1].iterations  # same problem, looser tolerance


def test_batch_not_converged_status():
    cfg = pmg.default_config()
    cfg.max_iter, cfg.rtol = 2, 1e-14
    probs = [pmg.make_problem(3, 4, 2, config=cfg), make(4, 3)]
    bt = pmg.batch_create(probs)
    bs = [dev(rhs_vector(3, 4, 2, 1)), dev(rhs_vector(3, 4, 3, 2))]
    xs = [torch.empty_like(b) for b in bs]
    infos = pmg.batch_solve(bt, bs, xs, pmg.FP32, raise_on_failure=False)
    assert infos[0].status == pmg.ERR_NOT_CONVERGED and infos[0].iterations == 2
    assert infos[1].status == pmg.OK and infos[1].rel_residual <= 1e-8
    with pytest.raises(pmg.PmgError) as e:
        pmg.batch_solve(bt, bs, xs, pmg.FP32)
    assert e.value.status == pmg.ERR_NOT_CONVERGED


def test_batch_stats_and_rejections():
    probs = [make(4, 2), make(4, 5), make(4, 7)]
    bt = pmg.batch_create(probs)
    stages, launches = pmg.batch_stats(bt, pmg.FP32)
    # one launch per degree in every sweep and residual stage: more launches than stages
    assert launches > stages > 0
    one = pmg.batch_create([make(4, 3), make(6, 3)])
    s1, l1 = pmg.batch_stats(one, pmg.FP64)
    assert s1 == l1
    # FP64 p=8: the patch arena of one Richardson step fits the LDS, that of two does not
    b8 = dev(rhs_vector(3, 2, 8, 3))
    x8 = torch.empty_like(b8)
    p8 = pmg.batch_create([make(2, 8)])
    assert pmg.batch_solve(p8, [b8], [x8], pmg.FP64)[0].rel_residual <= 1e-8
    cfg = pmg.default_config()
    cfg.n_local_iter = 2
    p8two = pmg.batch_create([pmg.make_problem(3, 2, 8, config=cfg)])
    with pytest.raises(pmg.PmgError) as e:
        pmg.batch_stats(p8two, pmg.FP64)
    assert e.value.status == pmg.ERR_UNSUPPORTED
    assert pmg.batch_solve(p8two, [b8], [x8], pmg.FP32)[0].rel_residual <= 1e-8
    for bad, code in (([pmg.make_problem(2, 8, 3)], pmg.ERR_UNSUPPORTED),
                      ([pmg.make_problem(3, 4, 3, vertices=jittered_vertices(3, 4, 0.1, 1))], pmg.ERR_UNSUPPORTED),
                      ([pmg.make_problem(3, 4, 3, p_levels=[1, 2, 3])], pmg.ERR_UNSUPPORTED),
                      ([probs[0], probs[0]], pmg.ERR_INVALID_ARG)):
        with pytest.raises(pmg.PmgError) as e:
            pmg.batch_create(bad)
        assert e.value.status == code


def test_tuning_cache_written_and_reused(tmp_path):
    path = str(tmp_path / "tune.json")
    probs = [make(6, 2), make(4, 5), make(4, 3)]
    bt = pmg.batch_create(probs, path)
    assert not os.path.exists(path)  # measured at the first use of a precision
    bs = [dev(rhs_vector(3, pr.cells[-1], pr.p, 9 + k)) for k, pr in enumerate(probs)]
    x1 = [torch.empty_like(b) for b in bs]
    i1 = pmg.batch_solve(bt, bs, x1, pmg.FP32)
    data = json.load(open(path))
    keys = set(data)
    assert any(k.endswith("fp32/smooth_wpc/p2") for k in keys) and any("fp64-outer/apply_wpc/p5" in k for k in keys)
    assert any(k.endswith("fp32/apply_tile/p5") for k in keys) and any(k.endswith("fp32/lane_items") for k in keys)
    assert not any("/fp64/" in k for k in keys)
    assert all(v in (0, 1, 2, 4, 8, 16) for v in data.values())
    before = os.stat(path).st_mtime_ns
    bt2 = pmg.batch_create(probs, path)
    x2 = [torch.empty_like(b) for b in bs]
    i2 = pmg.batch_solve(bt2, bs, x2, pmg.FP32)
    assert os.stat(path).st_mtime_ns == before
    assert [i.iterations for i in i1] == [i.iterations for i in i2]
    assert all(i.rel_residual <= 1e-8 for i in i1 + i2)
    z = [torch.empty_like(b) for b in bs]
    pmg.batch_vcycle(bt2, bs, z, pmg.FP64)
    torch.cuda.synchronize()
    assert any("/fp64/" in k for k in json.load(open(path)))


def test_full_size_16_problem_batch():
    # 16 Cartesian 3D problems, meshes 16^3..48^3, degrees 2..7 (88,993,752 DoFs in all)
    probs = [pmg.make_problem(3, n, p) for n, p in C5]
    assert sum(pr.n_nodes[-1] for pr in probs) == 88993752
    bt = pmg.batch_create(probs)
    bs = [dev(rhs_vector(3, n, p, 500 + k)) for k, (n, p) in enumerate(C5)]
    xs = [torch.empty_like(b) for b in bs]
    infos = pmg.batch_solve(bt, bs, xs, pmg.FP32)
    for k, ((n, p), pr) in enumerate(zip(C5, probs)):
        assert infos[k].status == pmg.OK and infos[k].rel_residual <= 1e-8 and infos[k].iterations <= 20, (n, p)
        r = torch.empty_like(bs[k])
        pmg.residual(pr, pr.finest, bs[k], xs[k], r)
        assert float(torch.linalg.norm(r) / torch.linalg.norm(bs[k])) <= 2e-8, (n, p)
        x1 = torch.empty_like(bs[k])
        ref = pmg.solve(pr, bs[k], x1, pmg.FP32)
        assert abs(ref.iterations - infos[k].iterations) <= 1, (n, p, ref.iterations, infos[k].iterations)
