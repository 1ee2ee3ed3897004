"""GPU parity of every compiled width of the Cartesian patch smoother against the oracle
(Alg. 1 with the local p-multigrid of Alg. 2/3), and the errors of FP32 multigrid against
the FP64 oracle per degree.

A color launch runs the per-degree lane count (64 lanes for p <= 3, 128 for p = 4, 256
or 512 above) or the 256-lane latency variant, each either in the variant compiled for the
default local solver (one half V-cycle, one Richardson step) or in the general one; 3D
degree-4 and degree-5 FP32 colors of at least 64 patches per CU run the default solver on
half the per-degree lanes (the configuration can force that kernel in both precisions).
Large problems take the per-degree width (or the half-lane kernel), small ones the latency
variant; the configuration fixes one of them here so that small meshes the oracle finishes
in seconds reach each, and one natural case has more than 1,024 patches per color (the
per-degree width at full size).  At 64^3 Q4 and Q5 the half-lane kernel that the
benchmark's finest levels run in FP32 is compared with the per-degree width on the same
inputs.

Tolerances as in test_gpu_parity.py: FP64 smoother / V-cycle 1e-11, FP32 2e-4 (max-norm
relative to the oracle's result).
"""
import json
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle.mesh import StructuredMesh, p_hierarchy  # noqa: E402
from oracle.smoother import LevelSmoother  # noqa: E402
from oracle.solver import MultigridProblem, solve as oracle_solve  # noqa: E402
from paper_2512_02577_amd import pmg  # noqa: E402
from paper_2512_02577_amd.inputs import rhs_vector  # noqa: E402

DEV = "cuda:0"
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device=DEV)


def host(t):
    torch.cuda.synchronize()
    return t.detach().to("cpu", torch.float64).numpy()


def relerr(x, ref):
    return float(abs(x - ref).max() / max(abs(ref).max(), 1e-300))


def omega_of(L):
    return [1.0] + [0.55 + 0.05 * l for l in range(1, L)]


def make(dim, n, p, lv=None, local="half", n_iter=1, omega=None, lanes=pmg.LANES_AUTO):
    cfg = pmg.default_config()
    cfg.local_solver = pmg.LOCAL_FULL_V if local == "full" else pmg.LOCAL_HALF_V
    cfg.n_local_iter = n_iter
    cfg.patch_lanes = lanes
    if omega is not None:
        cfg.n_omega = len(omega)
        for i, w in enumerate(omega):
            cfg.omega[i] = w
    return pmg.make_problem(dim, n, p, lv, config=cfg)


# (dim, n, p, levels): every degree whose per-degree width is below 256 lanes, in 3D with
# several patches per color, plus the 2D and one-step-hierarchy bodies
WIDTH_CASES = [(3, 5, 1, None), (3, 5, 2, None), (3, 4, 3, None), (3, 4, 4, None), (3, 3, 4, [1, 2, 3, 4]),
               (2, 6, 3, [1, 2, 3]), (2, 7, 4, None)]
SOLVERS = [("half", 1), ("full", 1), ("half", 2)]  # the first is the default solver's own variant


# the half-lane kernel exists for 3D degrees 4 and 5 (elsewhere LANES_HALF is the per-degree count)
WIDTH_PARAMS = [(c, lanes) for c in WIDTH_CASES for lanes in (pmg.LANES_NARROW, pmg.LANES_WIDE)] + \
    [(c, pmg.LANES_HALF) for c in WIDTH_CASES if c[0] == 3 and c[2] == 4]


@pytest.mark.parametrize("case,lanes", WIDTH_PARAMS)
def test_smoother_widths_fp64(case, lanes):
    dim, n, p, lv = case
    print(f"case smoother widths dim {dim} n {n} p {p} levels {lv} lanes {lanes}", flush=True)
    deg = lv or p_hierarchy(p)
    om = omega_of(len(deg))
    b = rhs_vector(dim, n, p, 41)
    u0 = np.random.default_rng(42).uniform(-1, 1, len(b))
    for local, it in SOLVERS:
        pr = make(dim, n, p, lv, local, it, om, lanes)
        ls = LevelSmoother(StructuredMesh(dim, n), deg, omega=om, local=local, n_local_iter=it)
        for direction in (1, -1):
            ud = dev(u0)
            pmg.smooth(pr, pr.finest, ud, dev(b), direction)
            ref = ls.smooth(u0, b, descending=direction < 0)
            assert relerr(host(ud), ref) <= 1e-11, (local, it, direction)


@pytest.mark.parametrize("dim,n,p,lanes", [(d, n, p, l) for (d, n, p) in [(3, 5, 2), (3, 4, 4), (2, 7, 3)]
                                             for l in (pmg.LANES_NARROW, pmg.LANES_WIDE)] + [(3, 4, 4, pmg.LANES_HALF)])
def test_smoother_widths_fp32(dim, n, p, lanes):
    print(f"case smoother widths fp32 dim {dim} n {n} p {p} lanes {lanes}", flush=True)
    deg = p_hierarchy(p)
    om = omega_of(len(deg))
    pr = make(dim, n, p, omega=om, lanes=lanes)
    ls = LevelSmoother(StructuredMesh(dim, n), deg, omega=om)
    b = rhs_vector(dim, n, p, 43)
    u0 = np.random.default_rng(44).uniform(-1, 1, len(b))
    ud = dev(u0, torch.float32)
    pmg.smooth(pr, pr.finest, ud, dev(b, torch.float32), 1)
    ref = ls.smooth(u0.astype(np.float32).astype(np.float64), b.astype(np.float32).astype(np.float64))
    assert relerr(host(ud), ref) <= 2e-4


def golden(name):
    """Oracle result of a case that takes the oracle minutes, written by
    tests/golden/make_oracle_refs.py (oracle only): sampled values, the max-norm of the full
    result and the damping the oracle used."""
    with np.load(os.path.join(ROOT, "tests", "golden", "oracle_refs", f"{name}.npz")) as z:
        return {k: z[k] for k in z.files}


def sampled_relerr(x, ref):
    return float(abs(x[ref["idx"]] - ref["val"]).max() / float(ref["absmax"]))


@pytest.mark.parametrize("name,p,direction,seeds", [("smooth_3d_n24_p2_asc", 2, 1, (45, 46)),
                                                    ("smooth_3d_n24_p3_desc", 3, -1, (51, 52))])
def test_smoother_natural_full_width_launch(name, p, direction, seeds):
    # 3D, 24^3 cells: 12,167 patches, more than 1,024 per color, so every color runs the
    # per-degree width of the default-solver kernel (64 lanes at Q2, 128 at Q3) that the
    # full-size solves run on their finest levels
    dim, n = 3, 24
    print(f"case natural width {name}", flush=True)
    ref = golden(name)
    pr = make(dim, n, p, omega=list(ref["omega"]))
    smallest_color = min(((n - 1 - f) // 2 + 1) for f in (1, 2)) ** 3
    assert pr.n_patches[-1] == (n - 1) ** 3 and smallest_color > 1024
    b = rhs_vector(dim, n, p, seeds[0])
    u0 = np.random.default_rng(seeds[1]).uniform(-1, 1, len(b))
    ud = dev(u0)
    pmg.smooth(pr, pr.finest, ud, dev(b), direction)
    assert sampled_relerr(host(ud), ref) <= 1e-11


@pytest.mark.parametrize("p", [4, 5])
def test_half_lane_kernel_at_the_benchmark_size(p):
    # 64^3 cells, Q4 / Q5 (17.0M / 33.1M nodes): every color has more than 64 patches per CU, so
    # the default configuration runs the half-lane kernel in FP32 (forced here for FP64 too);
    # the per-degree width (compared with the oracle above, at 24^3 and at Q5 below) on the same
    # inputs must give the same sweep up to the rounding of the coarsest p-level's block sum, in
    # both directions and both precisions
    dim, n = 3, 64
    print(f"case half-lane kernel 64^3 Q{p} against the per-degree width", flush=True)
    half, narrow = make(dim, n, p, lanes=pmg.LANES_HALF), make(dim, n, p, lanes=pmg.LANES_NARROW)
    b = rhs_vector(dim, n, p, 53)
    u0 = np.random.default_rng(54).uniform(-1, 1, len(b))
    for dtype, tol in ((torch.float64, 1e-12), (torch.float32, 1e-5)):
        bd = dev(b, dtype)
        for direction in (1, -1):
            uh, un = dev(u0, dtype), dev(u0, dtype)
            pmg.smooth(half, half.finest, uh, bd, direction)
            pmg.smooth(narrow, narrow.finest, un, bd, direction)
            assert relerr(host(uh), host(un)) <= tol, (dtype, direction)
            assert relerr(host(uh), u0) > 1e-3  # the sweep changed the iterate


@pytest.mark.parametrize("p", [5, 7])
def test_smoother_high_degree_3d(p):
    dim, n = 3, 3
    print(f"case high degree smoother p {p} n {n}", flush=True)
    b = rhs_vector(dim, n, p, 47)
    u0 = np.random.default_rng(48).uniform(-1, 1, len(b))
    for direction, tag in ((1, "asc"), (-1, "desc")):
        ref = golden(f"smooth_3d_n3_p{p}_{tag}")
        for lanes in (pmg.LANES_AUTO, pmg.LANES_NARROW) + ((pmg.LANES_HALF,) if p == 5 else ()):
            pr = make(dim, n, p, omega=list(ref["omega"]), lanes=lanes)
            ud = dev(u0)
            pmg.smooth(pr, pr.finest, ud, dev(b), direction)
            assert sampled_relerr(host(ud), ref) <= 1e-11, (lanes, direction)
            if direction == 1:
                # FP32 against the FP64 oracle on FP64 inputs: rounding of the inputs included
                ud = dev(u0, torch.float32)
                pmg.smooth(pr, pr.finest, ud, dev(b, torch.float32), 1)
                assert sampled_relerr(host(ud), ref) <= 2e-4


@pytest.mark.parametrize("p", [5, 7])
def test_vcycle_high_degree_3d(p):
    dim, n = 3, 4
    print(f"case high degree vcycle p {p} n {n}", flush=True)
    ref = golden(f"vcycle_3d_n4_p{p}")
    r = rhs_vector(dim, n, p, 49)
    for lanes in (pmg.LANES_AUTO, pmg.LANES_NARROW):
        pr = make(dim, n, p, omega=list(ref["omega"]), lanes=lanes)
        z = torch.empty(len(r), dtype=torch.float64, device=DEV)
        pmg.vcycle(pr, dev(r), z)
        assert sampled_relerr(host(z), ref) <= 1e-11
        pmg.vcycle(pr, dev(r), z, pmg.FP32)
        assert sampled_relerr(host(z), ref) <= 2e-4


# FP32 multigrid inside the FP64 flexible CG against the FP64 oracle's solution, per degree
# (reduced sizes): the solution error, and the iteration counts of both multigrid
# precisions against the oracle's.  The oracle solves in seconds up to 3D Q4 here; for 3D
# Q5..Q7 its solution comes sampled from tests/golden/oracle_refs (the error is then the
# relative 2-norm error over the sampled nodes).
ERR_CASES = [(3, 4, p) for p in range(2, 8)] + [(2, 8, p) for p in range(2, 9)]


@pytest.mark.parametrize("dim,n,p", ERR_CASES)
def test_fp32_mg_error_vs_oracle_per_degree(dim, n, p):
    print(f"case fp32-mg error dim {dim} n {n} p {p}", flush=True)
    b = rhs_vector(dim, n, p, 300 + p)
    if dim == 3 and p >= 5:
        ref = golden(f"solve_3d_n4_p{p}")
        idx, x_ref, it_ref, om = ref["idx"], ref["val"], int(ref["iterations"]), list(ref["omega"])
    else:
        pb = MultigridProblem(dim, n, p)
        x_full, it_ref, _ = oracle_solve(pb, b)
        idx, x_ref, om = np.arange(len(b)), x_full, list(pb.levels[-1].omega)
    cfg = pmg.default_config()
    cfg.n_omega = len(om)
    for i, w in enumerate(om):
        cfg.omega[i] = w
    pr = pmg.make_problem(dim, n, p, config=cfg)
    bd = dev(b)
    rec = {"dim": dim, "n": n, "p": p, "n_dofs": len(b), "oracle_iterations": it_ref, "compared_nodes": len(idx)}
    for prec, name in ((pmg.FP64, "fp64_mg"), (pmg.FP32, "fp32_mg")):
        x = torch.empty_like(bd)
        info = pmg.solve(pr, bd, x, prec)
        err = float(np.linalg.norm(host(x)[idx] - x_ref) / np.linalg.norm(x_ref))
        rec[name] = {"iterations": info.iterations, "rel_residual": info.rel_residual, "error_vs_oracle": err}
        assert info.rel_residual <= 1e-8
        assert abs(info.iterations - it_ref) <= 1, (name, info.iterations, it_ref)
        assert err <= 1e-6, (name, err)
    out = os.path.join(ROOT, "gpurun_out")
    if os.path.isdir(out):
        with open(os.path.join(out, "fp32mg_error_per_degree.jsonl"), "a") as f:
            f.write(json.dumps(rec) + "\n")
