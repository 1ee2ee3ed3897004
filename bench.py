#!/usr/bin/env python3
"""Benchmark of the local p-multigrid patch-smoother solver on one MI355X.

Headline workload: 3D Poisson on the unit cube, 64^3 hexahedra, Q4 Gauss-Lobatto elements
(16,974,593 nodes), homogeneous Dirichlet, right-hand side b = M f of a seeded uniform[-1,1]
nodal source f (M the consistent mass matrix, applied on the GPU before the timing; --rhs
nodal takes b = f instead); h-multigrid
V(1,1) (levels 2..64 cells) with the vertex-patch smoother whose local solver is one half
V-cycle over the p-levels 4 -> 3 -> 1, inside flexible CG, all FP64.  This is the largest
single-GPU configuration of the task's list (64^3, degrees 2..8) at the degree of its
roofline target; the other degrees are extra keys.

One step = one solve from x = 0 to |b - A x| <= 1e-8 |b| (apply, smoother color passes
with the fused local p-multigrid, residuals, transfers, coarse solve, dot products: the
whole path).  value = nodes x V-cycles / time (DoF/s per V-cycle).  Beside it:
  * the same solve with FP32 multigrid inside the FP64 CG (time to solution, iterations);
  * per-call rates (apply, one smoother application, one V-cycle) with HIP events on the
    launch stream (mean over back-to-back calls; per call mean and median, with warm caches
    and after a 512 MB flush write), and the roofline of the dominant kernel (the
    finest-level smoother color launch) and of the operator apply;
  * the degree sweep p = 2..8 at 64^3 (FP64-MG and FP32-MG time to 1e-8, iterations);
  * 128^3 Q4 (135M nodes, working set far beyond the 256 MB last-level cache): apply and
    smoother rates;
  * the local solver strategies of the paper's Table 3 (half and full p-V-cycles with Jacobi or
    Cartesian-reinforced smoothing, the exact fast-diagonalization solve), time and FLOPs per
    patch relative to the half V-cycle;
  * the 16-problem batch against the same solves one by one;
  * the CPU oracle on a bounded sample.

    python bench.py [--steps K] [--warmup W] [--no-cpu-baseline] [--no-batch] [--no-sweep]
                    [--rhs mass|nodal] [--extras]   (also the 48^3 Q6 perturbed mesh with a coefficient)
    python bench.py --counters       (short kernel runs for rocprofv3 counter passes)
    python bench.py --table1         (outer iteration counts on the grid of Table 1)
"""
import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0     # MI355X HBM3E
FP64_PEAK_TFLOPS = 78.6   # MI355X FP64 vector
FP32_PEAK_TFLOPS = 157.3

HEADLINE = (3, 64, 4, 2)  # dim, cells per direction, degree, right-hand-side seed


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def time_events(fn, reps, torch):
    """Mean milliseconds per call of fn() between HIP events on the current stream (the
    stream the binding passes to the library)."""
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    fn()
    e0.record(s)
    for _ in range(reps):
        fn()
    e1.record(s)
    e1.synchronize()
    return e0.elapsed_time(e1) / reps


def time_calls(fn, reps, torch, flush=None):
    """Per-call milliseconds of fn() with HIP events around each call on the current stream:
    (mean, median).  With `flush` (a 512 MB device buffer) the buffer is written between the
    calls, outside the timed events, so that every call starts with the last-level cache
    holding none of its data."""
    import statistics

    s = torch.cuda.current_stream()
    fn()
    ts = []
    for _ in range(reps):
        if flush is not None:
            flush.fill_(1.0)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        fn()
        e1.record(s)
        e1.synchronize()
        ts.append(e0.elapsed_time(e1))
    return {"mean_ms": sum(ts) / len(ts), "median_ms": statistics.median(ts)}


def measured_traffic(name):
    """HBM bytes per launch from a committed counter record profiles/<name>.traffic.json,
    or None when it is missing or a kernel source listed there has changed since the
    counters were taken."""
    import hashlib

    path = os.path.join(ROOT, "profiles", name + ".traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    for rel, digest in rec["sources_sha256"].items():
        full = os.path.join(ROOT, rel)
        if not os.path.exists(full):
            return None
        with open(full, "rb") as f:
            if hashlib.sha256(f.read()).hexdigest() != digest:
                return None
    return rec["fetch_bytes_per_launch"] + rec["write_bytes_per_launch"]


def cpu_baseline(dim, n, p, seed, budget_s=12.0):
    """The oracle (NumPy/SciPy, one thread) timed on V-cycles of a reduced mesh."""
    from threadpoolctl import threadpool_limits

    from oracle.solver import MultigridProblem
    from paper_2512_02577_amd.inputs import rhs_vector

    def rate(f, budget, least):
        t0 = time.perf_counter()
        k = 0
        while time.perf_counter() - t0 < budget or k < least:
            f()
            k += 1
        return k, time.perf_counter() - t0

    with threadpool_limits(1):
        pb = MultigridProblem(dim, n, p)
        r = rhs_vector(dim, n, p, seed)
        pb.vcycle(r)  # builds the patch caches (setup)
        k, t = rate(lambda: pb.vcycle(r), budget_s, 3)
        # the assembled operator's CSR apply and one smoother application on the finest level
        fin = len(pb.sizes) - 1
        ka, ta = rate(lambda: pb.A[fin] @ r, 1.0, 3)
        u = 0.0 * r
        ks, ts = rate(lambda: pb.smooth(fin, u, r), 2.0, 1)
    return {"vcycle": (pb.N * k / t, k, t), "apply": (pb.N * ka / ta, ka, ta), "smooth": (pb.N * ks / ts, ks, ts)}


# 16 independent 3D Cartesian problems (n cells per direction, degree p), seeds 500 + k
BATCH = [(16, 2), (24, 3), (32, 4), (48, 5), (16, 6), (24, 7), (32, 2), (48, 3), (16, 4), (24, 5), (32, 6), (48, 7),
         (16, 7), (24, 6), (32, 5), (48, 4)]


# 16 small problems, where the per-launch and per-iteration costs of one-by-one solves dominate
SMALL_BATCH = [(8, 2), (8, 3), (8, 4), (8, 5), (12, 2), (12, 3), (12, 4), (12, 6), (16, 2), (16, 3), (16, 4), (16, 7),
               (6, 5), (6, 6), (6, 7), (4, 8)]


def bench_small_batch(steps, torch, pmg, rhs_vector):
    """16 small 3D problems (4^3..16^3 cells, Q2..Q8), FP32-MG in FP64 CG: batched vs one by one."""
    dev = "cuda:0"
    probs = [pmg.make_problem(3, n, p) for n, p in SMALL_BATCH]
    bs = [torch.as_tensor(rhs_vector(3, n, p, 700 + k), dtype=torch.float64, device=dev)
          for k, (n, p) in enumerate(SMALL_BATCH)]
    xs = [torch.empty_like(b) for b in bs]
    bt = pmg.batch_create(probs, os.path.join(ROOT, "paper_2512_02577_amd", "tuning", "launch_params.json"))
    pmg.batch_solve(bt, bs, xs, pmg.FP32)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        infos = pmg.batch_solve(bt, bs, xs, pmg.FP32)
    torch.cuda.synchronize()
    t_batch = (time.perf_counter() - t0) / steps
    for pr, b, x in zip(probs, bs, xs):
        pmg.solve(pr, b, x, pmg.FP32)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        its1 = [pmg.solve(pr, b, x, pmg.FP32).iterations for pr, b, x in zip(probs, bs, xs)]
    torch.cuda.synchronize()
    t_seq = (time.perf_counter() - t0) / steps
    Ns = [pr.n_nodes[-1] for pr in probs]
    its = [i.iterations for i in infos]
    return {"problems": [f"{n}^3 Q{p}" for n, p in SMALL_BATCH], "n_dofs": sum(Ns),
            "time_to_solution_s": t_batch, "one_by_one_time_s": t_seq, "speedup_vs_one_by_one": t_seq / t_batch,
            "iterations": its, "one_by_one_iterations": its1,
            "value": sum(N * k for N, k in zip(Ns, its)) / t_batch, "unit": "DoF/s per V-cycle",
            "max_rel_residual": max(i.rel_residual for i in infos)}


def bench_batch(steps, torch, pmg, rhs_vector):
    """The 16-problem batch: FP32 multigrid in FP64 flexible CG, all problems in one batch
    (persistent stage launches, graph-captured), against the same 16 solves one by one."""
    dev = "cuda:0"
    probs = [pmg.make_problem(3, n, p) for n, p in BATCH]
    Ns = [pr.n_nodes[-1] for pr in probs]
    bs = [torch.as_tensor(rhs_vector(3, n, p, 500 + k), dtype=torch.float64, device=dev)
          for k, (n, p) in enumerate(BATCH)]
    xs = [torch.empty_like(b) for b in bs]
    cache = os.path.join(ROOT, "paper_2512_02577_amd", "tuning", "launch_params.json")
    os.makedirs(os.path.dirname(cache), exist_ok=True)
    t0 = time.perf_counter()
    bt = pmg.batch_create(probs, cache)
    t_create = time.perf_counter() - t0
    t0 = time.perf_counter()
    pmg.batch_solve(bt, bs, xs, pmg.FP32)  # measures missing launch parameters first
    torch.cuda.synchronize()
    t_first = time.perf_counter() - t0
    t0 = time.perf_counter()
    for _ in range(steps):
        infos = pmg.batch_solve(bt, bs, xs, pmg.FP32)
    torch.cuda.synchronize()
    t_batch = (time.perf_counter() - t0) / steps
    its = [i.iterations for i in infos]
    worst = max(i.rel_residual for i in infos)
    # one batched V-cycle (graph launch; includes copying r in and z out)
    zs = [torch.empty_like(b) for b in bs]
    t_vc = time_events(lambda: pmg.batch_vcycle(bt, bs, zs, pmg.FP32), 5, torch)
    stages, launches = pmg.batch_stats(bt, pmg.FP32)
    # the same solves one problem at a time
    for pr, b, x in zip(probs, bs, xs):
        pmg.solve(pr, b, x, pmg.FP32)
    torch.cuda.synchronize()
    t_vc1 = sum(time_events(lambda: pmg.vcycle(pr, b, z, pmg.FP32), 3, torch) for pr, b, z in zip(probs, bs, zs))
    t0 = time.perf_counter()
    its1 = []
    for _ in range(steps):
        its1 = [pmg.solve(pr, b, x, pmg.FP32).iterations for pr, b, x in zip(probs, bs, xs)]
    torch.cuda.synchronize()
    t_seq = (time.perf_counter() - t0) / steps
    work = sum(N * k for N, k in zip(Ns, its))
    return {"workload": "16 independent 3D Poisson problems, Cartesian, meshes 16^3..48^3, Q2..Q7, "
                        "FP32 h-MG(V(1,1), vertex-patch smoother, local half V-cycle) in FP64 flexible CG to 1e-8",
            "problems": [f"{n}^3 Q{p}" for n, p in BATCH], "n_dofs": sum(Ns),
            "value": work / t_batch, "unit": "DoF/s per V-cycle",
            "time_to_solution_s": t_batch, "iterations": its, "max_rel_residual": worst,
            "vcycle_ms": t_vc, "vcycle_dof_per_s": sum(Ns) / (t_vc * 1e-3),
            "stages_per_vcycle": stages, "launches_per_vcycle": launches,
            "one_by_one_time_s": t_seq, "one_by_one_iterations": its1,
            "one_by_one_dof_per_s_per_vcycle": sum(N * k for N, k in zip(Ns, its1)) / t_seq,
            "one_by_one_vcycle_ms": t_vc1, "vcycle_speedup_vs_one_by_one": t_vc1 / t_vc,
            "speedup_vs_one_by_one": t_seq / t_batch, "create_s": t_create,
            "first_solve_s_incl_tuning": t_first}


def _solve_times(torch, pmg, pr, b, precs, steps, warmup=1):
    """Time-to-solution, iterations and relative residual of each multigrid precision, and
    the relative difference of each solution to the FP64-multigrid one."""
    out, xref = {}, None
    for prec, name in precs:
        x = torch.empty_like(b)
        for _ in range(max(1, warmup)):
            pmg.solve(pr, b, x, prec)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            info = pmg.solve(pr, b, x, prec)
        torch.cuda.synchronize()
        t = (time.perf_counter() - t0) / steps
        N = pr.n_nodes[-1]
        rec = {"time_to_solution_s": t, "iterations": info.iterations, "rel_residual": info.rel_residual,
               "dof_per_s_per_vcycle": N * info.iterations / t}
        if xref is None:
            xref = x
        else:
            rec["solution_rel_diff_vs_fp64_mg"] = float(torch.linalg.vector_norm(x - xref) /
                                                        torch.linalg.vector_norm(xref))
        out[name] = rec
    return out


def make_rhs(torch, pmg, pr, f, mode):
    """The right-hand side on the device: b = M f (mass matrix of the finest level, on the
    GPU) or b = f (nodal mode).  f is zero on the Dirichlet boundary, and so is b."""
    fd = torch.as_tensor(f, dtype=torch.float64, device="cuda:0")
    if mode == "nodal":
        return fd
    b = torch.empty_like(fd)
    pmg.mass_operator(pr, pr.finest, fd, b)
    torch.cuda.synchronize()
    return b


def bench_degree_sweep(torch, pmg, rhs_vector, steps, degrees, rhs="mass"):
    """3D Poisson, 64^3 hexes, p = 2..8 (paper p-hierarchies), seeds 300 + p: FP64 and FP32
    multigrid inside the FP64 flexible CG.  (Cartesian meshes store no operator data, so a
    bfloat16-storage arm would equal FP32 and is not run.)"""
    res = []
    for p in degrees:
        log(f"bench: degree sweep 64^3 Q{p}")
        pr = pmg.make_problem(3, 64, p)
        b = make_rhs(torch, pmg, pr, rhs_vector(3, 64, p, 300 + p), rhs)
        rec = {"degree": p, "n_dofs": pr.n_nodes[-1]}
        rec.update(_solve_times(torch, pmg, pr, b, ((pmg.FP64, "fp64_mg"), (pmg.FP32, "fp32_mg")), steps))
        rec["fp32_mg_speedup"] = rec["fp64_mg"]["time_to_solution_s"] / rec["fp32_mg"]["time_to_solution_s"]
        res.append(rec)
        del pr, b
        torch.cuda.empty_cache()
    return res


def bench_general(torch, pmg, steps):
    """3D variable coefficient on a perturbed mesh: 48^3 hexes, Q6, interior vertices moved
    by 0.1 h, a = exp(seeded smooth field) in [0.1, 10]; FP64, FP32 and FP32 with bfloat16
    operator storage inside the FP64 flexible CG."""
    from paper_2512_02577_amd.inputs import CoefficientField, jittered_vertices, rhs_vector

    log("bench: general path 48^3 Q6 (setup)")
    t0 = time.perf_counter()
    pr = pmg.make_problem(3, 48, 6, vertices=jittered_vertices(3, 48, 0.1, 40), coefficient=CoefficientField(3, 41))
    t_setup = time.perf_counter() - t0
    b = torch.as_tensor(rhs_vector(3, 48, 6, 4), dtype=torch.float64, device="cuda:0")
    log("bench: general path solves")
    rec = {"workload": "3D -div(a grad u) = f, 48^3 perturbed hexes (jitter 0.1 h), Q6, a in [0.1, 10]",
           "n_dofs": pr.n_nodes[-1], "setup_s": t_setup}
    rec.update(_solve_times(torch, pmg, pr, b, ((pmg.FP64, "fp64_mg"), (pmg.FP32, "fp32_mg"),
                                                (pmg.FP32_BF16, "fp32_bf16_mg")), steps))
    del pr, b
    torch.cuda.empty_cache()
    return rec


def bench_hex(torch, pmg, perfmodel, np, reps):
    """General hex mesh with stored maps: a 3D L-shaped domain of 64^3 lattice cells minus a
    quadrant (196,608 hexes, renumbered, rotated and reflected, vertices jittered by 0.3 h,
    nodes numbered with locality as a DoF handler would), Q4; the stored-map apply and one smoother application (DSATUR colors) in FP64 and FP32,
    beside the same kernels with computed indices on the 64^3 distorted box."""
    from paper_2512_02577_amd.inputs import hex_mesh, jittered_vertices

    log("bench: general hex mesh 3D L 64^3 Q4 (mesh and setup)")
    t0 = time.perf_counter()
    h = hex_mesh(3, 64, 4, 50, shape="L", distortion=0.3, renumber_nodes=False)
    t_mesh = time.perf_counter() - t0
    t0 = time.perf_counter()
    hp = pmg.setup_hex(3, 4, h["vertices"], h["cell_vertices"], h["cell_dofs"], h["n_dofs"])
    t_host = time.perf_counter() - t0
    t0 = time.perf_counter()
    pmg.hex_device_init(hp)
    torch.cuda.synchronize()
    t_dev = time.perf_counter() - t0
    nd = h["n_dofs"]
    rng = np.random.default_rng(51)
    rec = {"workload": "3D Poisson on an L-shaped general hex mesh (64^3 lattice minus a quadrant, cells and vertices "
                       "renumbered at random, cells rotated and reflected, nodes in lattice order, vertices jittered "
                       "0.3 h), Q4, stored maps, DSATUR colors",
           "n_cells": hp.n_cells, "n_dofs": nd, "n_patches": hp.n_patches, "patch_colors": hp.n_patch_colors,
           "cell_colors": hp.n_cell_colors, "mesh_s": t_mesh, "host_setup_s": t_host, "device_init_s": t_dev,
           "ms": {}, "dof_per_s": {}, "frac_hbm": {}}
    bytes_sm = perfmodel.hex_smooth_bytes(3, 4, hp.degrees, hp.n_patches)
    bytes_ap = perfmodel.hex_apply_bytes(3, 4, hp.n_cells, nd)
    rec["bytes_per_application"] = {"smooth_fp64": bytes_sm, "apply_fp64": bytes_ap}
    for dt, tag in ((torch.float64, "fp64"), (torch.float32, "fp32")):
        u = torch.as_tensor(rng.uniform(-1, 1, nd), dtype=dt, device="cuda:0")
        b = torch.as_tensor(rng.uniform(-1, 1, nd), dtype=dt, device="cuda:0")
        v = torch.empty_like(u)
        ms_ap = time_events(lambda: pmg.hex_apply(hp, u, v), reps, torch)
        ms_sm = time_events(lambda: pmg.hex_smooth(hp, u, b, 1), max(2, reps // 4), torch)
        rec["ms"]["apply_" + tag], rec["ms"]["smooth_" + tag] = ms_ap, ms_sm
        rec["dof_per_s"]["apply_" + tag], rec["dof_per_s"]["smooth_" + tag] = nd / ms_ap * 1e3, nd / ms_sm * 1e3
        if tag == "fp64":
            rec["frac_hbm"]["apply_fp64"] = bytes_ap / (ms_ap * 1e-3) / 1e9 / HBM_PEAK_GBS
            rec["frac_hbm"]["smooth_fp64"] = bytes_sm / (ms_sm * 1e-3) / 1e9 / HBM_PEAK_GBS
        del u, b, v
    del hp, h
    torch.cuda.empty_cache()
    log("bench: the same kernels with computed indices on the 64^3 distorted box")
    pr = pmg.make_problem(3, 64, 4, vertices=jittered_vertices(3, 64, 0.3, 52))
    N = pr.n_nodes[-1]
    box = {"n_dofs": N, "ms": {}, "dof_per_s": {}}
    u = torch.as_tensor(rng.uniform(-1, 1, N), dtype=torch.float64, device="cuda:0")
    b = torch.as_tensor(rng.uniform(-1, 1, N), dtype=torch.float64, device="cuda:0")
    v = torch.empty_like(u)
    box["ms"]["apply_fp64"] = time_events(lambda: pmg.apply_operator(pr, pr.finest, u, v), reps, torch)
    box["ms"]["smooth_fp64"] = time_events(lambda: pmg.smooth(pr, pr.finest, u, b), max(2, reps // 4), torch)
    for k, ms in box["ms"].items():
        box["dof_per_s"][k] = N / ms * 1e3
    rec["distorted_box_computed_indices"] = box
    del pr, u, b, v
    torch.cuda.empty_cache()
    return rec


# Table 3's local solver strategies (Sec. 4.3), timed per patch in FP64
LOCAL_SOLVERS = [("half V-cycle (Jacobi)", 0, 0, False, "jacobi"), ("V-cycle (Jacobi)", 1, 0, True, "jacobi"),
                 ("half V-cycle (Cartesian-reinforced)", 0, 1, False, "reinforced"),
                 ("V-cycle (Cartesian-reinforced)", 1, 1, True, "reinforced"),
                 ("fast diagonalization (exact)", 2, 0, False, "jacobi")]
# the paper's relative times and FLOPs (normalized by the patch operator, p = 7, one CPU core)
PAPER_TABLE3 = {"half V-cycle (Jacobi)": (2.01, 1.17), "V-cycle (Jacobi)": (3.39, 2.27),
                "half V-cycle (Cartesian-reinforced)": (4.67, 1.87), "V-cycle (Cartesian-reinforced)": (8.68, 3.67),
                "fast diagonalization (exact)": (2.60, 0.68)}


def bench_local_solvers(torch, pmg, perfmodel, np, reps):
    """LocalSolve alone (pmg_local_solve) on every patch of the finest level of a 32^3 mesh,
    FP64, for each local solver strategy of Table 3: time and counted FLOPs relative to the
    half V-cycle with Jacobi smoothing (the paper's Table 3 divided by its half V-cycle row
    beside them)."""
    out = []
    for p in (4, 7):
        n = 32
        log(f"bench: local solvers 32^3 Q{p}")
        deg = None
        recs = []
        for name, loc, sm, full, smn in LOCAL_SOLVERS:
            cfg = pmg.default_config()
            cfg.local_solver, cfg.local_smoother = loc, sm
            pr = pmg.make_problem(3, n, p, config=cfg)
            deg = pr.degrees
            nb = pr.n_patches[-1]
            nd = (2 * p - 1) ** 3
            r = torch.as_tensor(np.random.default_rng(5).uniform(-1, 1, nb * nd), dtype=torch.float64, device="cuda:0")
            d = torch.empty_like(r)
            t = time_events(lambda: pmg.local_solve(pr, pr.finest, r, d), reps, torch)
            fl = perfmodel.local_solve_flops(3, deg, full=full, smoother=smn, direct=loc == 2) * nb
            recs.append({"solver": name, "ms": t, "gflops": fl / (t * 1e-3) / 1e9, "flops_per_patch": fl // nb})
            del pr, r, d
            torch.cuda.empty_cache()
        base_t, base_f = recs[0]["ms"], recs[0]["flops_per_patch"]
        pt = PAPER_TABLE3["half V-cycle (Jacobi)"]
        for rc in recs:
            rc["relative_time"] = rc["ms"] / base_t
            rc["relative_flops"] = rc["flops_per_patch"] / base_f
            paper = PAPER_TABLE3[rc["solver"]]
            rc["paper_p7_relative_time"] = paper[0] / pt[0]
            rc["paper_p7_relative_flops"] = paper[1] / pt[1]
        out.append({"degree": p, "patches": (n - 1) ** 3, "degrees": deg, "solvers": recs})
    return out


def bench_table1(torch, pmg):
    """Outer FCG iterations (FP64 multigrid) on the grid of Table 1: local solvers
    {1 V-cycle, 1 half V-cycle, 2 half V-cycles, 25 V-cycles} x interior-vertex distortion x
    p in {3, 7}, 2D 32^2 and 3D 16^3 cells (the paper's sizes are not given)."""
    from paper_2512_02577_amd.inputs import jittered_vertices, rhs_vector

    variants = [("1 V-cycle", pmg.LOCAL_FULL_V, 1), ("1 half V-cycle", pmg.LOCAL_HALF_V, 1),
                ("2 half V-cycles", pmg.LOCAL_HALF_V, 2), ("25 V-cycles", pmg.LOCAL_FULL_V, 25)]
    out = []
    for dim, n, deltas in ((2, 32, (0.0, 0.10, 0.25, 0.35)), (3, 16, (0.0, 0.10, 0.25, 0.30))):
        for p in (3, 7):
            for delta in deltas:
                log(f"bench: table 1 grid {dim}D {n} cells Q{p} distortion {delta}")
                verts = jittered_vertices(dim, n, delta, 91) if delta > 0 else None
                b = torch.as_tensor(rhs_vector(dim, n, p, 90), dtype=torch.float64, device="cuda:0")
                rec = {"dim": dim, "n": n, "p": p, "delta": delta}
                for name, loc, it in variants:
                    cfg = pmg.default_config()
                    cfg.local_solver, cfg.n_local_iter = loc, it
                    pr = pmg.make_problem(dim, n, p, config=cfg, vertices=verts)
                    x = torch.empty_like(b)
                    info = pmg.solve(pr, b, x, pmg.FP64)
                    rec[name] = info.iterations
                    del pr, x
                out.append(rec)
                torch.cuda.empty_cache()
    return out


def kernel_rates(torch, pmg, perfmodel, np, pr, dim, n, p, reps):
    """Per-call rates on the finest level (HIP events on the launch stream) and the roofline
    numbers of the smoother color launch and of the apply."""
    dev = "cuda:0"
    N = pr.n_nodes[-1]
    L = pr.finest
    u = torch.as_tensor(np.random.default_rng(3).uniform(-1, 1, N), dtype=torch.float64, device=dev)
    b = torch.as_tensor(np.random.default_rng(4).uniform(-1, 1, N), dtype=torch.float64, device=dev)
    v = torch.empty_like(u)
    t_apply = time_events(lambda: pmg.apply_operator(pr, L, u, v), reps, torch)
    u_s = u.clone()
    t_smooth = time_events(lambda: pmg.smooth(pr, L, u_s, b, 1), reps, torch)
    u32, b32 = u.float(), b.float()
    t_smooth32 = time_events(lambda: pmg.smooth(pr, L, u32, b32, 1), reps, torch)
    v32 = torch.empty_like(u32)
    t_apply32 = time_events(lambda: pmg.apply_operator(pr, L, u32, v32), reps, torch)
    ncol = 2 ** dim
    bytes_launches = sum(perfmodel.smooth_launch_bytes(dim, n, p, c) for c in range(ncol))
    patches = sum(perfmodel.smooth_launch_patches(dim, n, c) for c in range(ncol))
    flops = patches * perfmodel.patch_flops(dim, p, pr.degrees)
    t_launch = t_smooth / ncol * 1e-3
    rec = {"n_dofs": N, "ms": {"apply_fp64": t_apply, "smooth_fp64": t_smooth, "smooth_fp32": t_smooth32,
                               "apply_fp32": t_apply32},
           "dof_per_s": {"apply_fp64": N / (t_apply * 1e-3), "smooth_fp64": N / (t_smooth * 1e-3),
                         "smooth_fp32": N / (t_smooth32 * 1e-3), "apply_fp32": N / (t_apply32 * 1e-3)},
           "smooth_over_apply": t_smooth / t_apply}
    smooth = {"avg_launch_us": t_launch * 1e6, "bytes_per_launch": bytes_launches // ncol,
              "flops_per_launch": flops // ncol, "flop_per_byte": flops / bytes_launches,
              "achieved_gbs": bytes_launches / ncol / t_launch / 1e9,
              "achieved_tflops": flops / ncol / t_launch / 1e12,
              "fp32_avg_launch_us": t_smooth32 / ncol * 1e3,
              "fp32_achieved_gbs": bytes_launches / 2 / ncol / (t_smooth32 / ncol * 1e-3) / 1e9}
    # per-call statistics, with the caches warm and after a 512 MB flush write
    flush = torch.empty(2 ** 26, dtype=torch.float64, device=dev)
    z = torch.empty_like(u)
    rec["per_call"] = {}
    for name, fn in (("apply_fp64", lambda: pmg.apply_operator(pr, L, u, v)),
                     ("smooth_fp64", lambda: pmg.smooth(pr, L, u_s, b, 1)),
                     ("vcycle_fp64", lambda: pmg.vcycle(pr, b, z, pmg.FP64))):
        warm, cold = time_calls(fn, 10, torch), time_calls(fn, 10, torch, flush)
        rec["per_call"][name] = {**warm, "flushed_mean_ms": cold["mean_ms"], "flushed_median_ms": cold["median_ms"]}
    del flush, z
    apply_bytes = perfmodel.apply_bytes(dim, n, p)
    apply = {"avg_launch_us": t_apply * 1e3, "bytes_per_launch": apply_bytes,
             "achieved_gbs": apply_bytes / (t_apply * 1e-3) / 1e9,
             "fp32_avg_launch_us": t_apply32 * 1e3,
             "fp32_achieved_gbs": apply_bytes / 2 / (t_apply32 * 1e-3) / 1e9}
    return rec, smooth, apply


def counters_mode(torch, pmg, np):
    """Short runs of the kernels whose HBM traffic is recorded under profiles/, for
    `rocprofv3 --pmc FETCH_SIZE` and `--pmc WRITE_SIZE` passes: a plain device copy of
    1 GiB (the calibration: 1 GiB read and 1 GiB written per dispatch), then at 64^3 and
    128^3 Q4 two FP64 smoother applications (8 color launches each) and three applies, and
    at 64^3 Q8 three applies."""
    dev = "cuda:0"
    x = torch.empty(2 ** 27, dtype=torch.float64, device=dev).uniform_(-1, 1)
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    del x, y
    torch.cuda.empty_cache()
    for n, p in ((64, 4), (128, 4), (64, 8)):
        log(f"bench: counter runs at {n}^3 Q{p}")
        pr = pmg.make_problem(3, n, p)
        N = pr.n_nodes[-1]
        u = torch.as_tensor(np.random.default_rng(3).uniform(-1, 1, N), dtype=torch.float64, device=dev)
        b = torch.as_tensor(np.random.default_rng(4).uniform(-1, 1, N), dtype=torch.float64, device=dev)
        v = torch.empty_like(u)
        for _ in range(2 if p == 4 else 0):
            pmg.smooth(pr, pr.finest, u, b, 1)
        for _ in range(3):
            pmg.apply_operator(pr, pr.finest, u, v)
        torch.cuda.synchronize()
        del pr, u, b, v
        torch.cuda.empty_cache()
    print(json.dumps({"counters": "done"}), flush=True)
    return 0


def hex_counters_mode(torch, pmg, np):
    """Short runs of the general hex-mesh kernels for rocprofv3 passes: the 1 GiB device
    copy (calibration), then on the 3D L of 64^3 lattice cells Q4 (as in bench_hex) one FP64
    smoother application (one launch per DSATUR color) and three FP64 applies."""
    from paper_2512_02577_amd.inputs import hex_mesh

    dev = "cuda:0"
    x = torch.empty(2 ** 27, dtype=torch.float64, device=dev).uniform_(-1, 1)
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    del x, y
    torch.cuda.empty_cache()
    log("bench: hex counter runs (3D L 64^3 Q4)")
    h = hex_mesh(3, 64, 4, 50, shape="L", distortion=0.3, renumber_nodes=False)
    hp = pmg.setup_hex(3, 4, h["vertices"], h["cell_vertices"], h["cell_dofs"], h["n_dofs"])
    pmg.hex_device_init(hp)
    nd = h["n_dofs"]
    u = torch.as_tensor(np.random.default_rng(3).uniform(-1, 1, nd), dtype=torch.float64, device=dev)
    b = torch.as_tensor(np.random.default_rng(4).uniform(-1, 1, nd), dtype=torch.float64, device=dev)
    v = torch.empty_like(u)
    pmg.hex_smooth(hp, u, b, 1)
    for _ in range(3):
        pmg.hex_apply(hp, u, v)
    torch.cuda.synchronize()
    print(json.dumps({"hex_counters": "done", "patch_colors": hp.n_patch_colors, "cell_colors": hp.n_cell_colors}),
          flush=True)
    return 0


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--kernel-reps", type=int, default=20)
    ap.add_argument("--no-batch", action="store_true", help="leave out the 16-problem batch measurement")
    ap.add_argument("--no-sweep", action="store_true", help="leave out the degree sweep and the 128^3 rates")
    ap.add_argument("--no-hex", action="store_true", help="leave out the general hex-mesh measurement")
    ap.add_argument("--hex-only", action="store_true", help="only the general hex-mesh measurement")
    ap.add_argument("--hex-counters", action="store_true", help="short hex-mesh kernel runs for rocprofv3 passes")
    ap.add_argument("--extras", action="store_true", help="also the 48^3 Q6 perturbed-mesh problem")
    ap.add_argument("--counters", action="store_true", help="short kernel runs for rocprofv3 counter passes")
    ap.add_argument("--table1", action="store_true", help="only the Table 1 iteration-count grid (minutes)")
    ap.add_argument("--rhs", choices=("mass", "nodal"), default="mass",
                    help="b = M f (default) or b = f, f seeded uniform[-1,1] nodal values, zero on the boundary")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    from paper_2512_02577_amd import perfmodel, pmg
    from paper_2512_02577_amd.inputs import rhs_vector

    torch.cuda.set_device(0)
    if args.counters:
        return counters_mode(torch, pmg, np)
    if args.hex_counters:
        return hex_counters_mode(torch, pmg, np)
    if args.table1:
        print(json.dumps({"table1_fcg_iterations": bench_table1(torch, pmg)}), flush=True)
        return 0
    if args.hex_only:
        print(json.dumps({"hex_general": bench_hex(torch, pmg, perfmodel, np, max(4, args.kernel_reps // 2))}),
              flush=True)
        return 0
    dim, n, p, seed = HEADLINE
    dev = "cuda:0"
    log(f"bench: setup 3D n={n} Q{p}")
    t0 = time.perf_counter()
    pr = pmg.make_problem(dim, n, p)
    t_setup = time.perf_counter() - t0
    N = pr.n_nodes[-1]
    b = make_rhs(torch, pmg, pr, rhs_vector(dim, n, p, seed), args.rhs)
    x = torch.empty_like(b)

    def run_solves(prec, k):
        its = []
        for _ in range(k):
            info = pmg.solve(pr, b, x, prec)
            its.append(info.iterations)
        return its

    log("bench: warmup")
    run_solves(pmg.FP64, args.warmup)
    torch.cuda.synchronize()
    log(f"bench: timing {args.steps} FP64 solves")
    t0 = time.perf_counter()
    its = run_solves(pmg.FP64, args.steps)
    torch.cuda.synchronize()
    t64 = time.perf_counter() - t0
    relres64 = pmg.solve(pr, b, x, pmg.FP64).rel_residual
    x64 = x.clone()

    log("bench: FP32-MG solves")
    run_solves(pmg.FP32, args.warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    its32 = run_solves(pmg.FP32, args.steps)
    torch.cuda.synchronize()
    t32 = time.perf_counter() - t0
    info32 = pmg.solve(pr, b, x, pmg.FP32)
    diff32 = float(torch.linalg.vector_norm(x - x64) / torch.linalg.vector_norm(x64))
    del x64

    log("bench: per-call timings")
    reps = args.kernel_reps
    z = torch.empty_like(b)
    t_vc = time_events(lambda: pmg.vcycle(pr, b, z, pmg.FP64), max(5, reps // 4), torch)
    t_vc32 = time_events(lambda: pmg.vcycle(pr, b, z, pmg.FP32), max(5, reps // 4), torch)
    rates, sm, ap_ = kernel_rates(torch, pmg, perfmodel, np, pr, dim, n, p, reps)
    rates["ms"].update({"vcycle_fp64": t_vc, "vcycle_fp32": t_vc32})
    rates["dof_per_s"].update({"vcycle_fp64": N / (t_vc * 1e-3), "vcycle_fp32": N / (t_vc32 * 1e-3)})

    ridge = FP64_PEAK_TFLOPS * 1e12 / (HBM_PEAK_GBS * 1e9)
    if sm["flop_per_byte"] < ridge:
        roof = {"bound": "hbm", "achieved": round(sm["achieved_gbs"], 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(sm["achieved_gbs"] / HBM_PEAK_GBS, 4)}
    else:
        roof = {"bound": "alu", "achieved": round(sm["achieved_tflops"], 2), "peak": FP64_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": round(sm["achieved_tflops"] / FP64_PEAK_TFLOPS, 4)}
    # the library's choice for these launches: FP32 colors of 3D Q4 with at least 64 patches per
    # CU run one wave per patch (half the per-degree lanes), FP64 colors two
    ncu = torch.cuda.get_device_properties(0).multi_processor_count
    smallest_color = min((n - 1 - f) // 2 + 1 for f in (1, 2)) ** dim
    wave32 = dim == 3 and p == 4 and smallest_color >= 64 * ncu
    roof.update({"traffic": measured_traffic("k_smooth_fp64_q4_64cube"),
                 "kernel": f"k_smooth<3,double,4,{{1,3,4}},ONE> (finest level {n}^3, one color launch)",
                 "fp32_kernel": ("k_smooth_h<3,float,4,{1,3,4},64> (one wave per patch)" if wave32
                                 else "k_smooth<3,float,4,{1,3,4},ONE>"),
                 "avg_launch_us": round(sm["avg_launch_us"], 2), "bytes_per_launch": sm["bytes_per_launch"],
                 "flops_per_launch": sm["flops_per_launch"], "flop_per_byte": round(sm["flop_per_byte"], 2),
                 "achieved_tflops": round(sm["achieved_tflops"], 3), "achieved_gbs": round(sm["achieved_gbs"], 1),
                 "frac_fp64_valu": round(sm["achieved_tflops"] / FP64_PEAK_TFLOPS, 4),
                 "fp32_avg_launch_us": round(sm["fp32_avg_launch_us"], 2),
                 "fp32_frac_hbm": round(sm["fp32_achieved_gbs"] / HBM_PEAK_GBS, 4)})
    roof_apply = {"bound": "hbm", "achieved": round(ap_["achieved_gbs"], 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                  "frac": round(ap_["achieved_gbs"] / HBM_PEAK_GBS, 4),
                  "traffic": measured_traffic("k_march_fp64_q4_64cube"),
                  "kernel": f"k_march<double,4> (finest level {n}^3, v = A u, one launch)",
                  "avg_launch_us": round(ap_["avg_launch_us"], 2), "bytes_per_launch": ap_["bytes_per_launch"],
                  "fp32_avg_launch_us": round(ap_["fp32_avg_launch_us"], 2),
                  "fp32_frac_hbm": round(ap_["fp32_achieved_gbs"] / HBM_PEAK_GBS, 4)}

    out = {
        "metric": "DoF/s per V-cycle + time-to-1e-8 residual, FP64 vs FP32-MG, one MI355X",
        "value": N * sum(its) / t64,
        "unit": "DoF/s per V-cycle",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": t64 / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": ("synthetic: b = M f, f seeded uniform[-1,1] nodal values (zero on the boundary)"
                 if args.rhs == "mass" else "synthetic: b = f, seeded uniform[-1,1] nodal values"),
        "config": {"workload": f"3D Poisson, unit cube, {n}^3 hexes, Q{p} GLL, Dirichlet, FP64 h-MG(V(1,1), "
                               f"vertex-patch smoother, local half V-cycle p=4->3->1) in flexible CG to rtol 1e-8",
                   "n_dofs": N, "n_cells": n ** dim, "degree": p, "parallelism": "single GPU"},
        "setup_s": t_setup,
        "time_to_solution_s": {"fp64": t64 / args.steps, "fp32_mg": t32 / args.steps},
        "fp32_mg_speedup": t64 / t32,
        "iterations": {"fp64": its[-1], "fp32_mg": its32[-1]},
        "rel_residual": {"fp64": relres64, "fp32_mg": info32.rel_residual},
        "fp32_mg_solution_rel_diff_vs_fp64": diff32,
        "dof_per_s": rates["dof_per_s"],
        "ms": rates["ms"],
        "smooth_over_apply": rates["smooth_over_apply"],
        "per_call": rates["per_call"],
        "roofline": roof,
        "roofline_operator": roof_apply,
    }
    del pr, b, x, z
    torch.cuda.empty_cache()
    if not args.no_sweep:
        out["degree_sweep_64"] = bench_degree_sweep(torch, pmg, rhs_vector, 1, [2, 3, 5, 6, 7, 8], args.rhs)
        log("bench: 128^3 Q4 rates (working set beyond the last-level cache)")
        pr128 = pmg.make_problem(3, 128, 4)
        r128, sm128, ap128 = kernel_rates(torch, pmg, perfmodel, np, pr128, 3, 128, 4, max(3, reps // 4))
        r128.update({"smooth_launch_frac_hbm": sm128["achieved_gbs"] / HBM_PEAK_GBS,
                     "smooth_launch_us": sm128["avg_launch_us"],
                     "smooth_launch_frac_fp64_valu": sm128["achieved_tflops"] / FP64_PEAK_TFLOPS,
                     "apply_frac_hbm": ap128["achieved_gbs"] / HBM_PEAK_GBS, "apply_us": ap128["avg_launch_us"],
                     "smooth_traffic": measured_traffic("k_smooth_fp64_q4_128cube"),
                     "apply_traffic": measured_traffic("k_march_fp64_q4_128cube")})
        out["n128_q4"] = r128
        del pr128
        torch.cuda.empty_cache()
        out["local_solvers_32"] = bench_local_solvers(torch, pmg, perfmodel, np, max(3, reps // 2))
    if not args.no_batch:
        log("bench: 16-problem batch (FP32-MG in FP64 CG) and the same solves one by one")
        out["batched"] = bench_batch(max(1, min(args.steps, 3)), torch, pmg, rhs_vector)
        out["batched_small"] = bench_small_batch(max(1, min(args.steps, 3)), torch, pmg, rhs_vector)
    if not args.no_hex:
        out["hex_general"] = bench_hex(torch, pmg, perfmodel, np, max(4, reps // 2))
    if args.extras:
        out["general_48_q6"] = bench_general(torch, pmg, max(1, min(args.steps, 2)))
    if not args.no_cpu_baseline:
        log("bench: CPU oracle baseline (8^3 cells, Q4, V-cycles, CSR apply, smoother, one thread)")
        cb = cpu_baseline(3, 8, 4, seed, budget_s=10.0)
        (rate, k, t), (ra, ka, ta), (rs, ks, ts) = cb["vcycle"], cb["apply"], cb["smooth"]
        out["cpu_baseline"] = {"value": rate, "unit": "DoF/s per V-cycle", "cores": 1, "kind": "oracle",
                               "apply_dof_per_s": ra, "smooth_dof_per_s": rs,
                               "sample": f"{k} oracle V-cycles on 8^3 cells Q4 (35,937 DoFs; the 64^3 headline "
                                         f"is out of the oracle's reach), setup excluded, {t:.1f} s; beside them "
                                         f"{ka} applies of the assembled CSR operator ({ta:.1f} s) and {ks} "
                                         f"smoother applications ({ts:.1f} s) on the same mesh; rates at that "
                                         f"size, not extrapolated; host {platform.processor() or platform.machine()}, "
                                         f"{os.cpu_count()} logical CPUs"}
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
