#!/usr/bin/env python3
"""Benchmark of the local p-multigrid patch-smoother solver on one MI355X.

Workload: 3D Poisson on the unit cube, 32^3 hexahedra, Q4 Gauss-Lobatto elements
(2,146,689 nodes), homogeneous Dirichlet, seeded uniform[-1,1] right-hand side; h-multigrid
V(1,1) (levels 2..32 cells) with the vertex-patch smoother whose local solver is one half
V-cycle over the p-levels 4 -> 3 -> 1, inside flexible CG, all FP64.

One step = one solve from x = 0 to |b - A x| <= 1e-8 |b| (apply, smoother color passes
with the fused local p-multigrid, residuals, transfers, coarse solve, dot products: the
whole path).  value = nodes x V-cycles / time (DoF/s per V-cycle).  The same solve with
FP32 multigrid inside the FP64 CG is timed alongside, and the finest-level smoother kernel
(the dominant kernel) is timed with HIP events on the launch stream for the roofline.

    python bench.py [--steps K] [--warmup W] [--no-cpu-baseline] [--no-batch] [--extras]
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


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def time_events(fn, reps, torch):
    """Mean milliseconds per call of fn() between HIP events on the current stream."""
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    fn()
    e0.record(s)
    for _ in range(reps):
        fn()
    e1.record(s)
    e1.synchronize()
    return e0.elapsed_time(e1) / reps


def measured_traffic():
    """HBM bytes per finest-level smoother launch from the committed counter runs
    (profiles/k_smooth_fp64_q4_32cube.traffic.json), or None when a kernel source listed
    there has changed since the counters were taken."""
    import hashlib

    path = os.path.join(ROOT, "profiles", "k_smooth_fp64_q4_32cube.traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    for rel, digest in rec["sources_sha256"].items():
        with open(os.path.join(ROOT, rel), "rb") as f:
            if hashlib.sha256(f.read()).hexdigest() != digest:
                return None
    return rec["fetch_bytes_per_launch"] + rec["write_bytes_per_launch"]


def cpu_baseline(dim, n, p, seed, budget_s=12.0):
    """The oracle (NumPy/SciPy, one thread) timed on V-cycles of a reduced mesh."""
    from threadpoolctl import threadpool_limits

    from oracle.solver import MultigridProblem
    from paper_2512_02577_amd.inputs import rhs_vector

    with threadpool_limits(1):
        pb = MultigridProblem(dim, n, p)
        r = rhs_vector(dim, n, p, seed)
        pb.vcycle(r)  # builds the patch caches (setup)
        t0 = time.perf_counter()
        k = 0
        while time.perf_counter() - t0 < budget_s or k < 3:
            pb.vcycle(r)
            k += 1
        t = time.perf_counter() - t0
    return pb.N * k / t, k, t


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


def _solve_times(torch, pmg, pr, b, precs, steps):
    """Time-to-solution, iterations and relative residual of each multigrid precision, and
    the relative difference of each solution to the FP64-multigrid one."""
    out, xref = {}, None
    for prec, name in precs:
        x = torch.empty_like(b)
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


def bench_degree_sweep(torch, pmg, rhs_vector, steps):
    """3D Poisson, 64^3 hexes, p = 2..8 (paper p-hierarchies), seeds 300 + p: FP64 and FP32
    multigrid inside the FP64 flexible CG (on Cartesian meshes BF16 storage has no stored
    operator data to act on, so it equals FP32)."""
    res = []
    for p in range(2, 9):
        log(f"bench: degree sweep 64^3 Q{p}")
        pr = pmg.make_problem(3, 64, p)
        b = torch.as_tensor(rhs_vector(3, 64, p, 300 + p), dtype=torch.float64, device="cuda:0")
        rec = {"degree": p, "n_dofs": pr.n_nodes[-1]}
        rec.update(_solve_times(torch, pmg, pr, b, ((pmg.FP64, "fp64_mg"), (pmg.FP32, "fp32_mg")), steps))
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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--kernel-reps", type=int, default=50)
    ap.add_argument("--no-batch", action="store_true", help="leave out the 16-problem batch measurement")
    ap.add_argument("--extras", action="store_true",
                    help="also the 64^3 degree sweep and the 48^3 Q6 perturbed-mesh problem (minutes)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    from paper_2512_02577_amd import perfmodel, pmg
    from paper_2512_02577_amd.inputs import rhs_vector

    dim, n, p, seed = 3, 32, 4, 2
    torch.cuda.set_device(0)
    dev = "cuda:0"
    log(f"bench: setup 3D n={n} Q{p}")
    pr = pmg.make_problem(dim, n, p)
    N = pr.n_nodes[-1]
    b = torch.as_tensor(rhs_vector(dim, n, p, seed), dtype=torch.float64, device=dev)
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

    # per-call rates with HIP events on torch's current stream (the launch stream)
    log("bench: per-call timings")
    L = pr.finest
    u = torch.as_tensor(np.random.default_rng(3).uniform(-1, 1, N), dtype=torch.float64, device=dev)
    v = torch.empty_like(u)
    z = torch.empty_like(u)
    reps = args.kernel_reps
    t_apply = time_events(lambda: pmg.apply_operator(pr, L, u, v), reps, torch)
    u_s = u.clone()
    t_smooth = time_events(lambda: pmg.smooth(pr, L, u_s, b, 1), reps, torch)
    t_vc = time_events(lambda: pmg.vcycle(pr, b, z, pmg.FP64), max(5, reps // 5), torch)
    t_vc32 = time_events(lambda: pmg.vcycle(pr, b, z, pmg.FP32), max(5, reps // 5), torch)
    u32 = u.float()
    b32 = b.float()
    t_smooth32 = time_events(lambda: pmg.smooth(pr, L, u32, b32, 1), reps, torch)

    # dominant kernel: the finest-level smoother color kernel (8 launches per application)
    ncol = 2 ** dim
    bytes_launches = sum(perfmodel.smooth_launch_bytes(dim, n, p, c) for c in range(ncol))
    patches = sum(perfmodel.smooth_launch_patches(dim, n, c) for c in range(ncol))
    flops = patches * perfmodel.patch_flops(dim, p, pr.degrees)
    t_launch = t_smooth / ncol * 1e-3
    ach_gbs = bytes_launches / ncol / t_launch / 1e9
    ach_tf = flops / ncol / t_launch / 1e12
    ai = flops / bytes_launches
    ridge = FP64_PEAK_TFLOPS * 1e12 / (HBM_PEAK_GBS * 1e9)
    bound = "hbm" if ai < ridge else "alu"
    if bound == "hbm":
        roof = {"bound": "hbm", "achieved": round(ach_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(ach_gbs / HBM_PEAK_GBS, 4)}
    else:
        roof = {"bound": "alu", "achieved": round(ach_tf, 2), "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": round(ach_tf / FP64_PEAK_TFLOPS, 4)}
    traffic = measured_traffic()
    roof.update({"traffic": traffic, "kernel": "k_smooth<3,double,4,{1,3,4},ONE> (finest level, one color launch)",
                 "avg_launch_us": round(t_launch * 1e6, 2), "bytes_per_launch": bytes_launches // ncol,
                 "flops_per_launch": flops // ncol, "flop_per_byte": round(ai, 2),
                 "achieved_tflops": round(ach_tf, 3), "achieved_gbs": round(ach_gbs, 1)})

    # the operator apply v = A u on the finest level (one launch): reads u, writes v
    apply_bytes = 16 * N
    apply_gbs = apply_bytes / (t_apply * 1e-3) / 1e9
    roof_apply = {"bound": "hbm", "achieved": round(apply_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                  "frac": round(apply_gbs / HBM_PEAK_GBS, 4), "traffic": None,
                  "kernel": "k_apply<3,double,4> (finest level, v = A u, one launch)",
                  "avg_launch_us": round(t_apply * 1e3, 2), "bytes_per_launch": apply_bytes}

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
        "data": "synthetic (seeded uniform[-1,1] right-hand side)",
        "config": {"workload": "3D Poisson, unit cube, 32^3 hexes, Q4 GLL, Dirichlet, FP64 h-MG(V(1,1), vertex-patch "
                               "smoother, local half V-cycle p=4->3->1) in flexible CG to rtol 1e-8",
                   "n_dofs": N, "n_cells": n ** dim, "degree": p, "parallelism": "single GPU"},
        "time_to_solution_s": {"fp64": t64 / args.steps, "fp32_mg": t32 / args.steps},
        "iterations": {"fp64": its[-1], "fp32_mg": its32[-1]},
        "rel_residual": {"fp64": relres64, "fp32_mg": info32.rel_residual},
        "fp32_mg_solution_rel_diff_vs_fp64": diff32,
        "dof_per_s": {"apply_fp64": N / (t_apply * 1e-3), "smooth_fp64": N / (t_smooth * 1e-3),
                      "smooth_fp32": N / (t_smooth32 * 1e-3), "vcycle_fp64": N / (t_vc * 1e-3),
                      "vcycle_fp32": N / (t_vc32 * 1e-3)},
        "ms": {"apply_fp64": t_apply, "smooth_fp64": t_smooth, "smooth_fp32": t_smooth32, "vcycle_fp64": t_vc,
               "vcycle_fp32": t_vc32},
        "smooth_over_apply": t_smooth / t_apply,
        "roofline": roof,
        "roofline_operator": roof_apply,
    }
    if not args.no_batch:
        log("bench: 16-problem batch (FP32-MG in FP64 CG) and the same solves one by one")
        out["batched"] = bench_batch(max(1, min(args.steps, 3)), torch, pmg, rhs_vector)
        out["batched_small"] = bench_small_batch(max(1, min(args.steps, 3)), torch, pmg, rhs_vector)
    if args.extras:
        out["degree_sweep_64"] = bench_degree_sweep(torch, pmg, rhs_vector, max(1, min(args.steps, 2)))
        out["general_48_q6"] = bench_general(torch, pmg, max(1, min(args.steps, 2)))
    if not args.no_cpu_baseline:
        log("bench: CPU oracle baseline (8^3 cells, Q4, V-cycles, one thread)")
        rate, k, t = cpu_baseline(3, 8, 4, seed)
        out["cpu_baseline"] = {"value": rate, "unit": "DoF/s per V-cycle", "cores": 1, "kind": "oracle",
                               "sample": f"{k} oracle V-cycles on 8^3 cells Q4 (35,937 DoFs), setup excluded, "
                                         f"{t:.1f} s; host {platform.processor() or platform.machine()}, "
                                         f"{os.cpu_count()} logical CPUs"}
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
