"""The library's outer iteration counts on the grid of the paper's Table 1 (Sec. 2.2.1):
local solvers {1 V-cycle, 1 half V-cycle, 2 half V-cycles, 25 V-cycles} x mesh distortion x
p in {3, 7} x 2D/3D.  The GPU's flexible CG (FP64 multigrid) must need the oracle's FCG
count within one iteration on every configuration stored by
tests/golden/make_table1_counts.py (oracle only); the oracle's GMRES(30) counts, the
paper's solver, are reported beside them in the design notes (absolute counts: parity
unpinned, the paper's mesh, tolerance and damping are unknown)."""
import glob
import json
import os

import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from paper_2512_02577_amd import pmg  # noqa: E402
from paper_2512_02577_amd.inputs import jittered_vertices, rhs_vector  # noqa: E402

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
FILES = sorted(glob.glob(os.path.join(ROOT, "tests", "golden", "table1", "*.json")))
VARIANTS = {"1 V-cycle": (pmg.LOCAL_FULL_V, 1), "1 half V-cycle": (pmg.LOCAL_HALF_V, 1),
            "2 half V-cycles": (pmg.LOCAL_HALF_V, 2), "25 V-cycles": (pmg.LOCAL_FULL_V, 25)}


@pytest.mark.parametrize("path", FILES, ids=[os.path.basename(f)[:-5] for f in FILES])
def test_fcg_counts_match_the_oracle(path):
    rec = json.load(open(path))
    dim, n, p, delta = rec["dim"], rec["n"], rec["p"], rec["delta"]
    print(f"case table1 {dim}D n {n} p {p} delta {delta}", flush=True)
    verts = jittered_vertices(dim, n, delta, 91) if delta > 0 else None
    b = torch.as_tensor(rhs_vector(dim, n, p, 90), dtype=torch.float64, device="cuda:0")
    out = {}
    for name, (loc, it) in VARIANTS.items():
        cfg = pmg.default_config()
        cfg.local_solver, cfg.n_local_iter = loc, it
        pr = pmg.make_problem(dim, n, p, config=cfg, vertices=verts)
        x = torch.empty_like(b)
        info = pmg.solve(pr, b, x, pmg.FP64)
        assert info.rel_residual <= 1e-8
        out[name] = info.iterations
        assert abs(info.iterations - rec["counts"][name]["fcg"]) <= 1, (name, info.iterations, rec["counts"][name])
    outd = os.path.join(ROOT, "gpurun_out")
    if os.path.isdir(outd):
        with open(os.path.join(outd, "table1_gpu_counts.jsonl"), "a") as f:
            f.write(json.dumps({"dim": dim, "n": n, "p": p, "delta": delta, "gpu_fcg": out,
                                "oracle": rec["counts"]}) + "\n")
