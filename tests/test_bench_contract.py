"""bench.py contract on the CPU: it measures one GPU only and refuses other GPU counts with a
message and a non-zero status; the committed HBM traffic record matches the kernel sources it
lists (otherwise bench.py reports the traffic as unknown)."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_more_than_one_gpu():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert p.returncode == 2
    assert "one GPU" in p.stderr
    assert p.stdout == ""


def test_traffic_records_are_well_formed():
    # the records bench.py reads: HBM bytes per launch of the smoother color launch and of the
    # apply at 64^3 and 128^3 Q4, each naming its summary and the kernel sources it was taken with
    for name in ("k_smooth_fp64_q4_64cube", "k_smooth_fp64_q4_128cube", "k_march_fp64_q4_64cube",
                 "k_march_fp64_q4_128cube", "k_march_fp64_q8_64cube"):
        rec = json.load(open(os.path.join(ROOT, "profiles", name + ".traffic.json")))
        assert rec["fetch_bytes_per_launch"] > 0 and rec["write_bytes_per_launch"] > 0
        for rel in rec["sources_sha256"]:
            assert os.path.exists(os.path.join(ROOT, rel)), rel
        assert os.path.exists(os.path.join(ROOT, rec["summary"]))
