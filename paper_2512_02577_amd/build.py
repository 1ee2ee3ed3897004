"""Builds the HIP library libpmg.so (gfx950) and the CPU emulation library of its kernel
bodies, in-tree, next to this file.

    python -m paper_2512_02577_amd.build          # both libraries
    python -m paper_2512_02577_amd.build --asan   # also the bounds-checked emulation runner
    python -m paper_2512_02577_amd.build --tsan   # also the race-checked emulation runner

Every call compiles from scratch; objects go to paper_2512_02577_amd/_build/.
"""
from __future__ import annotations

import argparse
import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libpmg.so")
EMU = os.path.join(PKG, "libpmg_hostemu.so")

HIP_SOURCES = ["kernels_metric_3d_f32.hip", "kernels_metric_3d_bf16.hip", "kernels_metric_3d_f64.hip",
               "kernels_metric_2d_f64.hip", "kernels_metric_2d_f32.hip",
               "kernels_3d_f64.hip", "kernels_3d_f32.hip", "kernels_2d_f64.hip", "kernels_2d_f32.hip",
               "setup.hip", "blas.hip", "batch.hip", "capi.cpp", "batch_host.cpp", "kernels_dispatch.cpp",
               "host_tables.cpp", "geometry.cpp", "hex_setup.cpp", "hex_capi.cpp",
               "kernels_hex_3d_f64.hip", "kernels_hex_3d_f32.hip", "kernels_hex_2d_f64.hip", "kernels_hex_2d_f32.hip"]
HIPCC_FLAGS = ["-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC",
               # no packed FP32 instructions anywhere in the device code
               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
               "-I" + os.path.join(ROOT, "include"), "-I" + CSRC]


def _hipcc() -> str:
    for cand in ("/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def _run(cmd: list[str]) -> None:
    res = subprocess.run(cmd, capture_output=True, text=True)
    err = "\n".join(l for l in res.stderr.splitlines() if "packed-fp32-ops" not in l and l.strip())
    if res.returncode != 0:
        raise RuntimeError(f"command failed ({res.returncode}): {' '.join(cmd)}\n{err}")


def build_hip(jobs: int = 8, only: list[str] | None = None) -> str:
    """Compiles every source (or, with `only`, just those, reusing the other objects of
    an earlier build) and links libpmg.so."""
    os.makedirs(BUILD, exist_ok=True)
    hipcc = _hipcc()
    cmds, objs = [], []
    for src in HIP_SOURCES:
        obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
        lang = ["-x", "hip"] if src in ("capi.cpp", "batch_host.cpp", "kernels_dispatch.cpp", "hex_capi.cpp") else []
        if only is None or src in only or not os.path.exists(obj):
            cmds.append([hipcc, *HIPCC_FLAGS, *lang, "-c", os.path.join(CSRC, src), "-o", obj])
        objs.append(obj)
    with ThreadPoolExecutor(max_workers=max(1, min(jobs, len(cmds)))) as ex:
        list(ex.map(_run, cmds))
    tmp = LIB + ".tmp"
    _run([hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp, "-L/opt/rocm/lib", "-lhipsolver",
          "-lpthread", "-Wl,-rpath,/opt/rocm/lib"])
    os.replace(tmp, LIB)
    return LIB


def build_emulation(asan: bool = False, tsan: bool = False) -> str:
    """The CPU emulation library of the kernel bodies; with asan/tsan also the checked
    runner hostemu_check (AddressSanitizer + UndefinedBehaviorSanitizer, or
    ThreadSanitizer), a plain g++ build of host code only."""
    os.makedirs(BUILD, exist_ok=True)
    srcs = [os.path.join(CSRC, "hostemu.cpp"), os.path.join(CSRC, "host_tables.cpp"), os.path.join(CSRC, "geometry.cpp"),
            os.path.join(CSRC, "hex_setup.cpp")]
    tmp = EMU + ".tmp"
    _run(["g++", "-O2", "-std=c++17", "-shared", "-fPIC", "-I" + CSRC, "-I" + os.path.join(ROOT, "include"), *srcs, "-o", tmp, "-lpthread"])
    os.replace(tmp, EMU)
    out = EMU
    checked = os.path.join(CSRC, "hostemu_check.cpp")
    if asan:
        out = os.path.join(BUILD, "hostemu_asan")
        _run(["g++", "-O1", "-g", "-std=c++17", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
              "-I" + CSRC, "-I" + os.path.join(ROOT, "include"), checked, *srcs, "-o", out, "-lpthread"])
    if tsan:
        out = os.path.join(BUILD, "hostemu_tsan")
        _run(["g++", "-O1", "-g", "-std=c++17", "-fsanitize=thread", "-I" + CSRC, "-I" + os.path.join(ROOT, "include"), checked, *srcs, "-o", out,
              "-lpthread"])
    return out


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--asan", action="store_true")
    ap.add_argument("--tsan", action="store_true")
    ap.add_argument("--emulation-only", action="store_true")
    ap.add_argument("--jobs", type=int, default=8)
    ap.add_argument("--only", nargs="*", help="recompile only these sources (file names under csrc/)")
    args = ap.parse_args(argv)
    if not args.emulation_only:
        print(build_hip(args.jobs, args.only))
    print(build_emulation(args.asan, args.tsan))
    return 0


if __name__ == "__main__":
    sys.exit(main())
