"""Build the HIP library liblbm_lee.so in-tree for gfx950 with hipcc.

Usage: python -m paper_1601_08103_amd.build  (or build() from Python).
"""
from __future__ import annotations

import glob
import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "liblbm_lee.so")
# the C ABI, the step launch sequences (one translation unit per velocity set, compiled in
# parallel) and the host-side tables
SOURCES = ["api.hip", "tables.cpp"] + sorted(os.path.basename(p) for p in glob.glob(os.path.join(CSRC, "step_*.hip")))
ARCH = os.environ.get("LBM_OFFLOAD_ARCH", "gfx950")

# -packed-fp32-ops off: hipcc would otherwise form v_pk_*_f32 from plain float code.
DEVICE_FLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def hipcc() -> str:
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def _compile(src: str, obj: str, verbose: bool) -> None:
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-Wall",
           "-I", os.path.join(ROOT, "include")]
    if src.endswith(".hip"):
        cmd += DEVICE_FLAGS
    else:
        cmd += ["-x", "c++"]
    cmd += ["-c", os.path.join(CSRC, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), file=sys.stderr)
    subprocess.run(cmd, check=True)


def build(verbose: bool = False, jobs: int | None = None) -> str:
    """Compile every source (in parallel, `jobs` at a time) and link liblbm_lee.so."""
    build_dir = os.path.join(ROOT, "_build")
    os.makedirs(build_dir, exist_ok=True)
    objs = [os.path.join(build_dir, os.path.splitext(src)[0] + ".o") for src in SOURCES]
    if jobs is None:
        jobs = int(os.environ.get("MAX_JOBS", "0")) or min(len(SOURCES), os.cpu_count() or 1)
    with ThreadPoolExecutor(max_workers=max(1, jobs)) as ex:
        # the largest translation units first
        order = sorted(range(len(SOURCES)), key=lambda i: SOURCES[i] != "step_d3q7.hip")
        futs = [ex.submit(_compile, SOURCES[i], objs[i], verbose) for i in order]
        for f in futs:
            f.result()
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), file=sys.stderr)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
