"""Build the HIP library ``libhhg.so`` for gfx950 in-tree.

Every HIP source is compiled by hipcc for gfx950 only; packed FP32 VALU
instructions are disabled (``-packed-fp32-ops``).
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libhhg.so")
SOURCES = ["hhg_setup.cpp", "hhg_profile.cpp", "hhg_apply.hip", "hhg_solve.hip", "hhg_viscosity.hip",
           "hhg_batch.hip", "hhg_learned.hip", "hhg_mg.hip", "hhg2d.hip",
           "hhg_interior_f64_scaled.hip", "hhg_interior_f64_onthefly.hip",
           "hhg_interior_f32_scaled.hip", "hhg_interior_f32_onthefly.hip"]
ARCH = "gfx950"


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


FLAGS = ["-O3", "-std=c++17", "-fPIC", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-function", "-Wno-unknown-pragmas"]
BUILD_DIR = os.path.join(HERE, "_build")


def _run(cmd):
    res = subprocess.run(cmd, capture_output=True, text=True)
    errs = "\n".join(l for l in res.stderr.splitlines()
                     if "is not a recognized feature for this target" not in l)
    return res.returncode, errs


def build(verbose: bool = False) -> str:
    """Compile every source for gfx950 (always recompiles, sources in
    parallel), link libhhg.so in place and return its path."""
    from concurrent.futures import ThreadPoolExecutor
    os.makedirs(BUILD_DIR, exist_ok=True)
    cc = hipcc()
    jobs = []
    for src in SOURCES:
        obj = os.path.join(BUILD_DIR, src + ".o")
        jobs.append((obj, [cc, f"--offload-arch={ARCH}", *FLAGS, "-x", "hip", "-c",
                           os.path.join(CSRC, src), "-o", obj]))
    if verbose:
        for _, cmd in jobs:
            print(" ".join(cmd), flush=True)
    with ThreadPoolExecutor(max_workers=min(len(jobs), os.cpu_count() or 1, 8)) as ex:
        results = list(ex.map(lambda j: _run(j[1]), jobs))
    for (obj, cmd), (rc, errs) in zip(jobs, results):
        if rc != 0:
            raise RuntimeError(f"hipcc failed on {cmd[-3]} ({rc}):\n{errs}")
        if verbose and errs.strip():
            print(errs, file=sys.stderr)
    tmp = LIB + ".tmp"
    link = [cc, f"--offload-arch={ARCH}", "-shared", "-fPIC", *[j[0] for j in jobs], "-o", tmp]
    if verbose:
        print(" ".join(link), flush=True)
    rc, errs = _run(link)
    if rc != 0:
        raise RuntimeError(f"link failed ({rc}):\n{errs}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
