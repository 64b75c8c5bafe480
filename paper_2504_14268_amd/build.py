"""Builds libmpcg.so (gfx950) in-tree with hipcc.

Flags: IEEE semantics throughout (no fast math, no fp contraction: every fused
multiply-add in the kernels is written out), correctly rounded fp32 division
and square root, and packed-fp32 instructions disabled.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libmpcg.so")
SOURCES = ["kernels.hip", "mlp.hip", "api.hip"]
ARCH = os.environ.get("MPCG_OFFLOAD_ARCH", "gfx950")

HIPCC_FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    "-ffp-contract=off", "-fhip-fp32-correctly-rounded-divide-sqrt",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-const-variable",
    f"-I{os.path.join(ROOT, 'include')}", f"-I{CSRC}",
]


# (source, extra flags, object): kernels.hip is compiled as nine parts in
# parallel (its MPCG_KPART selects the kernels of each object).
UNITS = [("kernels.hip", [f"-DMPCG_KPART={k}"], f"kernels_p{k}.o") for k in range(1, 10)] + [
    ("mlp.hip", [], "mlp.o"), ("api.hip", [], "api.o")]


def build(verbose: bool = False, jobs: int = 0) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    jobs = jobs or min(len(UNITS), max(1, os.cpu_count() or 1))
    objs, running = [], []
    for src, extra, obj in UNITS:
        obj = os.path.join(CSRC, obj)
        cmd = [hipcc, *HIPCC_FLAGS, *extra, "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        while len(running) >= jobs:
            _wait_one(running)
        running.append((subprocess.Popen(cmd), cmd))
        objs.append(obj)
    while running:
        _wait_one(running)
    tmp = LIB + ".tmp"
    cmd = [hipcc, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


def _wait_one(running: list) -> None:
    proc, cmd = running.pop(0)
    if proc.wait() != 0:
        for p, _ in running:
            p.wait()
        raise subprocess.CalledProcessError(proc.returncode, cmd)


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
