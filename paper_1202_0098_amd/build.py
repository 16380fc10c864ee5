"""Compile libmarnoldi.so (HIP, gfx950) in-tree with hipcc.

The translation units (the launchers, one per basis-kernel family, the start
network and the host side) compile in parallel, then link into one library.
"""

from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libmarnoldi.so")
SOURCES = ["ma_atom.hip", "ma_basis_g9.hip", "ma_basis_g4.hip", "ma_basis_g0.hip", "ma_basis_s.hip",
           "ma_basis_m.hip", "ma_kernels.hip", "ma_post.hip", "ma_mlp.hip", "ma_noalloc.hip", "ma_host.cpp"]

# Packed FP32 instructions are disabled for all device code.
DEVICE_FLAGS = ["--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang",
                "-packed-fp32-ops"]


def _jobs() -> int:
    n = os.cpu_count() or 4
    return max(1, min(len(SOURCES), n, int(os.environ.get("MAX_JOBS", "16"))))


def build(verbose: bool = False) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

    def compile_one(src: str) -> str:
        obj = os.path.join(CSRC, src + ".o")
        cmd = [hipcc, "-O3", "-std=c++17", "-fPIC", "-fvisibility=hidden",
               "-ffp-contract=off" if src.endswith(".cpp") else "-ffp-contract=fast",
               *DEVICE_FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        return obj

    with ThreadPoolExecutor(max_workers=_jobs()) as pool:
        objs = list(pool.map(compile_one, SOURCES))
    tmp = LIB + ".tmp"
    cmd = [hipcc, "-shared", "-fPIC", *DEVICE_FLAGS, *objs, "-o", tmp, "-lpthread"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    for o in objs:
        os.remove(o)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
