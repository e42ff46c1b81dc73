"""Build step for the HIP library (gfx950): one hipcc compile per source file
(in parallel), then one link, in-tree output."""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libmtspd.so")
SOURCES = ["neighbors.hip", "layout.hip", "pd.hip", "pd_implicit.hip", "fe.hip", "fe_implicit.hip", "coupling.hip",
           "dense.hip", "solver.hip", "pool.hip", "energy.hip"]

HIPCC_FLAGS = [
    "-O3", "--offload-arch=gfx950", "-std=c++17", "-fPIC",
    # every expression evaluated as written (bit-exact neighbour criterion and
    # reproducible FP64 sums)
    "-ffp-contract=off",
    # no packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def build(verbose: bool = False, jobs: int = 0) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    os.makedirs(OBJ, exist_ok=True)
    jobs = jobs or min(len(SOURCES), max(1, min(os.cpu_count() or 1, 16)))

    def compile_one(f):
        obj = os.path.join(OBJ, os.path.splitext(f)[0] + ".o")
        cmd = [hipcc, *HIPCC_FLAGS, "-c", "-o", obj, os.path.join(CSRC, f)]
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        return f, obj, r

    with ThreadPoolExecutor(jobs) as ex:
        results = list(ex.map(compile_one, SOURCES))
    failed = [(f, r) for f, _, r in results if r.returncode != 0]
    for f, r in failed:
        sys.stderr.write(f"---- {f}\n" + r.stdout + r.stderr)
    if failed:
        raise RuntimeError("hipcc failed: " + ", ".join(f for f, _ in failed))
    cmd = [hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", LIB + ".tmp"] + [o for _, o, _ in results]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc link failed")
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
