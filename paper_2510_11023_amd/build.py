"""Compile libl1pr.so (all HIP sources of csrc/) for gfx950 with hipcc, in-tree."""
from __future__ import annotations

import concurrent.futures
import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libl1pr.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    # packed FP32 instructions stay off in every device code object
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", INCLUDE,
    "-I", CSRC,
]


# Per-file scheduling strategies, each the fastest of the default, max-ILP, memory-clause and
# the iterative ILP, min-register and max-occupancy strategies on its own workload, with the
# same results bit for bit:
# - the register-resident factor kernel, bound by its per-unit dependency chain: iterative ILP,
#   666 -> 646 us per 2048-unit launch at M = 256;
# - the blocked factorisation through device memory: iterative max-occupancy, 1384 -> 1328 ms
#   for the 2D fine sweep of 128 systems of 4096 coefficients (the compiler fails on this file
#   with the iterative ILP strategy).
# The other sources keep the default (measured on the 1D GEMMs and history sums, the 2D
# conjugate gradients, the full-history prefix sums and the MLP: within 2%).
FILE_FLAGS = {
    "step1d_reg.hip": ["-mllvm", "-amdgpu-sched-strategy=iterative-ilp"],
    "chol_blk.hip": ["-mllvm", "-amdgpu-sched-strategy=iterative-maxocc"],
}


def sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")) + glob.glob(os.path.join(CSRC, "*.cpp")))


def _compile(src: str, bdir: str, verbose: bool) -> str:
    obj = os.path.join(bdir, os.path.basename(src) + ".o")
    cmd = [HIPCC, "-x", "hip", "-c", src, "-o", obj] + FLAGS + FILE_FLAGS.get(os.path.basename(src), [])
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError(f"hipcc failed on {src}")
    return obj


def build(verbose: bool = False) -> str:
    bdir = os.path.join(HERE, "_build")
    os.makedirs(bdir, exist_ok=True)
    jobs = max(1, min(8, os.cpu_count() or 1))
    with concurrent.futures.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(lambda src: _compile(src, bdir, verbose), sources()))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("link of libl1pr.so failed")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
