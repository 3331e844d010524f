"""Build libsgsplat.so (HIP, gfx950) in-tree with hipcc.

    python -m paper_2501_00342_amd.build [--jobs N]

Each .hip file is compiled to an object, then linked into one shared
library next to this file.  The preprocess files are compiled with
-ffp-contract=off: their float64 key path (the values that decide radii,
rectangles and depth keys) must follow one fixed sequence of rounded
operations.  Packed-FP32 instructions are disabled for all device code.
"""
from __future__ import annotations

import argparse
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libsgsplat.so")
BUILD = os.path.join(ROOT, "_build")
ARCH = "gfx950"

SOURCES = {
    "host.hip": [],
    "preprocess.hip": ["-ffp-contract=off"],
    "preprocess_bwd.hip": ["-ffp-contract=off"],
    "sort.hip": [],
    "radix.hip": [],
    "bin.hip": [],
    "adam.hip": [],
    # the blends' atomics add values already reduced across the wave (the
    # work counters from one lane at a wave-uniform address): LLVM's atomic
    # optimizer would only wrap them in a second, redundant wave reduction
    "blend.hip": ["-mllvm", "-amdgpu-atomic-optimizer-strategy=None"],
}

COMMON = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-munsafe-fp-atomics", "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
    "-Wno-unused-command-line-argument",
    "-I", INCLUDE, "-I", CSRC,
]


def hipcc() -> str:
    for c in ("/opt/rocm/bin/hipcc", "hipcc"):
        if os.path.exists(c) or c == "hipcc":
            return c
    raise RuntimeError("hipcc not found")


def _compile(name: str, extra: list, verbose: bool) -> str:
    src = os.path.join(CSRC, name)
    obj = os.path.join(BUILD, name.replace(".hip", ".o"))
    cmd = [hipcc(), "-c", src, "-o", obj] + COMMON + extra
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {name}:\n{r.stdout}\n{r.stderr}")
    if r.stderr.strip() and verbose:
        print(r.stderr, file=sys.stderr)
    return obj


def build(jobs: int = 5, verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    with ThreadPoolExecutor(max_workers=max(1, jobs)) as ex:
        objs = list(ex.map(lambda kv: _compile(kv[0], kv[1], verbose), SOURCES.items()))
    tmp = LIB + ".tmp"
    cmd = [hipcc(), "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=5)
    ap.add_argument("-v", "--verbose", action="store_true")
    a = ap.parse_args()
    print(build(a.jobs, a.verbose))
