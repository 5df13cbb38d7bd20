"""Build the correlator's HIP library (libcorr_gfx950.so) in-tree with hipcc.

Every source is compiled for gfx950 only, with packed-FP32 instruction
selection disabled, fp-contraction limited to explicit fma calls in the
compensated paths (-ffp-contract=fast keeps ordinary mul+add fusion), and no
fast-math (the compensated sums rely on IEEE evaluation order).
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libcorr_gfx950.so")
HIPCC = "/opt/rocm/bin/hipcc"

SOURCES = ["corr_push.hip", "corr_deferred.hip", "corr_rhok.hip", "corr_rhok_mfma.hip",
           "corr_reduce.hip", "corr_window.hip", "corr_momentum.hip", "corr_runtime.cpp",
           "corr_autotune.cpp"]

FLAGS = [
    "-O3", "-std=c++17", "--offload-arch=gfx950", "-mcode-object-version=5", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-fno-fast-math", "-ffp-contract=fast",
    "-Wall", "-Wno-unused-result",
]


def build(verbose: bool = False) -> str:
    obj_dir = os.path.join(HERE, "_build")
    os.makedirs(obj_dir, exist_ok=True)
    cmds, objs = [], []
    for src in SOURCES:
        path = os.path.join(CSRC, src)
        obj = os.path.join(obj_dir, os.path.splitext(src)[0] + ".o")
        cmds.append([HIPCC] + FLAGS + ["-x", "hip", "-c", path, "-o", obj])
        objs.append(obj)

    def compile_one(cmd):
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)

    workers = max(1, min(len(cmds), os.cpu_count() or 1, 8))
    with ThreadPoolExecutor(max_workers=workers) as pool:
        list(pool.map(compile_one, cmds))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
