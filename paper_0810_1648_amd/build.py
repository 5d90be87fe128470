"""Builds libgabp_svm.so (HIP for gfx950) in the package directory.

Every HIP translation unit is compiled with hipcc for gfx950 only, with the
packed-FP32 instruction feature disabled, then linked into one shared
library that exports the C ABI of include/gabp_svm.h.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libgabp_svm.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

SOURCES = ["gabp_sweep_mixed.hip", "gabp_sweep_f32.hip", "gabp_sweep_f64.hip", "gabp_kernels.hip",
           "gabp_predict.hip", "gabp_sparse.hip", "gabp_svm.cpp", "gabp_serve.cpp"]
FLAGS = ["--offload-arch=gfx950", "-O3", "-fPIC", "-std=c++17", "-Wall", "-Wno-unused-result",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I", os.path.join(ROOT, "include")]
# per-file additions: the decision function's MFMA accumulators in ordinary
# VGPRs (its exp2 reads them directly instead of copying each out of an AGPR)
FILE_FLAGS = {"gabp_predict.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form"]}


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError(f"command failed ({r.returncode}): {' '.join(cmd)}")
    err = "\n".join(l for l in r.stderr.splitlines() if "packed-fp32-ops" not in l)
    if err.strip() and verbose:
        sys.stderr.write(err + "\n")


def build(verbose: bool = False, jobs: int = 6) -> str:
    os.makedirs(BUILD, exist_ok=True)
    objs = []
    procs = []
    for src in SOURCES:
        obj = os.path.join(BUILD, src + ".o")
        cmd = [HIPCC, *FLAGS, *FILE_FLAGS.get(src, []), "-c", os.path.join(CSRC, src), "-o", obj]
        if src.endswith(".cpp"):
            cmd.insert(1, "-xhip")
        objs.append(obj)
        procs.append(cmd)
    # compile in parallel
    running = []
    for cmd in procs:
        if verbose:
            print(" ".join(cmd), flush=True)
        running.append((cmd, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True)))
        if len(running) >= jobs:
            _wait(running.pop(0))
    for item in running:
        _wait(item)
    tmp = LIB + ".tmp"
    _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs, "-lpthread"], verbose)
    os.replace(tmp, LIB)
    return LIB


def _wait(item):
    cmd, p = item
    out, err = p.communicate()
    if p.returncode != 0:
        sys.stderr.write(out + err)
        raise RuntimeError(f"command failed ({p.returncode}): {' '.join(cmd)}")


if __name__ == "__main__":
    print(build(verbose=True))
