"""Builds libtlrmle.so (HIP for gfx950) in-tree.

    python -m paper_1804_09137_amd.build

Every HIP source is compiled with hipcc for gfx950 only, with the packed-FP32
instructions disabled (-packed-fp32-ops); the host-only helper is compiled with
g++.  Objects go to paper_1804_09137_amd/_build/.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libtlrmle.so")
INCLUDE = os.path.join(ROOT, "include")

HIP_SOURCES = ["matern.hip", "gemm.hip", "gemm_update.hip", "chol.hip", "tile_chol.hip", "compress.hip", "hqr.hip", "solve.hip",
               "grad.hip", "runtime.hip", "compress_cols.hip", "column_update.hip",
               "factor.hip", "api.hip",
               "predict.hip", "noalloc.hip", "aca.hip"]
CPP_SOURCES = ["morton.cpp"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
HIP_FLAGS = ["--offload-arch=gfx950", "-O3", "-fPIC", "-std=c++17", "-Wall", "-Wno-unused-function",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-I", INCLUDE, "-I", CSRC]
CXX_FLAGS = ["-O2", "-fPIC", "-std=c++17", "-Wall", "-I", INCLUDE]


def _run(cmd: list[str]) -> tuple[int, str]:
    p = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    return p.returncode, p.stdout


def build(verbose: bool = False, jobs: int | None = None) -> str:
    os.makedirs(BUILD, exist_ok=True)
    jobs = jobs or min(8, os.cpu_count() or 4)
    cmds = []
    objs = []
    for src in HIP_SOURCES:
        obj = os.path.join(BUILD, src.replace(".hip", ".o"))
        cmds.append([HIPCC, *HIP_FLAGS, "-c", os.path.join(CSRC, src), "-o", obj])
        objs.append(obj)
    for src in CPP_SOURCES:
        obj = os.path.join(BUILD, src.replace(".cpp", ".o"))
        cmds.append(["g++", *CXX_FLAGS, "-c", os.path.join(CSRC, src), "-o", obj])
        objs.append(obj)
    with cf.ThreadPoolExecutor(jobs) as ex:
        results = list(ex.map(_run, cmds))
    failed = False
    for cmd, (rc, out) in zip(cmds, results):
        noisy = [ln for ln in out.splitlines() if "packed-fp32-ops" not in ln and ln.strip()]
        if rc != 0 or (verbose and noisy):
            sys.stderr.write(" ".join(cmd) + "\n" + "\n".join(noisy) + "\n")
        failed |= rc != 0
    if failed:
        raise RuntimeError("HIP build failed")
    tmp = LIB + ".tmp"
    rc, out = _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs])
    if rc != 0:
        raise RuntimeError("link failed:\n" + out)
    shutil.move(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
