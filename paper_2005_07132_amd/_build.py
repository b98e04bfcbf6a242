"""Builds libfkkec.so (HIP kernels for gfx950 + the C ABI + host FP64 code)
in-tree, next to this file."""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libfkkec.so")
ARCH = os.environ.get("FKK_OFFLOAD_ARCH", "gfx950")

HIP_SOURCES = ["api.hip", "kernels.hip", "kernels_bf16.hip", "kernels_i8.hip", "plain.hip", "eig.hip", "serve.hip"]
HOST_SOURCES = ["host_math.cpp"]

# Packed FP32 instructions stay off: the compiler must not form them.
HIP_FLAGS = ["-O3", "-fPIC", "-std=c++17", f"--offload-arch={ARCH}",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wno-unused-command-line-argument"]
HOST_FLAGS = ["-O3", "-fPIC", "-std=c++17", "-march=x86-64-v3"]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError(f"build step failed: {' '.join(cmd[:3])} ...")
    return res


def build(verbose: bool = False, out: str = LIB) -> str:
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    gxx = shutil.which("g++") or "g++"
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    jobs = []
    for src in HOST_SOURCES:
        obj = os.path.join(objdir, src + ".o")
        jobs.append(([gxx, *HOST_FLAGS, "-I", INCLUDE, "-c", os.path.join(CSRC, src), "-o", obj], obj))
    for src in HIP_SOURCES:
        obj = os.path.join(objdir, src + ".o")
        jobs.append(([hipcc, *HIP_FLAGS, "-I", INCLUDE, "-I", CSRC, "-c", os.path.join(CSRC, src), "-o", obj], obj))
    # the translation units compile independently: in parallel
    workers = max(1, min(len(jobs), os.cpu_count() or 1, 8))
    with ThreadPoolExecutor(workers) as pool:
        list(pool.map(lambda job: _run(job[0], verbose), jobs))
    objs = [obj for _, obj in jobs]
    tmp = out + ".tmp"
    _run([hipcc, "-shared", f"--offload-arch={ARCH}", "-o", tmp, *objs, "-lpthread"], verbose)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
