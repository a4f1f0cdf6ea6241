"""Build libcpm.so in-tree: host band builder with g++ (IEEE double, no contraction,
OpenMP), HIP sources with hipcc for gfx950, linked into one shared library.

    python -m paper_1307_4354_amd.build          (or call build())
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
REPO = os.path.dirname(HERE)
OUT_DIR = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libcpm.so")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
ARCH = os.environ.get("CPM_OFFLOAD_ARCH", "gfx950")

HOST_SOURCES = ["band_build.cpp"]
HIP_SOURCES = ["kernels.hip", "capi.hip", "extras.hip", "mlp.hip", "batched.hip", "noalloc.hip", "coarse.hip"]

HIPCC_FLAGS = [
    "-O3", "-fPIC", "-std=c++17", "--offload-arch=" + ARCH,
    # keep the compiler from emitting packed-FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I" + os.path.join(REPO, "include"),
]
GXX_FLAGS = ["-O2", "-fPIC", "-std=c++17", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
             "-I" + os.path.join(REPO, "include")]


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout)
        raise RuntimeError("build step failed: " + " ".join(cmd))
    return r.stdout


def build(verbose: bool = False) -> str:
    os.makedirs(OUT_DIR, exist_ok=True)
    hipcc = os.path.join(ROCM, "bin", "hipcc")
    jobs = []
    objs = []
    for src in HOST_SOURCES:
        o = os.path.join(OUT_DIR, src + ".o")
        jobs.append(["g++"] + GXX_FLAGS + ["-c", os.path.join(CSRC, src), "-o", o])
        objs.append(o)
    for src in HIP_SOURCES:
        p = os.path.join(CSRC, src)
        if not os.path.exists(p):
            continue
        o = os.path.join(OUT_DIR, src + ".o")
        jobs.append([hipcc] + HIPCC_FLAGS + ["-c", p, "-o", o])
        objs.append(o)
    with ThreadPoolExecutor(max_workers=min(8, len(jobs))) as ex:
        outs = list(ex.map(_run, jobs))
    if verbose:
        for o in outs:
            if o.strip():
                print(o)
    tmp = LIB + ".tmp"
    _run([hipcc, "-shared", "-fPIC", "--offload-arch=" + ARCH, "-o", tmp] + objs +
         ["-L" + os.path.join(ROCM, "lib"), "-lamdhip64", "-lgomp", "-Wl,-rpath," + os.path.join(ROCM, "lib")])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
