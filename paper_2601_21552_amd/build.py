"""Build ``libscuba.so`` in-tree: host C++ with g++, the HIP kernels with
hipcc for gfx950, linked by hipcc.  ``python -m paper_2601_21552_amd.build``
or ``__graft_entry__.build()``."""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libscuba.so")
MICRO_LIB = os.path.join(HERE, "libkmicro.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

HOST_SRCS = ["api.cpp", "encode.cpp", "split.cpp", "verify.cpp"]
HIP_SRCS = ["device.hip", "mlp.hip"]
MICRO_SRC = "kmicro.hip"   # microbenchmarks, a library of their own

CXXFLAGS = ["-O2", "-std=c++17", "-fPIC", "-Wall", "-Wextra", "-Wno-unused-parameter",
            "-fvisibility=hidden"]
HIPFLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
            # packed FP32 instructions are kept out of every device build
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wno-unused-parameter"]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"command failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return r


def build(verbose: bool = False) -> str:
    os.makedirs(OBJ, exist_ok=True)
    jobs = []
    for s in HOST_SRCS:
        jobs.append(["g++", *CXXFLAGS, "-I", os.path.join(HERE, "..", "include"),
                     "-I", "/opt/rocm/include",
                     "-c", os.path.join(CSRC, s), "-o", os.path.join(OBJ, s + ".o")])
    for s in HIP_SRCS:
        jobs.append([HIPCC, *HIPFLAGS, "-I", os.path.join(HERE, "..", "include"),
                     "-c", os.path.join(CSRC, s), "-o", os.path.join(OBJ, s + ".o")])
    jobs.append([HIPCC, *HIPFLAGS, "-I", os.path.join(HERE, "..", "include"),
                 "-c", os.path.join(CSRC, MICRO_SRC), "-o", os.path.join(OBJ, MICRO_SRC + ".o")])
    with cf.ThreadPoolExecutor(max_workers=min(8, len(jobs))) as ex:
        for r in ex.map(_run, jobs):
            if verbose and (r.stdout or r.stderr):
                print(r.stdout, r.stderr, file=sys.stderr)
    objs = [os.path.join(OBJ, s + ".o") for s in HOST_SRCS + HIP_SRCS]
    tmp = LIB + ".tmp"
    _run([HIPCC, "-shared", f"--offload-arch={ARCH}", "-o", tmp, *objs])
    os.replace(tmp, LIB)
    tmp = MICRO_LIB + ".tmp"
    _run([HIPCC, "-shared", f"--offload-arch={ARCH}", "-o", tmp, os.path.join(OBJ, MICRO_SRC + ".o")])
    os.replace(tmp, MICRO_LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
