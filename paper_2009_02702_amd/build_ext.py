"""Compile libmg.so (host C++ builder + HIP kernels for gfx950), in-tree.

    python -m paper_2009_02702_amd.build_ext

Host C++ goes through g++; the HIP translation unit through hipcc for
gfx950 only, with packed fp32 instructions disabled; the shared library is
linked by hipcc and written next to this file.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
OUT = os.path.join(HERE, "libmg.so")
OBJ = os.path.join(HERE, "_build")

HOST_SOURCES = ["builder.cpp", "factorize.cpp", "stream.cpp", "runs.cpp", "api.cpp"]
HIP_SOURCES = ["kernels.hip"]
ARCH = "gfx950"


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        raise RuntimeError("build step failed:\n  %s\n%s" % (" ".join(cmd), r.stdout))
    return r.stdout


def build(verbose: bool = False) -> str:
    os.makedirs(OBJ, exist_ok=True)
    jobs = []
    objs = []
    for src in HOST_SOURCES:
        o = os.path.join(OBJ, src + ".o")
        objs.append(o)
        jobs.append(["g++", "-O3", "-std=c++17", "-fPIC", "-Wall", "-Wextra", "-Wno-unused-parameter",
                     "-I", INCLUDE, "-I", CSRC, "-c", os.path.join(CSRC, src), "-o", o])
    for src in HIP_SOURCES:
        o = os.path.join(OBJ, src + ".o")
        objs.append(o)
        jobs.append(["hipcc", "--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC",
                     "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                     "-I", INCLUDE, "-I", CSRC, "-c", os.path.join(CSRC, src), "-o", o])
    with ThreadPoolExecutor(max_workers=len(jobs)) as ex:
        logs = list(ex.map(_run, jobs))
    if verbose:
        for lg in logs:
            if lg.strip():
                print(lg)
    tmp = OUT + ".tmp%d" % os.getpid()
    _run(["hipcc", "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs + ["-lpthread"])
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
