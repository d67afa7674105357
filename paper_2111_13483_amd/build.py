"""Build libhschur.so (gfx950) in-tree.

Host integer phases are compiled with g++ without floating-point
contraction; the HIP kernels and the C-ABI with hipcc for gfx950 (packed
FP32 instructions disabled).
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libhschur.so")
BENCH_EXE = os.path.join(HERE, "hs_bench")
BUILD = os.path.join(HERE, "_build")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")
HIPCC = os.path.join(ROCM, "bin", "hipcc")

HIP_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-fPIC", "-std=c++17",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-result", "-I" + INCLUDE,
]
GXX_FLAGS = ["-O2", "-fPIC", "-std=c++17", "-ffp-contract=off", "-Wall"]

HIP_SOURCES = ["kernels_build.hip", "kernels_setup.hip", "kernels_elim.hip", "kernels_solve.hip", "kernels_sweep.hip", "abi.cpp"]
CXX_SOURCES = ["plan.cpp"]


def _run(cmd):
    p = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if p.returncode != 0:
        raise RuntimeError("build failed: %s\n%s" % (" ".join(cmd), p.stdout))
    return p.stdout


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    jobs = []
    objs = []
    for src in HIP_SOURCES:
        obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
        cmd = [HIPCC] + HIP_FLAGS + ["-c", os.path.join(CSRC, src), "-o", obj]
        if src.endswith(".cpp"):
            cmd = [HIPCC] + HIP_FLAGS + ["-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
        jobs.append(cmd)
        objs.append(obj)
    for src in CXX_SOURCES:
        obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
        jobs.append(["g++"] + GXX_FLAGS + ["-c", os.path.join(CSRC, src), "-o", obj])
        objs.append(obj)
    with ThreadPoolExecutor(max_workers=min(8, len(jobs))) as ex:
        outs = list(ex.map(_run, jobs))
    if verbose:
        for o in outs:
            if o.strip():
                print(o)
    tmp = OUT + ".tmp"
    _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs +
         ["-L" + os.path.join(ROCM, "lib"), "-lrocblas", "-Wl,-rpath," + os.path.join(ROCM, "lib")])
    os.replace(tmp, OUT)
    # C-ABI-only driver for hardware-counter runs (links the library by rpath)
    tmp = BENCH_EXE + ".tmp"
    _run([HIPCC, "--offload-arch=gfx950", "-O2", "-std=c++17", "-I" + INCLUDE, os.path.join(CSRC, "hs_bench.cpp"),
          "-o", tmp, "-L" + HERE, "-lhschur", "-Wl,-rpath,$ORIGIN"])
    os.replace(tmp, BENCH_EXE)
    return OUT


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
