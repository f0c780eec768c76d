"""Build libbgcr.so (HIP kernels + host driver + C ABI) in-tree for gfx950.

    python -m paper_1604_01713_amd.build

Every HIP translation unit is compiled with packed-FP32 instructions disabled
(`-Xclang -target-feature -Xclang -packed-fp32-ops`).
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libbgcr.so")
BUILD = os.path.join(ROOT, "_build")
ARCH = os.environ.get("BGCR_OFFLOAD_ARCH", "gfx950")

HIP_FLAGS = ["-O3", "-fPIC", "-std=c++17", f"--offload-arch={ARCH}", "-fcx-limited-range",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-I", INCLUDE, "-I", CSRC]
# complex products without the NaN-recovery path (operands are finite and checked)
CXX_FLAGS = ["-O3", "-fPIC", "-std=c++17", "-march=x86-64-v3", "-fcx-limited-range", "-fopenmp", "-I", INCLUDE, "-I", CSRC]

HIP_SOURCES = ["kernels.hip", "kernels_mfma_f64.hip", "kernels_mfma_f32.hip", "kernels_mfma_bf16.hip",
               "kernels_mfma_c128.hip", "ilu.hip", "stream_probe.hip",
               "solver.cpp"]
CXX_SOURCES = ["dense.cpp"]


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(l for l in r.stdout.splitlines()
                    if "packed-fp32-ops" not in l and "unknown target feature" not in l
                    and l.strip() != "1 warning generated.")
    if r.returncode != 0:
        raise RuntimeError(f"build step failed: {' '.join(cmd)}\n{out}")
    return out


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    jobs = []
    objs = []
    for s in HIP_SOURCES:
        o = os.path.join(BUILD, s + ".o")
        objs.append(o)
        jobs.append(["hipcc", "-x", "hip", *HIP_FLAGS, "-c", os.path.join(CSRC, s), "-o", o])
    for s in CXX_SOURCES:
        o = os.path.join(BUILD, s + ".o")
        objs.append(o)
        jobs.append(["g++", *CXX_FLAGS, "-c", os.path.join(CSRC, s), "-o", o])
    with cf.ThreadPoolExecutor(max_workers=min(6, len(jobs))) as ex:
        outs = list(ex.map(_run, jobs))
    if verbose:
        for o in outs:
            if o.strip():
                print(o)
    tmp = LIB + ".tmp"
    _run(["hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs, "-lgomp"])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
