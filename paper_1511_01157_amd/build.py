"""Build the gfx950 HIP library ``paper_1511_01157_amd/libmorse.so`` with hipcc.

Flags: -O3 for gfx950 only; -ffp-contract=off so the binary32 arithmetic of the ray
and sampling kernels is exactly the written operation sequence (no fused
multiply-add contraction); packed FP32 instructions disabled; IEEE division and
square root (hipcc's default correctly rounded FP32 divide/sqrt).
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libmorse.so")
SOURCES = ["maps.hip", "search.hip", "refine.hip", "stack.hip", "lines.hip", "simplex.hip",
           "fsmag.hip", "api_ctx.hip", "api_maps.hip", "api_lines.hip", "api_search.hip",
           "api_refine.hip", "api_fsmag.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-ffp-contract=off",
         "-fhip-fp32-correctly-rounded-divide-sqrt",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-function", "-Wno-unused-parameter"]


def build(verbose: bool = False) -> str:
    objs = []
    for src in SOURCES:
        obj = os.path.join(CSRC, src.replace(".hip", ".o"))
        cmd = [HIPCC, *FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        objs.append(obj)
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    for o in objs:
        os.remove(o)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
