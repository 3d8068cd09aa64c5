"""Build the C part of the oracle (test infrastructure): ``oracle/_rays_mirror32.so``.

gcc, -O2, -ffp-contract=off and no fast-math, so each FP32 operation in the C source is
one correctly rounded binary32 operation (x86-64 SSE2 scalar arithmetic).
"""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "rays_mirror32.c")
LIB = os.path.join(HERE, "_rays_mirror32.so")


def build(force: bool = True) -> str:
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= os.path.getmtime(SRC):
        return LIB
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
           "-shared", "-pthread", SRC, "-o", tmp, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build())
