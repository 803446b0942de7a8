"""Build step of the CPU oracle (test infrastructure): gcc, OpenMP, no FP
contraction, no fast-math, SSE arithmetic (no x87 excess precision)."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "mpir_oracle.c")
OUT = os.path.join(HERE, "libmpir_oracle.so")

CFLAGS = ["-O3", "-std=c11", "-fPIC", "-shared", "-fopenmp",
          "-ffp-contract=off", "-fno-fast-math", "-fexcess-precision=standard",
          "-mfpmath=sse", "-msse2", "-Wall", "-Wextra", "-Wno-unused-parameter"]


def build_oracle(force: bool = True) -> str:
    if not force and os.path.exists(OUT) and os.path.getmtime(OUT) >= os.path.getmtime(SRC):
        return OUT
    tmp = OUT + ".tmp"
    cmd = ["gcc", *CFLAGS, SRC, "-o", tmp, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build_oracle(force=True))
