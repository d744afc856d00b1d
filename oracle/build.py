"""Compile the CPU oracle into ``oracle/libgse_oracle.so`` (plain gcc, C99)."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "gse_oracle.c")
LIB = os.path.join(HERE, "libgse_oracle.so")

CMD = ["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
       "-shared", "-Wall", "-Wextra", "-o", LIB, SRC, "-lm"]


def build() -> str:
    subprocess.run(CMD, check=True, cwd=HERE)
    return LIB


if __name__ == "__main__":
    print(build())
