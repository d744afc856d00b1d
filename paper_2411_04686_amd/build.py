"""Build ``libgse.so`` (all HIP sources under ``csrc/``) for gfx950 with hipcc.

Each source is compiled to its own object in parallel (every object carries
its own device code), then hipcc links the shared library.
"""
from __future__ import annotations

import concurrent.futures as cf
import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libgse.so")
OBJ = os.path.join(HERE, "_build")
ARCH = os.environ.get("GSE_OFFLOAD_ARCH", "gfx950")


def sources():
    return sorted(glob.glob(os.path.join(HERE, "csrc", "*.hip")))


def _hipcc():
    return os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc")


def flags():
    return [f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
            # keep the compiler from emitting packed FP32 instructions
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wall", "-Wno-unused-function",
            "-I", os.path.join(ROOT, "include"), "-I", os.path.join(HERE, "csrc")]


def command(out: str = LIB):
    """One-shot command line (all sources, one hipcc call)."""
    return [_hipcc()] + flags() + ["-shared", "-o", out] + sources()


def _compile(src: str) -> str:
    obj = os.path.join(OBJ, os.path.basename(src) + ".o")
    subprocess.run([_hipcc()] + flags() + ["-c", "-o", obj, src], check=True, cwd=HERE)
    return obj


def build(out: str = LIB) -> str:
    os.makedirs(OBJ, exist_ok=True)
    srcs = sources()
    jobs = max(1, min(len(srcs), int(os.environ.get("MAX_JOBS", os.cpu_count() or 1))))
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = out + ".tmp"
    subprocess.run([_hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs,
                   check=True, cwd=HERE)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(sys.argv[1] if len(sys.argv) > 1 else LIB))
