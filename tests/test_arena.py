"""Host logic of the solver server: the first-fit arena allocator and the
request layout (csrc/arena.h), compiled with g++ and checked against an
explicit model (no GPU)."""
import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_arena_allocator_and_request_layout(tmp_path):
    exe = tmp_path / "arena_check"
    subprocess.run(["g++", "-std=c++17", "-O1", "-Wall", "-Wextra",
                    "-I", os.path.join(ROOT, "paper_2411_04686_amd", "csrc"),
                    os.path.join(ROOT, "tests", "native", "arena_check.cpp"), "-o", str(exe)],
                   check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0 and out.stdout.strip().endswith("ok"), out.stdout + out.stderr
