"""Host bounds check of the field solver's index arithmetic: tests/index_bounds.cpp compiles the
header the kernels use (paper_1410_0986_amd/csrc/krylov_index.h) with the host C++ compiler and
checks every partial-sum slot, flush row map, small-block element and block -> (system, chunk)
map over all deflation dimensions, cycle and Lanczos lengths, basis counts and block orders."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "index_bounds.cpp")
INC = os.path.join(ROOT, "paper_1410_0986_amd", "csrc")


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs a host C++ compiler")
def test_solver_index_arithmetic_in_bounds(tmp_path):
    exe = tmp_path / "index_bounds"
    # -fsanitize: any out-of-range vector access or signed overflow in the check itself fails too
    subprocess.run(["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                    "-I", INC, SRC, "-o", str(exe)], check=True, capture_output=True, text=True)
    res = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300)
    assert res.returncode == 0, res.stdout + res.stderr
    assert res.stdout.startswith("ok "), res.stdout
    assert int(res.stdout.split()[1]) > 1_000_000
