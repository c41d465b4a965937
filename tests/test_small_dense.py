"""The host-side dense routines of the eigensolver (small_dense.h), built with
g++ on the CPU and checked on seeded random Hermitian and positive definite
matrices of orders 1 to 64 (see tests/small_dense_check.cpp)."""
import os
import shutil
import subprocess
import tempfile

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_0910_2918_amd", "csrc")


@pytest.mark.skipif(shutil.which("g++") is None, reason="no host C++ compiler")
def test_jacobi_and_cholesky():
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "small_dense_check")
        subprocess.run(["g++", "-O2", "-std=c++17", "-I", CSRC, "-o", exe,
                        os.path.join(HERE, "small_dense_check.cpp")], check=True)
        out = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stdout + out.stderr
