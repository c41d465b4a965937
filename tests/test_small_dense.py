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
@pytest.mark.parametrize("flags", [["-O2"], ["-O1", "-g", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
                                            "-fno-sanitize-recover=all"]], ids=["plain", "asan_ubsan"])
def test_jacobi_and_cholesky(flags):
    """Built plain, and with AddressSanitizer and UndefinedBehaviorSanitizer
    (any report aborts the run), on the host only."""
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "small_dense_check")
        subprocess.run(["g++", *flags, "-std=c++17", "-I", CSRC, "-o", exe,
                        os.path.join(HERE, "small_dense_check.cpp")], check=True)
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1", UBSAN_OPTIONS="halt_on_error=1")
        out = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert out.returncode == 0, out.stdout + out.stderr
