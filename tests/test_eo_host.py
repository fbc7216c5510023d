"""The even-odd (symmetry) form of the 1D contractions used by the HIP kernels equals the
direct sums: the kernel header is compiled for the host with g++ and run on the CPU."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1910_03032_amd", "csrc")


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_even_odd_contractions_match_direct_sums(tmp_path):
    exe = str(tmp_path / "eo_check")
    src = os.path.join(ROOT, "tests", "eo_check.cpp")
    r = subprocess.run(["g++", "-std=c++17", "-O1", "-Wno-unknown-pragmas", "-I", CSRC, src, "-o", exe],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    r = subprocess.run([exe], capture_output=True, text=True)
    assert "FAIL" not in r.stdout, r.stdout
    assert r.returncode == 0, r.stdout
