"""The even-odd (symmetry) form of the 1D contractions used by the HIP kernels equals the
direct sums: the kernel header is compiled for the host with g++ and run on the CPU."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1910_03032_amd", "csrc")
# host-only build (g++, no GPU code): address and undefined-behaviour sanitizers, any
# report fails the run
SANITIZE = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer"]
SANITIZE_ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:exitcode=23",
                    UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_even_odd_contractions_match_direct_sums(tmp_path):
    exe = str(tmp_path / "eo_check")
    src = os.path.join(ROOT, "tests", "eo_check.cpp")
    r = subprocess.run(["g++", "-std=c++17", "-O1", "-g", "-Wno-unknown-pragmas", *SANITIZE, "-I", CSRC,
                        src, "-o", exe], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    r = subprocess.run([exe], capture_output=True, text=True, env=SANITIZE_ENV)
    assert "Sanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr
    assert "FAIL" not in r.stdout, r.stdout
    assert r.returncode == 0, r.stdout
