"""Host logic of the library's mesh preparation (map validation, map encoding and the
assembly plan): plan.cpp is compiled with g++ together with a checker that replays the
assembly list with integer element contributions against a direct scatter-add."""
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
def test_assembly_plan_replays_scatter_add(tmp_path):
    exe = str(tmp_path / "plan_check")
    r = subprocess.run(["g++", "-std=c++17", "-O1", "-g", "-Wall", *SANITIZE, "-I", CSRC, "-I",
                        os.path.join(ROOT, "include"), os.path.join(ROOT, "tests", "plan_check.cpp"),
                        os.path.join(CSRC, "plan.cpp"), "-o", exe], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    r = subprocess.run([exe], capture_output=True, text=True, env=SANITIZE_ENV)
    assert "Sanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr
    print(r.stdout)
    assert "FAIL" not in r.stdout, r.stdout
    assert r.returncode == 0, r.stdout
