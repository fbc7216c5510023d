"""Host-side behaviour of bench.py that needs no GPU: the one-GPU guard and the traffic
bookkeeping (measured HBM bytes are reported only for the kernel sources they were
taken with)."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    out = json.loads(r.stdout.strip().splitlines()[-1])
    assert out["n_gpus"] == 2 and "one GPU" in out["error"]


def test_kernel_hash_ignores_comments_but_not_code():
    sys.path.insert(0, ROOT)
    import bench
    src = {f: "int a; // note\n\nint b;\n" for f in bench.KERNEL_SOURCES}
    h0 = bench.kernel_source_hash(read=lambda f: src[f])
    src2 = {f: "int a; // other note\nint b;  \n" for f in bench.KERNEL_SOURCES}
    assert bench.kernel_source_hash(read=lambda f: src2[f]) == h0
    src3 = dict(src)
    src3[bench.KERNEL_SOURCES[0]] = "int a;\nint c;\n"
    assert bench.kernel_source_hash(read=lambda f: src3[f]) != h0
