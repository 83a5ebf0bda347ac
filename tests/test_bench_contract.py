"""bench.py's command-line contract on the CPU: a request for more than one
GPU ends with a JSON message and a non-zero status before any device work."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


def test_kernel_source_fingerprint_is_stable():
    sys.path.insert(0, ROOT)
    import bench
    a = bench.kernel_source_fingerprint()
    b = bench.kernel_source_fingerprint()
    assert a == b and len(a) == 16
