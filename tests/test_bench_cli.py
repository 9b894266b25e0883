"""The benchmark's command line on a machine without a GPU: a request for
more than one GPU ends at once with a message and a non-zero status, before
any device is touched (the build targets one GPU)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300, cwd=ROOT)
    assert r.returncode != 0
    msg = (r.stdout + r.stderr).lower()
    assert "one gpu" in msg or "1 gpu" in msg or "single gpu" in msg, msg[-500:]
    assert '"metric"' not in r.stdout
