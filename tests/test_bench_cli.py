"""bench.py's command line on the host: more than one GPU is refused with a message
before anything touches a device (the library is single-GPU)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=60)
    assert p.returncode == 2
    assert "one GPU only" in p.stderr
    assert p.stdout == ""
