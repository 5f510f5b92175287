"""bench.py's command line on the CPU: a request for more than one GPU is
refused with a message before anything touches a device."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    for n in (2, 8):
        p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", str(n)],
                           capture_output=True, text=True, timeout=60, cwd=ROOT)
        assert p.returncode == 2, (n, p.returncode, p.stderr)
        assert "one GPU" in p.stderr and p.stdout == "", (n, p.stderr, p.stdout)
