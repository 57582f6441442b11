"""bench.py's command line on a host without a GPU: a request for more than
one GPU is refused with a JSON message and exit status 2 before any device
is touched."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(*args):
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True, text=True,
                       timeout=300, cwd=ROOT)
    return p.returncode, p.stdout.strip().splitlines()


def test_more_than_one_gpu_is_refused():
    rc, out = _run("--gpus", "2")
    assert rc == 2
    msg = json.loads(out[-1])
    assert "one GPU" in msg["error"]
