"""bench.py's command line on a host without a GPU: it measures one GPU only, and a run
asked for more exits before touching a device, saying so."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    out = r.stdout + r.stderr
    assert r.returncode != 0
    assert "one GPU only" in out, out
    assert '"metric"' not in out  # no measurement line
