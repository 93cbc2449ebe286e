"""bench.py's command line without a GPU: it measures one GPU and refuses more
(a run on several GPUs is a design in the documentation, not a measurement)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300, cwd=ROOT)
    assert r.returncode == 2, r
    assert "one GPU only" in r.stderr
    assert r.stdout == ""  # no JSON line for a configuration that was not measured
