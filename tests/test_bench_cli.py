"""bench.py's command line on the CPU: the parser builds (every workload
name is offered) and a request for more than one GPU is refused with a
message before any device work."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args],
                          cwd=ROOT, stdout=subprocess.PIPE, stderr=subprocess.PIPE,
                          text=True, timeout=300)


def test_help_lists_workloads():
    r = _bench("--help")
    assert r.returncode == 0, r.stderr
    for name in ("plain", "generation", "uneven", "precision", "serving", "reward"):
        assert name in r.stdout


def test_more_than_one_gpu_is_refused():
    r = _bench("--gpus", "2")
    assert r.returncode != 0
    assert "one GPU" in r.stderr or "1 GPU" in r.stderr or "single" in r.stderr, r.stderr
