"""bench.py's command-line contract on the CPU: more than one GPU is refused
with a message (the benchmark measures one device), and the help lists the
workloads."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True, text=True,
                          timeout=120)


def test_more_than_one_gpu_is_refused():
    r = _run("--gpus", "2")
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_help_lists_the_workloads():
    r = _run("--help")
    assert r.returncode == 0
    for w in ("lfr_1m", "lfr_20m", "sbm_2k", "batch", "served", "robustness"):
        assert w in r.stdout
