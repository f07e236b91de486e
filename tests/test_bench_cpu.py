"""Host-side checks of the benchmark's command line (no GPU needed)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True, text=True,
                          timeout=120, cwd=ROOT)


def test_more_than_one_gpu_is_refused_with_a_message():
    r = _run("--gpus", "2")
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_help_lists_the_workloads_and_formulations():
    r = _run("--help")
    assert r.returncode == 0
    for w in ("bem2m", "batch64", "adjoint1m", "shell30m", "exterior_p1", "--retune", "--summarize-profile",
              "--summarize-counters"):
        assert w in r.stdout
