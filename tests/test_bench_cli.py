"""bench.py's command-line contract on the host (no GPU is touched): more
than one GPU is refused with a message, and the FP32 / mixed site
arithmetic is accepted only for the closed form."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args],
                          capture_output=True, text=True, timeout=120)


def test_more_than_one_gpu_is_refused():
    r = _run("--gpus", "2")
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_reduced_arithmetic_needs_the_closed_form():
    for arith in ("mixed", "fp32"):
        r = _run("--arith", arith)
        assert r.returncode == 2
        assert "closed form" in r.stderr
        r = _run("--arith", arith, "--only", "newton")
        assert r.returncode == 2
