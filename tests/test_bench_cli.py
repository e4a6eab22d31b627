"""CPU checks of bench.py's command line: it measures one GPU only and
refuses requests it cannot honour before touching a device."""
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


def test_oracle_to_tolerance_only_for_small_configs():
    r = _run("--cpu-to-tol")
    assert r.returncode == 2 and "tiny and medium" in r.stderr


def test_help_lists_the_patterns():
    r = _run("--help")
    assert r.returncode == 0
    for p in ("batched", "adjoint", "warmstart", "congested", "transit"):
        assert p in r.stdout
