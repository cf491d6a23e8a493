"""bench.py's command line, without a GPU: more than one GPU is refused with
a message (exit status 2) before anything touches a device, and the profiling
legs are offered."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True, text=True,
                          timeout=120, cwd=ROOT)


def test_bench_refuses_more_than_one_gpu():
    r = run("--gpus", "2")
    assert r.returncode == 2
    assert "single MI355X" in r.stderr or "one GPU" in r.stderr
    assert r.stdout == ""


def test_bench_help_lists_the_legs():
    r = run("--help")
    assert r.returncode == 0
    for leg in ("learned_step", "bank", "windows", "--dense", "--copy-calibration"):
        assert leg in r.stdout
