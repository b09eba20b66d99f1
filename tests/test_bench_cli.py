"""bench.py's command line, checked without a GPU: more than one GPU is refused with a
message before anything touches a device, and --help lists the single-workload flag."""
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
    assert "exactly one GPU" in r.stderr and "requested 2" in r.stderr
    assert r.stdout == ""  # no JSON line


def test_help_lists_single_workload_flag():
    r = _run("--help")
    assert r.returncode == 0
    for flag in ("--steps", "--warmup", "--gpus", "--only", "--no-cpu-baseline"):
        assert flag in r.stdout
