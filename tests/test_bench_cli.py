"""bench.py's command line, checked without a GPU: more than one GPU is
refused before anything touches a device, and the profiling modes exist."""
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
    assert r.stdout == ""


def test_profiling_modes_are_listed():
    r = _run("--help")
    assert r.returncode == 0
    for flag in ("--steps", "--warmup", "--only-main", "--only-zoom-to", "--only-fwd-bwd", "--only-u8", "--copy-calib",
                 "--no-cpu"):
        assert flag in r.stdout, flag
