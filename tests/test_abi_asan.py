"""The C ABI checks (tests/test_abi.py) once more against a build of the
library whose host code -- argument validation, overlap sweeps, workspace
layout, status strings -- runs under AddressSanitizer.  CPU only: nothing is
launched (validation fails before any device work, as in test_abi.py)."""
import os
import subprocess
import sys

import pytest

from paper_2312_00229_amd import build

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.slow
def test_abi_checks_under_address_sanitizer(tmp_path):
    lib = build.build_asan(str(tmp_path))
    nm = subprocess.run(["nm", "-D", lib], capture_output=True, text=True, check=True).stdout
    assert "__asan_report" in nm          # the host code is instrumented
    rt = build.asan_runtime()
    assert os.path.exists(rt), rt
    env = dict(os.environ, LD_PRELOAD=rt, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0", WENO_ZOOM_LIB=lib)
    res = subprocess.run([sys.executable, "-m", "pytest", os.path.join("tests", "test_abi.py"), "-q", "-p",
                          "no:cacheprovider", "-m", "not gpu"], cwd=ROOT, env=env, capture_output=True, text=True,
                         timeout=600)
    assert res.returncode == 0, res.stdout[-3000:] + res.stderr[-3000:]
    assert "ERROR: AddressSanitizer" not in res.stdout + res.stderr
    assert " passed" in res.stdout
