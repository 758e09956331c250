"""The library's host-only calls (validation, create-time tables, workspace
sizing, the hookstep subproblem, the Hessenberg eigenvalue routine, the
tile-cache reader and writer with malformed files) run clean under
AddressSanitizer (with leak detection) and UndefinedBehaviorSanitizer:
tests/sanitize/build_and_run.sh builds the sources with host-side
sanitizers and runs tests/sanitize/host_calls.cpp.  No GPU is used."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.mark.slow
@pytest.mark.skipif(not os.path.exists("/opt/rocm/bin/hipcc"), reason="needs hipcc")
def test_host_calls_clean_under_asan_and_ubsan(tmp_path):
    script = os.path.join(HERE, "sanitize", "build_and_run.sh")
    r = subprocess.run(["bash", script, str(tmp_path)], capture_output=True, text=True, timeout=900)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "host calls: 0 expectation failures" in out
    assert "ERROR: AddressSanitizer" not in out and "runtime error" not in out
    shutil.rmtree(tmp_path, ignore_errors=True)
