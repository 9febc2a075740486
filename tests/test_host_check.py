"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer
(CPU): a sanitizer build of libmpid plus a C++ checker of its ABI -- workspace
sizing over a grid of shapes and options, and every entry point's argument
validation (all of which return before any device call)."""
import os
import shutil
import subprocess

import pytest


@pytest.mark.slow
def test_host_code_clean_under_sanitizers(tmp_path):
    if not os.path.exists(os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")):
        pytest.skip("hipcc not available")
    from paper_2012_00706_amd.build import build_host_check
    exe = build_host_check(str(tmp_path / "host_check"))
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    res = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    out = res.stdout + res.stderr
    assert res.returncode == 0, out[-4000:]
    assert "host checks: 0 failed" in out
    assert "AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
    shutil.rmtree(tmp_path / "host_check", ignore_errors=True)
