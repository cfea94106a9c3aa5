"""The host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

paper_2411_00546_amd.build.build_host_check compiles the engine, server and tuner
sources with both sanitizers on their host pass and links them with the kernel objects
and tests/host/host_check.cpp, which drives every entry point that needs no GPU: the
partition of Section 4.2 against an independent restatement (cores tile the grid, boxes
are the clipped extensions, tile sizes) on random grids, the workspace sizes used for
serving admission, the validation of problems and options, the argument checks and
missing-device errors of the calls that need a GPU, and per-thread error messages.
"""
import os
import shutil
import subprocess

import pytest


def _hipcc():
    return shutil.which("hipcc") or ("/opt/rocm/bin/hipcc" if os.path.exists("/opt/rocm/bin/hipcc") else None)


@pytest.mark.skipif(_hipcc() is None, reason="hipcc not available")
def test_host_code_under_asan_and_ubsan():
    from paper_2411_00546_amd import build
    exe = build.build_host_check()
    env = dict(os.environ)
    env["ASAN_OPTIONS"] = "detect_leaks=1:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    # no device for this program, whatever the machine has
    env["HIP_VISIBLE_DEVICES"] = "-1"
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)
    out = r.stdout + r.stderr
    assert "AddressSanitizer" not in out and "LeakSanitizer" not in out, out[-4000:]
    assert "runtime error:" not in out, out[-4000:]
    assert r.returncode == 0, out[-4000:]
    assert "0 failed" in r.stdout, out[-4000:]
