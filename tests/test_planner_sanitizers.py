"""The host planner under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only):
tests/planner_sanitize.cpp plans every length 1..3000 in every kind and dtype, a set of
multi-dimensional shapes and a 3000-length ragged schedule; any sanitizer report or
planning failure fails the test."""
import os
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.mark.slow
def test_planner_clean_under_sanitizers(tmp_path):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    exe = str(tmp_path / "planner_sanitize")
    # sanitizers on the host pass only
    cmd = [HIPCC, "-O1", "-g", "-std=c++17", "--offload-arch=gfx950", "-Xarch_host", "-fsanitize=address",
           "-Xarch_host", "-fsanitize=undefined", "-I", os.path.join(ROOT, "include"),
           "-I", os.path.join(ROOT, "paper_1707_03776_amd", "csrc"), os.path.join(HERE, "planner_sanitize.cpp"),
           os.path.join(ROOT, "paper_1707_03776_amd", "csrc", "planner.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=900)
    assert r.returncode == 0, r.stderr[-3000:]
    env = dict(os.environ, UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", ASAN_OPTIONS="detect_leaks=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=900, env=env)
    assert r.returncode == 0 and "runtime error" not in r.stderr, (r.stdout[-2000:], r.stderr[-3000:])
    assert "fails=0" in r.stdout and "ragged st=0" in r.stdout
