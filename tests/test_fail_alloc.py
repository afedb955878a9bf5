"""Allocation-failure injection (MIFFT_TEST_FAIL_ALLOC=k) through the C ABI.

CPU: tests/fail_alloc_host.cpp links the library's host sources (api.cpp, planner.cpp)
against host stand-ins for the HIP runtime (tests/fake_hip.cpp) under AddressSanitizer
and LeakSanitizer; every k-th device allocation of a c2c, Bluestein, real, DCT and
ragged plan creation is made to fail, and each must return NULL with FFT_ERR_ALLOC and
leave no allocation, graph or host memory behind.

GPU: the same hook against the real runtime: creations fail cleanly and the device's
free memory returns to where it was."""
import os
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_1707_03776_amd", "csrc")


@pytest.mark.slow
def test_fail_alloc_host_under_asan(tmp_path):
    if not os.path.isdir("/opt/rocm/include/hip"):
        pytest.skip("HIP headers not available")
    exe = str(tmp_path / "fail_alloc_host")
    # host code only, built by g++ (no device code is involved)
    cmd = ["g++", "-O1", "-g", "-std=c++17", "-fsanitize=address", "-fsanitize=undefined",
           "-D__HIP_PLATFORM_AMD__", "-I", "/opt/rocm/include", "-I", os.path.join(ROOT, "include"), "-I", CSRC,
           os.path.join(HERE, "fail_alloc_host.cpp"), os.path.join(HERE, "fake_hip.cpp"),
           os.path.join(CSRC, "api.cpp"), os.path.join(CSRC, "planner.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-3000:]
    env = dict(os.environ, UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", ASAN_OPTIONS="detect_leaks=1")
    env.pop("MIFFT_TEST_FAIL_ALLOC", None)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)
    assert r.returncode == 0 and "runtime error" not in r.stderr, (r.stdout[-3000:], r.stderr[-3000:])
    assert "failures=0" in r.stdout
    for name in ("c2c 2^20", "bluestein", "r2c", "dct2", "ragged"):
        assert name in r.stdout


@pytest.mark.gpu
def test_fail_alloc_on_gpu(gpu_available, monkeypatch):
    import torch

    import paper_1707_03776_amd as mf
    cases = [
        lambda: mf.Plan((1 << 16,), 4, mf.FFT_C2C, mf.FFT_FORWARD, mf.FFT_F32),
        lambda: mf.Plan((4099,), 2, mf.FFT_C2C, mf.FFT_INVERSE, mf.FFT_F64),
        lambda: mf.Laplacian((32, 32, 32), 1, (1.0, 1.0, 1.0), mf.FFT_F32),
    ]
    def ragged():
        return mf.fft_plan_create_many([64, 97, 4096], [0, 64, 161], [0, 64, 161], mf.FFT_C2C, mf.FFT_FORWARD,
                                       mf.FFT_F32)
    # load every code object and runtime pool first (the first use of the library on a
    # device maps its kernels and static arrays), so the free-memory comparison below
    # sees only what the creations themselves allocate
    monkeypatch.delenv("MIFFT_TEST_FAIL_ALLOC", raising=False)
    for make in cases:
        make().close()
    mf.fft_plan_destroy(ragged())
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    for make in cases:
        for k in range(1, 40):
            monkeypatch.setenv("MIFFT_TEST_FAIL_ALLOC", str(k))
            try:
                obj = make()
            except mf.MifftError as e:
                assert e.status == mf.FFT_ERR_ALLOC, (k, e)
                continue
            obj.close()  # k beyond this creation's allocations: it succeeded
            break
        else:
            pytest.fail("creation kept failing")
    for k in range(1, 40):
        monkeypatch.setenv("MIFFT_TEST_FAIL_ALLOC", str(k))
        try:
            plan = ragged()
        except mf.MifftError as e:
            assert e.status == mf.FFT_ERR_ALLOC, (k, e)
            continue
        mf.fft_plan_destroy(plan)
        break
    monkeypatch.delenv("MIFFT_TEST_FAIL_ALLOC")
    torch.cuda.synchronize()
    assert torch.cuda.mem_get_info()[0] == free0
