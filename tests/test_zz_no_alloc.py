"""fft_execute_noalloc (the allocation-free entry point, tables and scratch in the
library's static per-GPU array) against fft_plan_create + fft_execute on the same
inputs: bitwise equal outputs (the same kernels run with the same arguments), and both
within the oracle bounds.  Several calls in a row, later ones smaller than earlier
ones, so a call that relied on anything left in the array by the previous one, or on
the array starting at zero, would show."""
import numpy as np
import pytest

import oracle
import paper_1707_03776_amd as mf
from gpu_util import TOL, assert_parity, cplx_input, real_input

pytestmark = pytest.mark.gpu

F32, F64 = mf.FFT_F32, mf.FFT_F64


@pytest.fixture(autouse=True, scope="module")
def _gpu(gpu_available):
    return gpu_available


def _bits(t):
    import torch
    return torch.view_as_real(t).view(torch.uint8) if t.is_complex() else t.view(torch.uint8)


def _case(dims, batch, kind, direction, dtype, seed, inplace=False):
    import torch
    rng = np.random.default_rng(seed)
    real_in = kind == mf.FFT_R2C
    x = real_input(rng, (batch,) + dims, dtype) if real_in else cplx_input(rng, (batch,) + dims, dtype)
    print(f"noalloc dims={dims} batch={batch} kind={kind} dir={direction} dtype={dtype} inplace={inplace}",
          flush=True)
    xd = torch.from_numpy(x).cuda()
    plan = mf.Plan(dims, batch, kind, direction, dtype)
    try:
        ref_dev = plan(xd)
    finally:
        plan.close()
    stream = torch.cuda.current_stream().cuda_stream
    if inplace:
        y = xd.clone()
        mf.fft_execute_noalloc(len(dims), dims, batch, kind, direction, dtype, y.data_ptr(), y.data_ptr(), stream)
    else:
        y = torch.empty_like(ref_dev)
        mf.fft_execute_noalloc(len(dims), dims, batch, kind, direction, dtype, xd.data_ptr(), y.data_ptr(), stream)
    torch.cuda.synchronize()
    assert torch.equal(_bits(y), _bits(ref_dev))
    if kind == mf.FFT_C2C:
        ref = oracle.c2c(x, dims, inverse=direction == mf.FFT_INVERSE)
    else:
        ref = oracle.r2c(x, dims)
    assert_parity(y.cpu().numpy(), ref, batch, TOL[dtype], int(np.prod(dims)), "noalloc")


def test_noalloc_matches_fft_execute_calls_in_a_row():
    # 256 MiB of complex64 scratch for one chunk: runs in chunks inside the 64 MiB array
    _case((1 << 20,), 32, mf.FFT_C2C, mf.FFT_FORWARD, F32, 1)
    # smaller: two passes, inverse, complex128
    _case((1 << 16,), 8, mf.FFT_C2C, mf.FFT_INVERSE, F64, 2)
    # smaller still: one pass, in place
    _case((4096,), 3, mf.FFT_C2C, mf.FFT_FORWARD, F32, 3, inplace=True)
    # a real multi-dimensional transform (staging scratch)
    _case((32, 24, 40), 2, mf.FFT_R2C, mf.FFT_FORWARD, F32, 4)
    # a staged real transform (its twist in the last pass; tables in the static array)
    _case((1 << 18,), 4, mf.FFT_R2C, mf.FFT_FORWARD, F32, 5)


def test_noalloc_rejects_what_it_cannot_hold():
    import torch
    x = torch.zeros(4099 * 2, dtype=torch.complex64, device="cuda")
    y = torch.empty_like(x)
    with pytest.raises(mf.MifftError) as e:
        mf.fft_execute_noalloc(1, (4099,), 2, mf.FFT_C2C, mf.FFT_FORWARD, F32, x.data_ptr(), y.data_ptr(), 0)
    assert e.value.status == mf.FFT_ERR_UNSUPPORTED
    # one 2^24-point transform needs 128 MiB of scratch and cannot be chunked further
    x = torch.zeros(1 << 24, dtype=torch.complex64, device="cuda")
    y = torch.empty_like(x)
    with pytest.raises(mf.MifftError) as e:
        mf.fft_execute_noalloc(1, (1 << 24,), 1, mf.FFT_C2C, mf.FFT_FORWARD, F32, x.data_ptr(), y.data_ptr(), 0)
    assert e.value.status == mf.FFT_ERR_UNSUPPORTED
