"""fft_execute under a stream capture: the kernels it enqueues are recorded into the
caller's graph, and every replay writes bitwise what the eager call wrote.  Replays
are interleaved with eager work of the same plans (and synchronisations), and the
output is cleared before each replay, so a replay that skipped or reused anything
would show.  Covered: a two-pass and a three-pass complex transform, in place, a real
3-D transform, a Bluestein length, a DCT-II, the Laplacian operator, and a ragged
batch (whose plan-owned graph cannot be launched into a capturing stream, so it
launches its phase kernels one by one there)."""
import numpy as np
import pytest

import paper_1707_03776_amd as mf
from gpu_util import cplx_input, real_input

pytestmark = pytest.mark.gpu

F32, F64 = mf.FFT_F32, mf.FFT_F64


@pytest.fixture(autouse=True, scope="module")
def _gpu(gpu_available):
    return gpu_available


def _bits(t):
    import torch
    return t.view(torch.uint8) if not t.is_complex() else torch.view_as_real(t).view(torch.uint8)


def _replays_equal_eager(run, out, eager_out, other=None):
    """Capture run() (which writes `out`), replay 3 times; each replay must equal
    eager_out bitwise.  `other` is eager work done between replays."""
    import torch
    g = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        with torch.cuda.graph(g, stream=side):
            run()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    for _ in range(3):
        out.zero_()
        if other is not None:
            other()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(_bits(out), _bits(eager_out))
    del g


CASES = [
    ((1 << 16,), 3, mf.FFT_C2C, mf.FFT_FORWARD, F32, False),
    ((1 << 21,), 1, mf.FFT_C2C, mf.FFT_INVERSE, F32, False),
    ((3 * 2 ** 12,), 4, mf.FFT_C2C, mf.FFT_FORWARD, F64, True),
    ((32, 24, 40), 2, mf.FFT_R2C, mf.FFT_FORWARD, F32, False),
    ((4099,), 2, mf.FFT_C2C, mf.FFT_FORWARD, F32, False),
    ((1000,), 3, mf.FFT_DCT2, mf.FFT_FORWARD, F64, False),
]


@pytest.mark.parametrize("dims,batch,kind,direction,dtype,inplace", CASES)
def test_capture_plan(dims, batch, kind, direction, dtype, inplace):
    import torch
    rng = np.random.default_rng(sum(dims) + batch)
    real_in = kind in (mf.FFT_R2C, mf.FFT_DCT2)
    x = real_input(rng, (batch,) + dims, dtype) if real_in else cplx_input(rng, (batch,) + dims, dtype)
    plan = mf.Plan(dims, batch, kind, direction, dtype)
    try:
        xd = torch.from_numpy(x).cuda()
        if inplace:
            work = xd.clone()
            plan(work, out=work)
            torch.cuda.synchronize()
            eager = work.clone()
            buf = xd.clone()

            def run():
                buf.copy_(xd)
                plan(buf, out=buf)
            _replays_equal_eager(run, buf, eager, other=lambda: plan(xd.clone()))
        else:
            eager = plan(xd)
            torch.cuda.synchronize()
            out = torch.empty_like(eager)
            _replays_equal_eager(lambda: plan(xd, out=out), out, eager, other=lambda: plan(xd))
    finally:
        plan.close()


def test_capture_laplacian():
    import torch
    dims = (24, 20, 18)
    u = torch.from_numpy(np.random.default_rng(3).standard_normal((2,) + dims)).cuda()
    lap = mf.Laplacian(dims, 2, (1.0, 2.0, 3.0), F64)
    try:
        eager = lap(u)
        torch.cuda.synchronize()
        out = torch.empty_like(eager)
        _replays_equal_eager(lambda: lap(u, out=out), out, eager, other=lambda: lap(u))
    finally:
        lap.close()


def test_capture_ragged():
    import torch
    lengths = [64, 97, 1000, 4096, 65536, 30011, 12288]
    offs = np.concatenate([[0], np.cumsum(lengths)])[:-1]
    total = int(sum(lengths))
    x = torch.from_numpy(cplx_input(np.random.default_rng(9), (total,), F32)).cuda()
    plan = mf.fft_plan_create_many(lengths, offs, offs, mf.FFT_C2C, mf.FFT_FORWARD, F32)
    try:
        eager = torch.empty_like(x)
        scratch_out = torch.empty_like(x)
        mf.fft_execute(plan, x.data_ptr(), eager.data_ptr(), torch.cuda.current_stream().cuda_stream)
        torch.cuda.synchronize()
        out = torch.empty_like(x)

        def run():
            mf.fft_execute(plan, x.data_ptr(), out.data_ptr(), torch.cuda.current_stream().cuda_stream)

        def other():
            # the plan's own graph, re-bound to other buffers between replays
            mf.fft_execute(plan, x.data_ptr(), scratch_out.data_ptr(), torch.cuda.current_stream().cuda_stream)

        _replays_equal_eager(run, out, eager, other=other)
        assert torch.equal(_bits(scratch_out), _bits(eager))
    finally:
        mf.fft_plan_destroy(plan)
