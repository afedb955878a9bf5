"""GPU parity of the pseudo-spectral Laplacian (fft_laplacian_*: r2c, the
-|kappa|^2 multiply, c2r) against the oracle's r2c / multiply / c2r in FP64.
White-noise fields on grids the oracle finishes in seconds (1-D, 2-D, 3-D, odd and
even sizes, several periods, batches), relative L2 per field <= 2e-6 (FP32) and
<= 1e-13 (FP64), with the element bound of gpu_util.assert_parity; the 512^3 grid of
the 3-D benchmark is compared at full size as well."""
import numpy as np
import pytest

import oracle
import paper_1707_03776_amd as mf
from gpu_util import TOL, assert_parity

pytestmark = pytest.mark.gpu

F32, F64 = mf.FFT_F32, mf.FFT_F64


@pytest.fixture(autouse=True, scope="module")
def _gpu(gpu_available):
    return gpu_available


def _run(dims, batch, lengths, dtype, u, inplace=False):
    import torch
    lap = mf.Laplacian(dims, batch, lengths, dtype)
    try:
        x = torch.from_numpy(np.ascontiguousarray(u)).cuda()
        y = lap(x, out=x if inplace else None)
        torch.cuda.synchronize()
        return y.cpu().numpy()
    finally:
        lap.close()


CASES = [((64,), 3, (1.0,)), ((1000,), 2, (6.0,)), ((97,), 2, (1.0,)), ((32, 48), 2, (1.0, 2.0)),
         ((17, 20), 3, (0.5, 3.0)), ((5, 7, 9), 2, (1.0, 1.0, 1.0)), ((32, 32, 32), 2, (2.0, 2.0, 2.0)),
         ((16, 12, 20), 1, (1.0, 0.7, 2.3)), ((48, 40, 36), 1, (3.0, 1.0, 2.0)), ((64, 64, 64), 1, (1.0, 1.0, 1.0)),
         ((1, 16), 2, (1.0, 1.0)), ((8, 1, 6), 1, (1.0, 1.0, 1.0))]


@pytest.mark.parametrize("dims,batch,lengths", CASES)
@pytest.mark.parametrize("dtype", [F32, F64])
def test_laplacian_vs_oracle(dims, batch, lengths, dtype):
    rng = np.random.default_rng(sum(dims) + batch)
    u = rng.standard_normal((batch,) + dims).astype(np.float64 if dtype == F64 else np.float32)
    y = _run(dims, batch, lengths, dtype, u)
    ref = oracle.laplacian(u.astype(np.float64), dims, lengths)
    if not np.any(ref):
        # a grid of single points (every axis of length 1) has a zero Laplacian
        assert np.max(np.abs(y)) == 0
        return
    assert_parity(y, ref, batch, TOL[dtype], int(np.prod(dims)), f"dims={dims} dtype={dtype}")


@pytest.mark.parametrize("dims,fused", [((32, 32, 32), True), ((64, 64, 64), True), ((32, 48), True),
                                        ((48, 40, 36), False), ((24, 20, 18), False), ((1000,), False)])
def test_laplacian_symbol_fused_where_eligible(dims, fused):
    # the multiply rides in the c2r plan's first pass when that pass is a specialised
    # kernel over one whole axis (here 32, 64 or 48-bin axes) and runs on its own
    # otherwise (a 20- or 40-point axis has no specialised kernel; a 1-D field's c2r plan
    # starts with the untwisting pass)
    lap = mf.Laplacian(dims, 2, (1.0,) * len(dims), F32)
    try:
        d = lap.describe()
    finally:
        lap.close()
    assert ("in the c2r plan's first pass" in d) == fused, d
    assert ("pro=sym" in d) == fused, d


@pytest.mark.parametrize("dims,batch,lengths", [((32, 32, 32), 2, (2.0, 2.0, 2.0)), ((32, 48), 2, (1.0, 2.0))])
@pytest.mark.parametrize("dtype", [F32, F64])
def test_laplacian_unfused_form_vs_oracle(dims, batch, lengths, dtype, monkeypatch):
    # MIFFT_LAPLACE_UNFUSED keeps the multiply a kernel of its own on grids that would fuse it
    monkeypatch.setenv("MIFFT_LAPLACE_UNFUSED", "1")
    rng = np.random.default_rng(sum(dims) + batch + 1)
    u = rng.standard_normal((batch,) + dims).astype(np.float64 if dtype == F64 else np.float32)
    lap = mf.Laplacian(dims, batch, lengths, dtype)
    try:
        assert "first pass" not in lap.describe()
    finally:
        lap.close()
    y = _run(dims, batch, lengths, dtype, u)
    ref = oracle.laplacian(u.astype(np.float64), dims, lengths)
    assert_parity(y, ref, batch, TOL[dtype], int(np.prod(dims)), f"unfused dims={dims} dtype={dtype}")


@pytest.mark.parametrize("dtype", [F32, F64])
def test_laplacian_in_place(dtype):
    dims, lengths = (24, 20, 18), (1.0, 2.0, 3.0)
    u = np.random.default_rng(5).standard_normal((2,) + dims).astype(np.float64 if dtype == F64 else np.float32)
    a = _run(dims, 2, lengths, dtype, u)
    b = _run(dims, 2, lengths, dtype, u.copy(), inplace=True)
    assert np.array_equal(a, b)


@pytest.mark.timeout(600)
@pytest.mark.parametrize("dtype", [F32, F64])
def test_laplacian_512_cubed_vs_oracle(dtype):
    # the full 512^3 grid, a white-noise field, against the oracle's r2c / multiply / c2r
    dims, lengths = (512, 512, 512), (2.0, 2.0, 2.0)
    u = np.random.default_rng(512).standard_normal((1,) + dims).astype(np.float64 if dtype == F64 else np.float32)
    y = _run(dims, 1, lengths, dtype, u)
    ref = oracle.laplacian(u.astype(np.float64), dims, lengths)
    assert_parity(y, ref, 1, TOL[dtype], 512 ** 3, f"512^3 dtype={dtype}")
