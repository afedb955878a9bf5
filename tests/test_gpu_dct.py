"""GPU parity of the real-to-real DCT-II / DCT-III plans (an element-wise
prologue, one real transform of the same length, an element-wise epilogue) against
the oracle's definition sums, per transform.  Bounds as for the other kinds:
relative L2 <= 1e-13 (FP64) and <= 2e-6 (FP32).  Above the sizes the O(n^2)
oracle finishes in seconds, the inverse relation DCT-III(DCT-II(x)) = 2n x and
the closed form for a constant input are checked instead."""
import numpy as np
import pytest

import oracle
import paper_1707_03776_amd as mf
from gpu_util import TOL, assert_parity, run_plan

pytestmark = pytest.mark.gpu

F32, F64 = mf.FFT_F32, mf.FFT_F64
DCT2, DCT3, FWD = mf.FFT_DCT2, mf.FFT_DCT3, mf.FFT_FORWARD


@pytest.fixture(autouse=True, scope="module")
def _gpu(gpu_available):
    return gpu_available


def _real(rng, shape, dtype):
    return rng.standard_normal(shape).astype(np.float64 if dtype == F64 else np.float32)


# every length to 20, smooth single- and multi-pass lengths, primes (Bluestein inside)
LENGTHS = list(range(1, 21)) + [32, 64, 97, 100, 128, 1000, 1024, 1009, 4096, 4099, 6125]


@pytest.mark.parametrize("n", LENGTHS)
@pytest.mark.parametrize("kind", [DCT2, DCT3])
@pytest.mark.parametrize("dtype", [F32, F64])
def test_dct_vs_oracle(n, kind, dtype):
    batch = 3 if n <= 1024 else 1
    x = _real(np.random.default_rng(n * 7 + kind), (batch, n), dtype)
    y = run_plan((n,), batch, kind, FWD, dtype, x)
    ref = oracle.dct(x.astype(np.float64), 2 if kind == DCT2 else 3)
    assert_parity(y, ref, batch, TOL[dtype], n, f"n={n} kind={kind} dtype={dtype}")


@pytest.mark.parametrize("n,dtype", [(16384, F64), (20000, F32), (8198, F32), (32768, F32)])
@pytest.mark.parametrize("kind", [DCT2, DCT3])
def test_dct_large_vs_oracle(n, dtype, kind):
    # real transforms staged through a complex one (n/2 above the single-pass limit, or
    # n/2 = 4099 through Bluestein): DCT-II then runs the fused twist-and-rotation op, or
    # in float32 that step in the last pass's stores where the pass takes mirrored tiles
    # (32768), DCT-III the fused rotation-and-untwist op
    d = mf.fft_plan_inspect(1, [n], 1, kind, FWD, dtype)
    if kind == DCT2:
        assert ("epi=dtwist" in d) == (n == 32768) and ("dct2_twpost" in d) != ("epi=dtwist" in d), d
    else:
        assert "dct3_preuntwist" in d, d
    x = _real(np.random.default_rng(3 + kind), (1, n), dtype)
    y = run_plan((n,), 1, kind, FWD, dtype, x)
    ref = oracle.dct(x.astype(np.float64), 2 if kind == DCT2 else 3)
    assert_parity(y, ref, 1, TOL[dtype], n, f"n={n} kind={kind}")


@pytest.mark.parametrize("n,dtype,batch", [(1009, F32, 9), (1000, F64, 17), (4096, F32, 19), (8198, F32, 11),
                                            (8198, F64, 9)])
@pytest.mark.parametrize("kind", [DCT2, DCT3])
def test_dct_many_rows(n, dtype, batch, kind):
    # more rows than one thread of the row-wise reorder / rotation kernels walks (8), a
    # ragged last group of rows, odd lengths (an unpaired middle sample); 8198 runs the
    # staged real transform, so its fused twist / untwist steps take the row-wise form too
    x = _real(np.random.default_rng(n + batch + kind), (batch, n), dtype)
    y = run_plan((n,), batch, kind, FWD, dtype, x)
    ref = oracle.dct(x.astype(np.float64), 2 if kind == DCT2 else 3)
    assert_parity(y, ref, batch, TOL[dtype], n, f"n={n} batch={batch} kind={kind} dtype={dtype}")


@pytest.mark.parametrize("n", [1 << 16, 1 << 20, 3 << 18, 65521])
@pytest.mark.parametrize("dtype", [F32, F64])
def test_dct_round_trip_large(n, dtype):
    # DCT-III(DCT-II(x)) = 2n x holds at any size; the error of the pair is at most
    # about twice that of one transform
    import torch
    batch = 2
    x = _real(np.random.default_rng(n), (batch, n), dtype)
    p2 = mf.Plan((n,), batch, DCT2, FWD, dtype)
    p3 = mf.Plan((n,), batch, DCT3, FWD, dtype)
    try:
        xd = torch.from_numpy(x).cuda()
        z = p3(p2(xd))
        torch.cuda.synchronize()
        z = z.cpu().numpy().astype(np.float64) / (2 * n)
    finally:
        p2.close()
        p3.close()
    assert_parity(z, x.astype(np.float64), batch, 2 * TOL[dtype], n, f"n={n} dtype={dtype}")


@pytest.mark.parametrize("n", [1 << 20, 65521])
def test_dct2_constant_input(n):
    # DCT-II of ones: 2n at k = 0 and zero elsewhere (the cosine sums cancel)
    x = np.ones((1, n))
    y = run_plan((n,), 1, DCT2, FWD, F64, x).reshape(-1)
    assert abs(y[0] - 2 * n) <= 1e-12 * 2 * n
    assert np.max(np.abs(y[1:])) <= 1e-12 * 2 * n


def test_dct_in_place_rejected():
    import torch
    p = mf.Plan((64,), 1, DCT2, FWD, F32)
    try:
        x = torch.zeros(64, dtype=torch.float32, device="cuda")
        with pytest.raises(mf.MifftError):
            p(x, out=x)
    finally:
        p.close()
