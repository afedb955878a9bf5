"""GPU parity of the split-BF16 MFMA forms (radix-16 stages on the matrix cores).

The three-term split (hi+mid+lo, six cross products) keeps ~27 significand bits per
operand, below FP32's 24, so it is held to the FP32 bound (relative L2 <= 2e-6).
The two-term split keeps ~18 bits; its error is stated rather than gated at the
FP32 level: each radix-16 stage contributes ~2^-18 relative error, so after five
such stages the relative L2 stays near 1e-5 (bound used here: 5e-5).
"""
import numpy as np
import pytest

import paper_1707_03776_amd as mf
from gpu_util import cplx_input, max_rel_err, reference, run_plan

pytestmark = pytest.mark.gpu

X2, X3 = mf.FFT_F32_BF16X2, mf.FFT_F32_BF16X3
BOUND = {X2: 5e-5, X3: 2e-6}


@pytest.fixture(autouse=True, scope="module")
def _gpu(gpu_available):
    return gpu_available


def errs(n, batch, dtype, direction, seed):
    rng = np.random.default_rng(seed)
    x = cplx_input(rng, (batch, n), mf.FFT_F32)
    y = run_plan((n,), batch, mf.FFT_C2C, direction, dtype, x)
    return max_rel_err(y, reference((n,), mf.FFT_C2C, direction, x), batch)


@pytest.mark.parametrize("n", [16, 64, 128, 256, 4096, 2 ** 16, 2 ** 18])
@pytest.mark.parametrize("dtype", [X2, X3])
def test_bf16_split_forms(n, dtype):
    for direction in (mf.FFT_FORWARD, mf.FFT_INVERSE):
        e = errs(n, 3, dtype, direction, seed=n + dtype)
        assert e <= BOUND[dtype], (n, dtype, direction, e)


def test_three_term_beats_two_term():
    e2 = errs(4096, 4, X2, mf.FFT_FORWARD, 11)
    e3 = errs(4096, 4, X3, mf.FFT_FORWARD, 11)
    ef = errs(4096, 4, mf.FFT_F32, mf.FFT_FORWARD, 11)
    assert e3 < e2 / 4, (e2, e3)
    assert e3 < 4 * ef + 1e-7, (e3, ef)


def test_bf16_precision_workload_full_size():
    # 2^20 points, batch 64: every transform against the oracle, error per transform
    n, b = 2 ** 20, 64
    rng = np.random.default_rng(4001)
    x = cplx_input(rng, (b, n), mf.FFT_F32)
    ref = reference((n,), mf.FFT_C2C, mf.FFT_FORWARD, x)
    import oracle
    for dtype in (X2, X3):
        y = run_plan((n,), b, mf.FFT_C2C, mf.FFT_FORWARD, dtype, x)
        e = oracle.rel_l2(y, ref)
        assert e.shape == (b,)
        assert float(e.max()) <= BOUND[dtype], (dtype, float(e.max()))


def test_bf16_non_mfma_lengths_fall_back_to_fp32():
    # lengths without a radix-16 MFMA shape still plan and meet the FP32 bound
    for n in (1000, 97, 48):
        assert errs(n, 2, X3, mf.FFT_FORWARD, n) <= 2e-6
