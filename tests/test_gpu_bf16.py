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


R64_CASES = [
    # (n, radix entries forcing radix-64 matrix-core stages, expected pass radices)
    (64, "L64:radix=r64", ["64"]),
    (256, "L256:radix=r64.4", ["64x4"]),
    (512, "L512:radix=r64.8", ["64x8"]),
    (1024, "L1024:radix=r64.16", ["64x16"]),
    (1024, "L1024:radix=r16.64", ["16x64"]),
    (4096, "L4096:radix=r64.64", ["64x64"]),
    (1 << 20, "L1024:radix=r64.16", ["64x16", "64x16"]),
]


@pytest.mark.parametrize("n,entry,expect", R64_CASES)
@pytest.mark.parametrize("dtype", [X2, X3])
def test_bf16_radix64_stages(n, entry, expect, dtype, monkeypatch):
    """Radix-64 stages as dense 128x128 DFT-matrix products (8 x 4 blocks of MFMA), the
    split DFT matrix in LDS: against the oracle at the bounds of the radix-16 form, both
    directions, and a batch that leaves a partial last tile."""
    import re
    pre = "bf2" if dtype == X2 else "bf3"
    monkeypatch.setenv("MIFFT_TUNE", f"{pre}:{entry}")
    batch = 3 if n < (1 << 20) else 2
    d = mf.fft_plan_inspect(1, [n], batch, mf.FFT_C2C, mf.FFT_FORWARD, dtype)
    got = re.findall(r"radices=([0-9x]+) mfma", d.split("  in place")[0])
    assert got == expect, d
    for direction in (mf.FFT_FORWARD, mf.FFT_INVERSE):
        e = errs(n, batch, dtype, direction, seed=n + dtype + 64)
        assert e <= BOUND[dtype], (n, entry, dtype, direction, e)
