"""GPU parity of the paths the default plans do not take: the runtime-radix kernel on
shapes that normally have specialised kernels (MIFFT_GENERIC_ONLY=1), and plans bent
by tuning-table entries of every kind the autotuner can write (pass splits, radix
orders, tile widths, workgroup sizes, LDS pitches).  Same bounds as the other parity
tests: relative L2 <= 2e-6 (FP32) / 1e-13 (FP64) against the FP64 oracle."""
import os

import pytest

import paper_1707_03776_amd as mf
from gpu_util import check

pytestmark = pytest.mark.gpu

F32, F64 = mf.FFT_F32, mf.FFT_F64
C2C, R2C, C2R = mf.FFT_C2C, mf.FFT_R2C, mf.FFT_C2R
FWD, INV = mf.FFT_FORWARD, mf.FFT_INVERSE


@pytest.fixture(autouse=True, scope="module")
def _gpu(gpu_available):
    return gpu_available


@pytest.fixture
def generic_only():
    os.environ["MIFFT_GENERIC_ONLY"] = "1"
    yield
    del os.environ["MIFFT_GENERIC_ONLY"]


@pytest.fixture
def table():
    saved = mf.fft_tune_get()
    yield lambda entries: mf.fft_tune_set(entries, replace=True)
    mf.fft_tune_set(saved, replace=True)


@pytest.mark.parametrize("n", [16, 64, 1024, 4096, 8192, 2 ** 16, 3 * 2 ** 12, 7 * 3 ** 6, 2 ** 20])
@pytest.mark.parametrize("dtype", [F32, F64])
def test_generic_kernel_on_specialised_shapes(generic_only, n, dtype):
    d = mf.fft_plan_inspect(1, [n], 2, C2C, FWD, dtype)
    assert " fixed " not in d and " generic " in d
    check((n,), 2, C2C, FWD, dtype, seed=n)
    check((n,), 2, C2C, INV, dtype, seed=n + 1)
    check((n,), 2, C2C, FWD, dtype, seed=n + 2, inplace=True)


@pytest.mark.parametrize("dims,kind", [((512, 32), R2C), ((64, 64, 64), C2R), ((4096,), R2C), ((30, 1024), C2C)])
def test_generic_kernel_real_and_multidim(generic_only, dims, kind):
    check(dims, 2, kind, INV if kind == C2R else FWD, F32, seed=sum(dims))


SPLITS = ["s256.256", "s1024.64", "s64.1024", "s16.64.64", "s4096.16", "s65536"]


@pytest.mark.parametrize("split", SPLITS)
@pytest.mark.parametrize("dtype", [F32, F64])
def test_tuned_pass_splits(table, split, dtype):
    dt = "f64" if dtype == F64 else "f32"
    table(f"{dt}:n65536:S1:split={split}")
    d = mf.fft_plan_inspect(1, [65536], 2, C2C, FWD, dtype)
    lengths = [int(x) for x in split[1:].split(".")]
    if len(lengths) > 1 or 65536 <= (4096 if dtype == F64 else 8192):
        assert [f"L={L} " in d for L in lengths] == [True] * len(lengths), d
    check((65536,), 2, C2C, FWD, dtype, seed=7)
    check((65536,), 2, C2C, INV, dtype, seed=8, inplace=True)


@pytest.mark.parametrize("radices", ["r8.8.16", "r4.16.16", "r16.4.16", "r2.16.32", "r8.16.8"])
def test_tuned_radix_orders(table, radices):
    table(f"f32:L1024:radix={radices}")
    d = mf.fft_plan_inspect(1, [1024], 4, C2C, FWD, F32)
    if radices != "r2.16.32":  # 32 is not a radix: the entry is ignored
        assert "radices=" + radices[1:].replace(".", "x") in d
    check((1024,), 4, C2C, FWD, F32, seed=3)
    check((1 << 20,), 1, C2C, INV, F32, seed=4)


@pytest.mark.parametrize("knobs", ["c1", "c2", "c32", "c8,t512", "c16,p4", "c4,t1024,p8"])
def test_tuned_tiles(table, knobs):
    table("\n".join(f"f32:L1024:16x8x8:{m}=" + knobs for m in ("CP:tw0", "CC:tw1", "PP:tw0"))
          + "\n" + "\n".join(f"f64:L1024:16x8x8:{m}=" + knobs for m in ("CP:tw0", "CC:tw1", "PP:tw0")))
    check((1024,), 9, C2C, FWD, F32, seed=11)
    check((1 << 20,), 1, C2C, FWD, F32, seed=12)
    check((1 << 20,), 1, C2C, INV, F64, seed=13)


def test_shipped_table_against_defaults(table):
    # the sizes the shipped table changes, with and without it
    for n, dtype in [(1 << 20, F32), (7 * 3 ** 9, F32), (3 * 2 ** 18, F64), (7 * 3 ** 9, F64)]:
        check((n,), 1, C2C, FWD, dtype, seed=n)
    table("")
    for n, dtype in [(1 << 20, F32), (7 * 3 ** 9, F32), (3 * 2 ** 18, F64), (7 * 3 ** 9, F64)]:
        check((n,), 1, C2C, FWD, dtype, seed=n)
