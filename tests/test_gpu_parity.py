"""GPU parity: every kernel family against the FP64 oracle, per transform, through
the C ABI (ctypes binding).  Bounds: relative L2 <= 1e-13 for FP64 and <= 2e-6 for
FP32 inputs (FP32 results), measured against the oracle run on the same inputs."""
import numpy as np
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


# single-pass lengths: every n to 64, then smooth sizes across the radix set
SMALL = list(range(1, 65)) + [81, 96, 100, 125, 128, 189, 243, 256, 343, 512, 640, 729, 768, 1000, 1024,
                              2048, 3000, 4096, 6125, 8192]


@pytest.mark.parametrize("n", SMALL)
@pytest.mark.parametrize("dtype", [F32, F64])
def test_c2c_1d_single_pass(n, dtype):
    batch = 3 if n > 1000 else 7
    if dtype == F64 and n > 4096:
        batch = 2
    check((n,), batch, C2C, FWD, dtype, seed=n)
    check((n,), batch, C2C, INV, dtype, seed=n + 1)


# multi-pass lengths: scaled-down relatives of the sweep sizes plus the sweep's odd one
MULTI = [2 ** 13, 2 ** 14, 2 ** 16, 3 * 2 ** 12, 5 * 2 ** 12, 7 * 3 ** 6, 2 ** 18, 7 * 3 ** 9, 2 ** 20, 3 * 2 ** 18,
         5 * 2 ** 16]


@pytest.mark.parametrize("n", MULTI)
@pytest.mark.parametrize("dtype", [F32, F64])
def test_c2c_1d_multi_pass(n, dtype):
    batch = 2
    check((n,), batch, C2C, FWD, dtype, seed=n)
    check((n,), batch, C2C, INV, dtype, seed=n + 1)


def test_c2c_three_passes():
    # 2^21 splits into three passes of <= 1024 points in both precisions
    check((1 << 21,), 1, C2C, FWD, F32, seed=21)
    check((1 << 21,), 1, C2C, INV, F64, seed=22)


@pytest.mark.parametrize("n", [2 ** 10, 4096, 2 ** 16, 3 * 2 ** 12, 97])
@pytest.mark.parametrize("dtype", [F32, F64])
def test_c2c_in_place_equals_out_of_place(n, dtype):
    check((n,), 3, C2C, FWD, dtype, seed=5, inplace=True)
    check((n,), 3, C2C, INV, dtype, seed=6, inplace=True)


PRIMES = [11, 13, 17, 97, 101, 257, 1009, 4099]


@pytest.mark.parametrize("n", PRIMES + [2 * 97, 3 * 101, 11 * 13, 2 ** 5 * 17])
@pytest.mark.parametrize("dtype", [F32, F64])
def test_c2c_bluestein(n, dtype):
    check((n,), 2, C2C, FWD, dtype, seed=n)
    check((n,), 2, C2C, INV, dtype, seed=n + 1)


@pytest.mark.parametrize("dtype", [F32, F64])
def test_c2c_bluestein_largest_prime(dtype):
    # the largest prime of the ragged workload: M = 2^17, multi-pass inner FFTs
    check((65521,), 1, C2C, FWD, dtype, seed=65521)


@pytest.mark.parametrize("dims", [(4, 6), (16, 16), (64, 48), (256, 512), (5, 7, 9), (32, 32, 32), (8, 12, 20),
                                  (1, 16), (16, 1), (3, 1, 5), (2048, 8), (8, 2048), (17, 20), (30, 1024)])
@pytest.mark.parametrize("dtype", [F32, F64])
def test_c2c_multidim(dims, dtype):
    check(dims, 2, C2C, FWD, dtype, seed=sum(dims))
    check(dims, 2, C2C, INV, dtype, seed=sum(dims) + 1)


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6, 7, 8, 9, 16, 30, 64, 100, 512, 1000, 4096, 8192, 16384, 2 ** 16,
                               2 * 97, 97, 3 * 2 ** 10 + 0])
@pytest.mark.parametrize("dtype", [F32, F64])
def test_real_1d(n, dtype):
    check((n,), 3, R2C, FWD, dtype, seed=n)
    check((n,), 3, C2R, INV, dtype, seed=n + 7)


@pytest.mark.parametrize("n", [2 ** 16, 18000, 2 * 9001])
@pytest.mark.parametrize("dtype", [F32, F64])
def test_real_1d_staged_many_rows(n, dtype):
    # staged real transforms (n/2 beyond one workgroup, or a prime n/2) over more rows than
    # one thread of the row-wise twist / untwist walks (8), with a ragged last group; an odd
    # n/2 (9001) has no self-paired middle bin
    check((n,), 11, R2C, FWD, dtype, seed=n + 11)
    check((n,), 11, C2R, INV, dtype, seed=n + 12)


@pytest.mark.parametrize("dims,batch,dtype", [((98304,), 5, F32), ((1 << 21,), 2, F32), ((1 << 22,), 1, F32),
                                              ((3 << 18,), 3, F32), ((1 << 17,), 3, F64), ((3, 1 << 16), 2, F32),
                                              ((1 << 16,), 1, F32), ((1 << 16,), 1, F64)])
def test_real_1d_twist_in_last_or_first_pass(dims, batch, dtype):
    # staged real transforms whose twist rides in the last pass (mirrored tiles: each tile
    # holds columns j and J - j; columns 0 and J/2 pair with themselves): last passes of
    # 192, 1024 and 128 points (three passes at 2^22), one line and several, a 2-D array
    # whose rows are staged, both precisions; and the inverses, whose untwist rides in the
    # first pass the same way
    check(dims, batch, R2C, FWD, dtype, seed=sum(dims) + batch)
    check(dims, batch, C2R, INV, dtype, seed=sum(dims) + batch + 1)


@pytest.mark.parametrize("dims", [(4, 6), (16, 16), (6, 10, 8), (32, 32, 32), (5, 7), (64, 64, 64), (7, 9, 11),
                                  (512, 32)])
@pytest.mark.parametrize("dtype", [F32, F64])
def test_real_multidim(dims, dtype):
    check(dims, 2, R2C, FWD, dtype, seed=sum(dims))
    check(dims, 2, C2R, INV, dtype, seed=sum(dims) + 3)


def test_config1_c128_4096_x64():
    # the FP64 workload at its full size: 64 transforms of 4096, all compared
    err = check((4096,), 64, C2C, FWD, F64, seed=1001)
    assert err <= 1e-13


def test_non_default_stream_and_repeat():
    import torch
    from gpu_util import cplx_input, reference, max_rel_err
    rng = np.random.default_rng(77)
    x = cplx_input(rng, (4, 3 * 2 ** 12), F32)
    plan = mf.Plan((3 * 2 ** 12,), 4, C2C, FWD, F32)
    s = torch.cuda.Stream()
    xin = torch.from_numpy(x).cuda()
    outs = []
    with torch.cuda.stream(s):
        for _ in range(3):
            outs.append(plan(xin, stream=s))
    s.synchronize()
    ref = reference((3 * 2 ** 12,), C2C, FWD, x)
    for o in outs:
        assert max_rel_err(o.cpu().numpy(), ref, 4) <= 2e-6
    # bitwise determinism run to run
    a, b = outs[0].cpu().numpy(), outs[2].cpu().numpy()
    assert np.array_equal(a.view(np.uint32), b.view(np.uint32))
    plan.close()


def test_input_is_not_modified():
    import torch
    from gpu_util import cplx_input
    rng = np.random.default_rng(3)
    for dims, kind, dt in [((3 * 2 ** 14,), C2C, F32), ((6, 10, 8), C2R, F64), ((4096,), R2C, F32)]:
        plan = mf.Plan(dims, 2, kind, INV if kind == C2R else FWD, dt)
        (ishape, idt), _ = plan._spec()
        if idt.is_complex:
            x = torch.from_numpy(cplx_input(rng, ishape, dt)).cuda()
        else:
            x = torch.randn(ishape, dtype=idt, device="cuda")
        x0 = x.clone()
        plan(x)
        torch.cuda.synchronize()
        assert torch.equal(x, x0)
        plan.close()


def test_unwritten_output_detection():
    # output pre-filled with NaN: any element the plan fails to write shows up
    import torch
    from gpu_util import cplx_input
    rng = np.random.default_rng(9)
    for n, b in [(3 * 2 ** 12, 3), (1000, 5), (97, 4), (2 ** 16, 2)]:
        plan = mf.Plan((n,), b, C2C, FWD, F32)
        x = torch.from_numpy(cplx_input(rng, (b, n), F32)).cuda()
        out = torch.full((b, n), float("nan"), dtype=torch.complex64, device="cuda")
        plan(x, out=out)
        torch.cuda.synchronize()
        assert torch.isfinite(torch.view_as_real(out)).all()
        plan.close()


@pytest.mark.parametrize("n", [6, 10, 12, 14, 15, 30, 126, 150, 180, 210, 1260, 2916, 3150, 6561, 44100, 30000, 6125])
@pytest.mark.parametrize("dtype", [F32, F64])
def test_c2c_composite_radices(n, dtype):
    # prime-factor butterflies (6, 10, 12, 14, 15) in single- and multi-pass plans
    check((n,), 3, C2C, FWD, dtype, seed=n)
    check((n,), 3, C2C, INV, dtype, seed=n + 1)


def _sweep_cases():
    from paper_1707_03776_amd import inputs
    for n in inputs.SWEEP_LENGTHS:
        for dt in (F32, F64):
            for d in (FWD, INV):
                yield n, dt, d


@pytest.mark.timeout(300)
@pytest.mark.parametrize("n,dtype,direction", list(_sweep_cases()))
def test_sweep_full_size(n, dtype, direction):
    """Every length of the 1-D sweep at its ~1 GiB batch, in the plan and launch
    configuration the benchmark times: the first, the last and two seeded transforms in
    between compared with the oracle (the whole batch is far beyond what the CPU oracle
    finishes in seconds at 2^24); inputs drawn on the GPU as the benchmark does."""
    import torch
    from gpu_util import assert_parity
    from paper_1707_03776_amd import inputs
    import oracle
    npdt = np.complex128 if dtype == F64 else np.complex64
    batch = inputs.sweep_batch(n, npdt)
    seed = inputs.seed_for(2, inputs.sweep_case_index(n, npdt))
    print(f"sweep n={n} batch={batch} dtype={dtype} dir={direction}", flush=True)
    x = inputs.device_complex_normal((batch, n), npdt, seed)
    plan = mf.Plan((n,), batch, C2C, direction, dtype)
    try:
        y = plan(x)
        torch.cuda.synchronize()
    finally:
        plan.close()
    rng = np.random.default_rng(seed)
    pick = sorted({0, batch - 1} | set(int(b) for b in rng.integers(0, batch, size=2)))
    xs = x[pick].cpu().numpy()
    ys = y[pick].cpu().numpy()
    del x, y
    ref = oracle.c2c(xs, (n,), inverse=direction == INV)
    assert_parity(ys, ref, len(pick), 1e-13 if dtype == F64 else 2e-6, n,
                  f"n={n} dtype={dtype} dir={direction} transforms={pick}")


@pytest.mark.timeout(300)
@pytest.mark.parametrize("dtype,batch", [(F32, 128), (F64, 64)])
def test_real_1d_2to20_chunked(dtype, batch):
    """2^20-point real lines at the DCT workload's ~512 MiB batch, in the configuration it
    times: the r2c plan runs in chunks whose last pass carries the twist (mirrored tiles),
    the c2r plan in chunks (a shorter last one in float32) whose first pass carries the
    untwist; the first, the last and two seeded lines compared with the oracle."""
    import torch
    from gpu_util import assert_parity
    from paper_1707_03776_amd import inputs
    import oracle
    n = 1 << 20
    npdt = np.complex128 if dtype == F64 else np.complex64
    rdt = torch.float64 if dtype == F64 else torch.float32
    seed = inputs.seed_for(7, 20 + int(dtype))
    print(f"real 2^20 batch={batch} dtype={dtype}", flush=True)
    x = torch.view_as_real(inputs.device_complex_normal((batch, n // 2), npdt, seed)).reshape(batch, n).to(rdt)
    spec = inputs.device_complex_normal((batch, n // 2 + 1), npdt, seed + 1)
    fwd = mf.Plan((n,), batch, R2C, FWD, dtype)
    inv = mf.Plan((n,), batch, C2R, INV, dtype)
    try:
        assert "epi=rtwist" in fwd.describe() and "pro=cuntwist" in inv.describe()
        y = fwd(x)
        z = inv(spec)
        torch.cuda.synchronize()
    finally:
        fwd.close()
        inv.close()
    rng = np.random.default_rng(seed)
    pick = sorted({0, batch - 1} | set(int(b) for b in rng.integers(0, batch, size=2)))
    tol = 1e-13 if dtype == F64 else 2e-6
    ref = oracle.r2c(x[pick].cpu().numpy(), (n,))
    assert_parity(y[pick].cpu().numpy(), ref, len(pick), tol, n, f"r2c 2^20 dtype={dtype} lines={pick}")
    ref = oracle.c2r(spec[pick].cpu().numpy(), (n,))
    assert_parity(z[pick].cpu().numpy(), ref, len(pick), tol, n, f"c2r 2^20 dtype={dtype} lines={pick}")


@pytest.mark.timeout(600)
def test_multidim_full_size_r2c_512_cubed():
    """The 3-D benchmark at full size: 512^3 float32 uniform[-1, 1) plus three tones,
    r2c, the whole half spectrum against the oracle (L2 bound; both bounds for the
    noise part alone, and for the tone bins, each relative to itself)."""
    from gpu_util import assert_parity, run_plan
    from paper_1707_03776_amd import inputs
    import oracle
    dims = (512, 512, 512)
    rng = np.random.default_rng(inputs.seed_for(3, 1))
    x, freqs, _, noise = inputs.real_with_tones(rng, dims, 3, np.float32)
    for arr, tones in ((x, True), (noise, False)):
        a = arr.reshape((1,) + dims)
        y = run_plan(dims, 1, R2C, FWD, F32, a)
        ref = oracle.r2c(a, dims)
        l2, el = assert_parity(y, ref, 1, 2e-6, 512 ** 3, f"r2c 512^3 tones={tones}", elem=not tones)
        print(f"r2c 512^3 tones={tones}: rel L2 {l2:.3e}, max element error {el:.3e}", flush=True)
        if tones:
            for k in freqs:
                assert abs(y[(0,) + tuple(k)] - ref[(0,) + tuple(k)]) <= 2e-6 * abs(ref[(0,) + tuple(k)])
        del y, ref


@pytest.mark.timeout(300)
@pytest.mark.parametrize("direction", [FWD, INV])
def test_multidim_full_size_c2c_4096_squared(direction):
    """The 2-D benchmark at full size: 4096^2 complex64 uniform[-1, 1) plus three
    complex tones, the whole output against the oracle (L2 bound; both bounds for the
    noise part alone, and for the tone bins, each relative to itself)."""
    from gpu_util import assert_parity, run_plan
    from paper_1707_03776_amd import inputs
    import oracle
    dims = (4096, 4096)
    rng = np.random.default_rng(inputs.seed_for(3, 2))
    x, freqs, _, noise = inputs.complex_with_tones(rng, dims, 3, np.complex64)
    for arr, tones in ((x, True), (noise, False)):
        a = arr.reshape((1,) + dims)
        y = run_plan(dims, 1, C2C, direction, F32, a)
        ref = oracle.c2c(a, dims, inverse=direction == INV)
        l2, el = assert_parity(y, ref, 1, 2e-6, 4096 ** 2, f"c2c 4096^2 dir={direction} tones={tones}",
                               elem=not tones)
        print(f"c2c 4096^2 dir={direction} tones={tones}: rel L2 {l2:.3e}, max element error {el:.3e}",
              flush=True)
        if tones:
            for k in freqs:
                kk = tuple(k) if direction == FWD else tuple((-np.asarray(k)) % 4096)
                assert abs(y[(0,) + kk] - ref[(0,) + kk]) <= 2e-6 * abs(ref[(0,) + kk])



@pytest.mark.parametrize("dims,batch,kind,dtype", [
    ((1 << 16,), 7, C2C, F32), ((3 * 2 ** 12,), 5, C2C, F64), ((4099,), 5, C2C, F32),
    ((64, 48), 5, R2C, F32), ((64, 48), 5, C2R, F64), ((30, 1024), 3, C2C, F32)])
def test_chunked_batch(dims, batch, kind, dtype, monkeypatch):
    """A multi-op plan runs its batch in chunks (a small chunk size forces several chunks
    and a shorter last one): every transform, out of place and (c2c) in place."""
    import re
    per = int(np.prod(dims)) * (16 if dtype == F64 else 8)
    monkeypatch.setenv("MIFFT_CHUNK_BYTES", str(2 * per))
    desc = mf.fft_plan_inspect(len(dims), list(dims), batch, kind, INV if kind == C2R else FWD, dtype)
    m = re.search(r"chunks of (\d+) transforms", desc)
    assert m and int(m.group(1)) < batch, desc
    direction = INV if kind == C2R else FWD
    check(dims, batch, kind, direction, dtype, seed=batch + len(dims))
    if kind == C2C:
        check(dims, batch, kind, INV, dtype, seed=batch, inplace=True)
