"""CPU-side checks of the C ABI: the library loads, exports every symbol the header
declares, and the host-only planner (fft_plan_inspect) decides sensibly and rejects
bad requests with the documented status codes.  No GPU calls."""
import ctypes
import os
import re
import subprocess

import numpy as np

import pytest

import paper_1707_03776_amd as mf

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(autouse=True, scope="module")
def planner_defaults():
    # these tests check the planner's own decisions: run them with an empty tuning
    # table and put the shipped one back afterwards
    saved = mf.fft_tune_get()
    mf.fft_tune_set("", replace=True)
    yield
    mf.fft_tune_set(saved, replace=True)


def header_functions():
    text = open(os.path.join(ROOT, "include", "mifft.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fft_[a-z_]+)\s*\(", text)))


def test_library_exports_every_header_symbol():
    lib = mf.load_library()
    names = header_functions()
    assert "fft_plan_create" in names and "fft_execute" in names and "fft_plan_destroy" in names
    for name in names:
        assert hasattr(lib, name), name
    assert sorted(mf.EXPORTED) == names
    out = subprocess.run(["nm", "-D", "--defined-only", mf.LIB_PATH], capture_output=True, text=True).stdout
    for name in names:
        assert re.search(rf"\bT {name}\b", out), name


def test_header_compiles_as_c():
    src = '#include "mifft.h"\nint main(void){ fft_plan p = 0; (void)p; return FFT_OK; }\n'
    r = subprocess.run(["gcc", "-std=c11", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"), "-x", "c", "-",
                        "-fsyntax-only"], input=src, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr


def inspect(dims, batch=1, kind=mf.FFT_C2C, direction=mf.FFT_FORWARD, dtype=mf.FFT_F32):
    return mf.fft_plan_inspect(len(dims), dims, batch, kind, direction, dtype)


def passes(desc):
    # the out-of-place op list (an in-place variant may follow it)
    return [l for l in desc.split("  in place")[0].splitlines() if " pass " in l]


@pytest.mark.parametrize("n,dtype,npass", [(2 ** 10, 0, 1), (4096, 1, 1), (8192, 0, 1), (2 ** 16, 0, 2),
                                           (2 ** 20, 0, 2), (2 ** 20, 1, 2), (2 ** 24, 0, 3), (2 ** 24, 1, 3),
                                           (3 * 2 ** 18, 0, 2), (5 * 2 ** 16, 1, 2), (7 * 3 ** 9, 0, 2)])
def test_sweep_decompositions(n, dtype, npass):
    d = inspect((n,), 2, dtype=dtype)
    ps = passes(d)
    assert len(ps) == npass, d
    prod = 1
    for p in ps:
        prod *= int(re.search(r"L=(\d+)", p).group(1))
        rad = [int(r) for r in re.search(r"radices=([0-9x]+)", p).group(1).split("x")]
        L = 1
        for r in rad:
            assert r in (1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 12, 14, 15, 16)
            L *= r
        assert L == int(re.search(r"L=(\d+)", p).group(1))
        lds = int(re.search(r"lds=(\d+)", p).group(1))
        assert lds <= 160 * 1024
        T = int(re.search(r" T=(\d+)", p).group(1))
        assert T % 64 == 0 and 64 <= T <= (512 if " fixed " in p else 256)
    assert prod == n


def test_multipass_twiddle_and_coalescing():
    d = inspect((2 ** 20,), 4)
    ps = passes(d)
    assert "twN" not in ps[0] and "twN=1048576" in ps[1]
    # column passes take several adjacent columns per workgroup (>= 64-byte runs)
    for p in ps:
        if "map=C" in p:
            assert int(re.search(r" c=(\d+)", p).group(1)) * 8 >= 32


@pytest.mark.parametrize("n", [97, 65521, 4099, 2 * 97])
def test_bluestein_chosen_for_large_primes(n):
    # contiguous lines: the element-wise steps fused into the passes (four or two passes,
    # no element-wise ops): pad on the first pass's loads, filter on the forward
    # transform's last stores, extraction on the last pass's stores
    d = inspect((n,), 1)
    M = int(re.search(r"M=(\d+)", d).group(1))
    # the next power of two at or above 2n - 1 (no wrap-around in the cyclic convolution)
    assert M >= 2 * n - 1 and M & (M - 1) == 0 and M < 2 * (2 * n - 1)
    ops = [l for l in d.splitlines() if re.match(r"\s+op\d", l)]
    assert all(" pass " in l for l in ops) and len(ops) in (2, 4)
    assert "pro=bpad" in ops[0] and "epi=bext" in ops[-1]
    assert sum("epi=bmul" in l for l in ops) == 1
    # strided lines (a leading axis) keep the element-wise ops
    d = inspect((n, 4), 1)
    assert "chirp_pad" in d and "mul_conj" in d and "chirp_extract" in d


def test_real_plans():
    d = inspect((512, 512, 512), 1, mf.FFT_R2C)
    assert "epi=r2c" in d and len(passes(d)) == 3
    d = inspect((512, 512, 512), 1, mf.FFT_C2R, mf.FFT_INVERSE)
    assert "pro=c2r" in d
    d = inspect((9,), 2, mf.FFT_R2C)
    assert "real_to_cplx" in d and "half_copy" in d


@pytest.mark.parametrize("args,status", [
    (dict(dims=(0,)), mf.FFT_ERR_INVALID_ARG),
    (dict(dims=(8,), batch=0), mf.FFT_ERR_INVALID_ARG),
    (dict(dims=(8,), kind=7), mf.FFT_ERR_INVALID_ARG),
    (dict(dims=(8,), direction=0), mf.FFT_ERR_INVALID_ARG),
    (dict(dims=(8,), dtype=9), mf.FFT_ERR_INVALID_ARG),
    (dict(dims=(8,), kind=mf.FFT_R2C, direction=mf.FFT_INVERSE), mf.FFT_ERR_INVALID_ARG),
    (dict(dims=(8,), kind=mf.FFT_C2R, direction=mf.FFT_FORWARD), mf.FFT_ERR_INVALID_ARG),
    (dict(dims=(8, 8), dtype=mf.FFT_F32_BF16X2), mf.FFT_ERR_UNSUPPORTED),
    (dict(dims=(8,), kind=mf.FFT_R2C, dtype=mf.FFT_F32_BF16X3), mf.FFT_ERR_UNSUPPORTED),
    (dict(dims=(1 << 20,), batch=1 << 13), mf.FFT_ERR_UNSUPPORTED),
    (dict(dims=(65521,), batch=1 << 15), mf.FFT_ERR_UNSUPPORTED),  # Bluestein lines x M reach 2^32
])
def test_invalid_requests(args, status):
    a = dict(dims=(8,), batch=1, kind=mf.FFT_C2C, direction=mf.FFT_FORWARD, dtype=mf.FFT_F32)
    a.update(args)
    with pytest.raises(mf.MifftError) as e:
        mf.fft_plan_inspect(len(a["dims"]), a["dims"], a["batch"], a["kind"], a["direction"], a["dtype"])
    assert e.value.status == status
    assert mf.fft_last_error() == status
    assert mf.fft_last_error_message()


def test_rank_out_of_range():
    lib = mf.load_library()
    d = (ctypes.c_int64 * 4)(2, 2, 2, 2)
    buf = ctypes.create_string_buffer(256)
    assert lib.fft_plan_inspect(4, d, 1, 0, -1, 0, buf, 256) == mf.FFT_ERR_INVALID_ARG
    assert lib.fft_plan_inspect(0, d, 1, 0, -1, 0, buf, 256) == mf.FFT_ERR_INVALID_ARG
    assert lib.fft_plan_inspect(1, None, 1, 0, -1, 0, buf, 256) == mf.FFT_ERR_INVALID_ARG


def test_null_plan_calls_are_safe():
    lib = mf.load_library()
    lib.fft_plan_destroy(None)
    assert lib.fft_execute(None, None, None, None) == mf.FFT_ERR_INVALID_ARG
    assert lib.fft_plan_describe(None) == b""
    assert lib.fft_plan_device_bytes(None) == 0


def test_every_smooth_length_to_8192_plans():
    # every 7-smooth length the ragged workload can draw plans without error
    from paper_1707_03776_amd.inputs import smooth_pool
    for n in smooth_pool(1, 65536):
        inspect((n,), 3)


def _ops(section):
    out = []
    for l in section.splitlines():
        m = re.match(r"\s+op\d+ (\w+) (\w+)->(\w+) (.*)", l)
        if m:
            out.append((m.group(1), m.group(2), m.group(3), m.group(4)))
    return out


@pytest.mark.parametrize("dims", [(12288,), (2 ** 16,), (2 ** 20,), (2 ** 24,), (7 * 3 ** 9,), (97,), (64, 4096),
                                  (4096, 4096), (30, 1024), (8, 2048), (17, 20)])
def test_buffer_hazards(dims):
    """Every op that reads and writes the same buffer must be one whose read and write
    element sets coincide per workgroup: a single pass, the last pass of a chain
    (Ns * L == n), or the in-place element-wise Bluestein product.  Checked for the
    out-of-place list and for the list used when in == out (in renamed to out)."""
    d = inspect(dims, 2)
    sections = d.split("  in place (in == out):")
    for idx, sec in enumerate(sections):
        for name, src, dst, rest in _ops(sec):
            if idx == 1 or len(sections) == 1:
                src = "out" if src == "in" else src
            if src != dst:
                continue
            if name == "mul_conj":
                continue
            assert name == "pass", (name, src, dst)
            L = int(re.search(r"L=(\d+)", rest).group(1))
            m = re.search(r"axis n=(\d+) Ns=(\d+)", rest)
            assert m and int(m.group(2)) * L == int(m.group(1)), rest


def _schedule(desc):
    line = [l for l in desc.splitlines() if l.strip().startswith("schedule:")][0]
    kv = dict(f.split("=") for f in line.split()[1:])
    return int(kv["whole"]), int(kv["split"]), int(kv["phases"]), [int(b) for b in kv["blocks"].split("+")]


def test_ragged_schedule_dry_run():
    # the 20,000-length workload: small transforms run whole, large ones (all primes
    # above a few thousand points go through Bluestein's four passes) are split by op
    from paper_1707_03776_amd import inputs
    lengths = inputs.ragged_lengths()
    for dtype in (mf.FFT_F32, mf.FFT_F64):
        whole, split, phases, blocks = _schedule(
            mf.fft_plan_inspect_many(lengths, mf.FFT_C2C, mf.FFT_FORWARD, dtype))
        assert whole + split == len(lengths)
        assert whole > 0 and split > 0
        assert phases == len(blocks) == 4  # Bluestein: two M-point transforms of two passes each
        assert all(b > 0 for b in blocks)
    # one small transform: a single whole block in a single phase
    assert _schedule(mf.fft_plan_inspect_many([64], mf.FFT_C2C, mf.FFT_FORWARD, mf.FFT_F32)) == (1, 0, 1, [1])
    # a large smooth transform alone: one phase per pass, every block a tile
    w, s, ph, blocks = _schedule(mf.fft_plan_inspect_many([65536], mf.FFT_C2C, mf.FFT_FORWARD, mf.FFT_F32))
    assert (w, s, ph) == (0, 1, 2) and blocks[0] == blocks[1] > 1
    with pytest.raises(mf.MifftError):
        mf.fft_plan_inspect_many([16], mf.FFT_R2C, mf.FFT_FORWARD, mf.FFT_F32)


def test_tuning_table_overrides_and_validation():
    saved = mf.fft_tune_get()
    assert saved == ""
    try:
        mf.fft_tune_set("", replace=True)
        assert mf.fft_tune_get() == ""
        base = mf.fft_plan_inspect(1, [1 << 20], 128, mf.FFT_C2C, mf.FFT_FORWARD, mf.FFT_F32)
        mf.fft_tune_set("# comment line\nf32:L1024:radix=r8.8.16;f32:n1048576:S1:split=s512.2048\n"
                        "f32:L512:8x8x8:CP:tw0=c4,t256", replace=True)
        assert "f32:L1024:radix=r8.8.16" in mf.fft_tune_get()
        d = mf.fft_plan_inspect(1, [1 << 20], 128, mf.FFT_C2C, mf.FFT_FORWARD, mf.FFT_F32)
        assert "L=512 radices=8x8x8" in d and "L=2048" in d
        assert " c=4 T=256 " in passes(d)[0]
        d = mf.fft_plan_inspect(1, [1024], 4, mf.FFT_C2C, mf.FFT_FORWARD, mf.FFT_F32)
        assert "radices=8x8x16" in d
        # entries the planner cannot honour are ignored: wrong product, unknown radix,
        # a split that does not multiply to n
        mf.fft_tune_set("f32:L1024:radix=r8.8.8;f32:L2048:radix=r11.2;f32:n1048576:S1:split=s1000.1000",
                        replace=True)
        assert mf.fft_plan_inspect(1, [1 << 20], 128, mf.FFT_C2C, mf.FFT_FORWARD, mf.FFT_F32) == base
        # merging keeps earlier entries; a later value for a key replaces the earlier
        mf.fft_tune_set("a=c2", replace=True)
        mf.fft_tune_set("b=c4;a=c8")
        assert mf.fft_tune_get() == "a=c8\nb=c4\n"
    finally:
        mf.fft_tune_set(saved, replace=True)


def test_shipped_tuning_table_plans_every_workload():
    # every entry of the shipped table parses, and every benchmark workload still
    # plans with it (the planner falls back to its default for entries it cannot use)
    import os
    from paper_1707_03776_amd import autotune
    if not os.path.exists(mf.TUNING_FILE):
        pytest.skip("no tuning table shipped")
    for line in open(mf.TUNING_FILE):
        line = line.strip()
        if line and not line.startswith("#"):
            key, val = line.split("=", 1)
            assert val and all(f[0] in "cptrswb" for f in val.split(",")), line
    for dims, batch, kind, dtype in list(autotune.sweep_problems()) + list(autotune.other_problems()):
        mf.fft_plan_inspect(len(dims), dims, batch, kind, mf.FFT_FORWARD if kind != mf.FFT_C2R else mf.FFT_INVERSE,
                            dtype)


@pytest.mark.parametrize("L,stages", [(210, 2), (180, 2), (150, 2), (126, 2), (30, 2), (1000, 3), (250, 3),
                                      (768, 3), (567, 3), (4096, 3)])
def test_composite_radices_cut_stages(L, stages):
    # radices 6, 10, 12, 14, 15 (two coprime primes in one butterfly) where they save a
    # stage; lengths with a specialised kernel keep its sequence
    d = inspect((L,), 2)
    rad = [int(r) for r in re.search(r"radices=([\dx]+)", d).group(1).split("x")]
    assert len(rad) == stages and np.prod(rad) == L
    if L in (768, 567, 4096):
        assert " fixed " in d


@pytest.mark.parametrize("n,dtype", [(2916, mf.FFT_F64), (2916, mf.FFT_F32), (6561, mf.FFT_F64), (1458, mf.FFT_F64)])
def test_lengths_that_need_many_threads_plan(n, dtype):
    # single-pass candidates whose runtime-radix tile needs more than 256 threads must
    # fall back to more passes instead of failing to tile
    d = mf.fft_plan_inspect(1, [n], 1, mf.FFT_C2C, mf.FFT_FORWARD, dtype)
    assert all(int(re.search(r" T=(\d+)", l).group(1)) <= (512 if " fixed " in l else 256)
               for l in d.splitlines() if " pass " in l)


@pytest.mark.parametrize("n", [1, 8, 97, 4096, 65536])
@pytest.mark.parametrize("kind", [mf.FFT_DCT2, mf.FFT_DCT3])
def test_dct_plans(n, kind):
    # element-wise prologue, one n-point transform (DCT-II: the real-input plan of the
    # reordered line, into scratch; DCT-III: a complex transform; any length), element-wise
    # epilogue (DCT-II on a staged real transform: the twist and the rotation in one op,
    # or in the last pass's stores when that pass takes mirrored tiles, and the reordering
    # folded into its first pass's loads when that pass is specialised)
    d = mf.fft_plan_inspect(1, [n], 3, kind, mf.FFT_FORWARD, mf.FFT_F32)
    ops = [l.split()[1:4] for l in d.splitlines() if re.match(r"\s+op\d", l)]
    name = "dct2" if kind == mf.FFT_DCT2 else "dct3"
    assert f"kind={name}" in d
    if n >= 65536 and name == "dct2":
        # the reordering folded into op0, the real transform's first pass: it alone reads
        # the input, nothing writes out before the fused twist and rotation
        first = [l for l in d.splitlines() if re.match(r"\s+op0 ", l)][0]
        assert "pro=dct2" in first and first.split()[2].startswith("in->s") and "dct2_pre" not in d, d
        last = [l for l in d.splitlines() if re.match(r"\s+op\d+ ", l)][-1]
        assert all(not o[1].startswith("in->") for o in ops[1:])
        assert (ops[-1][0] == "pass" and "epi=dtwist" in last) or ops[-1][0] == "dct2_twpost", d
        assert "r2c_twist" not in d and "epi=rtwist" not in d
        assert ops[-1][1].endswith("->out") and all(not o[1].endswith("->out") for o in ops[:-1])
        return
    if n >= 65536 and name == "dct3":
        # the inverse reordering folded into the last pass's stores: it alone writes out
        last = [l for l in d.splitlines() if re.match(r"\s+op\d+ ", l)][-1]
        assert "epi=dct3" in last and last.split()[2].endswith("->out") and "dct3_post" not in d, d
        assert ops[0][0] == "dct3_preuntwist" and all(not o[1].endswith("->out") for o in ops[:-1])
        return
    assert ops[0][0] == f"{name}_pre" or (name == "dct3" and ops[0][0] == "dct3_preuntwist")
    assert ops[-1][0] == f"{name}_post" or (name == "dct2" and ops[-1][0] == "dct2_twpost")
    if n >= 65536 and name == "dct2":
        assert ops[-1][0] == "dct2_twpost" and "r2c_twist" not in d
    if n >= 65536 and name == "dct3":
        assert ops[0][0] == "dct3_preuntwist" and "c2r_untwist" not in d
    assert "pass" in [o[0] for o in ops[1:-1]]
    assert ops[-1][1].endswith("->out") and all(not o[1].startswith("in->") for o in ops[1:])
    if kind == mf.FFT_DCT2:
        # the prologue writes the reordered reals to out; nothing else writes out
        # before the epilogue, which reads the half spectrum from scratch
        assert ops[0][1] == "in->out" and all(not o[1].endswith("->out") for o in ops[1:-1])


@pytest.mark.parametrize("n,dtype,folded", [(1 << 20, mf.FFT_F32, True), (1 << 16, mf.FFT_F64, True),
                                             (18000, mf.FFT_F32, False), (1 << 14, mf.FFT_F32, False)])
def test_r2c_twist_folding(n, dtype, folded, monkeypatch):
    # a staged real transform whose last pass is specialised over an even number of
    # columns per line takes the twist in that pass (mirrored tiles, epi=rtwist, straight
    # to out); runtime-radix passes keep the twist op; n/2 within one workgroup has the
    # single fused pass (epi=r2c); MIFFT_TWIST_UNFUSED keeps the op
    d = mf.fft_plan_inspect(1, [n], 5, mf.FFT_R2C, mf.FFT_FORWARD, dtype)
    passes = [l for l in d.splitlines() if re.match(r"\s+op\d+ pass ", l)]
    if folded:
        assert "epi=rtwist" in passes[-1] and passes[-1].split()[2].endswith("->out") and "r2c_twist" not in d, d
        assert all("epi=rtwist" not in l for l in passes[:-1])
        monkeypatch.setenv("MIFFT_TWIST_UNFUSED", "1")
        d = mf.fft_plan_inspect(1, [n], 5, mf.FFT_R2C, mf.FFT_FORWARD, dtype)
    assert "epi=rtwist" not in d, d
    if n // 2 > 8192:
        assert "r2c_twist" in d, d


@pytest.mark.parametrize("n,dtype,folded", [(1 << 20, mf.FFT_F32, True), (1 << 16, mf.FFT_F64, True),
                                             (18000, mf.FFT_F32, False)])
def test_c2r_untwist_folding(n, dtype, folded, monkeypatch):
    # the staged real inverse's untwist rides in the first pass of its chain (mirrored
    # tiles, pro=cuntwist reading the caller's bins) where that pass is specialised;
    # DCT-III keeps it as an op (fused there with the rotation)
    d = mf.fft_plan_inspect(1, [n], 5, mf.FFT_C2R, mf.FFT_INVERSE, dtype)
    first = [l for l in d.splitlines() if re.match(r"\s+op0 ", l)][0]
    if folded:
        assert " pass " in first and "pro=cuntwist" in first and first.split()[2].startswith("in->"), d
        assert "c2r_untwist" not in d and d.count("pro=cuntwist") == d.count(" op0 ")
        monkeypatch.setenv("MIFFT_TWIST_UNFUSED", "1")
        d = mf.fft_plan_inspect(1, [n], 5, mf.FFT_C2R, mf.FFT_INVERSE, dtype)
    assert "pro=cuntwist" not in d and "c2r_untwist" in d, d
    monkeypatch.delenv("MIFFT_TWIST_UNFUSED", raising=False)
    d3 = mf.fft_plan_inspect(1, [n], 5, mf.FFT_DCT3, mf.FFT_FORWARD, dtype)
    assert "pro=cuntwist" not in d3


def test_dct2_reorder_fusion_switch(monkeypatch):
    # MIFFT_DCT2_UNFUSED keeps the reordering an op of its own (as for lengths whose real
    # transform starts with a runtime-radix or Bluestein pass)
    n = 1 << 20
    assert "pro=dct2" in mf.fft_plan_inspect(1, [n], 4, mf.FFT_DCT2, mf.FFT_FORWARD, mf.FFT_F32)
    monkeypatch.setenv("MIFFT_DCT2_UNFUSED", "1")
    d = mf.fft_plan_inspect(1, [n], 4, mf.FFT_DCT2, mf.FFT_FORWARD, mf.FFT_F32)
    assert "pro=dct2" not in d and "dct2_pre" in d
    assert "dct2_pre" in mf.fft_plan_inspect(1, [8198], 1, mf.FFT_DCT2, mf.FFT_FORWARD, mf.FFT_F32)


def test_dct3_reorder_fusion_switch(monkeypatch):
    # MIFFT_DCT3_UNFUSED keeps the inverse reordering an op of its own
    n = 1 << 20
    assert "epi=dct3" in mf.fft_plan_inspect(1, [n], 4, mf.FFT_DCT3, mf.FFT_FORWARD, mf.FFT_F32)
    monkeypatch.setenv("MIFFT_DCT3_UNFUSED", "1")
    d = mf.fft_plan_inspect(1, [n], 4, mf.FFT_DCT3, mf.FFT_FORWARD, mf.FFT_F32)
    assert "epi=dct3" not in d and "dct3_post" in d


@pytest.mark.parametrize("n", [8198, 8194, 20000, 2 * 65521])
def test_dct3_fused_prologue_keeps_bluestein_scratch(n):
    # the fused DCT-III rotation-and-untwist needs no staged half spectrum, but the
    # Bluestein steps of a prime n/2 still need their padded lines in S2 (a plan that named
    # S2 without sizing it once wrote through a null scratch pointer)
    d = mf.fft_plan_inspect(1, [n], 2, mf.FFT_DCT3, mf.FFT_FORWARD, mf.FFT_F32)
    used = set(re.findall(r"op\d+ \w+ (\w+)->", d)) | set(re.findall(r"op\d+ \w+ \w+->(\w+)", d))
    for b in used:
        if b.startswith("s"):
            assert f"{b}_bytes=" in d, (b, d)


@pytest.mark.parametrize("args", [dict(rank=2), dict(direction=mf.FFT_INVERSE), dict(dtype=mf.FFT_F32_BF16X2)])
def test_dct_rejects(args):
    a = dict(rank=1, direction=mf.FFT_FORWARD, dtype=mf.FFT_F32)
    a.update(args)
    dims = [16] * a["rank"]
    with pytest.raises(mf.MifftError):
        mf.fft_plan_inspect(a["rank"], dims, 1, mf.FFT_DCT2, a["direction"], a["dtype"])


@pytest.mark.parametrize("rank,dims,lengths,dtype", [
    (0, [8], [1.0], mf.FFT_F32),                     # rank
    (4, [2, 2, 2, 2], [1.0] * 4, mf.FFT_F32),
    (1, [8], [0.0], mf.FFT_F32),                     # period not positive
    (2, [8, 8], [1.0, float("nan")], mf.FFT_F64),   # period not finite
    (1, [8], [1.0], mf.FFT_F32_BF16X2),              # dtype
])
def test_laplacian_rejects_before_touching_the_gpu(rank, dims, lengths, dtype):
    with pytest.raises(mf.MifftError) as e:
        mf.fft_laplacian_create(rank, dims, 1, lengths, dtype)
    assert e.value.status == mf.FFT_ERR_INVALID_ARG


def test_laplacian_null_operator_is_an_error():
    with pytest.raises(mf.MifftError):
        mf.fft_laplacian_execute(0, 0, 0)
    mf.fft_laplacian_destroy(0)  # NULL-safe


def test_bench_counts_chunk_launches():
    """bench.py counts the kernel dispatches of a chunked plan: passes x chunks, the
    shorter last chunk's own op list included."""
    import bench
    one = "mifft plan rank=1\n  op0 pass in->out L=1024\n  tables=1\n"
    assert bench.plan_launches(one) == (1, 1, 1)
    even = ("mifft plan\n  chunks of 32 transforms (4 chunks)\n  op0 pass in->s0 L=1024\n"
            "  op1 pass s0->out L=1024\n  tables=3\n")
    assert bench.plan_launches(even) == (2, 2, 8)
    ragged_tail = ("mifft plan\n  chunks of 22 transforms (8 chunks, the last of 16)\n  op0 pass in->s0 L=1024\n"
                   "  op1 pass s0->out L=768\n  last chunk:\n  op0 pass in->s0 L=1024\n  op1 pass s0->out L=768\n")
    assert bench.plan_launches(ragged_tail) == (2, 2, 16)
    import paper_1707_03776_amd as mf
    d = mf.fft_plan_inspect(1, [1 << 24], 8, mf.FFT_C2C, mf.FFT_FORWARD, mf.FFT_F32).split("  in place")[0]
    p, o, k = bench.plan_launches(d)
    assert p == o == d.count(" pass ") - (d.split("  last chunk:")[1].count(" pass ") if "last chunk" in d else 0)
    assert k % p == 0 and k >= p
