"""Pins for the FP64 oracle: each test checks it against something other than itself.

The oracle (``oracle/oracle.c``) is a recursive Cooley–Tukey; the pins below are
the DFT definition summed by brute force (FP64 and 50-digit mpmath), closed forms,
hand-worked fixtures, and invariants of the transform (inverse, Parseval,
linearity, shift and convolution theorems, adjointness, Hermitian symmetry).
Chosen so that a dropped term, a wrong sign, a wrong index, a transposed axis or
a missing scale each fails at least one of them (``test_planted_mistakes_are_caught``
checks exactly that against deliberately broken copies of the oracle).
"""
import json
import os
import subprocess

import mpmath
import numpy as np
import pytest

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))


def brute_dft(x, sign=-1):
    """O(n^2) DFT along the last axis, exponent reduced exactly mod n."""
    n = x.shape[-1]
    j = np.arange(n)
    e = np.outer(j, j) % n
    W = np.exp(sign * 2j * np.pi * e / n)
    return x @ W.T


def brute_dftn(x, ndim, sign=-1):
    """Brute-force multi-dimensional DFT over the trailing ``ndim`` axes."""
    y = np.asarray(x, dtype=np.complex128)
    for ax in range(y.ndim - ndim, y.ndim):
        y = np.moveaxis(brute_dft(np.moveaxis(y, ax, -1), sign), -1, ax)
    return y


def crandn(rng, shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def relerr(a, b):
    return np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(np.asarray(b).ravel()), 1e-300)


# --------------------------------------------------------------------------- brute force


@pytest.mark.parametrize("n", list(range(1, 129)))
def test_bruteforce_every_small_n(n):
    rng = np.random.default_rng(n)
    x = crandn(rng, (2, n))
    assert relerr(oracle.c2c(x, (n,)), brute_dft(x)) < 2e-15 * max(1.0, np.log2(n))
    assert relerr(oracle.c2c(x, (n,), inverse=True), brute_dft(x, +1) / n) < 2e-15 * max(1.0, np.log2(n))


PRIMES_TO_127 = [p for p in range(2, 128) if all(p % q for q in range(2, int(p ** 0.5) + 1))]
CONFIG_ANALOGUES = ([2 ** k for k in range(8, 13)] + [3 * 2 ** k for k in range(4, 9)]
                    + [5 * 2 ** k for k in range(4, 8)] + [7 * 3 ** k for k in range(1, 5)]
                    + [131, 257, 509, 1021])


@pytest.mark.parametrize("n", CONFIG_ANALOGUES)
def test_bruteforce_config_analogues(n):
    # powers of two to 4096, 3*2^k, 5*2^k, 7*3^k (small versions of the benchmark
    # lengths) and primes that need the direct-sum leaf
    rng = np.random.default_rng(1000 + n)
    x = crandn(rng, (1, n))
    assert relerr(oracle.c2c(x, (n,)), brute_dft(x)) < 1e-14


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6, 7, 8, 9, 12, 16, 25, 27, 31, 32])
def test_mpmath_50_digits(n):
    mpmath.mp.dps = 50
    rng = np.random.default_rng(7 * n)
    x = crandn(rng, n)
    got = oracle.c2c(x[None, :], (n,))[0]
    ref = []
    for k in range(n):
        s = mpmath.mpc(0)
        for j in range(n):
            s += mpmath.mpc(x[j].real, x[j].imag) * mpmath.expjpi(mpmath.mpf(-2 * ((j * k) % n)) / n)
        ref.append(complex(s))
    ref = np.array(ref)
    assert relerr(got, ref) < 1e-15


@pytest.mark.parametrize("dims", [(3, 5), (4, 4), (6, 7), (2, 3, 4), (5, 1, 3), (8, 8, 8), (1, 1, 9)])
def test_bruteforce_multidim(dims):
    rng = np.random.default_rng(sum(dims))
    x = crandn(rng, (2,) + dims)
    nd = len(dims)
    assert relerr(oracle.c2c(x, dims), brute_dftn(x, nd)) < 1e-14
    n = int(np.prod(dims))
    assert relerr(oracle.c2c(x, dims, inverse=True), brute_dftn(x, nd, +1) / n) < 1e-14


# --------------------------------------------------------------------------- hand-worked fixtures


def test_hand_worked_fixtures():
    with open(os.path.join(HERE, "golden", "hand_worked.json")) as f:
        cases = json.load(f)["cases"]
    for c in cases:
        dims = tuple(c["dims"])
        if c["kind"] == "c2c":
            x = (np.array(c["x_re"], float) + 1j * np.array(c["x_im"], float)).reshape((1,) + dims)
            X = (np.array(c["X_re"], float) + 1j * np.array(c["X_im"], float)).reshape((1,) + dims)
            np.testing.assert_allclose(oracle.c2c(x, dims), X, atol=1e-14, err_msg=c["derivation"])
            np.testing.assert_allclose(oracle.c2c(X, dims, inverse=True), x, atol=1e-14)
        elif c["kind"] == "r2c":
            x = np.array(c["x"], float).reshape((1,) + dims)
            X = np.array(c["X_re"], float) + 1j * np.array(c["X_im"], float)
            np.testing.assert_allclose(oracle.r2c(x, dims)[0], X, atol=1e-14, err_msg=c["derivation"])
        else:
            X = (np.array(c["X_re"], float) + 1j * np.array(c["X_im"], float))[None]
            x = np.array(c["x"], float)
            np.testing.assert_allclose(oracle.c2r(X, dims)[0], x, atol=1e-14, err_msg=c["derivation"])


# --------------------------------------------------------------------------- closed forms


@pytest.mark.parametrize("n", [1, 2, 7, 16, 60, 97, 1024, 4096, 3 * 2 ** 8, 5 * 2 ** 6, 7 * 27])
def test_closed_forms(n):
    j = np.arange(n)
    # delta at 0 -> all ones
    d0 = np.zeros((1, n), complex)
    d0[0, 0] = 1
    np.testing.assert_allclose(oracle.c2c(d0, (n,))[0], np.ones(n), atol=1e-15)
    # constant c -> c*n at DC only
    c = 0.75 - 0.25j
    out = oracle.c2c(np.full((1, n), c), (n,))[0]
    ref = np.zeros(n, complex)
    ref[0] = c * n
    np.testing.assert_allclose(out, ref, atol=1e-12 * n)
    if n < 3:
        return
    # delta at j0 -> exp(-2 pi i j0 k / n)  (sign of the exponent)
    j0 = n // 3
    dj = np.zeros((1, n), complex)
    dj[0, j0] = 1
    ref = np.exp(-2j * np.pi * ((j0 * j) % n) / n)
    np.testing.assert_allclose(oracle.c2c(dj, (n,))[0], ref, atol=1e-14)
    # tone exp(+2 pi i k0 j/n) -> n at k0 only (k0 != n - k0 catches a flipped sign)
    k0 = max(1, n // 5)
    tone = np.exp(2j * np.pi * ((k0 * j) % n) / n)[None]
    ref = np.zeros(n, complex)
    ref[k0] = n
    np.testing.assert_allclose(oracle.c2c(tone, (n,))[0], ref, atol=1e-12 * n)
    # cosine tone -> n/2 at +k0 and -k0
    if 2 * k0 != n:
        cs = np.cos(2 * np.pi * ((k0 * j) % n) / n)[None] + 0j
        ref = np.zeros(n, complex)
        ref[k0] += n / 2
        ref[n - k0] += n / 2
        np.testing.assert_allclose(oracle.c2c(cs, (n,))[0], ref, atol=1e-12 * n)


def test_separable_tone_multidim():
    # product of per-axis tones with distinct frequencies lands on one spike; a
    # transposed or skipped axis moves or smears it
    dims = (6, 10, 8)
    k = (1, 3, 2)
    grids = np.meshgrid(*[np.arange(d) for d in dims], indexing="ij")
    phase = sum(2 * np.pi * ((kk * g) % d) / d for kk, g, d in zip(k, grids, dims))
    x = np.exp(1j * phase)[None]
    out = oracle.c2c(x, dims)[0]
    ref = np.zeros(dims, complex)
    ref[k] = np.prod(dims)
    np.testing.assert_allclose(out, ref, atol=1e-11)


def test_unit_root_exact_points_and_accuracy():
    for n in [4, 8, 12, 16, 1024, 3 << 18, 1 << 24]:
        assert oracle.unit_root(n, 0) == 1 + 0j
        assert oracle.unit_root(n, n // 4) == complex(0, -1)
        assert oracle.unit_root(n, n // 2) == complex(-1, 0)
        assert oracle.unit_root(n, 3 * n // 4) == complex(0, 1)
        assert oracle.unit_root(n, n // 4, +1) == complex(0, 1)
        if n % 8 == 0:
            w8 = oracle.unit_root(n, n // 8)
            assert w8.real == -w8.imag
    mpmath.mp.dps = 40
    rng = np.random.default_rng(3)
    for _ in range(300):
        n = int(rng.integers(1, 1 << 24))
        m = int(rng.integers(-3 * n, 3 * n))
        w = oracle.unit_root(n, m)
        ref = mpmath.expjpi(mpmath.mpf(-2 * (m % n)) / n)
        assert abs(w - complex(ref)) < 2.5e-16


# --------------------------------------------------------------------------- invariants


@pytest.mark.parametrize("n", [12, 64, 105, 243, 1000, 4096, 3 * 2 ** 10, 7 * 3 ** 5, 65536, 1 << 20])
def test_invariants(n):
    rng = np.random.default_rng(n)
    x, y = crandn(rng, (1, n)), crandn(rng, (1, n))
    X, Y = oracle.c2c(x, (n,)), oracle.c2c(y, (n,))
    tol = 4e-16 * np.log2(n) * 8
    # inverse round trip
    assert relerr(oracle.c2c(X, (n,), inverse=True), x) < tol
    # Parseval
    assert abs(np.sum(abs(X) ** 2) - n * np.sum(abs(x) ** 2)) / (n * np.sum(abs(x) ** 2)) < tol
    # linearity
    a, b = 0.3 - 1.7j, -2.1 + 0.4j
    assert relerr(oracle.c2c(a * x + b * y, (n,)), a * X + b * Y) < tol
    # adjointness <F x, y> = <x, F^H y> = n <x, F^-1 y>
    lhs = np.vdot(y, X)
    rhs = n * np.vdot(oracle.c2c(y, (n,), inverse=True), x)
    assert abs(lhs - rhs) / (np.linalg.norm(X) * np.linalg.norm(y)) < tol
    # shift theorem: x[j - s] -> X[k] exp(-2 pi i s k / n)
    s = n // 7 + 1
    k = np.arange(n)
    ramp = np.exp(-2j * np.pi * ((s * k) % n) / n)
    assert relerr(oracle.c2c(np.roll(x, s, axis=1), (n,)), X * ramp) < tol


@pytest.mark.parametrize("n", [8, 30, 37, 64, 210])
def test_convolution_theorem(n):
    rng = np.random.default_rng(11 * n)
    a, b = crandn(rng, n), crandn(rng, n)
    direct = np.array([sum(a[j] * b[(k - j) % n] for j in range(n)) for k in range(n)])
    A = oracle.c2c(a[None], (n,))
    B = oracle.c2c(b[None], (n,))
    conv = oracle.c2c(A * B, (n,), inverse=True)[0]
    assert relerr(conv, direct) < 1e-14


def test_multidim_invariants():
    rng = np.random.default_rng(5)
    dims = (12, 18, 10)
    x = crandn(rng, (2,) + dims)
    X = oracle.c2c(x, dims)
    n = int(np.prod(dims))
    assert relerr(oracle.c2c(X, dims, inverse=True), x) < 1e-14
    np.testing.assert_allclose(np.sum(abs(X) ** 2, axis=(1, 2, 3)), n * np.sum(abs(x) ** 2, axis=(1, 2, 3)),
                               rtol=1e-13)


# --------------------------------------------------------------------------- real transforms


@pytest.mark.parametrize("dims", [(1,), (2,), (7,), (16,), (100,), (513,), (4, 6), (5, 9), (3, 4, 8), (6, 5, 7)])
def test_r2c_c2r(dims):
    rng = np.random.default_rng(len(dims) * 100 + dims[-1])
    x = rng.standard_normal((2,) + dims)
    X = oracle.r2c(x, dims)
    full = brute_dftn(x + 0j, len(dims))
    h = dims[-1] // 2 + 1
    assert relerr(X, full[..., :h]) < 1e-14
    # Hermitian symmetry of the full c2c of real input: X[-k] = conj X[k]
    flip = full
    for ax in range(1, full.ndim):
        flip = np.roll(np.flip(flip, axis=ax), 1, axis=ax)
    assert relerr(np.conj(flip), full) < 1e-14
    # DC (and Nyquist) bins of a 1-D real transform are exactly real in the oracle
    if len(dims) == 1:
        assert np.all(X[:, 0].imag == 0)
        if dims[0] % 2 == 0:
            assert np.all(X[:, -1].imag == 0)
    # c2r inverts r2c
    assert relerr(oracle.c2r(X, dims), x) < 1e-14


@pytest.mark.parametrize("n", [1, 2, 5, 8, 9, 64, 75])
def test_c2r_definition_on_non_hermitian_input(n):
    # numpy semantics: only Re X[0] and (n even) Re X[n/2] enter; the rest is the
    # 2 * sum Re(X[k] e^{2 pi i jk/n}) of the definition, summed directly here
    rng = np.random.default_rng(n + 500)
    X = crandn(rng, n // 2 + 1)
    np.testing.assert_allclose(oracle.c2r(X[None], (n,))[0], c2r_direct(X, n), atol=1e-14)


def c2r_direct(X, n):
    """The 1-D c2r definition summed term by term."""
    h = n // 2 + 1
    j = np.arange(n)
    ref = np.full(n, X[0].real)
    for k in range(1, h):
        if 2 * k == n:
            ref += ((-1.0) ** j) * X[k].real
        else:
            ref += 2 * np.real(X[k] * np.exp(2j * np.pi * ((j * k) % n) / n))
    return ref / n


def test_tone_spike_r2c_3d():
    # the added-tone pin used for the 3-D real workload: A cos(2 pi k.x/N + phi)
    # lands on (A N/2) e^{i phi} at +k (with the conjugate at -k folded away)
    dims = (8, 12, 16)
    k = (3, 5, 6)
    phi = 0.7
    grids = np.meshgrid(*[np.arange(d) for d in dims], indexing="ij")
    arg = sum(2 * np.pi * ((kk * g) % d) / d for kk, g, d in zip(k, grids, dims))
    x = np.cos(arg + phi)[None]
    X = oracle.r2c(x, dims)[0]
    N = np.prod(dims)
    assert abs(X[k] - N / 2 * np.exp(1j * phi)) < 1e-11
    mask = np.ones(X.shape, bool)
    mask[k] = False
    assert np.max(np.abs(X[mask])) < 1e-11


def test_numpy_cross_check():
    # third-party cross-check only (never used by the oracle or the GPU path)
    rng = np.random.default_rng(42)
    for dims in [(1000,), (3 * 2 ** 9,), (7 * 3 ** 4,), (64, 48), (10, 12, 14)]:
        x = crandn(rng, (2,) + dims)
        axes = tuple(range(1, 1 + len(dims)))
        assert relerr(oracle.c2c(x, dims), np.fft.fftn(x, axes=axes)) < 1e-14
        xr = x.real
        assert relerr(oracle.r2c(xr, dims), np.fft.rfftn(xr, axes=axes)) < 1e-14


def test_bad_arguments_raise():
    with pytest.raises(RuntimeError):
        oracle.c2c(np.zeros((1, 0), complex), (0,))


# --------------------------------------------------------------------------- pin strength

PLANTS = {
    # each is a one-token mistake somewhere in the oracle; each must fail a pin
    "sign": ("cplx w = {c, sigma > 0 ? s : -s};", "cplx w = {c, sigma > 0 ? -s : s};"),
    "dropped_term": ("for (int64_t r = 0; r < p; ++r) {\n                cplx t",
                     "for (int64_t r = 1; r < p; ++r) {\n                cplx t"),
    "index": ("const int64_t idx = k + q * m;", "const int64_t idx = q + k * p;"),
    "octant": ("case 3: c = -cos(psi); s = sin(psi);  break;", "case 3: c = -sin(psi); s = cos(psi);  break;"),
    "scale": ("const double sc = 1.0 / (double)per;", "const double sc = 1.0;"),
    "hermitian": ("y[n - k].im = -x[k].im;", "y[n - k].im = x[k].im;"),
}


@pytest.mark.parametrize("plant", sorted(PLANTS))
def test_planted_mistakes_are_caught(plant, tmp_path):
    """Compile a broken copy of the oracle and check the pin tests above reject it."""
    src = open(os.path.join(os.path.dirname(oracle.__file__), "oracle.c")).read()
    old, new = PLANTS[plant]
    assert old in src, plant
    bad = tmp_path / "oracle.c"
    bad.write_text(src.replace(old, new, 1))
    so = tmp_path / "liboracle.so"
    subprocess.run(["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-fopenmp", "-fPIC", "-shared", "-o", str(so),
                    str(bad), "-lm"], check=True)
    import ctypes
    lib = ctypes.CDLL(str(so))
    i64p = ctypes.POINTER(ctypes.c_int64)
    lib.oracle_c2c.argtypes = [ctypes.c_int, i64p, ctypes.c_int64, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p]
    lib.oracle_c2r.argtypes = [ctypes.c_int, i64p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p]

    def bad_c2c(x, n, inverse=False):
        x = np.ascontiguousarray(x, np.complex128)
        out = np.empty_like(x)
        d = (ctypes.c_int64 * 1)(n)
        lib.oracle_c2c(1, d, x.size // n, 1 if inverse else -1, x.ctypes.data, out.ctypes.data)
        return out

    def bad_c2r(X, n):
        X = np.ascontiguousarray(X, np.complex128)
        out = np.empty(X.shape[:-1] + (n,))
        d = (ctypes.c_int64 * 1)(n)
        lib.oracle_c2r(1, d, X.size // (n // 2 + 1), X.ctypes.data, out.ctypes.data)
        return out

    rng = np.random.default_rng(0)
    caught = False
    for n in [4, 6, 8, 9, 12, 30]:
        x = crandn(rng, (1, n))
        if relerr(bad_c2c(x, n), brute_dft(x)) > 1e-12:
            caught = True
        if relerr(bad_c2c(x, n, True), brute_dft(x, +1) / n) > 1e-12:
            caught = True
        X = crandn(rng, (1, n // 2 + 1))
        if relerr(bad_c2r(X, n)[0], c2r_direct(X[0], n)) > 1e-12:
            caught = True
    assert caught, f"planted mistake '{plant}' slipped through the pins"


# ----------------------------------------------------------------------------- DCT-II / DCT-III

@pytest.mark.parametrize("n", [1, 2, 3, 5, 8, 13, 64, 97, 100])
def test_dct_matches_scipy(n):
    # third-party cross-check: scipy.fft.dct, unnormalised (norm=None)
    import scipy.fft as sf
    x = np.random.default_rng(n).standard_normal((4, n))
    for t in (2, 3):
        ref = sf.dct(x, t)
        assert np.max(np.abs(oracle.dct(x, t) - ref)) <= 1e-13 * max(1.0, np.max(np.abs(ref)))


def test_dct_closed_forms():
    n = 12
    c = 0.75
    # DCT-II of a constant: 2 n c at k = 0, zero elsewhere (sum of cos over a full period)
    y = oracle.dct(np.full(n, c), 2)
    assert abs(y[0] - 2 * n * c) < 1e-13 and np.max(np.abs(y[1:])) < 1e-13
    # DCT-III of delta_0: all ones; of delta_j: 2 cos(pi j (2k+1)/(2n))
    assert np.max(np.abs(oracle.dct(np.eye(n)[0], 3) - 1.0)) < 1e-15
    j = 5
    k = np.arange(n)
    assert np.max(np.abs(oracle.dct(np.eye(n)[j], 3) - 2 * np.cos(np.pi * j * (2 * k + 1) / (2 * n)))) < 1e-14
    # n = 2 by hand: y0 = 2 (a + b), y1 = 2 (a cos(pi/4) + b cos(3 pi/4)) = sqrt(2) (a - b)
    a, b = 1.5, -0.25
    y = oracle.dct(np.array([a, b]), 2)
    assert abs(y[0] - 2 * (a + b)) < 1e-15 and abs(y[1] - np.sqrt(2) * (a - b)) < 1e-15


@pytest.mark.parametrize("n", [1, 4, 9, 31, 128])
def test_dct_round_trip_and_transpose(n):
    # type 3 of type 2 is 2n x; the type-3 matrix is the transpose of the type-2 matrix
    # with the first column halved
    rng = np.random.default_rng(100 + n)
    x = rng.standard_normal(n)
    assert np.max(np.abs(oracle.dct(oracle.dct(x, 2), 3) - 2 * n * x)) <= 1e-12 * max(1, n)
    C2 = oracle.dct(np.eye(n), 2).T  # column j = DCT-II of e_j -> C2[k, j]
    C3 = oracle.dct(np.eye(n), 3).T
    w = np.full(n, 1.0)
    w[0] = 0.5
    assert np.max(np.abs(C3 - C2.T * w[None, :])) < 1e-12


# ---------------------------------------------------------------------------
# Pseudo-spectral Laplacian.  The operator is linear and diagonal in the Fourier
# basis, so checking it on every grid mode (cosine and sine phases) of small grids
# fixes it completely; a smooth non-trigonometric field with a hand-derived
# Laplacian pins the physical scale 2 pi / L and the sign independently of the
# transforms; the second-order finite-difference stencil (the paper's laplace
# operator on a uniform grid) must approach it at rate h^2.

def _grid(dims, lengths):
    axes = [np.arange(n) * (L / n) for n, L in zip(dims, lengths)]
    return np.meshgrid(*axes, indexing="ij")


@pytest.mark.parametrize("dims,lengths", [((6,), (2.5,)), ((5,), (1.0,)), ((4, 6), (1.0, 3.0)),
                                          ((3, 4, 5), (2.0, 0.5, 7.0)), ((4, 2, 6), (1.0, 1.0, 1.0))])
def test_laplacian_every_mode(dims, lengths):
    X = _grid(dims, lengths)
    for f in np.ndindex(*dims):
        fs = [j if j <= n // 2 else j - n for j, n in zip(f, dims)]
        theta = sum(2 * np.pi * fa * x / L for fa, x, L in zip(fs, X, lengths))
        lam = -sum((2 * np.pi * fa / L) ** 2 for fa, L in zip(fs, lengths))
        for phase in (0.0, 0.5 * np.pi, 1.1):
            u = np.cos(theta + phase)
            lu = oracle.laplacian(u, dims, lengths)
            assert np.max(np.abs(lu - lam * u)) <= 1e-12 * max(1.0, abs(lam)), (dims, f, phase)


def test_laplacian_smooth_field_closed_form():
    # u = exp(sin(a x)) cos(b y) with a = 2 pi / Lx, b = 4 pi / Ly:
    # u_xx = a^2 (cos^2(a x) - sin(a x)) u, u_yy = -b^2 u
    dims, lengths = (64, 32), (3.0, 1.7)
    X, Y = _grid(dims, lengths)
    a, b = 2 * np.pi / lengths[0], 4 * np.pi / lengths[1]
    u = np.exp(np.sin(a * X)) * np.cos(b * Y)
    exact = (a * a * (np.cos(a * X) ** 2 - np.sin(a * X)) - b * b) * u
    lu = oracle.laplacian(u, dims, lengths)
    assert np.max(np.abs(lu - exact)) <= 1e-9 * np.max(np.abs(exact))


def test_laplacian_second_order_stencil_converges():
    # 2nd-order central differences on the same smooth field: error ~ h^2 against the
    # spectral result (ratio ~4 per halving of h)
    errs = []
    for n in (16, 32, 64):
        dims, lengths = (n, n), (1.0, 2.0)
        X, Y = _grid(dims, lengths)
        u = np.exp(np.sin(2 * np.pi * X)) * np.cos(np.pi * Y)
        h = [L / m for L, m in zip(lengths, dims)]
        fd = sum((np.roll(u, 1, ax) - 2 * u + np.roll(u, -1, ax)) / h[ax] ** 2 for ax in range(2))
        errs.append(np.max(np.abs(fd - oracle.laplacian(u, dims, lengths))))
    assert 3.5 < errs[0] / errs[1] < 4.5 and 3.5 < errs[1] / errs[2] < 4.5, errs


def test_laplacian_self_adjoint_and_mean_free():
    rng = np.random.default_rng(77)
    dims, lengths = (6, 5, 8), (1.0, 2.0, 0.5)
    u, v = rng.standard_normal(dims), rng.standard_normal(dims)
    lu, lv = oracle.laplacian(u, dims, lengths), oracle.laplacian(v, dims, lengths)
    assert abs(np.sum(lu * v) - np.sum(u * lv)) <= 1e-11 * np.sum(np.abs(lu * v))
    assert abs(np.sum(lu)) <= 1e-11 * np.sum(np.abs(lu))
    # a batch is independent fields
    w = np.stack([u, v])
    assert np.max(np.abs(oracle.laplacian(w, dims, lengths) - np.stack([lu, lv]))) < 1e-12


def test_laplacian_against_stencil_symbol():
    # on a single mode the 2nd-order stencil multiplies by -(4/h^2) sin^2(pi f/n) and the
    # spectral operator by -(2 pi f/L)^2; their ratio is (sin(t)/t)^2 with t = pi f/n
    n, L = 48, 3.0
    h = L / n
    x = np.arange(n) * h
    for f in (1, 5, 12, 23, 24):
        u = np.cos(2 * np.pi * f * x / L + 0.3)
        fd = (np.roll(u, 1) - 2 * u + np.roll(u, -1)) / h ** 2
        sp = oracle.laplacian(u, (n,), (L,))
        t = np.pi * f / n
        assert np.max(np.abs(fd + 4 / h ** 2 * np.sin(t) ** 2 * u)) < 1e-9
        assert np.max(np.abs(sp + (2 * np.pi * f / L) ** 2 * u)) < 1e-9
        assert abs(np.dot(fd, u) / np.dot(sp, u) - (np.sin(t) / t) ** 2) < 1e-12
