"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module only draws numbers; it holds none of the transform's arithmetic, and
both the GPU path and the CPU oracle receive exactly the arrays made here.

Seeds follow one rule: ``numpy.random.default_rng(1000*c + i)`` where ``c`` is the
workload number (1: c128 n=4096 x64; 2: the 1-D size sweep; 3: multi-dimensional;
4: the split-BF16 precision workload; 5: the ragged batch) and ``i`` its 1-based
case index.  Complex N(0,1) draws the real and imaginary parts independently in
FP64 and rounds to the requested dtype.
"""
from __future__ import annotations

import math

import numpy as np

# 1-D lengths of the size sweep, in order
SWEEP_LENGTHS = [2 ** 10, 2 ** 16, 2 ** 20, 2 ** 24, 3 * 2 ** 18, 5 * 2 ** 16, 7 * 3 ** 9]


def seed_for(workload: int, case: int) -> int:
    return 1000 * workload + case


def complex_normal(rng: np.random.Generator, shape, dtype=np.complex64) -> np.ndarray:
    """Real and imaginary parts i.i.d. N(0,1), drawn in FP64 then rounded to dtype."""
    re = rng.standard_normal(shape)
    im = rng.standard_normal(shape)
    out = np.empty(shape, dtype=dtype)
    out.real = re
    out.imag = im
    return out


def sweep_batch(n: int, dtype) -> int:
    """Batch that makes a ~1 GiB input: floor(2^30 / (n * bytes per element))."""
    return max(1, (1 << 30) // (n * np.dtype(dtype).itemsize))


def sweep_case_index(n: int, dtype) -> int:
    """1-based index of (n, dtype) in the sweep: lengths in order, complex64 first."""
    k = SWEEP_LENGTHS.index(n)
    return 2 * k + (1 if np.dtype(dtype) == np.complex64 else 2)


def tones_real(rng: np.random.Generator, dims, count: int = 3):
    """(frequency vectors, phases) for ``count`` distinct pure tones, each axis
    frequency an integer in [1, d/2 - 1] (never DC or Nyquist)."""
    freqs, phases = [], []
    while len(freqs) < count:
        k = tuple(int(rng.integers(1, max(2, d // 2))) for d in dims)
        if k in freqs:
            continue
        freqs.append(k)
        phases.append(float(rng.uniform(0.0, 2.0 * math.pi)))
    return freqs, phases


def _phase_grid(dims, k):
    grids = np.meshgrid(*[np.arange(d, dtype=np.int64) for d in dims], indexing="ij", sparse=True)
    arg = 0.0
    for kk, g, d in zip(k, grids, dims):
        arg = arg + (2.0 * math.pi / d) * ((kk * g) % d)
    return arg


def real_with_tones(rng: np.random.Generator, dims, count: int = 3, dtype=np.float32):
    """uniform[-1, 1) plus ``count`` unit-amplitude cosines cos(2 pi k.x/N + phi).
    Returns (array, freqs, phases, noise) with noise the uniform part alone."""
    noise = rng.uniform(-1.0, 1.0, size=tuple(dims))
    freqs, phases = tones_real(rng, dims, count)
    x = noise.copy()
    for k, ph in zip(freqs, phases):
        x += np.cos(_phase_grid(dims, k) + ph)
    return x.astype(dtype), freqs, phases, noise.astype(dtype)


def complex_with_tones(rng: np.random.Generator, dims, count: int = 3, dtype=np.complex64):
    """re, im uniform[-1, 1) plus ``count`` unit complex exponentials exp(i(2 pi k.x/N + phi))."""
    re = rng.uniform(-1.0, 1.0, size=tuple(dims))
    im = rng.uniform(-1.0, 1.0, size=tuple(dims))
    freqs, phases = tones_real(rng, dims, count)
    x = re + 1j * im
    for k, ph in zip(freqs, phases):
        x = x + np.exp(1j * (_phase_grid(dims, k) + ph))
    noise = (re + 1j * im).astype(dtype)
    return x.astype(dtype), freqs, phases, noise


# ---------------------------------------------------------------------------- ragged batch


def smooth_pool(lo: int = 64, hi: int = 65536):
    """All 2^a 3^b 5^c 7^d in [lo, hi], sorted."""
    out = []
    p2 = 1
    while p2 <= hi:
        p3 = p2
        while p3 <= hi:
            p5 = p3
            while p5 <= hi:
                p7 = p5
                while p7 <= hi:
                    if p7 >= lo:
                        out.append(p7)
                    p7 *= 7
                p5 *= 5
            p3 *= 3
        p2 *= 2
    return sorted(out)


def prime_pool(lo: int = 64, hi: int = 65536):
    sieve = np.ones(hi + 1, dtype=bool)
    sieve[:2] = False
    for p in range(2, int(hi ** 0.5) + 1):
        if sieve[p]:
            sieve[p * p::p] = False
    return [int(p) for p in np.nonzero(sieve)[0] if p >= lo]


def _nearest_log(pool, target_log):
    logs = np.log(np.asarray(pool, dtype=np.float64))
    i = int(np.searchsorted(logs, target_log))
    if i <= 0:
        return pool[0]
    if i >= len(pool):
        return pool[-1]
    # ties go to the smaller length
    return pool[i - 1] if target_log - logs[i - 1] <= logs[i] - target_log else pool[i]


def ragged_lengths(count: int = 20000, prime_fraction: float = 0.05, lo: int = 64, hi: int = 65536,
                   seed: int = 5001):
    """Lengths of the ragged batch: log-uniform in [lo, hi], snapped to the nearest
    7-smooth length, except round(prime_fraction*count) seeded slots snapped to
    the nearest prime."""
    rng = np.random.default_rng(seed)
    n_primes = int(round(prime_fraction * count))
    prime_slots = set(int(i) for i in rng.choice(count, n_primes, replace=False)) if n_primes else set()
    smooth, primes = smooth_pool(lo, hi), prime_pool(lo, hi)
    u = rng.uniform(math.log(lo), math.log(hi), size=count)
    return [(_nearest_log(primes, u[i]) if i in prime_slots else _nearest_log(smooth, u[i]))
            for i in range(count)]


def ragged_inputs(lengths, seed: int = 5001, dtype=np.complex64):
    """One packed buffer of complex N(0,1) values and the per-transform offsets."""
    offsets = np.zeros(len(lengths) + 1, dtype=np.int64)
    offsets[1:] = np.cumsum(np.asarray(lengths, dtype=np.int64))
    rng = np.random.default_rng(seed + 10 ** 6)
    data = complex_normal(rng, int(offsets[-1]), dtype)
    return data, offsets


def device_complex_normal(shape, dtype, seed: int, device="cuda"):
    """Complex N(0,1) drawn on the GPU with torch's seeded generator (for the ~1 GiB
    benchmark batches, which are too slow to draw on the host).  Real and imaginary
    parts are independent standard normals in the target precision."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    real_dt = torch.float64 if dtype in (np.complex128, torch.complex128) else torch.float32
    v = torch.randn(tuple(shape) + (2,), dtype=real_dt, device=device, generator=g)
    return torch.view_as_complex(v)
