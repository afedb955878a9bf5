"""FP64 CPU oracle for the discrete Fourier transform — TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU library never calls it and shares
no code with it; a product path that reached this module would be a bug.

The computation lives in ``oracle.c`` (plain C, FP64, recursive Cooley–Tukey
with exact roots of unity and direct sums for prime lengths).  This module only
compiles it with gcc on first use and marshals numpy arrays through ctypes.

Conventions (numpy.fft's; the paper has no Fourier transform):
forward ``X[k] = sum_j x[j] exp(-2 pi i jk/n)``, inverse with ``+`` and a
``1/prod(dims)`` scale, r2c keeps ``n//2+1`` bins on the last axis, c2r follows
``numpy.fft.irfftn``.  ``laplacian`` composes r2c, a diagonal multiply (numpy) and
c2r into the pseudo-spectral Laplacian of a periodic grid.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None


def build(force: bool = False) -> str:
    """Compile ``oracle.c`` into ``liboracle.so`` (gcc, -O2, OpenMP, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        cmd = ["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-fopenmp", "-fPIC", "-shared",
               "-Wall", "-Wextra", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is None:
            build()
            lib = ctypes.CDLL(_LIB)
            i64p = ctypes.POINTER(ctypes.c_int64)
            dp = ctypes.c_void_p
            lib.oracle_c2c.argtypes = [ctypes.c_int, i64p, ctypes.c_int64, ctypes.c_int, dp, dp]
            lib.oracle_r2c.argtypes = [ctypes.c_int, i64p, ctypes.c_int64, dp, dp]
            lib.oracle_c2r.argtypes = [ctypes.c_int, i64p, ctypes.c_int64, dp, dp]
            for f in (lib.oracle_c2c, lib.oracle_r2c, lib.oracle_c2r):
                f.restype = ctypes.c_int
            lib.oracle_dct.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_int64, dp, dp]
            lib.oracle_dct.restype = ctypes.c_int
            lib.oracle_unit_root.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_int,
                                             ctypes.POINTER(ctypes.c_double)]
            lib.oracle_unit_root.restype = None
            lib.oracle_max_threads.restype = ctypes.c_int
            lib.oracle_set_threads.argtypes = [ctypes.c_int]
            lib.oracle_set_threads.restype = None
            _lib = lib
    return _lib


def _dims(dims):
    dims = tuple(int(d) for d in dims)
    return dims, (ctypes.c_int64 * len(dims))(*dims)


def _check(status: int) -> None:
    if status != 0:
        raise RuntimeError(f"oracle returned status {status}")


def c2c(x: np.ndarray, dims, inverse: bool = False) -> np.ndarray:
    """Complex-to-complex DFT over the trailing ``len(dims)`` axes of ``x``.

    ``x`` has shape ``[..., *dims]``; leading axes are a batch.  Computed in FP64
    (inputs are upcast exactly).  Returns complex128 of the same shape.
    """
    dims, cd = _dims(dims)
    a = np.ascontiguousarray(x, dtype=np.complex128)
    assert a.shape[a.ndim - len(dims):] == dims, (a.shape, dims)
    per = int(np.prod(dims))
    batch = a.size // per if per else 0
    out = np.empty_like(a)
    _check(_load().oracle_c2c(len(dims), cd, batch, 1 if inverse else -1,
                              a.ctypes.data, out.ctypes.data))
    return out


def r2c(x: np.ndarray, dims) -> np.ndarray:
    """Real-to-complex forward DFT (``numpy.fft.rfftn`` layout) over the trailing axes."""
    dims, cd = _dims(dims)
    a = np.ascontiguousarray(x, dtype=np.float64)
    assert a.shape[a.ndim - len(dims):] == dims, (a.shape, dims)
    per = int(np.prod(dims))
    batch = a.size // per if per else 0
    oshape = a.shape[:a.ndim - 1] + (dims[-1] // 2 + 1,)
    out = np.empty(oshape, dtype=np.complex128)
    _check(_load().oracle_r2c(len(dims), cd, batch, a.ctypes.data, out.ctypes.data))
    return out


def c2r(x: np.ndarray, dims) -> np.ndarray:
    """Complex-to-real inverse DFT (``numpy.fft.irfftn`` semantics); ``dims`` are the real sizes."""
    dims, cd = _dims(dims)
    a = np.ascontiguousarray(x, dtype=np.complex128)
    hshape = dims[:-1] + (dims[-1] // 2 + 1,)
    assert a.shape[a.ndim - len(dims):] == hshape, (a.shape, hshape)
    per_h = int(np.prod(hshape))
    batch = a.size // per_h if per_h else 0
    out = np.empty(a.shape[:a.ndim - len(dims)] + dims, dtype=np.float64)
    _check(_load().oracle_c2r(len(dims), cd, batch, a.ctypes.data, out.ctypes.data))
    return out


def dct(x: np.ndarray, type: int = 2) -> np.ndarray:
    """Unnormalised DCT of type 2 or 3 along the last axis, by the definition
    (``scipy.fft.dct(x, type)`` with ``norm=None``); type 3 of type 2 gives ``2n x``."""
    a = np.ascontiguousarray(x, dtype=np.float64)
    n = a.shape[-1]
    batch = a.size // n if n else 0
    out = np.empty_like(a)
    _check(_load().oracle_dct(int(type), n, batch, a.ctypes.data, out.ctypes.data))
    return out


def wavenumbers_sq(dims, lengths) -> np.ndarray:
    """``|kappa|^2`` on the half-spectrum grid of ``dims``: kappa_a = 2 pi f_a / L_a with
    the signed frequency f_a = j for j <= n_a/2, else j - n_a (numpy.fft.fftfreq times
    n_a, with the Nyquist bin taken as +n_a/2; its square is the same either way); the
    last axis keeps j = 0..n/2 (the rfftn layout)."""
    dims = tuple(int(d) for d in dims)
    total = np.zeros(dims[:-1] + (dims[-1] // 2 + 1,))
    for a, (n, L) in enumerate(zip(dims, lengths)):
        m = n // 2 + 1 if a == len(dims) - 1 else n
        f = np.array([j if j <= n // 2 else j - n for j in range(m)], dtype=np.float64)
        shape = [1] * len(dims)
        shape[a] = m
        total = total + ((2.0 * np.pi * f / float(L)) ** 2).reshape(shape)
    return total


def laplacian(u: np.ndarray, dims, lengths) -> np.ndarray:
    """Pseudo-spectral Laplacian of a real field sampled on a periodic grid: the
    gradient-squared operator is diagonal in the Fourier basis, so
    ``lap u = c2r(-|kappa|^2 * r2c(u))`` with grid spacing L_a / n_a along axis a.
    ``u`` has shape ``[..., *dims]`` (leading axes a batch); FP64 throughout."""
    dims = tuple(int(d) for d in dims)
    spec = r2c(u, dims)
    spec = spec * (-wavenumbers_sq(dims, lengths))
    return c2r(spec, dims)


def unit_root(n: int, m: int, sign: int = -1) -> complex:
    """``exp(sign * 2 pi i m / n)`` exactly as the oracle evaluates it."""
    buf = (ctypes.c_double * 2)()
    _load().oracle_unit_root(int(n), int(m), int(sign), buf)
    return complex(buf[0], buf[1])


def max_threads() -> int:
    """OpenMP threads the oracle will use (``OMP_NUM_THREADS`` or all cores)."""
    return int(_load().oracle_max_threads())


def set_threads(n: int) -> None:
    """Threads the oracle may use for calls made from the calling thread."""
    _load().oracle_set_threads(int(n))


def rel_l2(y: np.ndarray, ref: np.ndarray, batch_axes: int = 1) -> np.ndarray:
    """Relative L2 error per transform: ``||y_b - ref_b|| / ||ref_b||`` over the
    trailing axes, for each index of the leading ``batch_axes`` axes."""
    y = np.asarray(y)
    ref = np.asarray(ref)
    lead = ref.shape[:batch_axes]
    d = (y.astype(np.complex128) - ref).reshape(lead + (-1,))
    r = ref.reshape(lead + (-1,))
    num = np.sqrt(np.sum(np.abs(d) ** 2, axis=-1))
    den = np.sqrt(np.sum(np.abs(r) ** 2, axis=-1))
    return num / np.where(den == 0, 1.0, den)


def max_elem_err(y: np.ndarray, ref: np.ndarray, batch_axes: int = 1) -> np.ndarray:
    """Largest element error per transform, each element's error taken relative to the
    larger of its own magnitude and the transform's RMS:
    ``max_e |y_b[e] - ref_b[e]| / max(|ref_b[e]|, rms(ref_b))``.  Rounding errors of a
    bin well above the RMS (a spike built by coherent summation) scale with the bin
    itself, those of the other bins with the RMS.  Unlike ``rel_l2`` it does not
    average a few wrong bins away over a long transform."""
    y = np.asarray(y)
    ref = np.asarray(ref)
    lead = ref.shape[:batch_axes]
    d = np.abs(y.astype(np.complex128) - ref).reshape(lead + (-1,))
    r = np.abs(ref).reshape(lead + (-1,))
    rms = np.sqrt(np.mean(r ** 2, axis=-1, keepdims=True))
    scale = np.maximum(r, np.where(rms == 0, 1.0, rms))
    return np.max(d / scale, axis=-1)
