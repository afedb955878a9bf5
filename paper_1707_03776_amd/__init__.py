"""mifft: discrete Fourier transforms on one MI355X (gfx950).

Thin ctypes binding over ``libmifft.so`` (``include/mifft.h``): the functions
below carry the C names and only marshal arguments; every step of a transform
runs in the library's HIP kernels.  PyTorch supplies device memory and streams.
There is no fallback: if the built library is missing, loading fails loudly.
"""
from __future__ import annotations

import ctypes
import os
import threading

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libmifft.so")

# enum fft_kind / fft_direction / fft_dtype / fft_status
FFT_C2C, FFT_R2C, FFT_C2R, FFT_DCT2, FFT_DCT3 = 0, 1, 2, 3, 4
FFT_FORWARD, FFT_INVERSE = -1, 1
FFT_F32, FFT_F64, FFT_F32_BF16X2, FFT_F32_BF16X3 = 0, 1, 2, 3
FFT_OK, FFT_ERR_INVALID_ARG, FFT_ERR_UNSUPPORTED, FFT_ERR_ALLOC, FFT_ERR_HIP, FFT_ERR_INTERNAL = range(6)

EXPORTED = ["fft_plan_create", "fft_execute", "fft_plan_destroy", "fft_plan_create_many", "fft_last_error",
            "fft_last_error_message", "fft_plan_describe", "fft_plan_inspect", "fft_plan_inspect_many",
            "fft_tune_set", "fft_tune_get", "fft_plan_device_bytes", "fft_laplacian_create",
            "fft_laplacian_execute", "fft_laplacian_destroy", "fft_laplacian_describe", "fft_execute_noalloc"]


class MifftError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"mifft status {status}: {message}")
        self.status = status


_lock = threading.Lock()
_lib = None


TUNING_FILE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning", "mi355x.txt")


def load_library(path: str = LIB_PATH):
    """Load ``libmifft.so`` (torch first, so both share one HIP runtime)."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        import torch  # noqa: F401  (loads the HIP runtime libmifft links against)
        if not os.path.exists(path):
            raise ImportError(f"{path} is not built; run `python -m paper_1707_03776_amd.build` "
                              "(or __graft_entry__.build()) first")
        lib = ctypes.CDLL(path)
        i64, i64p, vp = ctypes.c_int64, ctypes.POINTER(ctypes.c_int64), ctypes.c_void_p
        lib.fft_plan_create.argtypes = [ctypes.c_int, i64p, i64, ctypes.c_int, ctypes.c_int, ctypes.c_int]
        lib.fft_plan_create.restype = vp
        lib.fft_execute.argtypes = [vp, vp, vp, vp]
        lib.fft_execute.restype = ctypes.c_int
        lib.fft_plan_destroy.argtypes = [vp]
        lib.fft_plan_destroy.restype = None
        lib.fft_plan_create_many.argtypes = [i64, i64p, i64p, i64p, ctypes.c_int, ctypes.c_int, ctypes.c_int]
        lib.fft_plan_create_many.restype = vp
        lib.fft_last_error.argtypes = []
        lib.fft_last_error.restype = ctypes.c_int
        lib.fft_last_error_message.argtypes = []
        lib.fft_last_error_message.restype = ctypes.c_char_p
        lib.fft_plan_describe.argtypes = [vp]
        lib.fft_plan_describe.restype = ctypes.c_char_p
        lib.fft_plan_inspect.argtypes = [ctypes.c_int, i64p, i64, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                         ctypes.c_char_p, ctypes.c_size_t]
        lib.fft_plan_inspect.restype = ctypes.c_int
        lib.fft_plan_inspect_many.argtypes = [i64, i64p, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_char_p,
                                              ctypes.c_size_t]
        lib.fft_plan_inspect_many.restype = ctypes.c_int
        lib.fft_tune_set.argtypes = [ctypes.c_char_p, ctypes.c_int]
        lib.fft_tune_set.restype = ctypes.c_int
        lib.fft_tune_get.argtypes = [ctypes.c_char_p, ctypes.c_size_t]
        lib.fft_tune_get.restype = ctypes.c_int
        lib.fft_execute_noalloc.argtypes = [ctypes.c_int, i64p, i64, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                            vp, vp, vp]
        lib.fft_execute_noalloc.restype = ctypes.c_int
        lib.fft_plan_device_bytes.argtypes = [vp]
        lib.fft_plan_device_bytes.restype = i64
        lib.fft_laplacian_create.argtypes = [ctypes.c_int, i64p, i64, ctypes.POINTER(ctypes.c_double), ctypes.c_int]
        lib.fft_laplacian_create.restype = vp
        lib.fft_laplacian_execute.argtypes = [vp, vp, vp, vp]
        lib.fft_laplacian_execute.restype = ctypes.c_int
        lib.fft_laplacian_destroy.argtypes = [vp]
        lib.fft_laplacian_destroy.restype = None
        lib.fft_laplacian_describe.argtypes = [vp]
        lib.fft_laplacian_describe.restype = ctypes.c_char_p
        # the autotuner's table for this GPU, unless the caller names a file of its own
        # (MIFFT_TUNE_FILE, read by the library) or asks for the planner's defaults
        if not os.environ.get("MIFFT_TUNE_FILE") and os.environ.get("MIFFT_NO_TUNING") != "1" \
                and os.path.exists(TUNING_FILE):
            with open(TUNING_FILE) as f:
                lib.fft_tune_set(f.read().encode(), 0)
        _lib = lib
        return lib


def _i64_array(vals):
    vals = [int(v) for v in vals]
    return (ctypes.c_int64 * max(1, len(vals)))(*vals)


def _raise_last():
    lib = load_library()
    raise MifftError(lib.fft_last_error(), (lib.fft_last_error_message() or b"").decode())


# ---------------------------------------------------------------------------- C names


def fft_plan_create(rank: int, dims, batch: int, kind: int, direction: int, dtype: int) -> int:
    lib = load_library()
    p = lib.fft_plan_create(int(rank), _i64_array(dims), int(batch), int(kind), int(direction), int(dtype))
    if not p:
        _raise_last()
    return p


def fft_execute(plan: int, in_ptr: int, out_ptr: int, stream: int = 0) -> None:
    lib = load_library()
    st = lib.fft_execute(plan, in_ptr, out_ptr, stream or None)
    if st != FFT_OK:
        _raise_last()


def fft_execute_noalloc(rank: int, dims, batch: int, kind: int, direction: int, dtype: int, in_ptr: int,
                        out_ptr: int, stream: int = 0) -> None:
    """Plan and run one transform without allocating device memory (tables and scratch
    in the library's static per-GPU array)."""
    lib = load_library()
    st = lib.fft_execute_noalloc(int(rank), _i64_array(dims), int(batch), int(kind), int(direction), int(dtype),
                                 in_ptr, out_ptr, stream or None)
    if st != FFT_OK:
        _raise_last()


def fft_plan_destroy(plan: int) -> None:
    if plan:
        load_library().fft_plan_destroy(plan)


def fft_plan_create_many(lengths, in_offsets, out_offsets, kind: int = FFT_C2C, direction: int = FFT_FORWARD,
                         dtype: int = FFT_F32) -> int:
    lib = load_library()
    p = lib.fft_plan_create_many(len(lengths), _i64_array(lengths), _i64_array(in_offsets), _i64_array(out_offsets),
                                 int(kind), int(direction), int(dtype))
    if not p:
        _raise_last()
    return p


def fft_laplacian_create(rank: int, dims, batch: int, lengths, dtype: int) -> int:
    lib = load_library()
    L = [float(v) for v in lengths]
    p = lib.fft_laplacian_create(int(rank), _i64_array(dims), int(batch),
                                 (ctypes.c_double * max(1, len(L)))(*L), int(dtype))
    if not p:
        _raise_last()
    return p


def fft_laplacian_execute(op: int, in_ptr: int, out_ptr: int, stream: int = 0) -> None:
    lib = load_library()
    if lib.fft_laplacian_execute(op, in_ptr, out_ptr, stream or None) != FFT_OK:
        _raise_last()


def fft_laplacian_destroy(op: int) -> None:
    if op:
        load_library().fft_laplacian_destroy(op)


def fft_laplacian_describe(op: int) -> str:
    return (load_library().fft_laplacian_describe(op) or b"").decode()


def fft_last_error() -> int:
    return load_library().fft_last_error()


def fft_last_error_message() -> str:
    return (load_library().fft_last_error_message() or b"").decode()


def fft_plan_describe(plan: int) -> str:
    return (load_library().fft_plan_describe(plan) or b"").decode()


def fft_plan_device_bytes(plan: int) -> int:
    return int(load_library().fft_plan_device_bytes(plan))


def fft_plan_inspect(rank: int, dims, batch: int, kind: int, direction: int, dtype: int) -> str:
    """Host-only planner dry run; raises MifftError with the planner's message on failure."""
    lib = load_library()
    buf = ctypes.create_string_buffer(1 << 16)
    st = lib.fft_plan_inspect(int(rank), _i64_array(dims), int(batch), int(kind), int(direction), int(dtype),
                              buf, len(buf))
    if st != FFT_OK:
        raise MifftError(st, buf.value.decode())
    return buf.value.decode()


def fft_tune_set(entries: str, replace: bool = False) -> None:
    """Merge (or with replace=True, replace) entries of the process-wide tuning table."""
    lib = load_library()
    st = lib.fft_tune_set(entries.encode(), 1 if replace else 0)
    if st != FFT_OK:
        _raise_last()


def fft_tune_get() -> str:
    """The process-wide tuning table as "key=value" lines."""
    lib = load_library()
    size = 1 << 16
    while True:
        buf = ctypes.create_string_buffer(size)
        if lib.fft_tune_get(buf, size) == FFT_OK:
            return buf.value.decode()
        size *= 4


def fft_plan_inspect_many(lengths, kind: int, direction: int, dtype: int) -> str:
    """Host-only dry run of fft_plan_create_many (per-length plans and phase schedule)."""
    lib = load_library()
    buf = ctypes.create_string_buffer(1 << 22)
    st = lib.fft_plan_inspect_many(len(lengths), _i64_array(lengths), int(kind), int(direction), int(dtype), buf,
                                   len(buf))
    if st != FFT_OK:
        raise MifftError(st, buf.value.decode())
    return buf.value.decode()


# ---------------------------------------------------------------------------- torch convenience


class Plan:
    """A plan bound to shapes; call it with torch device tensors.

    ``Plan(dims, batch, kind=FFT_C2C, direction=FFT_FORWARD, dtype=FFT_F32)``;
    ``plan(inp, out=None, stream=None)`` runs on ``stream`` (default: torch's current
    stream) and returns ``out``.
    """

    def __init__(self, dims, batch: int = 1, kind: int = FFT_C2C, direction: int = FFT_FORWARD,
                 dtype: int = FFT_F32):
        self.dims = tuple(int(d) for d in dims)
        self.batch, self.kind, self.direction, self.dtype = int(batch), int(kind), int(direction), int(dtype)
        self.handle = fft_plan_create(len(self.dims), self.dims, self.batch, self.kind, self.direction,
                                      self.dtype)

    # shapes and dtypes of the two sides
    def _spec(self):
        import torch
        cd = torch.complex128 if self.dtype == FFT_F64 else torch.complex64
        rd = torch.float64 if self.dtype == FFT_F64 else torch.float32
        half = self.dims[:-1] + (self.dims[-1] // 2 + 1,)
        full = (self.batch,) + self.dims
        hs = (self.batch,) + half
        if self.kind == FFT_C2C:
            return (full, cd), (full, cd)
        if self.kind in (FFT_DCT2, FFT_DCT3):
            return (full, rd), (full, rd)
        if self.kind == FFT_R2C:
            return (full, rd), (hs, cd)
        return (hs, cd), (full, rd)

    def __call__(self, inp, out=None, stream=None):
        import torch
        (ishape, idt), (oshape, odt) = self._spec()
        if inp.dtype != idt or not inp.is_cuda or not inp.is_contiguous() or inp.numel() != _prod(ishape):
            raise ValueError(f"input must be a contiguous {idt} CUDA tensor of {_prod(ishape)} elements")
        if out is None:
            out = torch.empty(oshape, dtype=odt, device=inp.device)
        if out.dtype != odt or not out.is_cuda or not out.is_contiguous() or out.numel() != _prod(oshape):
            raise ValueError(f"output must be a contiguous {odt} CUDA tensor of {_prod(oshape)} elements")
        s = stream if stream is not None else torch.cuda.current_stream(inp.device)
        fft_execute(self.handle, inp.data_ptr(), out.data_ptr(), s.cuda_stream)
        return out

    def describe(self) -> str:
        return fft_plan_describe(self.handle)

    def device_bytes(self) -> int:
        return fft_plan_device_bytes(self.handle)

    def close(self):
        if getattr(self, "handle", None):
            fft_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Laplacian:
    """Owning wrapper of an ``fft_laplacian`` operator: ``lap(u)`` for torch tensors of
    shape ``[batch, *dims]`` (float32 for FFT_F32, float64 for FFT_F64) on the GPU."""

    def __init__(self, dims, batch: int, lengths, dtype: int = FFT_F32):
        self.dims = tuple(int(d) for d in dims)
        self.batch = int(batch)
        self.dtype = dtype
        self.handle = fft_laplacian_create(len(self.dims), self.dims, self.batch, lengths, dtype)

    def __call__(self, inp, out=None, stream=None):
        import torch
        dt = torch.float64 if self.dtype == FFT_F64 else torch.float32
        n = self.batch * _prod(self.dims)
        if inp.dtype != dt or not inp.is_cuda or not inp.is_contiguous() or inp.numel() != n:
            raise ValueError(f"input must be a contiguous {dt} CUDA tensor of {n} elements")
        if out is None:
            out = torch.empty((self.batch,) + self.dims, dtype=dt, device=inp.device)
        if out.dtype != dt or not out.is_cuda or not out.is_contiguous() or out.numel() != n:
            raise ValueError(f"output must be a contiguous {dt} CUDA tensor of {n} elements")
        s = stream if stream is not None else torch.cuda.current_stream(inp.device)
        fft_laplacian_execute(self.handle, inp.data_ptr(), out.data_ptr(), s.cuda_stream)
        return out

    def describe(self) -> str:
        return fft_laplacian_describe(self.handle)

    def close(self):
        if getattr(self, "handle", None):
            fft_laplacian_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _prod(t):
    p = 1
    for v in t:
        p *= int(v)
    return p
