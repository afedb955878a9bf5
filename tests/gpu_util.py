"""Helpers shared by the GPU parity tests: run a plan on seeded numpy inputs and
compare with the FP64 oracle per transform.

Two bounds per transform: the relative L2 error (the stated tolerance: 2e-6 FP32,
1e-13 FP64), and the largest single-element error, each element's error relative to
the larger of its own magnitude and the transform's RMS (oracle.max_elem_err), held
to ``2 * tol * sqrt(log2 N)``.  Rounding errors of an N-point FFT grow like
sqrt(log2 N) and the largest of N roughly Gaussian element errors sits a few RMS
above the mean, so correct kernels stay well inside it, while one wrong bin — which
the L2 norm dilutes by 1/sqrt(N) — does not."""
from __future__ import annotations

import numpy as np

import oracle
import paper_1707_03776_amd as mf

TOL = {mf.FFT_F64: 1e-13, mf.FFT_F32: 2e-6}


def to_device(x: np.ndarray):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def run_plan(dims, batch, kind, direction, dtype, x: np.ndarray, inplace: bool = False):
    """Execute one plan on host array x (shape [batch, *in_dims]); returns host output."""
    import torch
    plan = mf.Plan(dims, batch, kind, direction, dtype)
    try:
        xin = to_device(x)
        if inplace:
            plan(xin, out=xin)
            out = xin
        else:
            out = plan(xin)
        torch.cuda.synchronize()
        return out.cpu().numpy()
    finally:
        plan.close()


def reference(dims, kind, direction, x: np.ndarray):
    if kind == mf.FFT_C2C:
        return oracle.c2c(x, dims, inverse=direction == mf.FFT_INVERSE)
    if kind == mf.FFT_R2C:
        return oracle.r2c(x, dims)
    return oracle.c2r(x, dims)


def elem_bound(tol: float, n: int) -> float:
    return 2.0 * tol * float(np.sqrt(max(1.0, np.log2(max(int(n), 2)))))


def assert_parity(y, ref, batch, tol, n, what="", elem=True):
    """Both bounds for every one of `batch` transforms of N = n points; returns
    (max relative L2, max element error).  elem=False keeps the L2 bound only: for
    inputs with strong pure tones the rounding errors of a multi-dimensional transform
    gather along the lines through each tone's bin (every partial transform of such a
    line carries the tone's large partial sum), so the element-error model of the
    noise inputs does not hold there."""
    y = np.asarray(y).reshape(batch, -1)
    ref = np.asarray(ref).reshape(batch, -1)
    l2 = float(np.max(oracle.rel_l2(y, ref)))
    el = float(np.max(oracle.max_elem_err(y, ref)))
    assert l2 <= tol, f"{what}: rel L2 {l2:.3e} > {tol:g}"
    eb = elem_bound(tol, n)
    if elem:
        assert el <= eb, f"{what}: max element error {el:.3e} > {eb:.3e}"
    return l2, el


def max_rel_err(y, ref, batch):
    return float(np.max(oracle.rel_l2(y.reshape(batch, -1), ref.reshape(batch, -1))))


def cplx_input(rng, shape, dtype):
    from paper_1707_03776_amd.inputs import complex_normal
    return complex_normal(rng, shape, np.complex128 if dtype == mf.FFT_F64 else np.complex64)


def real_input(rng, shape, dtype):
    return rng.standard_normal(shape).astype(np.float64 if dtype == mf.FFT_F64 else np.float32)


def check(dims, batch, kind, direction, dtype, seed=0, inplace=False, tol=None):
    rng = np.random.default_rng(seed)
    dims = tuple(dims)
    if kind == mf.FFT_C2R:
        # a Hermitian-consistent half spectrum: r2c (oracle) of a real input
        xr = real_input(rng, (batch,) + dims, dtype).astype(np.float64)
        x = oracle.r2c(xr, dims).astype(np.complex128 if dtype == mf.FFT_F64 else np.complex64)
    elif kind == mf.FFT_R2C:
        x = real_input(rng, (batch,) + dims, dtype)
    else:
        x = cplx_input(rng, (batch,) + dims, dtype)
    y = run_plan(dims, batch, kind, direction, dtype, x, inplace=inplace)
    ref = reference(dims, kind, direction, x)
    bound = TOL[dtype] if tol is None else tol
    what = f"dims={dims} batch={batch} kind={kind} dir={direction} dtype={dtype}"
    err, _ = assert_parity(y, ref, batch, bound, int(np.prod(dims)), what)
    return err
