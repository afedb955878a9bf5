"""Helpers shared by the GPU parity tests: run a plan on seeded numpy inputs and
compare with the FP64 oracle per transform."""
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
    err = max_rel_err(y, ref, batch)
    bound = TOL[dtype] if tol is None else tol
    assert err <= bound, f"dims={dims} batch={batch} kind={kind} dir={direction} dtype={dtype}: rel L2 {err:.3e}"
    return err
