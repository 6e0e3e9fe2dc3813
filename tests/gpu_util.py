"""Helpers for GPU tests: run the library on numpy inputs, compare with the oracle."""
from __future__ import annotations

import numpy as np

import oracle

# Float tolerance: per output, |y - y64| <= REL_TOL * sum_c |x_c| (the sum's own
# condition number; a plain relative error is undefined for sums near zero).
# The kernels sum channels in blocks of 32 in float32, which bounds the error by
# (31 + ceil(nchans/32)) * 2^-24 * sum_c |x_c| <= 1e-5 for nchans <= 4096.
REL_TOL = 1e-5


def torch_dtype(code: str):
    import torch
    return {"f32": torch.float32, "f16": torch.float16, "u8": torch.uint8}[code]


def to_device(x: np.ndarray):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(x))
    return t.to("cuda")


def run(plan, x: np.ndarray, nsamp: int, variant: int | None = None) -> np.ndarray:
    """Execute ``plan`` on host array ``x`` and return the host result."""
    import torch
    if variant is not None:
        plan.variant = variant
    xin = to_device(x)
    odt = torch.int32 if x.dtype == np.uint8 else torch.float32
    out = torch.full((plan.ndm, nsamp), -7, dtype=odt, device="cuda")
    plan.execute(xin, out, nsamp, torch.cuda.current_stream())
    torch.cuda.synchronize()
    return out.cpu().numpy()


def abs_sum(x: np.ndarray, shift: np.ndarray, nsamp: int, rows=None, t_begin=0, t_count=None) -> np.ndarray:
    """sum_c |x_c[t + shift]|: the scale the float tolerance is relative to."""
    ax = np.abs(x.astype(np.float32)) if x.dtype != np.uint8 else x
    return oracle.dedisperse(ax, shift, nsamp, rows=rows, t_begin=t_begin, t_count=t_count).astype(np.float64)


def check_float(got: np.ndarray, want: np.ndarray, scale: np.ndarray, tol: float = REL_TOL) -> float:
    """Assert the per-output bound; return the largest error / scale."""
    err = np.abs(got.astype(np.float64) - want)
    bound = tol * scale
    bad = err > bound
    if bad.any():
        i = np.unravel_index(np.argmax(err - bound), err.shape)
        raise AssertionError("float mismatch at %s: got %r want %r scale %r (%d bad of %d)"
                             % (i, got[i], want[i], scale[i], int(bad.sum()), bad.size))
    return float((err / np.maximum(scale, 1e-30)).max()) if err.size else 0.0


def per_dm_error(got: np.ndarray, want: np.ndarray) -> np.ndarray:
    """Per trial: max_t |y - y64| / max_t |y64|."""
    num = np.abs(got.astype(np.float64) - want).max(axis=1)
    den = np.maximum(np.abs(want).max(axis=1), 1e-30)
    return num / den
