"""Shared helpers of the GPU parity tests (not collected by pytest)."""
import numpy as np
import torch

import oracle as O

DEV = "cuda:0"


def dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to(DEV)


def matrix(mxl, ctx, A, dtype=torch.float64):
    rp, col = dev(A.row_ptr), dev(A.col)
    val = dev(A.val, dtype)
    return mxl.csr(ctx, rp, col, val, ncols=A.ncols)


def round32(a):
    return np.asarray(a, np.float32).astype(np.float64)


def spmv_reference(A, x, alpha, beta, y0, fp32):
    """Oracle result and the per-row bound |alpha| sum|a||x| + |beta||y0|.

    FP32: the oracle evaluates in FP64 on the FP32-rounded operands, so only
    the kernel's own rounding is charged against the tolerance."""
    if fp32:
        A = type(A)(A.nrows, A.ncols, A.row_ptr, A.col, round32(A.val), A.name)
        x, y0 = round32(x), round32(y0)
        alpha, beta = float(np.float32(alpha)), float(np.float32(beta))
    y = O.spmv(A, x, alpha, beta, y0)
    rows = np.repeat(np.arange(A.nrows), A.row_lengths())
    absax = np.bincount(rows, weights=np.abs(A.val) * np.abs(x[A.col]), minlength=A.nrows)
    bound = abs(alpha) * absax + (abs(beta) * np.abs(y0) if beta != 0 else 0.0)
    return y, bound


def assert_rows_close(got, want, bound, tau, what=""):
    got = np.asarray(got, np.float64)
    err = np.abs(got - want)
    ok = (err <= tau * bound) | (got == want)
    if not ok.all():
        i = int(np.nonzero(~ok)[0][0])
        raise AssertionError(f"{what}: row {i} got {got[i]!r} want {want[i]!r} "
                             f"err {err[i]:.3e} bound {tau * bound[i]:.3e} "
                             f"({int((~ok).sum())} rows fail)")


def assert_bicgstab_tracks_oracle(info, g, head=10, rtol=1e-8):
    """BiCGSTAB at the full sizes: the method fixes its iteration count only
    up to rounding.  The oracle's own count moves by several iterations when
    b changes at rounding level (its stored spread, `perturbed_counts`),
    while the first residuals agree to many digits.  So: residuals 1..head
    within rtol of the oracle's, and the count inside the oracle's spread
    widened by 2."""
    h = np.asarray(info["history"][:head + 1])
    want = np.asarray(g["history_head"][:head + 1])
    assert h.size == want.size
    assert np.all(np.abs(h - want) <= rtol * want), (h, want)
    counts = list(g["perturbed_counts"]) + [g["iterations"]]
    assert min(counts) - 2 <= info["iterations"] <= max(counts) + 2, (info["iterations"], counts)
