"""CPU oracle for the sparse-operator hot path -- TEST INFRASTRUCTURE ONLY.

Only the test-suite, ``__graft_entry__.smoke()`` and the benchmark's
``cpu_baseline`` leg may import this package.  The product library never
loads it, and it shares no code with the GPU path: it is plain FP64 C
(``oracle.c``, built with ``-ffp-contract=off``) driven through ctypes, plus
the exact-rational routines in ``oracle.exact``.

Functions without an independent pin are marked "parity unpinned" in their
docstring (none at present; the pins live in ``tests/test_oracle_pins.py``).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")
SRC = os.path.join(_HERE, "oracle.c")

CONVERGED, MAX_ITERS, TIME, BREAKDOWN, NONFINITE = 1, 2, 3, 4, 5


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (plain C99, no FMA contraction)."""
    if force or not os.path.exists(LIB_PATH):
        tmp = LIB_PATH + ".tmp"
        subprocess.check_call([
            "gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fno-fast-math",
            "-fPIC", "-shared", "-Wall", "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


class _Crit(C.Structure):
    _fields_ = [("max_iters", C.c_int64), ("reduction", C.c_double),
                ("nonfinite_check", C.c_int32)]


class _Info(C.Structure):
    _fields_ = [("iterations", C.c_int64), ("spmv_count", C.c_int64),
                ("rel_residual", C.c_double), ("stop_reason", C.c_int32),
                ("inner_iterations", C.c_int64)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        _lib = C.CDLL(LIB_PATH)
        _declare(_lib)
    return _lib


def _p(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def _declare(L):
    vp, i64, i32, f64 = C.c_void_p, C.c_int64, C.c_int32, C.c_double
    L.orc_csr_check.restype = C.c_int
    L.orc_csr_check.argtypes = [i64, i64, i64, vp, vp]
    L.orc_csr_spmv.restype = None
    L.orc_csr_spmv.argtypes = [i64, vp, vp, vp, f64, vp, f64, vp]
    L.orc_csr_to_coo.argtypes = [i64, vp, vp]
    L.orc_coo_spmv.argtypes = [i64, i64, vp, vp, vp, f64, vp, f64, vp]
    L.orc_max_row_len.restype = i32
    L.orc_max_row_len.argtypes = [i64, vp]
    L.orc_csr_to_ell.argtypes = [i64, vp, vp, vp, i32, i64, vp, vp]
    L.orc_ell_spmv.argtypes = [i64, i64, i32, vp, vp, f64, vp, f64, vp]
    L.orc_hyb_width.restype = i32
    L.orc_hyb_width.argtypes = [i64, vp, f64]
    L.orc_hyb_tail_count.restype = i64
    L.orc_hyb_tail_count.argtypes = [i64, vp, i32]
    L.orc_csr_to_hyb.argtypes = [i64, vp, vp, vp, i32, i64, vp, vp, vp, vp, vp]
    L.orc_hyb_spmv.argtypes = [i64, i64, i32, vp, vp, i64, vp, vp, vp, f64, vp, f64, vp]
    L.orc_jacobi_dinv.restype = i64
    L.orc_jacobi_dinv.argtypes = [i64, vp, vp, vp, vp]
    for name in ("orc_pcg", "orc_bicgstab"):
        f = getattr(L, name)
        f.restype = C.c_int
        f.argtypes = [i64, vp, vp, vp, vp, vp, vp, _Crit, C.POINTER(_Info), vp]
    L.orc_pcg_f32.restype = C.c_int
    L.orc_pcg_f32.argtypes = [i64, vp, vp, vp, vp, vp, vp, _Crit, C.POINTER(_Info)]
    L.orc_ir.restype = C.c_int
    L.orc_ir.argtypes = [i64, vp, vp, vp, vp, vp, i64, f64, i64, f64, C.POINTER(_Info), vp]
    L.orc_pcg_f32_block.restype = C.c_int
    L.orc_pcg_f32_block.argtypes = [i64, vp, vp, vp, i64, vp, vp, vp, vp, _Crit, C.POINTER(_Info)]
    L.orc_ir_block_var.restype = C.c_int
    L.orc_ir_block_var.argtypes = [i64, vp, vp, vp, vp, vp, i64, f64, i64, f64, i64, vp, f64,
                                   C.POINTER(_Info), vp]
    L.orc_ir_block.restype = C.c_int
    L.orc_ir_block.argtypes = [i64, vp, vp, vp, vp, vp, i64, f64, i64, f64, i32, f64, C.POINTER(_Info), vp]
    L.orc_batch_pcg.argtypes = [i64, vp, vp, vp, vp, vp, vp, f64, i64, vp, vp, vp]
    L.orc_features.argtypes = [i64, i64, vp, vp, vp]
    L.orc_mlp_loss_grad.restype = f64
    L.orc_mlp_loss_grad.argtypes = [i32, vp, vp, i64, vp, vp, vp, f64, vp, vp]
    L.orc_adam_step.argtypes = [i64, vp, vp, vp, vp, i64, f64, f64, f64, f64]
    L.orc_round_f16.restype = f64
    L.orc_round_f16.argtypes = [f64]
    L.orc_bj_choose_precision.restype = C.c_int
    L.orc_bj_choose_precision.argtypes = [C.c_int, vp, f64, f64]
    L.orc_bj_supervariable_blocks.restype = i64
    L.orc_bj_supervariable_blocks.argtypes = [i64, vp, vp, C.c_int, vp]
    L.orc_bj_generate.restype = i64
    L.orc_bj_generate.argtypes = [i64, vp, vp, vp, i64, vp, C.c_int, f64, vp, vp, vp]
    L.orc_bj_apply.argtypes = [i64, vp, vp, vp, vp]
    L.orc_bicgstab_block.restype = C.c_int
    L.orc_bicgstab_block.argtypes = [i64, vp, vp, vp, i64, vp, vp, vp, vp, _Crit, C.POINTER(_Info), vp]
    L.orc_pcg_block.restype = C.c_int
    L.orc_pcg_block.argtypes = [i64, vp, vp, vp, i64, vp, vp, vp, vp, _Crit, C.POINTER(_Info), vp]
    L.orc_gmres.restype = C.c_int
    L.orc_gmres.argtypes = [i64, vp, vp, vp, vp, vp, vp, i32, _Crit, C.POINTER(_Info), vp]
    L.orc_gmres_block.restype = C.c_int
    L.orc_ilu0.restype = i64
    L.orc_ilu0.argtypes = [i64, vp, vp, vp, vp]
    L.orc_parilu.restype = i64
    L.orc_parilu.argtypes = [i64, vp, vp, vp, i32, vp]
    L.orc_ilu_apply.argtypes = [i64, vp, vp, vp, i32, i32, vp, vp]
    L.orc_gmres_ilu.restype = C.c_int
    L.orc_gmres_ilu.argtypes = [i64, vp, vp, vp, vp, i32, i32, vp, vp, i32, _Crit, C.POINTER(_Info), vp]
    L.orc_gmres_block.argtypes = [i64, vp, vp, vp, i64, vp, vp, vp, vp, i32, _Crit, C.POINTER(_Info),
                                  vp]


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


def _csr(A):
    return _c(A.row_ptr, np.int32), _c(A.col, np.int32), _c(A.val, np.float64)


# ---------------------------------------------------------------- wrappers
def csr_check(A) -> int:
    rp, col, _ = _csr(A)
    return lib().orc_csr_check(A.nrows, A.ncols, col.size, _p(rp), _p(col))


def spmv(A, x, alpha=1.0, beta=0.0, y=None):
    rp, col, val = _csr(A)
    x = _c(x, np.float64)
    y = np.zeros(A.nrows) if y is None else _c(y, np.float64).copy()
    lib().orc_csr_spmv(A.nrows, _p(rp), _p(col), _p(val), alpha, _p(x), beta, _p(y))
    return y


def csr_to_coo(A):
    rp = _c(A.row_ptr, np.int32)
    row = np.empty(int(rp[-1]), np.int32)
    lib().orc_csr_to_coo(A.nrows, _p(rp), _p(row))
    return row


def coo_spmv(nrows, row, col, val, x, alpha=1.0, beta=0.0, y=None):
    row, col, val, x = _c(row, np.int32), _c(col, np.int32), _c(val, np.float64), _c(x, np.float64)
    y = np.zeros(nrows) if y is None else _c(y, np.float64).copy()
    lib().orc_coo_spmv(nrows, row.size, _p(row), _p(col), _p(val), alpha, _p(x), beta, _p(y))
    return y


def max_row_len(A) -> int:
    return lib().orc_max_row_len(A.nrows, _p(_c(A.row_ptr, np.int32)))


def pad_rows(n: int) -> int:
    """ELL row padding: n rounded up to a multiple of 64."""
    return ((n + 63) // 64) * 64


def csr_to_ell(A, width=None):
    rp, col, val = _csr(A)
    w = max_row_len(A) if width is None else width
    n_pad = pad_rows(A.nrows)
    ec = np.empty(max(w * n_pad, 1), np.int32)
    ev = np.empty(max(w * n_pad, 1), np.float64)
    lib().orc_csr_to_ell(A.nrows, _p(rp), _p(col), _p(val), w, n_pad, _p(ec), _p(ev))
    return w, n_pad, ec[:w * n_pad], ev[:w * n_pad]


def ell_spmv(nrows, n_pad, w, ec, ev, x, alpha=1.0, beta=0.0, y=None):
    ec, ev, x = _c(ec, np.int32), _c(ev, np.float64), _c(x, np.float64)
    y = np.zeros(nrows) if y is None else _c(y, np.float64).copy()
    lib().orc_ell_spmv(nrows, n_pad, w, _p(ec), _p(ev), alpha, _p(x), beta, _p(y))
    return y


def hyb_width(A, q: float) -> int:
    return lib().orc_hyb_width(A.nrows, _p(_c(A.row_ptr, np.int32)), q)


def csr_to_hyb(A, q: float = None, k: int = None):
    rp, col, val = _csr(A)
    if k is None:
        k = hyb_width(A, q)
    n_pad = pad_rows(A.nrows)
    nt = lib().orc_hyb_tail_count(A.nrows, _p(rp), k)
    ec = np.empty(max(k * n_pad, 1), np.int32)
    ev = np.empty(max(k * n_pad, 1), np.float64)
    tr = np.empty(max(nt, 1), np.int32)
    tc = np.empty(max(nt, 1), np.int32)
    tv = np.empty(max(nt, 1), np.float64)
    lib().orc_csr_to_hyb(A.nrows, _p(rp), _p(col), _p(val), k, n_pad, _p(ec), _p(ev),
                         _p(tr), _p(tc), _p(tv))
    return dict(k=k, n_pad=n_pad, ell_col=ec[:k * n_pad], ell_val=ev[:k * n_pad],
                tail_row=tr[:nt], tail_col=tc[:nt], tail_val=tv[:nt])


def hyb_spmv(nrows, H, x, alpha=1.0, beta=0.0, y=None):
    x = _c(x, np.float64)
    y = np.zeros(nrows) if y is None else _c(y, np.float64).copy()
    ec, ev = _c(H["ell_col"], np.int32), _c(H["ell_val"], np.float64)
    tr, tc, tv = (_c(H["tail_row"], np.int32), _c(H["tail_col"], np.int32),
                  _c(H["tail_val"], np.float64))
    lib().orc_hyb_spmv(nrows, H["n_pad"], H["k"], _p(ec), _p(ev), tr.size, _p(tr), _p(tc),
                       _p(tv), alpha, _p(x), beta, _p(y))
    return y


def jacobi_dinv(A):
    """Returns (dinv, bad_row) with bad_row = -1 on success."""
    rp, col, val = _csr(A)
    d = np.zeros(A.nrows)
    bad = lib().orc_jacobi_dinv(A.nrows, _p(rp), _p(col), _p(val), _p(d))
    return d, int(bad)


def _solve(fn, A, b, x0, dinv, max_iters, reduction, nonfinite_check, history):
    rp, col, val = _csr(A)
    b = _c(b, np.float64)
    x = np.zeros(A.nrows) if x0 is None else _c(x0, np.float64).copy()
    info = _Info()
    hist = np.full(max_iters + 1, np.nan) if history else None
    d = None if dinv is None else _c(dinv, np.float64)
    fn(A.nrows, _p(rp), _p(col), _p(val), _p(d), _p(b), _p(x),
       _Crit(max_iters, reduction, nonfinite_check), C.byref(info), _p(hist))
    out = dict(x=x, iterations=info.iterations, spmv_count=info.spmv_count,
               rel_residual=info.rel_residual, stop_reason=info.stop_reason)
    if history:
        out["history"] = hist[:info.iterations + 1]
    return out


def pcg(A, b, x0=None, dinv=None, max_iters=10_000, reduction=1e-10,
        nonfinite_check=1, history=False):
    """Jacobi-PCG; ``dinv=None`` means no preconditioner (plain CG)."""
    return _solve(lib().orc_pcg, A, b, x0, dinv, max_iters, reduction, nonfinite_check, history)


def bicgstab(A, b, x0=None, dinv=None, max_iters=10_000, reduction=1e-10,
             nonfinite_check=1, history=False):
    return _solve(lib().orc_bicgstab, A, b, x0, dinv, max_iters, reduction, nonfinite_check,
                  history)


def pcg_f32(A, b32, dinv32, max_iters=10_000, reduction=1e-4):
    rp, col, _ = _csr(A)
    v32 = _c(A.val, np.float32)
    b32 = _c(b32, np.float32)
    d32 = _c(dinv32, np.float32)
    x = np.zeros(A.nrows, np.float32)
    info = _Info()
    lib().orc_pcg_f32(A.nrows, _p(rp), _p(col), _p(v32), _p(d32), _p(b32), _p(x),
                      _Crit(max_iters, reduction, 1), C.byref(info))
    return dict(x=x, iterations=info.iterations, rel_residual=info.rel_residual,
                stop_reason=info.stop_reason)


def pcg_f32_block(A, b32, bptr, inv, max_iters=10_000, reduction=1e-4):
    """FP32 CG (vectors and matrix values FP32, scalars FP64) with block
    Jacobi: z = blockdiag(inv) r evaluated in FP64 and rounded to FP32."""
    rp, col, _ = _csr(A)
    v32 = _c(A.val, np.float32)
    b32 = _c(b32, np.float32)
    bptr = _c(bptr, np.int32)
    inv = _c(inv, np.float64)
    x = np.zeros(A.nrows, np.float32)
    info = _Info()
    lib().orc_pcg_f32_block(A.nrows, _p(rp), _p(col), _p(v32), bptr.size - 1, _p(bptr), _p(inv), _p(b32),
                            _p(x), _Crit(max_iters, reduction, 1), C.byref(info))
    return dict(x=x, iterations=info.iterations, rel_residual=info.rel_residual,
                stop_reason=info.stop_reason)


def ir(A, b, x0=None, max_outer=50, outer_reduction=1e-12, inner_max_iters=10_000,
       inner_reduction=1e-4, block_size=0, block_accuracy=0.1, bptr=None):
    """Mixed-precision iterative refinement (Sec. 3.2): FP64 residual and
    update, FP32 Jacobi-CG inner solve; block_size > 0 switches the inner
    preconditioner to adaptive block Jacobi over uniform blocks of that size,
    bptr (block boundaries) to adaptive block Jacobi over those blocks."""
    rp, col, val = _csr(A)
    b = _c(b, np.float64)
    x = np.zeros(A.nrows) if x0 is None else _c(x0, np.float64).copy()
    info = _Info()
    hist = np.full(max_outer + 1, np.nan)
    if bptr is not None:
        bp = _c(bptr, np.int32)
        lib().orc_ir_block_var(A.nrows, _p(rp), _p(col), _p(val), _p(b), _p(x), max_outer, outer_reduction,
                               inner_max_iters, inner_reduction, bp.size - 1, _p(bp), block_accuracy,
                               C.byref(info), _p(hist))
    elif block_size > 0:
        lib().orc_ir_block(A.nrows, _p(rp), _p(col), _p(val), _p(b), _p(x), max_outer, outer_reduction,
                           inner_max_iters, inner_reduction, block_size, block_accuracy, C.byref(info),
                           _p(hist))
    else:
        lib().orc_ir(A.nrows, _p(rp), _p(col), _p(val), _p(b), _p(x), max_outer,
                     outer_reduction, inner_max_iters, inner_reduction, C.byref(info), _p(hist))
    return dict(x=x, outer=info.iterations, inner_iterations=info.inner_iterations,
                spmv_count=info.spmv_count, rel_residual=info.rel_residual,
                stop_reason=info.stop_reason, history=hist[:info.iterations + 1])


def batch_pcg(B, reduction=1e-10, iter_factor=10):
    nsys = B.nsys
    x = np.zeros(int(B.sys_ptr[-1]))
    iters = np.zeros(nsys, np.int32)
    rel = np.zeros(nsys)
    st = np.zeros(nsys, np.uint8)
    sp, rp, col, val, b = (_c(B.sys_ptr, np.int32), _c(B.row_ptr, np.int32),
                           _c(B.col, np.int32), _c(B.val, np.float64), _c(B.b, np.float64))
    lib().orc_batch_pcg(nsys, _p(sp), _p(rp), _p(col), _p(val), _p(b), _p(x), reduction,
                        iter_factor, _p(iters), _p(rel), _p(st))
    return dict(x=x, iterations=iters, rel_residual=rel, status=st)


def features(A):
    rp, col, _ = _csr(A)
    out = np.zeros(16)
    lib().orc_features(A.nrows, A.ncols, _p(rp), _p(col), _p(out))
    return out


def mlp_param_count(dims) -> int:
    return sum(dims[i + 1] * dims[i] + dims[i + 1] for i in range(len(dims) - 1))


def mlp_loss_grad(dims, theta, X, Y, M, lam=1e-4, want_grad=True, want_pred=False):
    dims_a = np.asarray(dims, np.int32)
    theta = _c(theta, np.float64)
    X, Y, M = _c(X, np.float64), _c(Y, np.float64), _c(M, np.float64)
    g = np.zeros_like(theta) if want_grad else None
    pred = np.zeros((X.shape[0], dims[-1])) if want_pred else None
    loss = lib().orc_mlp_loss_grad(len(dims) - 1, _p(dims_a), _p(theta), X.shape[0], _p(X),
                                   _p(Y), _p(M), lam, _p(g), _p(pred))
    return loss, g, pred


def adam_step(theta, grad, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """In-place Adam update of float64 arrays theta, m, v."""
    for a in (theta, m, v):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    g = _c(grad, np.float64)
    lib().orc_adam_step(theta.size, _p(theta), _p(g), _p(m), _p(v), t, lr, b1, b2, eps)


# ------------------------------------------------------------ block Jacobi
P64, P32, P16 = 0, 1, 2


def round_f16(x: float) -> float:
    """Nearest-even IEEE binary16 rounding (from the format's definition)."""
    return lib().orc_round_f16(float(x))


def uniform_blocks(n: int, bs: int) -> np.ndarray:
    """Block row pointers of consecutive blocks of bs rows (last one ragged)."""
    return np.minimum(np.arange(0, n + bs, bs), n).astype(np.int32)[:(n + bs - 1) // bs + 1]


def supervariable_blocks(A, max_bs: int) -> np.ndarray:
    """Block row pointers by supervariable agglomeration: runs of rows with
    identical column sets, cut into pieces of at most max_bs rows, packed
    greedily into blocks of at most max_bs rows."""
    rp, col, _ = _csr(A)
    bptr = np.zeros(A.nrows + 1, np.int32)
    nb = lib().orc_bj_supervariable_blocks(A.nrows, _p(rp), _p(col), int(max_bs), _p(bptr))
    return bptr[:nb + 1].copy()


def bj_choose_precision(inv: np.ndarray, cond: float, accuracy: float = 0.1) -> int:
    m = inv.shape[0]
    return lib().orc_bj_choose_precision(m, _p(_c(inv, np.float64)), cond, accuracy)


def bj_generate(A, bptr, adaptive: bool = True, accuracy: float = 0.1):
    """Block-Jacobi inverses (Sec. 3.2): returns (inv packed block after
    block, each m x m row-major and rounded to its storage precision, cond
    per block, precision per block).  Raises ValueError on a singular
    diagonal block."""
    rp, col, val = _csr(A)
    bptr = _c(bptr, np.int32)
    nb = bptr.size - 1
    sizes = np.diff(bptr).astype(np.int64)
    inv = np.zeros(max(int((sizes ** 2).sum()), 1))
    cond = np.zeros(max(nb, 1))
    prec = np.zeros(max(nb, 1), np.int32)
    bad = lib().orc_bj_generate(A.nrows, _p(rp), _p(col), _p(val), nb, _p(bptr), int(adaptive),
                                accuracy, _p(inv), _p(cond), _p(prec))
    if bad >= 0:
        raise ValueError(f"diagonal block {bad} is singular")
    return inv, cond[:nb], prec[:nb]


def bj_apply(bptr, inv, r):
    bptr = _c(bptr, np.int32)
    r = _c(r, np.float64)
    z = np.zeros_like(r)
    lib().orc_bj_apply(bptr.size - 1, _p(bptr), _p(_c(inv, np.float64)), _p(r), _p(z))
    return z


def bicgstab_block(A, b, bptr, inv, x0=None, max_iters=10_000, reduction=1e-10, nonfinite_check=1,
                   history=False):
    """BiCGSTAB with the block-Jacobi preconditioner (right preconditioning)."""
    rp, col, val = _csr(A)
    b = _c(b, np.float64)
    bptr = _c(bptr, np.int32)
    inv = _c(inv, np.float64)
    x = np.zeros(A.nrows) if x0 is None else _c(x0, np.float64).copy()
    info = _Info()
    hist = np.full(max_iters + 1, np.nan) if history else None
    lib().orc_bicgstab_block(A.nrows, _p(rp), _p(col), _p(val), bptr.size - 1, _p(bptr), _p(inv), _p(b),
                             _p(x), _Crit(max_iters, reduction, nonfinite_check), C.byref(info), _p(hist))
    out = dict(x=x, iterations=info.iterations, spmv_count=info.spmv_count,
               rel_residual=info.rel_residual, stop_reason=info.stop_reason)
    if history:
        out["history"] = hist[:info.iterations + 1]
    return out


def pcg_block(A, b, bptr, inv, x0=None, max_iters=10_000, reduction=1e-10, nonfinite_check=1,
              history=False):
    """CG with the block-Jacobi preconditioner z = blockdiag(inv) r."""
    rp, col, val = _csr(A)
    b = _c(b, np.float64)
    bptr = _c(bptr, np.int32)
    inv = _c(inv, np.float64)
    x = np.zeros(A.nrows) if x0 is None else _c(x0, np.float64).copy()
    info = _Info()
    hist = np.full(max_iters + 1, np.nan) if history else None
    lib().orc_pcg_block(A.nrows, _p(rp), _p(col), _p(val), bptr.size - 1, _p(bptr), _p(inv), _p(b),
                        _p(x), _Crit(max_iters, reduction, nonfinite_check), C.byref(info), _p(hist))
    out = dict(x=x, iterations=info.iterations, spmv_count=info.spmv_count,
               rel_residual=info.rel_residual, stop_reason=info.stop_reason)
    if history:
        out["history"] = hist[:info.iterations + 1]
    return out


def gmres(A, b, x0=None, dinv=None, krylov_dim=100, max_iters=10_000, reduction=1e-10,
          nonfinite_check=1, history=False, bptr=None, inv=None):
    """Restarted GMRES(krylov_dim) preconditioned from the right with point
    Jacobi (``dinv``), block Jacobi (``bptr``/``inv``) or nothing; modified
    Gram-Schmidt Arnoldi, Givens rotations (Sec. 3.1, Table 2).  The
    iteration count is the number of Arnoldi steps; ``history`` holds the
    residual estimates |g| / ||b||."""
    rp, col, val = _csr(A)
    b = _c(b, np.float64)
    x = np.zeros(A.nrows) if x0 is None else _c(x0, np.float64).copy()
    info = _Info()
    hist = np.full(max_iters + 1, np.nan) if history else None
    crit = _Crit(max_iters, reduction, nonfinite_check)
    if bptr is not None:
        bptr = _c(bptr, np.int32)
        inv = _c(inv, np.float64)
        lib().orc_gmres_block(A.nrows, _p(rp), _p(col), _p(val), bptr.size - 1, _p(bptr), _p(inv),
                              _p(b), _p(x), int(krylov_dim), crit, C.byref(info), _p(hist))
    else:
        d = None if dinv is None else _c(dinv, np.float64)
        lib().orc_gmres(A.nrows, _p(rp), _p(col), _p(val), _p(d), _p(b), _p(x), int(krylov_dim),
                        crit, C.byref(info), _p(hist))
    out = dict(x=x, iterations=info.iterations, spmv_count=info.spmv_count,
               rel_residual=info.rel_residual, stop_reason=info.stop_reason)
    if history:
        out["history"] = hist[:info.iterations + 1]
    return out


def ilu0(A):
    """ILU(0) factors on A's pattern (L strictly lower with unit diagonal,
    U the rest) by row-wise elimination; returns (lu, bad_row), bad_row = -1
    on success."""
    rp, col, val = _csr(A)
    lu = np.zeros(A.nnz)
    bad = lib().orc_ilu0(A.nrows, _p(rp), _p(col), _p(val), _p(lu))
    return lu, int(bad)


def parilu(A, sweeps):
    """ParILU factors after `sweeps` synchronous fixed-point sweeps."""
    rp, col, val = _csr(A)
    lu = np.zeros(A.nnz)
    bad = lib().orc_parilu(A.nrows, _p(rp), _p(col), _p(val), int(sweeps), _p(lu))
    return lu, int(bad)


def ilu_apply(A, lu, r, mode=0, sweeps=0):
    """z = U^{-1} L^{-1} r with the factors on A's pattern; mode 0 exact
    substitution, 1 `sweeps` Jacobi sweeps per triangular system."""
    rp, col, _ = _csr(A)
    lu = _c(lu, np.float64)
    r = _c(r, np.float64)
    z = np.zeros(A.nrows)
    lib().orc_ilu_apply(A.nrows, _p(rp), _p(col), _p(lu), int(mode), int(sweeps), _p(r), _p(z))
    return z


def gmres_ilu(A, b, lu, trs_mode=0, trs_sweeps=0, x0=None, krylov_dim=100, max_iters=10_000,
              reduction=1e-10, nonfinite_check=1, history=False):
    """Restarted GMRES right-preconditioned by the incomplete LU factors lu."""
    rp, col, val = _csr(A)
    b = _c(b, np.float64)
    lu = _c(lu, np.float64)
    x = np.zeros(A.nrows) if x0 is None else _c(x0, np.float64).copy()
    info = _Info()
    hist = np.full(max_iters + 1, np.nan) if history else None
    lib().orc_gmres_ilu(A.nrows, _p(rp), _p(col), _p(val), _p(lu), int(trs_mode), int(trs_sweeps), _p(b),
                        _p(x), int(krylov_dim), _Crit(max_iters, reduction, nonfinite_check),
                        C.byref(info), _p(hist))
    out = dict(x=x, iterations=info.iterations, spmv_count=info.spmv_count,
               rel_residual=info.rel_residual, stop_reason=info.stop_reason)
    if history:
        out["history"] = hist[:info.iterations + 1]
    return out
