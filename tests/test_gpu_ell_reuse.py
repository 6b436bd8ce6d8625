"""ELL products with neighbour reuse of gathered x values.

Entry (i, s) whose column equals that of entry (i+1, s-1) takes x from that
entry instead of gathering it.  The value moved is x at the same column, so
the product must equal, bit for bit, the one that gathers every entry (the
LDS-staged variant never reuses), and stay within the oracle's per-row bound.
The conversion enables reuse when at least a quarter of the entries (of HYB's
ELL part) hit; the rule is recomputed here from the CSR arrays.
"""
import numpy as np
import pytest
import torch

import workloads as W
from tests._gpu import assert_rows_close, dev, matrix, spmv_reference

pytestmark = pytest.mark.gpu


def _hits(A, w=None):
    """Entries (i, s), 1 <= s < w, whose column equals that of (i+1, s-1),
    counting the first w entries of each row only (the ELL part of HYB)."""
    rp = A.row_ptr.astype(np.int64)
    w = int(np.diff(rp).max(initial=0)) if w is None else w
    h = 0
    for i in range(A.nrows - 1):
        a0, la = rp[i], min(rp[i + 1] - rp[i], w)
        b0, lb = rp[i + 1], min(rp[i + 2] - rp[i + 1], w)
        m = int(min(la - 1, lb))
        if m > 0:
            h += int(np.count_nonzero(A.col[a0 + 1:a0 + 1 + m] == A.col[b0:b0 + m]))
    return h


def _stored(A, w):
    return int(np.minimum(np.diff(A.row_ptr.astype(np.int64)), w).sum())


def _band_dropout(n, half, keep, seed):
    """Banded rows [i-half, i+half] with each off-diagonal entry kept with
    probability `keep`: runs of consecutive columns broken at random, so only
    part of the entries can reuse."""
    rng = np.random.default_rng(seed)
    rows, cols = [], []
    for i in range(n):
        c = np.arange(max(0, i - half), min(n, i + half + 1))
        m = (rng.random(c.size) < keep) | (c == i)
        rows.append(np.full(int(m.sum()), i))
        cols.append(c[m])
    rows = np.concatenate(rows)
    cols = np.concatenate(cols).astype(np.int32)
    rp = np.zeros(n + 1, np.int64)
    np.add.at(rp, rows + 1, 1)
    rp = np.cumsum(rp).astype(np.int32)
    val = rng.standard_normal(cols.size)
    return W.Csr(n, n, rp, cols, val, f"band{half}_keep{keep}_{n}")


MATS = [W.stencil_3d27(11), W.stencil_2d5(37), W.aniso_3d7(13), W.convdiff_2d5(29),
        _band_dropout(3001, 6, 0.85, 3), _band_dropout(517, 3, 0.6, 4)]


@pytest.fixture(scope="module")
def mxl():
    import paper_2006_16852_amd as m
    return m


@pytest.fixture(scope="module")
def ctx(mxl):
    return mxl.Context(0)


@pytest.mark.parametrize("A", MATS, ids=[a.name for a in MATS])
def test_reuse_flag_follows_rule(mxl, ctx, A):
    print(f"[ell-reuse flag] {A.name}", flush=True)
    base = matrix(mxl, ctx, A)
    want = 1 if 4 * _hits(A) >= A.nnz else 0
    for var in (0, mxl.ELL_DELTA16):
        assert base.convert("ell", variant=var).describe()["ell_reuse"] == want
    assert base.convert("ell", variant=mxl.ELL_LDS).describe()["ell_reuse"] == 0


@pytest.mark.parametrize("q", [0.66, 0.9])
@pytest.mark.parametrize("A", MATS, ids=[a.name for a in MATS])
def test_reuse_hyb_flag_and_bitwise(mxl, ctx, A, q):
    """HYB reuses within its ELL part; the tail is unchanged.  Against the
    LDS-staged HYB (which never reuses), bit for bit."""
    print(f"[hyb-reuse] {A.name} q={q}", flush=True)
    base = matrix(mxl, ctx, A)
    op = base.convert("hyb", hyb_quantile=q)
    d = op.describe()
    w = d["ell_width"]
    want = 1 if _stored(A, w) > 0 and 4 * _hits(A, w) >= _stored(A, w) else 0
    assert d["ell_reuse"] == want
    ref = base.convert("hyb", variant=mxl.ELL_LDS, hyb_quantile=q)
    assert ref.describe()["ell_reuse"] == 0
    rng = np.random.default_rng(5)
    x = dev(rng.uniform(-1, 1, A.ncols))
    y0 = rng.uniform(-1, 1, A.nrows)
    ya, yb = dev(y0), dev(y0)
    op.apply(x, ya, alpha=1.1, beta=0.3)
    ref.apply(x, yb, alpha=1.1, beta=0.3)
    assert np.array_equal(ya.cpu().numpy(), yb.cpu().numpy())


def test_reuse_off_on_scattered_columns(mxl, ctx):
    A = W.random_sparse(4000, 4000, 0.003, 5)
    base = matrix(mxl, ctx, A)
    assert 4 * _hits(A) < A.nnz
    assert base.convert("ell").describe()["ell_reuse"] == 0


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
@pytest.mark.parametrize("rpt", [1, 2, 4])
@pytest.mark.parametrize("A", MATS, ids=[a.name for a in MATS])
def test_reuse_bitwise_and_bound(mxl, ctx, A, rpt, dtype):
    print(f"[ell-reuse] {A.name} R={rpt} {dtype}", flush=True)
    base = matrix(mxl, ctx, A, dtype)
    ref = base.convert("ell", variant=mxl.ELL_LDS, vector_width=rpt)
    ops = {"ell": base.convert("ell", vector_width=rpt),
           "ell16": base.convert("ell", variant=mxl.ELL_DELTA16, vector_width=rpt)}
    rng = np.random.default_rng(11)
    x = rng.uniform(-1, 1, A.ncols)
    y0 = rng.uniform(-1, 1, A.nrows)
    xd = dev(x, dtype)
    for alpha, beta in ((1.0, 0.0), (1.3, 0.7)):
        yr = dev(y0, dtype)
        ref.apply(xd, yr, alpha=alpha, beta=beta)
        yr = yr.cpu().numpy()
        want, bound = spmv_reference(A, x, alpha, beta, y0, dtype == torch.float32)
        for name, op in ops.items():
            yd = dev(y0, dtype)
            op.apply(xd, yd, alpha=alpha, beta=beta)
            got = yd.cpu().numpy()
            assert np.array_equal(got, yr), f"{name}: differs from the gathering product"
            assert_rows_close(got, want, bound, 1e-12 if dtype == torch.float64 else 1e-5, name)


@pytest.mark.parametrize("fmt,q", [("ell", 0.0), ("hyb", 0.9)], ids=["ell", "hyb"])
@pytest.mark.parametrize("A", [MATS[0], MATS[2], MATS[4]], ids=lambda a: a.name)
def test_reuse_cg_bitwise(mxl, ctx, A, fmt, q):
    """Jacobi-CG through the fused product with reuse (and the dot's w rows
    loaded with the first slots) equals, bit for bit, the same solve through
    the LDS-staged variant, which neither reuses nor prefetches: every
    product and every partial of the fused dot is the same (on the
    nonsymmetric band matrix down to the same breakdown)."""
    print(f"[ell-reuse cg] {A.name} {fmt}", flush=True)
    base = matrix(mxl, ctx, A)
    kw = {"hyb_quantile": q} if fmt == "hyb" else {}
    ops = [base.convert(fmt, **kw), base.convert(fmt, variant=mxl.ELL_LDS, **kw)]
    if fmt == "ell":
        ops.append(base.convert("ell", variant=mxl.ELL_DELTA16))
    assert ops[0].describe()["ell_reuse"] == 1 and ops[1].describe()["ell_reuse"] == 0
    rng = np.random.default_rng(9)
    b = dev(rng.uniform(-1, 1, A.nrows))
    outs = []
    for op in ops:
        S = mxl.solver("cg", op, mxl.jacobi(op), max_iters=2000, reduction=1e-10, check_every=8,
                       launch_mode=1)
        x = torch.zeros(A.nrows, dtype=torch.float64, device="cuda:0")
        info = S.solve(b, x)
        outs.append((info["stop_reason"], info["iterations"], x.cpu().numpy()))
    if A.name.startswith(("stencil", "aniso")):  # SPD: CG converges
        assert outs[0][0] == mxl.STOP_CONVERGED
    for stop, it, x in outs[1:]:  # the nonsymmetric band matrix breaks down, identically
        assert stop == outs[0][0] and it == outs[0][1] and np.array_equal(x, outs[0][2])


@pytest.mark.parametrize("A", [W.aniso_3d7(24), W.stencil_3d27(22)], ids=lambda a: a.name)
def test_reuse_refinement_bitwise(mxl, ctx, A):
    """FP32-inner refinement: the FP32 copy keeps the reuse of the FP64
    operator, and the refined solution equals, bit for bit, the one through
    the LDS-staged operator (no reuse in either precision)."""
    print(f"[ell-reuse ir] {A.name}", flush=True)
    base = matrix(mxl, ctx, A)
    ops = [base.convert("ell", variant=mxl.ELL_DELTA16), base.convert("ell", variant=mxl.ELL_LDS)]
    assert ops[0].describe()["ell_reuse"] == 1 and ops[1].describe()["ell_reuse"] == 0
    b = dev(np.random.default_rng(12).uniform(-1, 1, A.nrows))
    outs = []
    for op in ops:
        I = mxl.ir(op, outer=dict(max_iters=30, reduction=1e-12),
                   inner=dict(reduction=1e-3, max_iters=5000, check_every=8, launch_mode=1))
        x = torch.zeros(A.nrows, dtype=torch.float64, device="cuda:0")
        info = I.solve(b, x)
        assert info["stop_reason"] == mxl.STOP_CONVERGED
        outs.append((info["iterations"], info["inner_iterations"], x.cpu().numpy()))
    assert outs[0][:2] == outs[1][:2] and np.array_equal(outs[0][2], outs[1][2])
