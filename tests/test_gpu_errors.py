"""Every error status of the C ABI is reachable and is raised on the host,
before any kernel runs (the paper's apply checks sizes, checked casts throw,
and unimplemented combinations throw)."""
import ctypes as C

import numpy as np
import pytest
import torch

import workloads as W
from tests._gpu import DEV, dev, matrix

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mxl():
    import paper_2006_16852_amd as m
    return m


@pytest.fixture(scope="module")
def ctx(mxl):
    return mxl.Context(0)


def _status(mxl, fn, *a):
    with pytest.raises(mxl.MxlError) as e:
        fn(*a)
    return e.value.status


def test_invalid_args(mxl, ctx):
    A = W.stencil_2d5(8)
    M = matrix(mxl, ctx, A)
    x = torch.ones(64, dtype=torch.float64, device=DEV)
    assert _status(mxl, M.apply, x, x) == mxl.ERR_INVALID_ARG           # aliasing
    st = mxl.lib.mxl_apply_adv(M.h, 1.0, None, 0.0, C.c_void_p(x.data_ptr()))
    assert st == mxl.ERR_INVALID_ARG                                    # NULL
    host = np.ones(64)
    y = torch.zeros(64, dtype=torch.float64, device=DEV)
    st = mxl.lib.mxl_apply_adv(M.h, 1.0, host.ctypes.data_as(C.c_void_p), 0.0,
                               C.c_void_p(y.data_ptr()))
    assert st == mxl.ERR_INVALID_ARG                                    # host memory
    assert "device memory" in mxl.lib.mxl_last_error().decode()
    assert mxl.lib.mxl_apply(None, None, None) == mxl.ERR_INVALID_ARG
    assert _status(mxl, lambda: mxl.solver("cg", M, None, max_iters=-1)) == mxl.ERR_INVALID_ARG
    bad = mxl.lib.mxl_convert(M.h, 3, None, C.byref(C.c_void_p()))
    assert bad == mxl.OK  # NULL params mean defaults


def test_dtype_and_dims(mxl, ctx):
    A = W.stencil_2d5(8)
    M64 = matrix(mxl, ctx, A)
    M32 = matrix(mxl, ctx, A, torch.float32)
    P32 = mxl.jacobi(M32)
    assert _status(mxl, mxl.solver, "cg", M64, P32) == mxl.ERR_DTYPE
    assert _status(mxl, mxl.ir, M32) == mxl.ERR_DTYPE
    B = W.stencil_2d5(9)
    PB = mxl.jacobi(matrix(mxl, ctx, B))
    assert _status(mxl, mxl.solver, "cg", M64, PB) == mxl.ERR_DIM_MISMATCH
    R = W.random_sparse(10, 12, 0.3, 1)
    assert _status(mxl, mxl.jacobi, matrix(mxl, ctx, R)) == mxl.ERR_NOT_IMPLEMENTED
    assert _status(mxl, mxl.solver, "cg", matrix(mxl, ctx, R)) == mxl.ERR_DIM_MISMATCH


def test_not_implemented(mxl, ctx):
    M = matrix(mxl, ctx, W.stencil_2d5(8))
    assert _status(mxl, M.convert, "csr", 7) == mxl.ERR_NOT_IMPLEMENTED
    assert _status(mxl, M.convert, "ell", 5) == mxl.ERR_NOT_IMPLEMENTED
    assert _status(mxl, M.convert, "csr", 1, 3) == mxl.ERR_INVALID_ARG  # width 3


def test_invalid_matrix_validation(mxl, ctx):
    A = W.random_sparse(40, 40, 0.2, 3)
    r = next(i for i in range(40) if A.row_ptr[i + 1] - A.row_ptr[i] >= 2)
    k = A.row_ptr[r]
    col = A.col.copy()
    col[k], col[k + 1] = col[k + 1], col[k]
    rp, c, v = dev(A.row_ptr), dev(col), dev(A.val)
    assert _status(mxl, mxl.csr, ctx, rp, c, v, None, False, True) == mxl.ERR_INVALID_MATRIX
    col2 = A.col.copy()
    col2[0] = 40
    assert _status(mxl, mxl.csr, ctx, rp, dev(col2), v, None, False, True) == mxl.ERR_INVALID_MATRIX
    ok = mxl.csr(ctx, rp, dev(A.col), v, validate=True)
    assert ok.describe()["nnz"] == A.nnz


def test_zero_diagonal(mxl, ctx):
    A = W.stencil_2d5(6)
    A.val[A.row_ptr[7] + 2] = 0.0     # row 7's diagonal (interior row: 5 entries, diag 3rd)
    assert A.col[A.row_ptr[7] + 2] == 7
    assert _status(mxl, mxl.jacobi, matrix(mxl, ctx, A)) == mxl.ERR_ZERO_DIAG
    assert "row 7" in mxl.lib.mxl_last_error().decode()


def test_infeasible_ell(mxl, ctx):
    n = 200_000
    rows = [([i], [1.0]) for i in range(n)]
    rows[5] = (list(range(10_000)), [1.0] * 10_000)
    rp = np.zeros(n + 1, np.int64)
    rp[1:] = np.cumsum([len(c) for c, _ in rows])
    col = np.concatenate([np.array(c, np.int32) for c, _ in rows])
    val = np.concatenate([np.array(v) for _, v in rows])
    A = W.Csr(n, n, rp.astype(np.int32), col, val)
    M = matrix(mxl, ctx, A)
    assert _status(mxl, M.convert, "ell") == mxl.ERR_INFEASIBLE_FORMAT
    H = M.convert("hyb", hyb_quantile=0.9)        # the tail absorbs the long row
    d = H.describe()
    assert d["ell_width"] == 1 and d["tail_nnz"] == 9_999


def test_handles_freed_in_any_order(mxl):
    """Handles that die together in a reference cycle are finalized in an
    arbitrary order (the context may go first); the library keeps a
    context alive while any object still uses it, so nothing is used after
    it is freed, and the library keeps working afterwards."""
    import gc

    class Holder:
        pass

    ctx = mxl.Context(0)
    A = matrix(mxl, ctx, W.stencil_2d5(8))
    h = Holder()
    h.me, h.ctx, h.A, h.P = h, ctx, A, mxl.jacobi(A)
    h.S = mxl.solver("cg", A, h.P, max_iters=50)
    x = torch.zeros(64, dtype=torch.float64, device=DEV)
    h.S.solve(torch.ones(64, dtype=torch.float64, device=DEV), x)
    del ctx, A, h
    gc.collect()
    ctx2 = mxl.Context(0)
    B = matrix(mxl, ctx2, W.stencil_2d5(8))
    y = torch.empty(64, dtype=torch.float64, device=DEV)
    B.apply(torch.ones(64, dtype=torch.float64, device=DEV), y)
    assert float(y.sum()) == float(W.stencil_2d5(8).val.sum())


def test_repeated_create_solve_destroy_releases_memory(mxl, ctx):
    """Every kind of operator created, used and dropped many times (GMRES
    with its captured graphs, CG, BiCGSTAB, refinement with point and block
    Jacobi, block Jacobi, ParILU, a batch with its ELL copy, a selector's
    features): the device's free memory comes back."""
    import gc
    A = W.convdiff_2d5(48)
    S2 = W.stencil_2d5(48)
    Bt = W.batch_systems(nsys=40, seed=3)
    b = dev(W.uniform_vec(A.nrows, 1))

    def cycle():
        M = matrix(mxl, ctx, A).convert("ell", variant=mxl.ELL_DELTA16)
        Ms = matrix(mxl, ctx, S2)
        x = torch.zeros(A.nrows, dtype=torch.float64, device=DEV)
        for kind, P in (("gmres", mxl.jacobi(M)), ("bicgstab", mxl.jacobi(M)),
                        ("gmres", mxl.ilu(matrix(mxl, ctx, A), sweeps=2, trisolve="jacobi", trs_sweeps=2))):
            S = mxl.solver(kind, M, P, max_iters=200, reduction=1e-8, check_every=8)
            x.zero_()
            S.solve(b, x)
        for P in (mxl.jacobi(Ms), mxl.bjacobi(Ms, 8, True)):
            x.zero_()
            mxl.solver("cg", Ms, P, max_iters=200, reduction=1e-8).solve(b, x)
        for bs in (0, 8):
            x.zero_()
            mxl.ir(Ms, block_size=bs).solve(b, x)
        Ms.features()
        op = mxl.batch(ctx, Bt.sys_ptr, dev(Bt.sys_ptr), dev(Bt.row_ptr), dev(Bt.col), dev(Bt.val))
        bb = dev(Bt.b)
        xb = torch.zeros_like(bb)
        it = torch.zeros(Bt.nsys, dtype=torch.int32, device=DEV)
        rel = torch.zeros(Bt.nsys, dtype=torch.float64, device=DEV)
        st = torch.zeros(Bt.nsys, dtype=torch.uint8, device=DEV)
        op.solve(bb, xb, it, rel, st, reduction=1e-10)
        torch.cuda.synchronize()

    cycle()
    gc.collect()
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    for _ in range(25):
        cycle()
    gc.collect()
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    print(f"[leak] free before {free0 / 2**20:.1f} MiB after {free1 / 2**20:.1f} MiB", flush=True)
    assert free0 - free1 < 32 * 2**20


CSR_RULES = {1: "row_ptr[0] != 0", 2: "row_ptr decreases", 3: "row_ptr[n] != nnz",
             4: "column out of range", 5: "columns not strictly increasing"}


def _violations(seed=3):
    """One matrix per canonical-form rule, each breaking only that rule; the
    expected oracle verdict (orc_csr_check's code) with it."""
    A = W.random_sparse(300, 300, 0.05, seed)
    n, nnz = A.nrows, A.nnz
    out = []
    rp = A.row_ptr.copy(); rp[0] = 1                        # bad start (row 0 loses an entry)
    out.append((1, rp, A.col.copy()))
    rp = A.row_ptr.copy()
    i = next(i for i in range(1, n) if rp[i + 1] - rp[i] >= 2)
    rp[i] = rp[i + 1] + 1 if rp[i + 1] + 1 <= nnz else rp[i + 1]
    assert rp[i] > rp[i + 1]                                 # row i ends before it starts
    out.append((2, rp, A.col.copy()))
    rp = A.row_ptr.copy(); rp[n] = nnz - 1                   # last row ends early
    out.append((3, rp, A.col.copy()))
    col = A.col.copy(); col[nnz // 2] = -1                   # negative column
    out.append((4, A.row_ptr.copy(), col))
    col = A.col.copy(); k = A.row_ptr[n - 1]; col[k] = 300   # column == ncols
    out.append((4, A.row_ptr.copy(), col))
    col = A.col.copy()
    r = next(r for r in range(n) if A.row_ptr[r + 1] - A.row_ptr[r] >= 2)
    col[A.row_ptr[r] + 1] = col[A.row_ptr[r]]                # duplicate column
    out.append((5, A.row_ptr.copy(), col))
    col = A.col.copy()
    r = next(r for r in range(n - 1, 0, -1) if A.row_ptr[r + 1] - A.row_ptr[r] >= 2)
    k = A.row_ptr[r]
    col[k], col[k + 1] = col[k + 1], col[k]                  # unsorted row
    out.append((5, A.row_ptr.copy(), col))
    return A, out


@pytest.mark.parametrize("case", range(7))
def test_csr_validation_matches_oracle(mxl, ctx, case):
    """Each canonical-form rule broken alone: the oracle's verdict is that
    rule, and the device validation fails with INVALID_MATRIX naming the
    same rule first (and setting its bit in the mask)."""
    import oracle as O
    A, cases = _violations()
    kind, rp, col = cases[case]
    bad = W.Csr(A.nrows, A.ncols, rp, col, A.val)
    assert O.csr_check(bad) == kind
    st = _status(mxl, mxl.csr, ctx, dev(rp), dev(col), dev(A.val), None, False, True)
    assert st == mxl.ERR_INVALID_MATRIX
    msg = mxl.lib.mxl_last_error().decode()
    print(f"[validate case {case} kind {kind}] {msg}", flush=True)
    assert f"first: {CSR_RULES[kind]}" in msg
    mask = int(msg.split("mask 0x")[1].split(";")[0], 16)
    assert mask & (1 << (kind - 1))


def test_csr_validation_accepts_canonical(mxl, ctx):
    import oracle as O
    for A in [W.random_sparse(300, 300, 0.05, 3), W.stencil_2d5(16)] + W.edge_matrices():
        assert O.csr_check(A) == 0
        M = mxl.csr(ctx, dev(A.row_ptr), dev(A.col), dev(A.val), ncols=A.ncols, validate=True)
        assert M.describe()["nnz"] == A.nnz
