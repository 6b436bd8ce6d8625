"""Matrix-free stencil operator (the user-defined operator of the paper's
Sec. 4) against the oracle: its products equal the oracle's CSR products of
the same operator (built by the input generators) within the SpMV contract,
and the solvers reach the oracle's iteration counts with it."""
import numpy as np
import pytest
import torch

import oracle as O
import workloads as W
from tests._gpu import DEV, assert_rows_close, dev, spmv_reference

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mxl():
    import paper_2006_16852_amd as m
    return m


@pytest.fixture(scope="module")
def ctx(mxl):
    return mxl.Context(0)


CASES = [("3d27_9", (9, 9, 9), W.points_3d27()),
         ("3d27_ragged", (13, 7, 5), W.points_3d27()),
         ("aniso7_11", (11, 11, 11), W.points_aniso7()),
         ("2d5_37", (37, 37, 1), W.points_2d5()),
         ("convdiff_17", (17, 17, 1), W.points_convdiff()),
         ("3d27_even", (12, 7, 5), W.points_3d27()),     # even nx: two points per thread
         ("aniso7_even", (10, 9, 8), W.points_aniso7()),
         ("2d5_even", (36, 37, 1), W.points_2d5()),
         ("line_3", (70, 1, 1), ([(-1, 0, 0), (0, 0, 0), (1, 0, 0)], [-1.0, 2.5, -1.0])),
         ("line_2", (2, 3, 1), ([(-1, 0, 0), (0, 0, 0), (1, 0, 0)], [-1.0, 2.5, -1.0])),
         ("single", (1, 1, 1), W.points_3d27())]


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
@pytest.mark.parametrize("name,shape,pc", CASES, ids=[c[0] for c in CASES])
def test_stencil_apply_parity(mxl, ctx, name, shape, pc, dtype):
    pts, cf = pc
    A = W.stencil_grid(*shape, pts, cf)
    op = mxl.stencil(ctx, shape, pts, cf, dtype)
    d = op.describe()
    assert d["format"] == mxl.STENCIL and d["nnz"] == A.nnz and d["stored_bytes"] == 0
    x = W.uniform_vec(A.nrows, 3)
    y0 = W.uniform_vec(A.nrows, 4)
    fp32 = dtype == torch.float32
    for alpha, beta in ((1.0, 0.0), (-0.5, 2.0)):
        want, bound = spmv_reference(A, x, alpha, beta, y0, fp32)
        y = dev(y0, dtype)
        op.apply(dev(x, dtype), y, alpha, beta)
        assert_rows_close(y.cpu().double().numpy(), want, bound, 1e-5 if fp32 else 1e-12, name)


def test_stencil_nan_only_through_neighbours(mxl, ctx):
    """A NaN in x reaches exactly the rows whose stencil covers it (the
    out-of-grid points never multiply x)."""
    pts, cf = W.points_3d27()
    shape = (6, 5, 4)
    A = W.stencil_grid(*shape, pts, cf)
    op = mxl.stencil(ctx, shape, pts, cf)
    for j in (0, A.nrows - 1, 37):
        x = np.ones(A.nrows)
        x[j] = np.nan
        y = torch.zeros(A.nrows, dtype=torch.float64, device=DEV)
        op.apply(dev(x), y)
        rows = np.repeat(np.arange(A.nrows), A.row_lengths())
        want = np.zeros(A.nrows, bool)
        want[rows[A.col == j]] = True
        assert np.array_equal(np.isnan(y.cpu().numpy()), want)


def test_stencil_full_size_rowsums(mxl, ctx):
    """128^3 27-point: A 1 equals the exact integer row sums, and sampled
    rows of A x match the oracle one by one."""
    N = 128
    pts, cf = W.points_3d27()
    op = mxl.stencil(ctx, (N, N, N), pts, cf)
    n = N ** 3
    idx = np.arange(n)
    c = [np.where((t == 0) | (t == N - 1), 2, 3) for t in (idx % N, (idx // N) % N, idx // N ** 2)]
    rowsum = (27 - c[0] * c[1] * c[2]).astype(np.float64)
    y = torch.empty(n, dtype=torch.float64, device=DEV)
    op.apply(torch.ones(n, dtype=torch.float64, device=DEV), y)
    assert np.array_equal(y.cpu().numpy(), rowsum)
    A = W.stencil_3d27(N)
    x = W.uniform_vec(n, 2)
    op.apply(dev(x), y)
    rows = np.unique(np.random.default_rng(0).integers(0, n, 3000))
    sub = W.Csr(rows.size, n, np.concatenate([[0], np.cumsum(A.row_lengths()[rows])]).astype(np.int32),
                np.concatenate([A.col[A.row_ptr[r]:A.row_ptr[r + 1]] for r in rows]),
                np.concatenate([A.val[A.row_ptr[r]:A.row_ptr[r + 1]] for r in rows]))
    want, bound = spmv_reference(sub, x, 1.0, 0.0, np.zeros(rows.size), False)
    assert_rows_close(y.cpu().numpy()[rows], want, bound, 1e-12, "stencil128")


def test_stencil_solvers(mxl, ctx):
    """Jacobi-PCG, BiCGSTAB and IR with the matrix-free operator reach the
    oracle's iteration counts (within 2) and the requested residual."""
    N = 16
    pts, cf = W.points_3d27()
    A = W.stencil_3d27(N)
    op = mxl.stencil(ctx, (N, N, N), pts, cf)
    P = mxl.jacobi(op)
    assert np.allclose(P.export("dinv").cpu().numpy(), 1.0 / 26.0, rtol=0, atol=0)
    b = O.spmv(A, W.uniform_vec(A.nrows, 1))
    d, _ = O.jacobi_dinv(A)
    ref = O.pcg(A, b, dinv=d, reduction=1e-10)
    S = mxl.solver("cg", op, P, max_iters=2000, reduction=1e-10)
    x = torch.zeros(A.nrows, dtype=torch.float64, device=DEV)
    info = S.solve(dev(b), x)
    assert info["stop_reason"] == mxl.STOP_CONVERGED
    assert abs(info["iterations"] - ref["iterations"]) <= 2
    assert np.linalg.norm(b - O.spmv(A, x.cpu().numpy())) <= 1.01e-10 * np.linalg.norm(b)
    # nonsymmetric: BiCGSTAB on convection-diffusion
    pts2, cf2 = W.points_convdiff()
    C = W.convdiff_2d5(24)
    opc = mxl.stencil(ctx, (24, 24, 1), pts2, cf2)
    bc = O.spmv(C, W.uniform_vec(C.nrows, 5))
    dc, _ = O.jacobi_dinv(C)
    refc = O.bicgstab(C, bc, dinv=dc, reduction=1e-10)
    Sb = mxl.solver("bicgstab", opc, mxl.jacobi(opc), max_iters=2000, reduction=1e-10)
    xc = torch.zeros(C.nrows, dtype=torch.float64, device=DEV)
    ib = Sb.solve(dev(bc), xc)
    assert ib["stop_reason"] == mxl.STOP_CONVERGED
    assert abs(ib["iterations"] - refc["iterations"]) <= 2
    # mixed precision: FP32 inner CG on the cast operator
    pts3, cf3 = W.points_aniso7()
    Q = W.aniso_3d7(20)
    opq = mxl.stencil(ctx, (20, 20, 20), pts3, cf3)
    bq = W.uniform_vec(Q.nrows, 4)
    I = mxl.ir(opq, outer=dict(reduction=1e-12), inner=dict(reduction=1e-4))
    xq = torch.zeros(Q.nrows, dtype=torch.float64, device=DEV)
    ii = I.solve(dev(bq), xq)
    assert ii["stop_reason"] == mxl.STOP_CONVERGED
    assert np.linalg.norm(bq - O.spmv(Q, xq.cpu().numpy())) <= 1.01e-12 * np.linalg.norm(bq)


def test_stencil_errors(mxl, ctx):
    pts, cf = W.points_3d27()
    with pytest.raises(mxl.MxlError) as e:
        mxl.stencil(ctx, (4, 4, 4), [(2, 0, 0)], [1.0])
    assert e.value.status == mxl.ERR_INVALID_ARG
    with pytest.raises(mxl.MxlError) as e:
        mxl.stencil(ctx, (4, 4, 4), [(0, 0, 0), (0, 0, 0)], [1.0, 2.0])
    assert e.value.status == mxl.ERR_INVALID_ARG
    with pytest.raises(mxl.MxlError) as e:
        mxl.stencil(ctx, (0, 4, 4), pts, cf)
    assert e.value.status == mxl.ERR_INVALID_ARG
    op = mxl.stencil(ctx, (4, 4, 4), [(-1, 0, 0), (1, 0, 0)], [1.0, 1.0])
    with pytest.raises(mxl.MxlError) as e:
        mxl.jacobi(op)
    assert e.value.status == mxl.ERR_ZERO_DIAG
    with pytest.raises(mxl.MxlError) as e:
        op.convert("ell")
    assert e.value.status == mxl.ERR_NOT_IMPLEMENTED
    with pytest.raises(mxl.MxlError) as e:
        op.features()
    assert e.value.status == mxl.ERR_NOT_IMPLEMENTED
