"""Batched persistent Jacobi-PCG against the oracle's per-system PCG.

Bar: every system converges; iteration counts within 2 of the oracle's for
at least 99% of systems (summation order differs); the residual recomputed
in FP64 on the CPU meets 1e-10; schedules that share the workgroup size give
bitwise-identical results, and so do the CSR and the per-system ELL kernels
(the ELL product keeps each row's stored order)."""
import numpy as np
import pytest
import torch

import oracle as O
import workloads as W
from tests._gpu import DEV, dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mxl():
    import paper_2006_16852_amd as m
    return m


@pytest.fixture(scope="module")
def ctx(mxl):
    return mxl.Context(0)


def _run(mxl, ctx, B, tuning=None, **crit):
    op = mxl.batch(ctx, B.sys_ptr, dev(B.sys_ptr), dev(B.row_ptr), dev(B.col), dev(B.val))
    b = dev(B.b)
    x = torch.zeros_like(b)
    it = torch.zeros(B.nsys, dtype=torch.int32, device=DEV)
    rel = torch.zeros(B.nsys, dtype=torch.float64, device=DEV)
    st = torch.zeros(B.nsys, dtype=torch.uint8, device=DEV)
    op.solve(b, x, it, rel, st, tuning=tuning, reduction=1e-10, **crit)
    return op, x.cpu().numpy(), it.cpu().numpy(), rel.cpu().numpy(), st.cpu().numpy()


def _check_residuals(B, x, tol=1.01e-10):
    for s in range(B.nsys):
        A = B.system(s)
        r0, r1 = B.sys_ptr[s], B.sys_ptr[s + 1]
        r = B.b[r0:r1] - O.spmv(A, x[r0:r1])
        assert np.linalg.norm(r) <= tol * np.linalg.norm(B.b[r0:r1]), s


@pytest.mark.parametrize("tuning", [None, (64, 4, 1), (128, 2, 0), (256, 1, 1), (512, 1, 0)],
                         ids=["default", "64x4", "128x2", "256x1", "512x1"])
def test_batch_parity(mxl, ctx, tuning):
    B = W.batch_systems(nsys=300, seed=77)
    ref = O.batch_pcg(B, reduction=1e-10)
    _, x, it, rel, st = _run(mxl, ctx, B, tuning)
    print(f"[batch {tuning}] iters gpu {it.sum()} oracle {ref['iterations'].sum()}", flush=True)
    assert np.all(st == 1)
    assert np.mean(np.abs(it - ref["iterations"]) <= 2) >= 0.99
    assert np.allclose(rel, ref["rel_residual"], rtol=0.5, atol=1e-13)
    _check_residuals(B, x)


def test_batch_schedules_same_wg_size_bitwise(mxl, ctx):
    B = W.batch_systems(nsys=120, seed=3)
    _, x1, it1, _, _ = _run(mxl, ctx, B, (128, 1, 0))
    _, x2, it2, _, _ = _run(mxl, ctx, B, (128, 8, 1))
    assert np.array_equal(it1, it2) and np.array_equal(x1, x2)


@pytest.mark.parametrize("fmt", [1, 2], ids=["csr", "ell"])
def test_batch_large_system_scratch_path(mxl, ctx, fmt):
    """A system larger than the LDS capacity runs from global scratch: the
    64x64 Poisson system as a batch of one, plus small systems around it."""
    A = W.stencil_2d5(64)
    b1 = O.spmv(A, W.uniform_vec(A.nrows, 1))
    S = W.batch_systems(nsys=5, seed=8)
    rp = np.concatenate([A.row_ptr[:-1], S.row_ptr + A.nnz]).astype(np.int32)
    sp = np.concatenate([[0], S.sys_ptr + A.nrows]).astype(np.int32)
    Bb = W.Batch(6, sp, rp, np.concatenate([A.col, S.col]), np.concatenate([A.val, S.val]),
                 np.concatenate([b1, S.b]))
    ref = O.batch_pcg(Bb, reduction=1e-10)
    _, x, it, rel, st = _run(mxl, ctx, Bb, (1024, 1, 1, fmt))
    assert np.all(st == 1)
    assert abs(int(it[0]) - int(ref["iterations"][0])) <= 2
    _check_residuals(Bb, x)


@pytest.mark.parametrize("wg,wpc", [(64, 4), (128, 2), (256, 1), (512, 1), (1024, 1)])
def test_batch_ell_equals_csr_bitwise(mxl, ctx, wg, wpc):
    B = W.batch_systems(nsys=150, seed=21)
    _, x1, it1, r1, s1 = _run(mxl, ctx, B, (wg, wpc, 0, 1))
    _, x2, it2, r2, s2 = _run(mxl, ctx, B, (wg, wpc, 1, 2))
    assert np.all(s1 == 1)
    assert np.array_equal(it1, it2) and np.array_equal(x1, x2) and np.array_equal(r1, r2) and np.array_equal(s1, s2)


def _batch_from(systems, rhs_seed=3):
    rps, cols, vals, sp = [], [], [], [0]
    off = 0
    for A in systems:
        rps.append(A.row_ptr[:-1] + off)
        cols.append(A.col)
        vals.append(A.val)
        off += A.nnz
        sp.append(sp[-1] + A.nrows)
    rp = np.concatenate(rps + [[off]]).astype(np.int32)
    b = W.uniform_vec(sp[-1], rhs_seed)
    return W.Batch(len(systems), np.array(sp, np.int32), rp, np.concatenate(cols).astype(np.int32),
                   np.concatenate(vals), b)


def test_batch_tiny_systems_ell_equals_csr(mxl, ctx):
    """Systems of one and two rows, a diagonal system and a dense 5x5 one:
    the ELL kernel (padding slots included) equals the CSR kernel bit for
    bit and the oracle's counts."""
    one = W.Csr(1, 1, np.array([0, 1], np.int32), np.array([0], np.int32), np.array([3.0]), "one")
    two = W.Csr(2, 2, np.array([0, 2, 4], np.int32), np.array([0, 1, 0, 1], np.int32),
                np.array([4.0, 1.0, 1.0, 3.0]), "two")
    diag = W.Csr(7, 7, np.arange(8, dtype=np.int32), np.arange(7, dtype=np.int32), np.linspace(1, 2, 7), "diag")
    D = np.full((5, 5), 0.5) + np.eye(5) * 4.0
    r, c = np.nonzero(D)
    dense = W.Csr(5, 5, np.arange(0, 26, 5, dtype=np.int32), c.astype(np.int32), D[r, c], "dense5")
    Bb = _batch_from([one, two, W.stencil_2d5(5), diag, dense, one])
    ref = O.batch_pcg(Bb, reduction=1e-10)
    for wg in (64, 256):
        _, x1, it1, _, s1 = _run(mxl, ctx, Bb, (wg, 2, 0, 1))
        _, x2, it2, _, s2 = _run(mxl, ctx, Bb, (wg, 2, 0, 2))
        assert np.all(s1 == 1) and np.array_equal(it1, it2) and np.array_equal(x1, x2)
        assert np.all(np.abs(it1 - ref["iterations"]) <= 2)
    _check_residuals(Bb, x1)


def test_batch_skewed_rows_keep_csr(mxl, ctx):
    """One dense row in a system makes the padded copy too large: the batch
    has no ELL copy, format 2 is refused and format 0 runs the CSR kernel."""
    n = 200
    D = np.eye(n) * (n + 1.0)
    D[0, :] += 1.0
    D[:, 0] += 1.0
    D[0, 0] = 4.0 * n
    r, c = np.nonzero(D)
    A = W.Csr(n, n, np.concatenate([[0], np.cumsum(np.bincount(r, minlength=n))]).astype(np.int32),
              c.astype(np.int32), D[r, c], "arrow")
    Bb = _batch_from([A, W.stencil_2d5(6)])
    with pytest.raises(mxl.MxlError) as e:
        _run(mxl, ctx, Bb, (128, 2, 0, 2))
    assert e.value.status == mxl.ERR_NOT_IMPLEMENTED
    ref = O.batch_pcg(Bb, reduction=1e-10)
    _, x, it, rel, st = _run(mxl, ctx, Bb, (128, 2, 0, 0))
    assert np.all(st == 1) and np.all(np.abs(it - ref["iterations"]) <= 2)
    _check_residuals(Bb, x)


def test_batch_column_outside_system_rejected(mxl, ctx):
    Bb = _batch_from([W.stencil_2d5(4), W.stencil_2d5(3)])
    Bb.col[Bb.row_ptr[17]] = 9  # a row of the second (9-row) system points at local column 9
    with pytest.raises(mxl.MxlError) as e:
        mxl.batch(ctx, Bb.sys_ptr, dev(Bb.sys_ptr), dev(Bb.row_ptr), dev(Bb.col), dev(Bb.val))
    assert e.value.status == mxl.ERR_INVALID_MATRIX


def test_batch_max_iters_and_zero_rhs(mxl, ctx):
    B = W.batch_systems(nsys=20, seed=5)
    B.b[B.sys_ptr[3]:B.sys_ptr[4]] = 0.0
    _, x, it, rel, st = _run(mxl, ctx, B, None, max_iters=3)
    assert st[3] == 1 and it[3] == 0 and not x[B.sys_ptr[3]:B.sys_ptr[4]].any()
    others = np.delete(np.arange(20), 3)
    assert np.all(it[others] == 3) and np.all(st[others] == 2)


def test_batch_autotune(mxl, ctx):
    B = W.batch_systems(nsys=400, seed=11)
    op = mxl.batch(ctx, B.sys_ptr, dev(B.sys_ptr), dev(B.row_ptr), dev(B.col), dev(B.val))
    b = dev(B.b)
    xs = torch.zeros_like(b)
    best, ms = op.autotune(b, xs, reps=1, reduction=1e-10)
    assert best[0] in (64, 128, 256, 512) and best[3] in (1, 2) and ms > 0
    x = torch.zeros_like(b)
    it = torch.zeros(B.nsys, dtype=torch.int32, device=DEV)
    rel = torch.zeros(B.nsys, dtype=torch.float64, device=DEV)
    st = torch.zeros(B.nsys, dtype=torch.uint8, device=DEV)
    op.solve(b, x, it, rel, st, reduction=1e-10)      # uses the tuned schedule
    assert np.all(st.cpu().numpy() == 1)
    _check_residuals(B, x.cpu().numpy())


def test_batch_full_size(mxl, ctx):
    """All 10,000 systems (seed 5000) against the oracle."""
    B = W.batch_systems()
    ref = O.batch_pcg(B, reduction=1e-10)
    _, x, it, rel, st = _run(mxl, ctx, B, None)
    assert np.all(st == 1)
    assert np.mean(np.abs(it - ref["iterations"]) <= 2) >= 0.99
    bad = 0
    for s in range(0, B.nsys, 7):
        r0, r1 = B.sys_ptr[s], B.sys_ptr[s + 1]
        r = B.b[r0:r1] - O.spmv(B.system(s), x[r0:r1])
        bad += np.linalg.norm(r) > 1.01e-10 * np.linalg.norm(B.b[r0:r1])
    assert bad == 0
