"""Pins of the oracle's block-Jacobi (Sec. 3.2) against what mathematics and
independent libraries fix: binary16 rounding against numpy's float16,
inverses against numpy.linalg.inv and the identity, condition numbers
against numpy.linalg.cond, the precision rule on blocks with known
condition numbers and exponent ranges, block size 1 = point Jacobi, and a
single block holding the whole matrix = an exact preconditioner."""
import numpy as np
import pytest

import oracle as O
import workloads as W


def test_round_f16_matches_numpy():
    rng = np.random.default_rng(0)
    xs = np.concatenate([rng.standard_normal(4000) * 10.0 ** rng.integers(-9, 6, 4000),
                         [0.0, -0.0, 65504.0, 65519.99, 65520.0, -70000.0, 2.0 ** -24, 2.0 ** -25,
                          3 * 2.0 ** -26, 2.0 ** -14, 1.0 + 2.0 ** -11, 1.0 + 3 * 2.0 ** -11,
                          np.inf, -np.inf]])
    got = np.array([O.round_f16(x) for x in xs])
    with np.errstate(over="ignore"):
        want = xs.astype(np.float16).astype(np.float64)
    assert np.array_equal(got, want, equal_nan=True)


def _dense(A):
    D = np.zeros((A.nrows, A.ncols))
    rows = np.repeat(np.arange(A.nrows), A.row_lengths())
    D[rows, A.col] = A.val
    return D


@pytest.mark.parametrize("bs", [1, 3, 8, 32])
def test_inverses_and_condition(bs):
    A = W.random_sparse(100, 100, 0.08, 3)
    # make it block-diagonally dominant so every block is invertible
    Dn = _dense(A) + np.eye(100) * 5.0
    rows, cols = np.nonzero(Dn)
    rp = np.concatenate([[0], np.cumsum(np.bincount(rows, minlength=100))]).astype(np.int32)
    A = W.Csr(100, 100, rp, cols.astype(np.int32), Dn[rows, cols], "dd100")
    bp = O.uniform_blocks(100, bs)
    inv, cond, prec = O.bj_generate(A, bp, adaptive=False)
    off = 0
    for b in range(bp.size - 1):
        r0, m = bp[b], bp[b + 1] - bp[b]
        D = Dn[r0:r0 + m, r0:r0 + m]
        Inv = inv[off:off + m * m].reshape(m, m)
        assert np.allclose(Inv, np.linalg.inv(D), rtol=1e-12, atol=1e-14)
        assert np.allclose(D @ Inv, np.eye(m), atol=1e-12)
        assert np.isclose(cond[b], np.linalg.cond(D, 1), rtol=1e-10)
        assert prec[b] == O.P64
        off += m * m


def test_exact_integer_inverse():
    """A unimodular integer block has an integer inverse that Gauss-Jordan
    reproduces exactly (every intermediate is a small integer or an exact
    binary fraction)."""
    D = np.array([[2.0, 1.0], [1.0, 1.0]])  # det 1, inverse [[1,-1],[-1,2]]
    A = W.Csr(2, 2, np.array([0, 2, 4], np.int32), np.array([0, 1, 0, 1], np.int32), D.ravel(), "unimod")
    inv, cond, prec = O.bj_generate(A, np.array([0, 2], np.int32), adaptive=False)
    assert np.array_equal(inv.reshape(2, 2), np.array([[1.0, -1.0], [-1.0, 2.0]]))
    assert cond[0] == 3.0 * 3.0


@pytest.mark.parametrize("d,lo_entry,want", [
    ((1.0, 2.0), None, O.P16),          # cond 2: 2 * 2^-11 <= 0.1
    ((1.0, 1e3), None, O.P32),          # cond 1e3 too large for binary16, fine for binary32
    ((1.0, 1e7), None, O.P64),          # cond 1e7: 1e7 * 2^-24 = 0.6 > 0.1
    ((1.0, 1e20), None, O.P64),
    ((1.0, 1.0), 1e6, O.P32),           # inverse entry 1e-6 below binary16's normal range
])
def test_precision_rule(d, lo_entry, want):
    D = np.diag(np.array(d, float))
    if lo_entry is not None:
        D = np.array([[1.0, 0.0], [0.0, lo_entry]])
    inv = np.linalg.inv(D)
    c = np.linalg.cond(D, 1)
    assert O.bj_choose_precision(inv, c, 0.1) == want, (d, c)


def test_adaptive_storage_is_rounded():
    A = W.aniso_3d7(6)
    bp = O.uniform_blocks(A.nrows, 6)
    inv64, cond, _ = O.bj_generate(A, bp, adaptive=False)
    inv, cond2, prec = O.bj_generate(A, bp, adaptive=True)
    assert np.array_equal(cond, cond2)
    off = 0
    for b in range(bp.size - 1):
        m = bp[b + 1] - bp[b]
        blk, ref = inv[off:off + m * m], inv64[off:off + m * m]
        if prec[b] == O.P16:
            assert np.array_equal(blk, ref.astype(np.float16).astype(np.float64))
        elif prec[b] == O.P32:
            assert np.array_equal(blk, ref.astype(np.float32).astype(np.float64))
        else:
            assert np.array_equal(blk, ref)
        off += m * m


def test_apply_is_block_diagonal_product():
    A = W.stencil_3d27(5)
    bp = O.uniform_blocks(A.nrows, 4)
    inv, _, _ = O.bj_generate(A, bp)
    M = np.zeros((A.nrows, A.nrows))
    off = 0
    for b in range(bp.size - 1):
        r0, m = bp[b], bp[b + 1] - bp[b]
        M[r0:r0 + m, r0:r0 + m] = inv[off:off + m * m].reshape(m, m)
        off += m * m
    r = W.uniform_vec(A.nrows, 7)
    assert np.allclose(O.bj_apply(bp, inv, r), M @ r, rtol=1e-14, atol=1e-15)


def test_block_size_one_is_point_jacobi():
    A = W.stencil_2d5(20)
    b = O.spmv(A, W.uniform_vec(A.nrows, 1))
    d, _ = O.jacobi_dinv(A)
    inv, _, _ = O.bj_generate(A, O.uniform_blocks(A.nrows, 1), adaptive=False)
    assert np.array_equal(inv, d)
    r0 = O.pcg(A, b, dinv=d, reduction=1e-10)
    r1 = O.pcg_block(A, b, O.uniform_blocks(A.nrows, 1), inv, reduction=1e-10)
    assert r0["iterations"] == r1["iterations"] and np.array_equal(r0["x"], r1["x"])


def test_single_block_is_exact():
    """With one block holding the whole SPD matrix, M = A^{-1} and CG stops
    after one iteration."""
    A = W.stencil_2d5(5)
    b = O.spmv(A, W.uniform_vec(A.nrows, 2))
    bp = np.array([0, A.nrows], np.int32)
    inv, _, _ = O.bj_generate(A, bp, adaptive=False)
    r = O.pcg_block(A, b, bp, inv, reduction=1e-10)
    assert r["iterations"] == 1 and r["stop_reason"] == O.CONVERGED


def test_singular_block_is_reported():
    A = W.Csr(2, 2, np.array([0, 1, 2], np.int32), np.array([1, 0], np.int32), np.array([1.0, 1.0]), "offdiag")
    with pytest.raises(ValueError):
        O.bj_generate(A, np.array([0, 1, 2], np.int32))
    inv, _, _ = O.bj_generate(A, np.array([0, 2], np.int32), adaptive=False)  # [[0,1],[1,0]] is its own inverse
    assert np.array_equal(inv.reshape(2, 2), np.array([[0.0, 1.0], [1.0, 0.0]]))
