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


# ----------------------------------------- FP32 inner CG and IR with blocks
def _a_norm_min(D, Minv, b, k):
    """argmin ||x - D^{-1} b||_D over x in Minv K_k(D Minv, b) (x0 = 0), by an
    explicit normalised power basis and its D-orthogonal projection."""
    B = np.zeros((len(b), k))
    v = b / np.linalg.norm(b)
    for i in range(k):
        B[:, i] = Minv @ v
        v = D @ (Minv @ v)
        v /= np.linalg.norm(v)
    Q, _ = np.linalg.qr(B)
    c = np.linalg.solve(Q.T @ D @ Q, Q.T @ b)
    return Q @ c


@pytest.mark.parametrize("bs", [3, 8])
@pytest.mark.parametrize("k", [1, 2, 4])
def test_f32_block_cg_iterate_is_a_norm_minimiser(k, bs):
    """Preconditioned CG's k-th iterate minimises the energy-norm error over
    the preconditioned Krylov space; the FP32 vectors hold it to single
    precision (a wrong block offset or row of the inverse breaks it)."""
    A = W.aniso_3d7(5)
    D = _dense(A)
    bp = O.uniform_blocks(A.nrows, bs)
    inv, _, _ = O.bj_generate(A, bp, adaptive=False)
    M = np.zeros_like(D)
    off = 0
    for s in range(bp.size - 1):
        m = bp[s + 1] - bp[s]
        M[bp[s]:bp[s + 1], bp[s]:bp[s + 1]] = inv[off:off + m * m].reshape(m, m)
        off += m * m
    b = W.uniform_vec(A.nrows, 3).astype(np.float32)
    out = O.pcg_f32_block(A, b, bp, inv, max_iters=k, reduction=0.0)
    assert out["iterations"] == k and out["stop_reason"] == O.MAX_ITERS
    D32 = _dense(W.Csr(A.nrows, A.ncols, A.row_ptr, A.col, A.val.astype(np.float32).astype(np.float64), "a"))
    want = _a_norm_min(D32, M, b.astype(np.float64), k)
    assert np.linalg.norm(out["x"] - want) <= 2e-5 * np.linalg.norm(want)


def test_ir_block_whole_matrix_block_takes_one_inner_step():
    """One block holding the whole matrix is an exact preconditioner: every
    inner solve stops after one step and the outer loop contracts at the
    single-precision rate."""
    A = W.aniso_3d7(4)
    b = W.uniform_vec(A.nrows, 5)
    res = O.ir(A, b, outer_reduction=1e-13, inner_reduction=1e-4, block_size=A.nrows)
    assert res["stop_reason"] == O.CONVERGED
    assert res["inner_iterations"] == res["outer"] <= 4


def test_ir_block_true_residual_and_fewer_inner_steps():
    A = W.aniso_3d7(16)
    b = W.uniform_vec(A.nrows, 4)
    pt = O.ir(A, b, outer_reduction=1e-12, inner_reduction=1e-4)
    for acc in (1e-1, 1e-8):
        blk = O.ir(A, b, outer_reduction=1e-12, inner_reduction=1e-4, block_size=8, block_accuracy=acc)
        assert blk["stop_reason"] == O.CONVERGED
        r = b - O.spmv(A, blk["x"])
        assert np.linalg.norm(r) <= 1e-12 * np.linalg.norm(b)
        # the strong coupling runs along consecutive rows, which the blocks absorb
        assert blk["inner_iterations"] < 0.6 * pt["inner_iterations"]


# ------------------------------------------------- BiCGSTAB with blocks
def test_bicgstab_block_size_one_is_point_jacobi():
    A = W.convdiff_2d5(30)
    b = W.uniform_vec(A.nrows, 3)
    d, _ = O.jacobi_dinv(A)
    inv, _, _ = O.bj_generate(A, O.uniform_blocks(A.nrows, 1), adaptive=False)
    r0 = O.bicgstab(A, b, dinv=d, reduction=1e-10)
    r1 = O.bicgstab_block(A, b, O.uniform_blocks(A.nrows, 1), inv, reduction=1e-10)
    assert r0["iterations"] == r1["iterations"] and np.array_equal(r0["x"], r1["x"])


def test_bicgstab_single_block_is_exact():
    """One block holding the whole nonsymmetric matrix: p_hat = A^{-1} r, so
    v = r, alpha = 1, s = 0 up to rounding and the half step converges in
    the first iteration."""
    A = W.convdiff_2d5(6)
    b = W.uniform_vec(A.nrows, 4)
    bp = np.array([0, A.nrows], np.int32)
    inv, _, _ = O.bj_generate(A, bp, adaptive=False)
    r = O.bicgstab_block(A, b, bp, inv, reduction=1e-10)
    assert r["stop_reason"] == O.CONVERGED and r["iterations"] == 1 and r["spmv_count"] == 2


@pytest.mark.parametrize("bs", [4, 8, 32])
def test_bicgstab_block_true_residual(bs):
    A = W.convdiff_3d7(10)
    b = W.uniform_vec(A.nrows, 5)
    bp = O.uniform_blocks(A.nrows, bs)
    inv, _, _ = O.bj_generate(A, bp, adaptive=True)
    r = O.bicgstab_block(A, b, bp, inv, reduction=1e-10)
    assert r["stop_reason"] == O.CONVERGED
    res = b - O.spmv(A, r["x"])
    assert np.linalg.norm(res) <= 2e-10 * np.linalg.norm(b)
    d, _ = O.jacobi_dinv(A)
    assert r["iterations"] <= O.bicgstab(A, b, dinv=d, reduction=1e-10)["iterations"]


# ----------------------------------------------- variable-size blocks
def _grouped(sizes, seed, extra=0.15):
    """A symmetric sparse matrix whose rows come in consecutive groups of the
    given sizes, all rows of a group sharing one column set (a group couples
    densely to itself and to a few random other groups), plus a dominant
    diagonal."""
    rng = np.random.default_rng(seed)
    g = len(sizes)
    start = np.concatenate([[0], np.cumsum(sizes)])
    n = int(start[-1])
    G = rng.random((g, g)) < extra
    G = G | G.T | np.eye(g, dtype=bool)
    D = np.zeros((n, n))
    for a in range(g):
        for b in np.nonzero(G[a])[0]:
            D[start[a]:start[a + 1], start[b]:start[b + 1]] = 1.0
    V = rng.uniform(0.1, 1.0, (n, n))
    D = -(D * (V + V.T) / 2)
    np.fill_diagonal(D, 0.0)
    np.fill_diagonal(D, np.abs(D).sum(1) + 1.0)
    r, c = np.nonzero(np.abs(D) + np.eye(n))
    rp = np.concatenate([[0], np.cumsum(np.bincount(r, minlength=n))]).astype(np.int32)
    return W.Csr(n, n, rp, c.astype(np.int32), D[r, c], f"grouped{n}"), start


def _units(A, max_bs):
    """Supervariables found from whole-row pattern tuples (a different route
    than a scan of neighbouring rows), cut into pieces of max_bs rows."""
    pats = [tuple(A.col[A.row_ptr[i]:A.row_ptr[i + 1]]) for i in range(A.nrows)]
    bounds = [0] + [i for i in range(1, A.nrows) if pats[i] != pats[i - 1]] + [A.nrows]
    units = []
    for s, e in zip(bounds[:-1], bounds[1:]):
        units += [(p, min(e, p + max_bs)) for p in range(s, e, max_bs)]
    return units


def _check_greedy(A, bptr, max_bs):
    """The three properties that single out the greedy agglomeration: no
    block exceeds max_bs rows, no unit is split, and every block is maximal
    (the unit after it would not fit)."""
    sizes = np.diff(bptr)
    assert bptr[0] == 0 and bptr[-1] == A.nrows and np.all(sizes >= 1) and np.all(sizes <= max_bs)
    units = _units(A, max_bs)
    ustarts = {s: e - s for s, e in units}
    for t in range(1, bptr.size - 1):
        assert bptr[t] in ustarts, f"block boundary {bptr[t]} splits a unit"
        assert sizes[t - 1] + ustarts[bptr[t]] > max_bs, f"block {t - 1} is not maximal"


@pytest.mark.parametrize("max_bs", [1, 4, 13, 32])
def test_supervariable_blocks_on_a_stencil_are_uniform(max_bs):
    """Every row of a stencil matrix has its own column set, so the rule
    reduces to consecutive blocks of max_bs rows (the last one shorter)."""
    A = W.stencil_3d27(6)
    assert np.array_equal(O.supervariable_blocks(A, max_bs), O.uniform_blocks(A.nrows, max_bs))


def test_supervariable_blocks_follow_the_node_structure():
    """Groups of 1..6 rows with shared column sets: with max_bs = 6 every
    group is a block of its own unless the next group still fits; with
    max_bs = 1 the rule gives point Jacobi."""
    sizes = np.random.default_rng(3).integers(1, 7, 60)
    A, start = _grouped(list(sizes), 4)
    for mb in (6, 8, 32):
        bp = O.supervariable_blocks(A, mb)
        _check_greedy(A, bp, mb)
        assert set(bp.tolist()) <= set(start.tolist())     # node boundaries only
    assert np.array_equal(O.supervariable_blocks(A, 1), np.arange(A.nrows + 1))


@pytest.mark.parametrize("seed", [5, 6, 7])
def test_supervariable_blocks_long_groups_are_cut(seed):
    """Groups up to 70 rows with max_bs = 16 and 32: long groups are cut into
    max_bs pieces, and the greedy properties hold."""
    sizes = np.random.default_rng(seed).integers(1, 71, 12)
    A, _ = _grouped(list(sizes), seed)
    for mb in (16, 32):
        bp = O.supervariable_blocks(A, mb)
        _check_greedy(A, bp, mb)


def test_supervariable_blocks_node_block_workload():
    A = W.node_block_3d7(6, kmax=6, seed=7)
    for mb in (8, 32):
        _check_greedy(A, O.supervariable_blocks(A, mb), mb)


def test_supervariable_blocks_empty_and_one_row():
    E = W.Csr(0, 0, np.zeros(1, np.int32), np.zeros(0, np.int32), np.zeros(0))
    assert list(O.supervariable_blocks(E, 8)) == [0]
    one = W.Csr(1, 1, np.array([0, 1], np.int32), np.zeros(1, np.int32), np.ones(1))
    assert list(O.supervariable_blocks(one, 8)) == [0, 1]


def test_variable_blocks_inverses_and_product():
    """Mixed block sizes: every inverse against numpy.linalg.inv of its
    diagonal block, cond_1 against numpy, and the product against the dense
    block-diagonal matrix."""
    A, _ = _grouped([3, 1, 5, 2, 6, 4, 1, 1, 6], 8)
    Dn = _dense(A)
    bp = O.supervariable_blocks(A, 8)
    assert len(set(np.diff(bp))) > 2
    inv, cond, prec = O.bj_generate(A, bp, adaptive=False)
    M = np.zeros_like(Dn)
    off = 0
    for b in range(bp.size - 1):
        r0, m = bp[b], bp[b + 1] - bp[b]
        D = Dn[r0:r0 + m, r0:r0 + m]
        Inv = inv[off:off + m * m].reshape(m, m)
        assert np.allclose(Inv, np.linalg.inv(D), rtol=1e-12, atol=1e-14)
        assert np.isclose(cond[b], np.linalg.cond(D, 1), rtol=1e-10)
        M[r0:r0 + m, r0:r0 + m] = Inv
        off += m * m
    r = W.uniform_vec(A.nrows, 9)
    assert np.allclose(O.bj_apply(bp, inv, r), M @ r, rtol=1e-14, atol=1e-15)


def test_variable_blocks_reduce_to_uniform_and_exact_cases():
    """Variable boundaries that happen to be uniform give the uniform
    preconditioner's solve bit for bit; one block over the whole matrix is
    exact (one CG step)."""
    A = W.node_block_3d7(4, kmax=3, seed=2)
    b = W.uniform_vec(A.nrows, 3)
    bp = O.supervariable_blocks(W.stencil_3d27(6), 5)[: (A.nrows + 4) // 5 + 1].copy()
    bp[-1] = A.nrows
    ub = O.uniform_blocks(A.nrows, 5)
    assert np.array_equal(bp, ub)
    i1, _, _ = O.bj_generate(A, bp)
    i2, _, _ = O.bj_generate(A, ub)
    r1 = O.pcg_block(A, b, bp, i1, reduction=1e-10)
    r2 = O.pcg_block(A, b, ub, i2, reduction=1e-10)
    assert r1["iterations"] == r2["iterations"] and np.array_equal(r1["x"], r2["x"])
    whole = np.array([0, A.nrows], np.int32)
    iw, _, _ = O.bj_generate(A, whole, adaptive=False)
    assert O.pcg_block(A, b, whole, iw, reduction=1e-10)["iterations"] == 1


def test_node_respecting_blocks_beat_uniform_blocks():
    """On the node-block workload, blocks that keep every node whole need
    fewer CG iterations than uniform blocks of the same maximum size."""
    A = W.node_block_3d7(8, kmax=6, seed=7)
    b = W.uniform_vec(A.nrows, 3)
    its = {}
    for name, bp in (("uniform", O.uniform_blocks(A.nrows, 32)), ("super", O.supervariable_blocks(A, 32))):
        inv, _, _ = O.bj_generate(A, bp)
        r = O.pcg_block(A, b, bp, inv, reduction=1e-10)
        assert r["stop_reason"] == O.CONVERGED
        assert np.linalg.norm(b - O.spmv(A, r["x"])) <= 1.01e-10 * np.linalg.norm(b)
        its[name] = r["iterations"]
    assert its["super"] < its["uniform"]


def test_ir_with_given_blocks_reduces_to_uniform():
    """Refinement with given block boundaries equal to uniform blocks is the
    uniform-block refinement bit for bit; with supervariable blocks on the
    node-block workload it reaches 1e-12 in the recomputed FP64 residual."""
    A = W.aniso_3d7(10)
    b = W.uniform_vec(A.nrows, 4)
    r1 = O.ir(A, b, outer_reduction=1e-12, block_size=8)
    r2 = O.ir(A, b, outer_reduction=1e-12, bptr=O.uniform_blocks(A.nrows, 8))
    assert r1["outer"] == r2["outer"] and r1["inner_iterations"] == r2["inner_iterations"]
    assert np.array_equal(r1["x"], r2["x"])
    B = W.node_block_3d7(6, kmax=6, seed=7)
    bb = W.uniform_vec(B.nrows, 5)
    r = O.ir(B, bb, outer_reduction=1e-12, bptr=O.supervariable_blocks(B, 32))
    assert r["stop_reason"] == O.CONVERGED
    assert np.linalg.norm(bb - O.spmv(B, r["x"])) <= 1e-12 * np.linalg.norm(bb)
