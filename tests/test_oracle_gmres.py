"""Pins of the oracle's restarted, right-preconditioned GMRES (Sec. 3.1,
Table 2) against what the mathematics fixes independently of its Arnoldi
process: after k steps of a cycle the iterate is the minimiser of
||b - A x|| over x0 + M^{-1} K_k(A M^{-1}, r0), computed here from an
explicit Krylov basis and numpy's least squares; restarts chain such
minimisations; GMRES(1) is the minimal-residual iteration; finite
termination in at most n steps and after as many steps as there are
distinct eigenvalues; an exact preconditioner converges in one step; on
SPD systems the residual never exceeds CG's; and the special cases (zero
right-hand side, non-finite data)."""
import numpy as np
import pytest

import oracle as O
import workloads as W


def _from_dense(D, name):
    rows, cols = np.nonzero(D)
    n = D.shape[0]
    rp = np.concatenate([[0], np.cumsum(np.bincount(rows, minlength=n))]).astype(np.int32)
    return W.Csr(n, n, rp, cols.astype(np.int32), D[rows, cols], name)


def _nonsym(n, seed, shift=3.0):
    rng = np.random.default_rng(seed)
    D = rng.standard_normal((n, n)) / np.sqrt(n)
    D[rng.random((n, n)) < 0.5] = 0.0
    D += np.diag(shift + rng.random(n))
    return D


def _krylov_min(D, Minv, b, x0, k):
    """argmin ||b - D x|| over x0 + Minv K_k(D Minv, r0), by an explicit
    (normalised power) basis, its QR and least squares."""
    r0 = b - D @ x0
    B = np.zeros((len(b), k))
    v = r0 / np.linalg.norm(r0)
    for i in range(k):
        B[:, i] = v
        v = D @ (Minv @ v)
        v /= np.linalg.norm(v)
    Q, _ = np.linalg.qr(B)
    c, *_ = np.linalg.lstsq(D @ (Minv @ Q), r0, rcond=None)
    return x0 + Minv @ (Q @ c)


@pytest.mark.parametrize("precond", [False, True], ids=["plain", "jacobi"])
@pytest.mark.parametrize("k", [1, 2, 3, 5, 8])
def test_iterate_minimises_over_krylov_space(k, precond):
    n = 40
    D = _nonsym(n, 7)
    A = _from_dense(D, "nonsym40")
    rng = np.random.default_rng(1)
    b, x0 = rng.uniform(-1, 1, n), rng.uniform(-1, 1, n)
    dinv = 1.0 / np.diag(D) if precond else None
    Minv = np.diag(dinv) if precond else np.eye(n)
    out = O.gmres(A, b, x0=x0, dinv=dinv, krylov_dim=10, max_iters=k, reduction=0.0)
    assert out["iterations"] == k and out["stop_reason"] == O.MAX_ITERS
    want = _krylov_min(D, Minv, b, x0, k)
    assert np.linalg.norm(out["x"] - want) <= 1e-10 * np.linalg.norm(want)
    true_rel = np.linalg.norm(b - D @ want) / np.linalg.norm(b)
    assert abs(out["rel_residual"] - true_rel) <= 1e-9 * true_rel + 1e-13  # b - D x in rounding


def test_restarts_chain_minimisations():
    n = 30
    D = _nonsym(n, 11, shift=2.0)
    A = _from_dense(D, "nonsym30")
    rng = np.random.default_rng(2)
    b = rng.uniform(-1, 1, n)
    dinv = 1.0 / np.diag(D)
    out = O.gmres(A, b, dinv=dinv, krylov_dim=3, max_iters=9, reduction=0.0)
    assert out["iterations"] == 9
    x = np.zeros(n)
    for _ in range(3):
        x = _krylov_min(D, np.diag(dinv), b, x, 3)
    assert np.linalg.norm(out["x"] - x) <= 1e-10 * np.linalg.norm(x)
    # 9 products in the cycles plus the initial residual and two restarts
    assert out["spmv_count"] == 12


def test_gmres1_is_minimal_residual_iteration():
    n = 25
    D = _nonsym(n, 5, shift=4.0)
    A = _from_dense(D, "nonsym25")
    b = np.random.default_rng(3).uniform(-1, 1, n)
    out = O.gmres(A, b, krylov_dim=1, max_iters=6, reduction=0.0)
    x = np.zeros(n)
    for _ in range(6):
        r = b - D @ x
        Ar = D @ r
        x = x + (r @ Ar) / (Ar @ Ar) * r
    assert np.linalg.norm(out["x"] - x) <= 1e-12 * np.linalg.norm(x)


def test_finite_termination_in_n_steps():
    n = 15
    D = _nonsym(n, 9, shift=1.0)
    A = _from_dense(D, "nonsym15")
    b = np.random.default_rng(4).uniform(-1, 1, n)
    out = O.gmres(A, b, krylov_dim=n, max_iters=n, reduction=1e-12)
    assert out["stop_reason"] == O.CONVERGED and out["iterations"] <= n
    assert np.linalg.norm(b - D @ out["x"]) <= 1e-11 * np.linalg.norm(b)


def test_distinct_eigenvalues_bound_the_steps():
    n = 30
    d = np.array([1.0, 2.0, 5.0])[np.arange(n) % 3]
    A = _from_dense(np.diag(d), "diag3")
    b = np.random.default_rng(5).uniform(-1, 1, n)
    two = O.gmres(A, b, krylov_dim=10, max_iters=2, reduction=0.0)
    assert two["rel_residual"] > 1e-3
    out = O.gmres(A, b, krylov_dim=10, max_iters=50, reduction=1e-13)
    assert out["iterations"] == 3 and out["stop_reason"] == O.CONVERGED
    assert np.abs(out["x"] - b / d).max() <= 1e-13 * np.abs(b / d).max()
    # Jacobi turns the diagonal system into the identity: one step
    one = O.gmres(A, b, dinv=1.0 / d, krylov_dim=10, reduction=1e-14)
    assert one["iterations"] == 1 and one["stop_reason"] == O.CONVERGED


def test_exact_block_preconditioner_converges_in_one_step():
    n = 24
    D = _nonsym(n, 13, shift=2.0)
    A = _from_dense(D, "nonsym24")
    b = np.random.default_rng(6).uniform(-1, 1, n)
    bp = O.uniform_blocks(n, 32)  # one block holding the whole matrix
    inv, _, _ = O.bj_generate(A, bp, adaptive=False)
    out = O.gmres(A, b, bptr=bp, inv=inv, krylov_dim=5, reduction=1e-12)
    assert out["iterations"] == 1 and out["stop_reason"] == O.CONVERGED
    assert np.linalg.norm(b - D @ out["x"]) <= 1e-12 * np.linalg.norm(b)


def test_residual_never_above_cg_on_spd():
    A = W.stencil_2d5(12)
    b = W.uniform_vec(A.nrows, 8)
    cg = O.pcg(A, b, max_iters=40, reduction=0.0, history=True)
    gm = O.gmres(A, b, krylov_dim=100, max_iters=40, reduction=0.0, history=True)
    assert np.all(gm["history"] <= cg["history"] * (1 + 1e-9))
    assert np.min(gm["history"][1:] / cg["history"][1:]) < 0.9  # a different iterate from CG's


def test_history_monotone_and_estimate_matches_true_residual():
    A = W.stencil_2d5(20)
    b = W.uniform_vec(A.nrows, 9)
    dinv, _ = O.jacobi_dinv(A)
    for m in (4, 30):
        out = O.gmres(A, b, dinv=dinv, krylov_dim=m, max_iters=5000, reduction=1e-10, history=True)
        assert out["stop_reason"] == O.CONVERGED
        h = out["history"]
        assert np.all(np.diff(h) <= 1e-14 * h[0])
        true_rel = np.linalg.norm(b - O.spmv(A, out["x"])) / np.linalg.norm(b)
        assert true_rel <= 1.01e-10
        assert abs(true_rel - out["rel_residual"]) <= 1e-3 * out["rel_residual"]


def test_zero_rhs_and_nonfinite():
    A = W.stencil_2d5(6)
    out = O.gmres(A, np.zeros(A.nrows), x0=np.ones(A.nrows))
    assert out["iterations"] == 0 and out["stop_reason"] == O.CONVERGED
    assert np.all(out["x"] == 0.0)
    one = _from_dense(np.array([[2.0]]), "one")
    nan = O.gmres(one, np.array([np.nan]), krylov_dim=10, max_iters=100)
    assert nan["stop_reason"] == O.NONFINITE
    # without the check the solver runs to the iteration limit (Table 1's protocol)
    run = O.gmres(one, np.array([np.nan]), krylov_dim=10, max_iters=100, nonfinite_check=0)
    assert run["stop_reason"] == O.MAX_ITERS and run["iterations"] == 100
