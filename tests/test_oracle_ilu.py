"""Pins of the oracle's incomplete LU (the ILU-type preconditioners of
Sec. 3.2: ILU(0), its ParILU fixed-point generation, the two triangular
solves) against what the definitions fix independently of the code:
(L U)_ij = a_ij on A's pattern checked with dense products; complete LU
(L U = A) wherever the pattern admits no fill; U = D L^T for symmetric A;
ParILU's fixed point is ILU(0) and is reached after finitely many
synchronous sweeps; triangular solves against numpy's dense solves; Jacobi
sweeps on a triangular system become exact after as many sweeps as the
system's dependency depth; GMRES with an exact factorization converges in
one step."""
import numpy as np
import pytest

import oracle as O
import workloads as W


def _dense(A):
    D = np.zeros((A.nrows, A.ncols))
    rows = np.repeat(np.arange(A.nrows), A.row_lengths())
    D[rows, A.col] = A.val
    return D


def _from_dense(D, name):
    rows, cols = np.nonzero(D)
    n = D.shape[0]
    rp = np.concatenate([[0], np.cumsum(np.bincount(rows, minlength=n))]).astype(np.int32)
    return W.Csr(n, n, rp, cols.astype(np.int32), D[rows, cols], name)


def _factors(A, lu):
    """Dense unit-lower L and upper U from factors on A's pattern."""
    n = A.nrows
    rows = np.repeat(np.arange(n), A.row_lengths())
    L, U = np.eye(n), np.zeros((n, n))
    low = A.col < rows
    L[rows[low], A.col[low]] = lu[low]
    U[rows[~low], A.col[~low]] = lu[~low]
    return L, U


def _nonsym(n, seed, density=0.15):
    rng = np.random.default_rng(seed)
    D = rng.standard_normal((n, n)) * (rng.random((n, n)) < density)
    D += np.diag(np.abs(D).sum(axis=1) + 1.0)
    return _from_dense(D, f"nonsym{n}")


MATS = [W.stencil_2d5(9), W.convdiff_2d5(8), W.convdiff_3d7(5), _nonsym(60, 1), W.stencil_3d27(4)]


@pytest.mark.parametrize("A", MATS, ids=[a.name for a in MATS])
def test_ilu0_matches_a_on_its_pattern(A):
    lu, bad = O.ilu0(A)
    assert bad == -1
    L, U = _factors(A, lu)
    P = L @ U
    rows = np.repeat(np.arange(A.nrows), A.row_lengths())
    scale = np.abs(A.val).max()
    assert np.abs(P[rows, A.col] - A.val).max() <= 1e-13 * scale
    # a pattern that does admit fill leaves L U != A off the pattern
    off = np.ones_like(P, bool)
    off[rows, A.col] = False
    if A.name.startswith("stencil2d5"):
        assert np.abs(P[off]).max() > 1e-3


@pytest.mark.parametrize("kind", ["tridiag", "lower", "arrow_last"])
def test_no_fill_pattern_gives_complete_lu(kind):
    n = 40
    rng = np.random.default_rng(3)
    if kind == "tridiag":
        D = np.diag(4.0 + rng.random(n)) + np.diag(rng.standard_normal(n - 1), 1) + np.diag(rng.standard_normal(n - 1), -1)
    elif kind == "lower":
        D = np.tril(rng.standard_normal((n, n)) * (rng.random((n, n)) < 0.2), -1) + np.diag(2.0 + rng.random(n))
    else:  # dense last row and column: the elimination creates no new entries
        D = np.diag(5.0 + rng.random(n))
        D[-1, :] += rng.standard_normal(n) * 0.1
        D[:, -1] += rng.standard_normal(n) * 0.1
    A = _from_dense(D, kind)
    lu, bad = O.ilu0(A)
    assert bad == -1
    L, U = _factors(A, lu)
    assert np.abs(L @ U - D).max() <= 1e-13 * np.abs(D).max()


def test_symmetric_matrix_gives_u_equal_d_lt():
    A = W.stencil_3d27(4)
    lu, _ = O.ilu0(A)
    L, U = _factors(A, lu)
    Dg = np.diag(np.diag(U))
    assert np.abs(U - Dg @ L.T).max() <= 1e-13 * np.abs(U).max()


def test_missing_or_zero_pivot_reported():
    D = np.array([[0.0, 1.0], [1.0, 2.0]])
    assert O.ilu0(_from_dense(D, "zero_pivot"))[1] == 0
    assert O.parilu(_from_dense(D, "zero_pivot"), 3)[1] == 0
    D = np.array([[2.0, 1.0, 0.0], [1.0, 0.5, 1.0], [0.0, 1.0, 2.0]])
    assert O.ilu0(_from_dense(D, "zero_u11"))[1] == 1  # u_11 = 0.5 - 0.5 * 1 = 0


@pytest.mark.parametrize("A", MATS, ids=[a.name for a in MATS])
def test_parilu_initial_guess_and_fixed_point(A):
    n = A.nrows
    rows = np.repeat(np.arange(n), A.row_lengths())
    diag = _dense(A).diagonal()
    p0, _ = O.parilu(A, 0)
    want0 = np.where(A.col < rows, A.val / diag[A.col], A.val)
    assert np.array_equal(p0, want0)
    lu, _ = O.ilu0(A)
    errs = [np.abs(O.parilu(A, s)[0] - lu).max() for s in (1, 3, 10)]
    assert errs[0] > errs[1] > errs[2]
    # the synchronous sweep map reaches its fixed point after finitely many sweeps
    full, _ = O.parilu(A, n)
    assert np.abs(full - lu).max() <= 1e-13 * np.abs(lu).max()
    again, _ = O.parilu(A, n + 1)
    assert np.abs(again - full).max() <= 1e-15 * np.abs(lu).max()


@pytest.mark.parametrize("A", MATS, ids=[a.name for a in MATS])
def test_triangular_solves(A):
    lu, _ = O.ilu0(A)
    L, U = _factors(A, lu)
    r = W.uniform_vec(A.nrows, 4)
    want = np.linalg.solve(U, np.linalg.solve(L, r))
    z = O.ilu_apply(A, lu, r, mode=0)
    assert np.abs(z - want).max() <= 1e-12 * np.abs(want).max()
    # Jacobi sweeps: zero sweeps = diagonal scaling, enough sweeps = exact
    z0 = O.ilu_apply(A, lu, r, mode=1, sweeps=0)
    assert np.allclose(z0, r / np.diag(U), rtol=0, atol=1e-15 * np.abs(r / np.diag(U)).max())
    zn = O.ilu_apply(A, lu, r, mode=1, sweeps=A.nrows)
    assert np.abs(zn - want).max() <= 1e-12 * np.abs(want).max()
    # one sweep each: y1 = r - (L - I) r,  z1 = D^-1 (y1 - (U - D) D^-1 y1)
    Dg = np.diag(np.diag(U))
    y1 = r - (L - np.eye(A.nrows)) @ r
    z1 = np.linalg.solve(Dg, y1 - (U - Dg) @ np.linalg.solve(Dg, y1))
    assert np.abs(O.ilu_apply(A, lu, r, mode=1, sweeps=1) - z1).max() <= 1e-13 * np.abs(z1).max()


def test_gmres_with_exact_factorization_converges_in_one_step():
    n = 50
    rng = np.random.default_rng(8)
    D = np.diag(4.0 + rng.random(n)) + np.diag(rng.standard_normal(n - 1), 1) + np.diag(rng.standard_normal(n - 1), -1)
    A = _from_dense(D, "tridiag50")
    lu, _ = O.ilu0(A)
    b = rng.uniform(-1, 1, n)
    out = O.gmres_ilu(A, b, lu, krylov_dim=10, reduction=1e-12)
    assert out["iterations"] == 1 and out["stop_reason"] == O.CONVERGED


def test_ilu_preconditioning_beats_jacobi():
    A = W.convdiff_2d5(30)
    b = W.uniform_vec(A.nrows, 2)
    lu, _ = O.ilu0(A)
    ilu = O.gmres_ilu(A, b, lu, krylov_dim=50, reduction=1e-10)
    jac = O.gmres(A, b, dinv=O.jacobi_dinv(A)[0], krylov_dim=50, reduction=1e-10)
    assert ilu["stop_reason"] == O.CONVERGED
    assert ilu["iterations"] < 0.7 * jac["iterations"]
    assert np.linalg.norm(b - O.spmv(A, ilu["x"])) <= 1.01e-10 * np.linalg.norm(b)
