"""Pins of the CPU oracle to facts fixed outside it (no GPU needed).

Each test checks the oracle against something it does not compute itself:
closed-form eigenpairs of the stencil operators, exact rational arithmetic,
integer-exact products, CG's finite termination, textbook convergence bounds,
independent brute-force constructions and finite differences.  A plausible
slip in the oracle (dropped term, wrong sign or index, transposed operand)
fails at least one of them.
"""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle as O
from oracle import exact as E
import workloads as W

U64 = 2.0 ** -53
GOLD = os.path.join(os.path.dirname(__file__), "golden")


def gamma(k, u=U64):
    return k * u / (1 - k * u)


@pytest.fixture(scope="module", autouse=True)
def _built(oracle_lib):
    return oracle_lib


# ------------------------------------------------------------------ CSR
def test_csr_check_accepts_generators():
    for A in [W.stencil_2d5(9), W.stencil_3d27(5), W.aniso_3d7(6), W.convdiff_2d5(7),
              W.random_sparse(30, 20, 0.2, 3)] + W.edge_matrices():
        assert O.csr_check(A) == 0, A.name


def test_csr_check_rejects_each_violation():
    A = W.random_sparse(12, 10, 0.4, 5)
    def bad(**kw):
        B = W.Csr(A.nrows, A.ncols, A.row_ptr.copy(), A.col.copy(), A.val.copy())
        for k, v in kw.items():
            setattr(B, k, v)
        return B
    rp = A.row_ptr.copy(); rp[0] = 1
    assert O.csr_check(bad(row_ptr=rp)) == 1
    rp = A.row_ptr.copy(); rp[4] = rp[3] - 1
    assert rp[3] >= 1 and O.csr_check(bad(row_ptr=rp)) == 2
    rp = A.row_ptr.copy(); rp[-1] += 1
    assert O.csr_check(bad(row_ptr=rp)) in (3,)
    col = A.col.copy(); col[2] = A.ncols
    assert O.csr_check(bad(col=col)) == 4
    col = A.col.copy()
    r = next(i for i in range(A.nrows) if A.row_ptr[i + 1] - A.row_ptr[i] >= 2)
    k = A.row_ptr[r]
    col[k], col[k + 1] = col[k + 1], col[k]
    assert O.csr_check(bad(col=col)) == 5
    col = A.col.copy(); col[k + 1] = col[k]
    assert O.csr_check(bad(col=col)) == 5


# ----------------------------------------------------------------- SpMV
@pytest.mark.parametrize("seed", [1, 2, 3])
def test_spmv_exact_rational_bound(seed):
    """FP64 result within the rigorous sequential-summation error bound of the
    exact rational product (alpha, beta general)."""
    A = W.random_sparse(45, 37, 0.25, seed, empty_row_frac=0.1)
    rng = np.random.default_rng(seed)
    x = rng.standard_normal(A.ncols)
    y0 = rng.standard_normal(A.nrows)
    for alpha, beta in [(1.0, 0.0), (-0.75, 1.0), (2.5, -0.3)]:
        y = O.spmv(A, x, alpha, beta, y0)
        D = E.frac_mat(A.dense())
        ye = E.matvec(D, E.frac_vec(x))
        a, b_ = Fraction(alpha), Fraction(beta)
        absb = np.abs(A.dense()) @ np.abs(x)
        lens = A.row_lengths()
        for i in range(A.nrows):
            exact = a * ye[i] + b_ * Fraction(float(y0[i]))
            bound = gamma(int(lens[i]) + 2) * (abs(alpha) * absb[i] + abs(beta) * abs(y0[i]))
            assert abs(Fraction(float(y[i])) - exact) <= Fraction(bound) + Fraction(0), (i, alpha, beta)


def test_spmv_beta_zero_ignores_nan_y():
    A = W.random_sparse(20, 20, 0.3, 9)
    x = np.ones(20)
    y = O.spmv(A, x, 1.0, 0.0, np.full(20, np.nan))
    assert np.all(np.isfinite(y))


@pytest.mark.parametrize("seed", [4, 5])
def test_spmv_integer_exact(seed):
    """Integer A and x with partial sums < 2^53: every correct summation order
    gives the exact integer, so the oracle must equal integer arithmetic bitwise."""
    A = W.random_sparse(300, 250, 0.05, seed, integer=True, int_range=1000)
    rng = np.random.default_rng(seed)
    xi = rng.integers(-10_000, 10_001, A.ncols)
    Di = np.rint(A.dense()).astype(np.int64)
    exact = Di @ xi
    y = O.spmv(A, xi.astype(np.float64))
    assert np.array_equal(y, exact.astype(np.float64))


def _sin_mode(N, ps):
    g = np.arange(1, N + 1)
    vs = [np.sin(p * math.pi * g / (N + 1)) for p in ps]
    v = vs[0]
    for w in vs[1:]:
        v = np.multiply.outer(w, v)   # later dimensions vary slowest
    return v.ravel()


def _check_eigenpair(A, v, lam):
    Av = O.spmv(A, v)
    absA = np.abs(A.val)
    rows = np.repeat(np.arange(A.nrows), A.row_lengths())
    scale = np.bincount(rows, weights=absA * np.abs(v[A.col]), minlength=A.nrows)
    err = np.abs(Av - lam * v)
    assert np.all(err <= 1e-12 * (scale + abs(lam) * np.abs(v)) + 1e-300)


@pytest.mark.parametrize("p,q", [(1, 1), (3, 7), (64, 1), (40, 33)])
def test_stencil_2d5_eigenpairs(p, q):
    N = 64
    A = W.stencil_2d5(N)
    lam = 4 - 2 * math.cos(p * math.pi / (N + 1)) - 2 * math.cos(q * math.pi / (N + 1))
    _check_eigenpair(A, _sin_mode(N, [p, q]), lam)


@pytest.mark.parametrize("ps", [(1, 1, 1), (2, 5, 9), (17, 3, 11)])
def test_stencil_3d27_eigenpairs(ps):
    N = 17
    A = W.stencil_3d27(N)
    lam = 27 - np.prod([1 + 2 * math.cos(p * math.pi / (N + 1)) for p in ps])
    _check_eigenpair(A, _sin_mode(N, ps), lam)


@pytest.mark.parametrize("ps", [(1, 1, 1), (4, 2, 9)])
def test_aniso_3d7_eigenpairs(ps):
    N, a, s = 14, (1.0, 1e-2, 1e-4), 1e-3
    A = W.aniso_3d7(N, a, s)
    lam = sum(ad * (2 - 2 * math.cos(p * math.pi / (N + 1))) for ad, p in zip(a, ps)) + s
    _check_eigenpair(A, _sin_mode(N, ps), lam)


def test_stencil_3d27_row_sums_exact():
    N = 11
    A = W.stencil_3d27(N)
    y = O.spmv(A, np.ones(A.nrows))
    idx = np.arange(A.nrows)
    c = [np.where((t == 0) | (t == N - 1), 2, 3) for t in (idx % N, (idx // N) % N, idx // N ** 2)]
    assert np.array_equal(y, (27 - c[0] * c[1] * c[2]).astype(np.float64))


def test_stencil_nnz_formulas():
    assert W.stencil_2d5(64).nnz == 5 * 64 ** 2 - 4 * 64
    assert W.stencil_3d27(20).nnz == (3 * 20 - 2) ** 3
    assert W.aniso_3d7(16).nnz == 7 * 16 ** 3 - 6 * 16 ** 2


# ------------------------------------------------------ COO / ELL / HYB
def _brute_ell(A, w, n_pad):
    ec = -np.ones((w, n_pad), np.int32)
    ev = np.zeros((w, n_pad))
    for i in range(A.nrows):
        for s, k in enumerate(range(A.row_ptr[i], A.row_ptr[i + 1])):
            ec[s, i] = A.col[k]
            ev[s, i] = A.val[k]
    return ec.ravel(), ev.ravel()


@pytest.mark.parametrize("A", W.edge_matrices()[:3] + [W.random_sparse(70, 50, 0.1, 8)],
                         ids=lambda a: a.name)
def test_formats_brute_force(A):
    x = np.random.default_rng(0).standard_normal(A.ncols)
    y0 = O.spmv(A, x)
    # COO: explicit row of each entry
    row = O.csr_to_coo(A)
    assert np.array_equal(row, np.repeat(np.arange(A.nrows), A.row_lengths()).astype(np.int32))
    assert np.array_equal(O.coo_spmv(A.nrows, row, A.col, A.val, x), y0)
    # ELL: slot-major layout, sentinel -1 padding
    w, n_pad, ec, ev = O.csr_to_ell(A)
    assert w == (A.row_lengths().max() if A.nrows else 0)
    assert n_pad % 64 == 0 and n_pad >= A.nrows
    bc, bv = _brute_ell(A, w, n_pad)
    assert np.array_equal(ec, bc) and np.array_equal(ev, bv)
    assert np.array_equal(O.ell_spmv(A.nrows, n_pad, w, ec, ev, x), y0)
    # HYB: quantile width; tail = entries beyond k in CSR order
    for q in (0.5, 0.66, 0.9):
        lens = np.sort(A.row_lengths())
        k_exp = int(lens[max(1, math.ceil(q * A.nrows)) - 1]) if A.nrows else 0
        H = O.csr_to_hyb(A, q=q)
        assert H["k"] == k_exp
        tr, tc, tv = [], [], []
        for i in range(A.nrows):
            for s, kk in enumerate(range(A.row_ptr[i], A.row_ptr[i + 1])):
                if s >= k_exp:
                    tr.append(i); tc.append(A.col[kk]); tv.append(A.val[kk])
        assert np.array_equal(H["tail_row"], np.array(tr, np.int32))
        assert np.array_equal(H["tail_col"], np.array(tc, np.int32))
        assert np.array_equal(H["tail_val"], np.array(tv))
        bc, bv = _brute_ell(W.Csr(A.nrows, A.ncols,
                                  np.concatenate([[0], np.cumsum(np.minimum(A.row_lengths(), k_exp))]).astype(np.int32),
                                  np.concatenate([A.col[A.row_ptr[i]:A.row_ptr[i] + min(k_exp, A.row_ptr[i+1]-A.row_ptr[i])] for i in range(A.nrows)] + [np.zeros(0, np.int32)]),
                                  np.concatenate([A.val[A.row_ptr[i]:A.row_ptr[i] + min(k_exp, A.row_ptr[i+1]-A.row_ptr[i])] for i in range(A.nrows)] + [np.zeros(0)])),
                            k_exp, H["n_pad"])
        assert np.array_equal(H["ell_col"], bc) and np.array_equal(H["ell_val"], bv)
        yh = O.hyb_spmv(A.nrows, H, x)
        assert np.allclose(yh, y0, rtol=1e-13, atol=1e-13 * np.abs(x).max() * (np.abs(A.val).max() if A.nnz else 1))


def test_ell_nan_propagation():
    A = W.random_sparse(50, 40, 0.1, 12)
    A.val[3] = 0.0   # an explicit zero still sees the NaN
    x = np.ones(40)
    j = int(A.col[3])
    x[j] = np.nan
    w, n_pad, ec, ev = O.csr_to_ell(A)
    y = O.ell_spmv(A.nrows, n_pad, w, ec, ev, x)
    stores_j = np.array([j in A.col[A.row_ptr[i]:A.row_ptr[i + 1]] for i in range(A.nrows)])
    assert np.array_equal(np.isnan(y), stores_j)


# --------------------------------------------------------------- Jacobi
def test_jacobi_dinv_and_zero_diag():
    A = W.random_sparse(25, 25, 0.3, 4)
    D = A.dense()
    d, bad = O.jacobi_dinv(A)
    diag = np.diag(D)
    first_bad = next((i for i in range(25) if diag[i] == 0), -1)
    assert bad == first_bad
    B = W.aniso_3d7(5)
    d, bad = O.jacobi_dinv(B)
    assert bad == -1 and np.array_equal(d, 1.0 / np.diag(B.dense()))


# ------------------------------------------------------------------- CG
def _dense_csr(D):
    D = np.asarray(D, dtype=np.float64)
    r, c = np.nonzero(D)
    rp = np.concatenate([[0], np.cumsum(np.bincount(r, minlength=D.shape[0]))]).astype(np.int32)
    return W.Csr(D.shape[0], D.shape[1], rp, c.astype(np.int32), D[r, c])


@pytest.mark.parametrize("n,seed", [(3, 1), (5, 2), (7, 3), (8, 4)])
def test_cg_exact_termination(n, seed):
    """Exact-rational CG reaches r = 0 in <= n steps and equals Gaussian
    elimination; the FP64 oracle agrees with that exact solution."""
    Ai = W.spd_integer_small(n, seed)
    b = np.random.default_rng(seed).integers(-5, 6, n).astype(float)
    if not b.any():
        b[0] = 1
    Af = [[Fraction(int(v)) for v in row] for row in Ai]
    bf = [Fraction(int(v)) for v in b]
    xs = E.solve(Af, bf)
    xe, k, r = E.cg(Af, bf)
    assert k <= n and all(t == 0 for t in r) and xe == xs
    dinv = [Fraction(1, int(Ai[i, i])) for i in range(n)]
    xj, kj, rj = E.cg(Af, bf, dinv)
    assert kj <= n and all(t == 0 for t in rj) and xj == xs
    A = _dense_csr(Ai)
    d, _ = O.jacobi_dinv(A)
    res = O.pcg(A, b, dinv=d, reduction=1e-13, max_iters=10 * n)
    assert res["stop_reason"] == O.CONVERGED
    xsf = np.array([float(t) for t in xs])
    kappa = np.linalg.cond(Ai.astype(float))
    assert np.linalg.norm(res["x"] - xsf) <= 1e-13 * kappa * 10 * np.linalg.norm(xsf)


def test_cg_rank_one_update_two_steps():
    rng = np.random.default_rng(3)
    n = 30
    u = rng.standard_normal(n)
    A = _dense_csr(np.eye(n) + np.outer(u, u))
    res = O.pcg(A, rng.standard_normal(n), reduction=1e-10)
    assert res["stop_reason"] == O.CONVERGED and res["iterations"] == 2


def test_cg_diagonal_jacobi_one_step():
    d = np.arange(1.0, 41.0)
    A = _dense_csr(np.diag(d))
    dinv, _ = O.jacobi_dinv(A)
    res = O.pcg(A, np.ones(40), dinv=dinv, reduction=1e-14)
    assert res["iterations"] == 1 and res["stop_reason"] == O.CONVERGED
    assert np.allclose(res["x"], 1 / d, rtol=1e-15)


def test_constant_diagonal_jacobi_equals_cg():
    A = W.stencil_2d5(32)
    b = O.spmv(A, W.uniform_vec(A.nrows, 1))
    d, _ = O.jacobi_dinv(A)
    r1 = O.pcg(A, b, dinv=d, reduction=1e-10, history=True)
    r0 = O.pcg(A, b, dinv=None, reduction=1e-10, history=True)
    assert r1["iterations"] == r0["iterations"]
    assert np.allclose(r1["history"], r0["history"], rtol=1e-8)


def test_cg_textbook_bound_and_monotone_error():
    """||e_k||_A <= 2 ((sqrt(k)-1)/(sqrt(k)+1))^k ||e_0||_A with the closed-form
    condition number of the 64x64 Laplacian; the A-norm error decreases."""
    N = 64
    A = W.stencil_2d5(N)
    xs = W.uniform_vec(A.nrows, 1)
    b = O.spmv(A, xs)
    lmin = 8 * math.sin(math.pi / (2 * (N + 1))) ** 2
    lmax = 8 * math.cos(math.pi / (2 * (N + 1))) ** 2
    kap = lmax / lmin
    rho = (math.sqrt(kap) - 1) / (math.sqrt(kap) + 1)
    def anorm(e):
        return math.sqrt(float(e @ O.spmv(A, e)))
    e0 = anorm(xs)
    prev = e0
    for k in (5, 20, 60, 100, 150, 190):
        res = O.pcg(A, b, max_iters=k, reduction=0.0)
        ek = anorm(res["x"] - xs)
        assert ek <= 2 * rho ** k * e0 * (1 + 1e-9)
        assert ek < prev
        prev = ek


def test_cg_iteration_count_matches_scipy_poisson2d_64():
    import scipy.sparse as sp
    import scipy.sparse.linalg as spl
    A = W.stencil_2d5(64)
    b = O.spmv(A, W.uniform_vec(A.nrows, 1))
    d, _ = O.jacobi_dinv(A)
    res = O.pcg(A, b, dinv=d, reduction=1e-10)
    S = sp.csr_matrix((A.val, A.col, A.row_ptr), shape=(A.nrows, A.ncols))
    it = [0]
    spl.cg(S, b, rtol=1e-10, atol=0.0, maxiter=5000, callback=lambda xk: it.__setitem__(0, it[0] + 1))
    assert abs(res["iterations"] - it[0]) <= 2
    xr = res["x"]
    assert np.linalg.norm(b - S @ xr) <= 1e-10 * np.linalg.norm(b) * 1.01


def test_golden_listing_protocol():
    """The introductory example: Iteration(20) OR ResidualNormReduction(1e-15)
    on a non-trivial system stops after exactly 20 iterations by the
    iteration criterion; x is overwritten in place."""
    g = json.load(open(os.path.join(GOLD, "listing_cg_jacobi.json")))
    A = W.stencil_2d5(32)
    b = O.spmv(A, W.uniform_vec(A.nrows, 3))
    d, _ = O.jacobi_dinv(A)
    res = O.pcg(A, b, dinv=d, max_iters=g["max_iters"], reduction=g["reduction_factor"])
    assert res["iterations"] == g["expected_iterations"]
    assert res["stop_reason"] == O.MAX_ITERS


def test_golden_nan_rhs_protocol():
    """The polymorphism-cost protocol: size-1 matrix, x = 0, b = NaN -- the
    solver runs all iterations without stopping early or crashing."""
    g = json.load(open(os.path.join(GOLD, "nan_rhs_protocol.json")))
    A = _dense_csr([[2.0]])
    b = np.array([np.nan])
    for fn in (O.pcg, O.bicgstab):
        res = fn(A, b, max_iters=g["iterations"], nonfinite_check=0)
        assert res["iterations"] == g["iterations"] and res["stop_reason"] == O.MAX_ITERS
        res = fn(A, b, max_iters=g["iterations"], nonfinite_check=1)
        assert res["stop_reason"] == O.NONFINITE


def test_cg_breakdown_and_zero_rhs():
    A = _dense_csr(np.diag([1.0, -1.0]))
    res = O.pcg(A, np.array([1.0, 1.0]))
    assert res["stop_reason"] == O.BREAKDOWN and res["iterations"] == 0
    res = O.pcg(W.stencil_2d5(4), np.zeros(16), x0=np.ones(16))
    assert res["stop_reason"] == O.CONVERGED and res["iterations"] == 0
    assert not res["x"].any()


# ------------------------------------------------------------- BiCGSTAB
@pytest.mark.parametrize("seed", [1, 2, 3])
def test_bicgstab_exact_solution_small(seed):
    rng = np.random.default_rng(seed)
    n = 9
    D = rng.integers(-3, 4, (n, n)).astype(float) + np.diag(np.full(n, 12.0))
    b = rng.integers(-4, 5, n).astype(float)
    xs = np.array([float(t) for t in E.solve(E.frac_mat(D), E.frac_vec(b))])
    A = _dense_csr(D)
    d, _ = O.jacobi_dinv(A)
    res = O.bicgstab(A, b, dinv=d, reduction=1e-13, max_iters=200)
    assert res["stop_reason"] == O.CONVERGED
    assert np.linalg.norm(res["x"] - xs) <= 1e-11 * np.linalg.norm(xs)


def test_bicgstab_diagonal_half_step():
    d = np.linspace(1, 5, 17)
    A = _dense_csr(np.diag(d))
    dinv, _ = O.jacobi_dinv(A)
    res = O.bicgstab(A, np.ones(17), dinv=dinv, reduction=1e-14)
    assert res["iterations"] == 1 and res["spmv_count"] == 2
    assert np.allclose(res["x"], 1 / d, rtol=1e-15)


@pytest.mark.parametrize("A", [W.convdiff_2d5(40), W.stencil_2d5(40)], ids=lambda a: a.name)
def test_bicgstab_true_residual(A):
    b = O.spmv(A, W.uniform_vec(A.nrows, 5))
    d, _ = O.jacobi_dinv(A)
    res = O.bicgstab(A, b, dinv=d, reduction=1e-10)
    assert res["stop_reason"] == O.CONVERGED
    r = b - O.spmv(A, res["x"])
    assert np.linalg.norm(r) <= 2e-10 * np.linalg.norm(b)


# ------------------------------------------------------------------- IR
def test_ir_reaches_fp64_accuracy_fp32_cg_does_not():
    N = 28
    A = W.aniso_3d7(N)
    b = W.uniform_vec(A.nrows, 4)
    res = O.ir(A, b, outer_reduction=1e-12, inner_reduction=1e-4)
    assert res["stop_reason"] == O.CONVERGED
    r = b - O.spmv(A, res["x"])
    assert np.linalg.norm(r) <= 1e-12 * np.linalg.norm(b)
    # contraction: log(1e-12)/log(1e-4) = 3 outer steps plus slack for the
    # FP32 precision floor (kappa * u32)
    assert res["outer"] <= 6
    # pure FP32 CG: its recurrence residual can go low but the true FP64
    # residual is stuck near kappa * u32
    d, _ = O.jacobi_dinv(A)
    f = O.pcg_f32(A, b.astype(np.float32), d.astype(np.float32), reduction=1e-9, max_iters=3000)
    rt = b - O.spmv(A, f["x"].astype(np.float64))
    assert np.linalg.norm(rt) > 1e-9 * np.linalg.norm(b)


def test_ir_small_exact():
    Ai = W.spd_integer_small(6, 9)
    b = np.arange(1.0, 7.0)
    xs = np.array([float(t) for t in E.solve([[Fraction(int(v)) for v in r] for r in Ai],
                                             [Fraction(v) for v in b])])
    res = O.ir(_dense_csr(Ai), b, outer_reduction=1e-14, inner_reduction=1e-3)
    assert res["stop_reason"] == O.CONVERGED
    assert np.linalg.norm(res["x"] - xs) <= 1e-12 * np.linalg.norm(xs) * np.linalg.cond(Ai)


# -------------------------------------------------------------- batched
def test_batch_pcg_residuals():
    B = W.batch_systems(nsys=40, seed=77)
    out = O.batch_pcg(B, reduction=1e-10)
    assert np.all(out["status"] == O.CONVERGED)
    for s in range(B.nsys):
        A = B.system(s)
        r0, r1 = B.sys_ptr[s], B.sys_ptr[s + 1]
        D = A.dense()
        assert np.allclose(D, D.T)
        assert np.all(np.diag(D) >= np.abs(D).sum(1) - np.abs(np.diag(D)) + 1 - 1e-12)
        r = B.b[r0:r1] - D @ out["x"][r0:r1]
        assert np.linalg.norm(r) <= 1.5e-10 * np.linalg.norm(B.b[r0:r1])
        assert 0 < out["iterations"][s] <= A.nrows


# ------------------------------------------------------------- features
def _features_numpy(A):
    lens = A.row_lengths().astype(np.int64)
    n, nnz = A.nrows, A.nnz
    s = np.sort(lens)
    rank = lambda P: s[(P * n + 99) // 100 - 1]
    rows = np.repeat(np.arange(n), lens)
    bw = np.abs(A.col.astype(np.int64) - rows)
    mu = nnz / n
    sd = lens.std()
    from scipy.stats import skew
    sk = skew(lens, bias=True) if sd > 0 else 0.0
    return np.array([math.log10(n), math.log10(max(nnz, 1)), mu, sd, sd / mu, s[-1], s[0],
                     rank(50), rank(90), rank(99), np.mean(lens > 2 * mu), n * s[-1] / nnz,
                     bw.max() / n, bw.mean() / n, np.mean(bw <= 64), sk])


@pytest.mark.parametrize("m", [0, 7, 42])
def test_features_brute_force(m):
    A = W.zipf_suite_matrix(m, scale_n=0.02)
    f = O.features(A)
    g = _features_numpy(A)
    assert np.allclose(f, g, rtol=1e-12, atol=1e-14)
    ints = [5, 6, 7, 8, 9]
    assert np.array_equal(f[ints], g[ints])


# ------------------------------------------------------------------ MLP
def _theta(dims, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(O.mlp_param_count(dims)) * 0.3


def test_mlp_gradient_finite_differences():
    dims = [16, 8, 8, 5]
    rng = np.random.default_rng(0)
    X = rng.standard_normal((12, 16))
    Y = rng.standard_normal((12, 5))
    M = (rng.random((12, 5)) < 0.8).astype(float)
    th = _theta(dims, 1)
    loss, g, _ = O.mlp_loss_grad(dims, th, X, Y, M, lam=1e-2)
    h = 1e-6
    for j in rng.choice(th.size, 60, replace=False):
        tp, tm = th.copy(), th.copy()
        tp[j] += h
        tm[j] -= h
        fd = (O.mlp_loss_grad(dims, tp, X, Y, M, 1e-2, False)[0]
              - O.mlp_loss_grad(dims, tm, X, Y, M, 1e-2, False)[0]) / (2 * h)
        assert abs(fd - g[j]) <= 1e-6 * max(1.0, abs(g[j])), j


def test_mlp_linear_closed_form():
    """Zero hidden layers: loss = |M.(XW^T+b-Y)|^2/sum(M) + lam|W|^2 has
    gradient (2/sum M) (M.E)^T X + 2 lam W."""
    rng = np.random.default_rng(2)
    dims = [16, 4]
    X = rng.standard_normal((20, 16)); Y = rng.standard_normal((20, 4))
    M = (rng.random((20, 4)) < 0.7).astype(float)
    th = _theta(dims, 3)
    Wm, b = th[:64].reshape(4, 16), th[64:]
    lam = 1e-3
    loss, g, pred = O.mlp_loss_grad(dims, th, X, Y, M, lam, True, True)
    Ee = X @ Wm.T + b - Y
    assert np.allclose(pred, X @ Wm.T + b, rtol=1e-13)
    assert np.isclose(loss, (M * Ee ** 2).sum() / M.sum() + lam * (Wm ** 2).sum(), rtol=1e-13)
    gW = 2 / M.sum() * (M * Ee).T @ X + 2 * lam * Wm
    gb = 2 / M.sum() * (M * Ee).sum(0)
    assert np.allclose(g[:64], gW.ravel(), rtol=1e-12) and np.allclose(g[64:], gb, rtol=1e-12)


def test_adam_first_step_closed_form():
    rng = np.random.default_rng(4)
    th = rng.standard_normal(50); g = rng.standard_normal(50)
    m = np.zeros(50); v = np.zeros(50)
    t0 = th.copy()
    O.adam_step(th, g, m, v, 1, lr=1e-2)
    # with zero moments the bias-corrected step is lr * g / (|g| + eps)
    assert np.allclose(th, t0 - 1e-2 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=1e-15)


def test_adam_constant_gradient_every_step():
    """With a constant gradient g the bias-corrected moments are exactly g and
    g^2 at every step t, so each of the T steps moves theta by
    lr g / (|g| + eps): a dropped beta carry-over of m or v, or a bias
    correction with the wrong power of beta, fails from t = 2 on."""
    rng = np.random.default_rng(5)
    th = rng.standard_normal(40); g = rng.standard_normal(40) * np.logspace(-3, 2, 40)
    m = np.zeros(40); v = np.zeros(40)
    t0 = th.copy()
    lr, eps = 3e-3, 1e-8
    for t in range(1, 26):
        O.adam_step(th, g, m, v, t, lr=lr, eps=eps)
        assert np.allclose(th, t0 - t * lr * g / (np.abs(g) + eps), rtol=1e-11, atol=1e-14), t
        assert np.allclose(m, (1 - 0.9 ** t) * g, rtol=1e-12), t
        assert np.allclose(v, (1 - 0.999 ** t) * g * g, rtol=1e-12), t


def test_adam_moments_are_discounted_sums():
    """Varying gradients g_1..g_T: the moments equal the discounted sums
    m_t = (1-b1) sum_k b1^(t-k) g_k and v_t = (1-b2) sum_k b2^(t-k) g_k^2,
    and theta moves by lr (m_t/(1-b1^t)) / (sqrt(v_t/(1-b2^t)) + eps) at
    step t."""
    rng = np.random.default_rng(6)
    T, P = 12, 30
    G = rng.standard_normal((T, P))
    b1, b2, lr, eps = 0.8, 0.95, 1e-2, 1e-8
    th = rng.standard_normal(P); m = np.zeros(P); v = np.zeros(P)
    want = th.copy()
    for t in range(1, T + 1):
        O.adam_step(th, G[t - 1], m, v, t, lr=lr, b1=b1, b2=b2, eps=eps)
        w1 = (1 - b1) * b1 ** (t - np.arange(1, t + 1))
        w2 = (1 - b2) * b2 ** (t - np.arange(1, t + 1))
        ms = w1 @ G[:t]
        vs = w2 @ G[:t] ** 2
        assert np.allclose(m, ms, rtol=1e-12, atol=1e-15), t
        assert np.allclose(v, vs, rtol=1e-12, atol=1e-15), t
        want -= lr * (ms / (1 - b1 ** t)) / (np.sqrt(vs / (1 - b2 ** t)) + eps)
        assert np.allclose(th, want, rtol=1e-11, atol=1e-14), t
