"""ILU-type preconditioner (Sec. 3.2) on the GPU against the oracle.

ParILU sweeps recompute every factor entry from the previous sweep with the
sum over k in ascending order and no contraction, so the factors after any
number of sweeps equal the oracle's bit for bit; the triangular solves
(level-scheduled exact substitution and Jacobi sweeps) evaluate each row in
the oracle's order and equal it bit for bit too.  GMRES with the ILU
preconditioner reaches the oracle's iteration count within two steps, at
small sizes and at the full 128^3 size."""
import json
import os

import numpy as np
import pytest
import torch

import oracle as O
import workloads as W
from tests._gpu import DEV, dev, matrix

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def mxl():
    import paper_2006_16852_amd as m
    return m


@pytest.fixture(scope="module")
def ctx(mxl):
    return mxl.Context(0)


def _nonsym(n, seed, density=0.05):
    rng = np.random.default_rng(seed)
    D = rng.standard_normal((n, n)) * (rng.random((n, n)) < density)
    D += np.diag(np.abs(D).sum(axis=1) + 1.0)
    r, c = np.nonzero(D)
    rp = np.concatenate([[0], np.cumsum(np.bincount(r, minlength=n))]).astype(np.int32)
    return W.Csr(n, n, rp, c.astype(np.int32), D[r, c], f"nonsym{n}")


MATS = [W.stencil_2d5(23), W.convdiff_2d5(31), W.convdiff_3d7(13), W.stencil_3d27(9), _nonsym(517, 4)]


@pytest.mark.parametrize("sweeps", [0, 1, 3, 10])
@pytest.mark.parametrize("A", MATS, ids=[a.name for a in MATS])
def test_parilu_factors_bitwise(mxl, ctx, A, sweeps):
    P = mxl.ilu(matrix(mxl, ctx, A), sweeps=sweeps)
    got = P.info(factors=True)["lu"]
    want, bad = O.parilu(A, sweeps)
    assert bad == -1
    assert np.array_equal(got, want), np.abs(got - want).max()


@pytest.mark.parametrize("mode,ts", [("exact", 0), ("jacobi", 0), ("jacobi", 1), ("jacobi", 4)])
@pytest.mark.parametrize("A", MATS, ids=[a.name for a in MATS])
def test_triangular_solves_bitwise(mxl, ctx, A, mode, ts):
    M = matrix(mxl, ctx, A)
    P = mxl.ilu(M, sweeps=3, trisolve=mode, trs_sweeps=ts)
    lu = P.info(factors=True)["lu"]
    r = W.uniform_vec(A.nrows, 5)
    z = torch.empty(A.nrows, dtype=torch.float64, device=DEV)
    P.apply(dev(r), z)
    want = O.ilu_apply(A, lu, r, mode=0 if mode == "exact" else 1, sweeps=ts)
    assert np.array_equal(z.cpu().numpy(), want), np.abs(z.cpu().numpy() - want).max()
    # advanced apply: z = 2 M^{-1} r - 0.5 z
    z0 = W.uniform_vec(A.nrows, 6)
    zz = dev(z0)
    P.apply(dev(r), zz, 2.0, -0.5)
    err = np.abs(zz.cpu().numpy() - (2.0 * want - 0.5 * z0))
    assert np.all(err <= 2e-16 * (2.0 * np.abs(want) + 0.5 * np.abs(z0)))


def test_levels_of_a_grid(mxl, ctx):
    """The 2D N x N five-point pattern has 2N - 1 dependency levels in each
    triangle (the anti-diagonals i + j)."""
    N = 17
    P = mxl.ilu(matrix(mxl, ctx, W.stencil_2d5(N)), sweeps=1)
    info = P.info()
    assert info["levels_lower"] == 2 * N - 1 and info["levels_upper"] == 2 * N - 1


def test_converged_parilu_is_ilu0(mxl, ctx):
    A = W.convdiff_2d5(12)
    P = mxl.ilu(matrix(mxl, ctx, A), sweeps=A.nrows)
    lu0, _ = O.ilu0(A)
    assert np.abs(P.info(factors=True)["lu"] - lu0).max() <= 1e-13 * np.abs(lu0).max()


@pytest.mark.parametrize("mode,ts,sw", [("exact", 0, 3), ("jacobi", 2, 2), ("jacobi", 4, 5)])
@pytest.mark.parametrize("A", MATS[1:3] + MATS[4:], ids=[a.name for a in MATS[1:3] + MATS[4:]])
def test_gmres_with_ilu_matches_oracle(mxl, ctx, A, mode, ts, sw):
    b = W.uniform_vec(A.nrows, 7)
    M = matrix(mxl, ctx, A)
    P = mxl.ilu(M, sweeps=sw, trisolve=mode, trs_sweeps=ts)
    S = mxl.solver("gmres", M, P, krylov_dim=30, max_iters=2000, reduction=1e-10)
    x = torch.zeros(A.nrows, dtype=torch.float64, device=DEV)
    info = S.solve(dev(b), x)
    lu, _ = O.parilu(A, sw)
    ref = O.gmres_ilu(A, b, lu, trs_mode=0 if mode == "exact" else 1, trs_sweeps=ts, krylov_dim=30,
                      max_iters=2000, reduction=1e-10)
    assert ref["stop_reason"] == O.CONVERGED and info["stop_reason"] == mxl.STOP_CONVERGED
    assert abs(info["iterations"] - ref["iterations"]) <= 2, (info["iterations"], ref["iterations"])
    xh = x.cpu().numpy()
    assert np.linalg.norm(b - O.spmv(A, xh)) <= 1.01e-10 * np.linalg.norm(b)


def test_gmres_ilu_iterate_before_convergence(mxl, ctx):
    A = W.convdiff_3d7(11)
    b = W.uniform_vec(A.nrows, 8)
    M = matrix(mxl, ctx, A)
    P = mxl.ilu(M, sweeps=2, trisolve="jacobi", trs_sweeps=3)
    S = mxl.solver("gmres", M, P, krylov_dim=8, max_iters=13, reduction=0.0)
    x = torch.zeros(A.nrows, dtype=torch.float64, device=DEV)
    info = S.solve(dev(b), x)
    lu, _ = O.parilu(A, 2)
    ref = O.gmres_ilu(A, b, lu, trs_mode=1, trs_sweeps=3, krylov_dim=8, max_iters=13, reduction=0.0)
    assert info["iterations"] == 13 == ref["iterations"]
    assert np.linalg.norm(x.cpu().numpy() - ref["x"]) <= 1e-11 * np.linalg.norm(ref["x"])


def test_full_size(mxl, ctx):
    """128^3 convection-diffusion, GMRES(100) with ParILU(3) and 4 Jacobi
    sweeps per triangle: the oracle's stored count, residual recomputed."""
    g = json.load(open(os.path.join(GOLD, "solver_counts.json")))["convdiff3d7_128_gmres100_parilu3_jacobi4_1e-10"]
    A = W.convdiff_3d7(128)
    b = W.uniform_vec(A.nrows, 5)
    base = matrix(mxl, ctx, A)
    P = mxl.ilu(base, sweeps=3, trisolve="jacobi", trs_sweeps=4)
    M = base.convert("ell")
    S = mxl.solver("gmres", M, P, krylov_dim=100, max_iters=5000, reduction=1e-10, check_every=25)
    x = torch.zeros(A.nrows, dtype=torch.float64, device=DEV)
    info = S.solve(dev(b), x)
    assert info["stop_reason"] == mxl.STOP_CONVERGED
    assert abs(info["iterations"] - g["iterations"]) <= 2, (info["iterations"], g["iterations"])
    r = dev(b).clone()
    M.apply(x, r, -1.0, 1.0)
    assert float(torch.linalg.norm(r)) <= 1.01e-10 * float(np.linalg.norm(b))


def test_ilu_errors(mxl, ctx):
    A = matrix(mxl, ctx, W.convdiff_2d5(8))
    for kw in (dict(sweeps=-1), dict(trs_sweeps=-2, trisolve="jacobi")):
        with pytest.raises(mxl.MxlError) as e:
            mxl.ilu(A, **kw)
        assert e.value.status == mxl.ERR_INVALID_ARG
    Z = W.Csr(2, 2, np.array([0, 1, 3], np.int32), np.array([1, 0, 1], np.int32), np.array([1.0, 1.0, 2.0]), "nodiag")
    with pytest.raises(mxl.MxlError) as e:
        mxl.ilu(matrix(mxl, ctx, Z))
    assert e.value.status == mxl.ERR_ZERO_DIAG
    with pytest.raises(mxl.MxlError) as e:
        mxl.ilu(matrix(mxl, ctx, W.convdiff_2d5(8), torch.float32))
    assert e.value.status == mxl.ERR_NOT_IMPLEMENTED
    pts, cf = W.points_2d5()
    with pytest.raises(mxl.MxlError) as e:
        mxl.ilu(mxl.stencil(ctx, (8, 8, 1), pts, cf))
    assert e.value.status == mxl.ERR_NOT_IMPLEMENTED
    P = mxl.ilu(A)
    for kind in ("cg", "bicgstab"):
        with pytest.raises(mxl.MxlError) as e:
            mxl.solver(kind, A, P)
        assert e.value.status == mxl.ERR_NOT_IMPLEMENTED
    with pytest.raises(mxl.MxlError) as e:
        mxl.solver("gmres", matrix(mxl, ctx, W.convdiff_2d5(9)), P)
    assert e.value.status == mxl.ERR_DIM_MISMATCH
