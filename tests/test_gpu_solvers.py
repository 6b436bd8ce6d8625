"""Krylov solver parity (Jacobi-PCG, Jacobi-BiCGSTAB, FP32-inner iterative
refinement) of the HIP library against the CPU oracle, through the C ABI.

The bar: the stop reason equals the oracle's, the iteration count is within
max(2, 2%) of the oracle's (summation order differs, so the count may move
by a step near the threshold), and the residual recomputed in FP64 on the
CPU meets the tolerance.
"""
import json
import os

import numpy as np
import pytest
import torch

import oracle as O
import workloads as W
from tests._gpu import assert_bicgstab_tracks_oracle, DEV, dev, matrix

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def mxl():
    import paper_2006_16852_amd as m
    return m


@pytest.fixture(scope="module")
def ctx(mxl):
    return mxl.Context(0)


def _close_iters(a, b):
    return abs(a - b) <= max(2, int(0.02 * b))


def _true_rel(A, b, x):
    return np.linalg.norm(b - O.spmv(A, x)) / np.linalg.norm(b)


FORMATS = [("csr", dict(variant=1)), ("csr", dict(variant=2)), ("csr", dict(variant=0)),
           ("csr", dict(variant=3)), ("coo", {}), ("ell", {}), ("ell", dict(variant=2)),
           ("hyb", dict(hyb_quantile=0.66))]


@pytest.mark.parametrize("fmt,kw", FORMATS, ids=["vec", "merge", "scalar", "stream", "coo", "ell", "ell16", "hyb"])
def test_pcg_poisson2d_64_all_formats(mxl, ctx, fmt, kw):
    A = W.stencil_2d5(64)
    b = O.spmv(A, W.uniform_vec(A.nrows, 1))
    d, _ = O.jacobi_dinv(A)
    ref = O.pcg(A, b, dinv=d, reduction=1e-10)
    M = matrix(mxl, ctx, A).convert(fmt, **kw)
    P = mxl.jacobi(M)
    S = mxl.solver("cg", M, P, max_iters=10_000, reduction=1e-10)
    x = torch.zeros(A.nrows, dtype=torch.float64, device=DEV)
    info = S.solve(dev(b), x, history=400)
    print(f"[pcg poisson2d {fmt}] gpu {info['iterations']} oracle {ref['iterations']}", flush=True)
    assert info["stop_reason"] == mxl.STOP_CONVERGED
    assert _close_iters(info["iterations"], ref["iterations"])
    assert _true_rel(A, b, x.cpu().numpy()) <= 1.01e-10
    h = np.array(info["history"])
    assert h[0] == pytest.approx(1.0) and h[-1] <= 1e-10
    assert np.allclose(h[:50], ref_hist(A, b, d)[:50], rtol=1e-6)


def ref_hist(A, b, d):
    return O.pcg(A, b, dinv=d, reduction=1e-10, history=True)["history"]


def test_pcg_check_every_independent(mxl, ctx):
    A = W.aniso_3d7(20)
    b = W.uniform_vec(A.nrows, 4)
    M = matrix(mxl, ctx, A)
    P = mxl.jacobi(M)
    xs = []
    its = []
    for ce in (1, 7, 64):
        S = mxl.solver("cg", M, P, max_iters=5000, reduction=1e-11, check_every=ce, launch_mode=1)
        x = torch.zeros(A.nrows, dtype=torch.float64, device=DEV)
        info = S.solve(dev(b), x)
        xs.append(x.cpu().numpy())
        its.append(info["iterations"])
    assert its[0] == its[1] == its[2]
    assert np.array_equal(xs[0], xs[1]) and np.array_equal(xs[0], xs[2])
    ref = O.pcg(A, b, dinv=O.jacobi_dinv(A)[0], reduction=1e-11, max_iters=5000)
    assert _close_iters(its[0], ref["iterations"])


def test_pcg_fp32_matches_oracle_definition(mxl, ctx):
    A = W.aniso_3d7(16)
    b32 = W.uniform_vec(A.nrows, 6).astype(np.float32)
    d, _ = O.jacobi_dinv(A)
    ref = O.pcg_f32(A, b32, d.astype(np.float32), reduction=1e-5, max_iters=2000)
    M = matrix(mxl, ctx, A, torch.float32)
    P = mxl.jacobi(M)
    S = mxl.solver("cg", M, P, max_iters=2000, reduction=1e-5)
    x = torch.zeros(A.nrows, dtype=torch.float32, device=DEV)
    info = S.solve(dev(b32), x)
    assert info["stop_reason"] == mxl.STOP_CONVERGED == ref["stop_reason"]
    assert _close_iters(info["iterations"], ref["iterations"])


@pytest.mark.parametrize("A", [W.stencil_2d5(64), W.aniso_3d7(16), W.convdiff_2d5(20), W.stencil_2d5(8),
                               W.stencil_2d5(11), W.stencil_3d27(5)],
                         ids=lambda a: a.name)
def test_single_launch_matches_per_step(mxl, ctx, A):
    """The whole-solve-in-one-workgroup path (small systems; n <= 128 with
    at most 8 entries per row takes the one-wave register shape) against
    the per-step kernels and the oracle, with a nonzero initial guess."""
    b = O.spmv(A, W.uniform_vec(A.nrows, 1))
    x0 = W.uniform_vec(A.nrows, 9) * 0.1
    d, _ = O.jacobi_dinv(A)
    ref = O.pcg(A, b, x0=x0, dinv=d, reduction=1e-10, max_iters=5000)
    M = matrix(mxl, ctx, A)
    P = mxl.jacobi(M)
    out = {}
    for mode in (1, 2):
        S = mxl.solver("cg", M, P, max_iters=5000, reduction=1e-10, launch_mode=mode)
        x = dev(x0)
        out[mode] = (S.solve(dev(b), x), x.cpu().numpy())
    for mode in (1, 2):
        info, x = out[mode]
        assert info["stop_reason"] == ref["stop_reason"], (mode, info)
        assert _close_iters(info["iterations"], ref["iterations"]), (mode, info["iterations"], ref["iterations"])
        if ref["stop_reason"] == mxl.STOP_CONVERGED:
            assert _true_rel(A, b, x) <= 1.01e-10


@pytest.mark.parametrize("A", [W.convdiff_2d5(64), W.convdiff_2d5(20), W.stencil_2d5(11), W.convdiff_2d5(5),
                               W.convdiff_3d7(9), W.stencil_3d27(5)],
                         ids=lambda a: a.name)
def test_single_launch_bicgstab_matches_per_step(mxl, ctx, A):
    """BiCGSTAB in one workgroup (n <= 4096, shapes of 64, 256 and 512
    threads; the 27-point case has no shape and runs per step) against the
    per-step kernels and the oracle, with a nonzero initial guess.  The
    matrices are well-conditioned: on the anisotropic 1e-4 couplings
    BiCGSTAB's irregular residual lets rounding move its count by 10%."""
    b = W.uniform_vec(A.nrows, 2)
    x0 = W.uniform_vec(A.nrows, 8) * 0.1
    d, _ = O.jacobi_dinv(A)
    ref = O.bicgstab(A, b, x0=x0, dinv=d, reduction=1e-10, max_iters=5000)
    M = matrix(mxl, ctx, A)
    P = mxl.jacobi(M)
    for mode in (1, 2):
        S = mxl.solver("bicgstab", M, P, max_iters=5000, reduction=1e-10, launch_mode=mode)
        x = dev(x0)
        info = S.solve(dev(b), x)
        assert info["stop_reason"] == ref["stop_reason"] == mxl.STOP_CONVERGED, (mode, info)
        assert _close_iters(info["iterations"], ref["iterations"]), (mode, info["iterations"], ref["iterations"])
        assert _true_rel(A, b, x.cpu().numpy()) <= 1.01e-10
        assert info["spmv_count"] in (2 * info["iterations"], 2 * info["iterations"] + 1)


def test_single_launch_bicgstab_special_cases(mxl, ctx):
    """Half-step exit, zero right-hand side, the size-1 NaN protocol with and
    without the non-finite check, and the iteration limit, in one workgroup."""
    # a diagonal system: the half step of the first iteration is exact
    n = 50
    A = W.Csr(n, n, np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32), 1.0 + np.arange(n) / n, "diag50")
    b = W.uniform_vec(n, 3)
    M = matrix(mxl, ctx, A)
    S = mxl.solver("bicgstab", M, mxl.jacobi(M), max_iters=100, reduction=1e-12, launch_mode=2)
    x = torch.zeros(n, dtype=torch.float64, device=DEV)
    info = S.solve(dev(b), x)
    ref = O.bicgstab(A, b, dinv=O.jacobi_dinv(A)[0], max_iters=100, reduction=1e-12)
    assert info["iterations"] == ref["iterations"] == 1 and info["spmv_count"] == ref["spmv_count"] == 2
    assert np.allclose(x.cpu().numpy(), b / A.val, rtol=1e-14, atol=0)
    x = dev(np.ones(n))
    info = S.solve(dev(np.zeros(n)), x)
    assert info["iterations"] == 0 and info["stop_reason"] == mxl.STOP_CONVERGED and float(x.abs().max()) == 0.0
    one = W.Csr(1, 1, np.array([0, 1], np.int32), np.array([0], np.int32), np.array([2.0]), "one")
    M1 = matrix(mxl, ctx, one)
    for chk, want in ((1, mxl.STOP_NONFINITE), (0, mxl.STOP_MAX_ITERS)):
        S1 = mxl.solver("bicgstab", M1, None, max_iters=1000, nonfinite_check=chk, launch_mode=2)
        x1 = torch.zeros(1, dtype=torch.float64, device=DEV)
        info = S1.solve(dev(np.array([np.nan])), x1)
        ref = O.bicgstab(one, np.array([np.nan]), max_iters=1000, nonfinite_check=chk)
        assert info["stop_reason"] == want == ref["stop_reason"]
        assert info["iterations"] == ref["iterations"]
    A = W.convdiff_2d5(16)
    b = W.uniform_vec(A.nrows, 4)
    M = matrix(mxl, ctx, A)
    S = mxl.solver("bicgstab", M, mxl.jacobi(M), max_iters=7, reduction=0.0, launch_mode=2)
    x = torch.zeros(A.nrows, dtype=torch.float64, device=DEV)
    info = S.solve(dev(b), x)
    ref = O.bicgstab(A, b, dinv=O.jacobi_dinv(A)[0], max_iters=7, reduction=0.0)
    assert info["iterations"] == 7 == ref["iterations"] and info["stop_reason"] == mxl.STOP_MAX_ITERS
    assert np.linalg.norm(x.cpu().numpy() - ref["x"]) <= 1e-11 * np.linalg.norm(ref["x"])


def test_listing_protocol(mxl, ctx):
    g = json.load(open(os.path.join(GOLD, "listing_cg_jacobi.json")))
    A = W.stencil_2d5(32)
    b = O.spmv(A, W.uniform_vec(A.nrows, 3))
    M = matrix(mxl, ctx, A)
    S = mxl.solver("cg", M, mxl.jacobi(M), max_iters=g["max_iters"], reduction=g["reduction_factor"])
    x = torch.zeros(A.nrows, dtype=torch.float64, device=DEV)
    info = S.solve(dev(b), x)
    assert info["iterations"] == g["expected_iterations"]
    assert info["stop_reason"] == mxl.STOP_MAX_ITERS
    ref = O.pcg(A, b, dinv=O.jacobi_dinv(A)[0], max_iters=20, reduction=1e-15)
    assert np.allclose(x.cpu().numpy(), ref["x"], rtol=1e-9, atol=1e-12)


@pytest.mark.parametrize("kind", ["cg", "bicgstab"])
def test_nan_rhs_protocol(mxl, ctx, kind):
    g = json.load(open(os.path.join(GOLD, "nan_rhs_protocol.json")))
    A = W.Csr(1, 1, np.array([0, 1], np.int32), np.array([0], np.int32), np.array([2.0]))
    M = matrix(mxl, ctx, A)
    b = torch.full((1,), float("nan"), dtype=torch.float64, device=DEV)
    for chk, want in ((0, mxl.STOP_MAX_ITERS), (1, mxl.STOP_NONFINITE)):
        S = mxl.solver(kind, M, None, max_iters=g["iterations"], reduction=1e-10,
                       nonfinite_check=chk, check_every=g["iterations"])
        x = torch.zeros(1, dtype=torch.float64, device=DEV)
        info = S.solve(b, x)
        assert info["stop_reason"] == want
        if chk == 0:
            assert info["iterations"] == g["iterations"]


def test_breakdown_zero_rhs_and_initial_guess(mxl, ctx):
    A = W.Csr(2, 2, np.array([0, 1, 2], np.int32), np.array([0, 1], np.int32), np.array([1.0, -1.0]))
    M = matrix(mxl, ctx, A)
    S = mxl.solver("cg", M, None, max_iters=10)
    x = torch.zeros(2, dtype=torch.float64, device=DEV)
    info = S.solve(dev(np.array([1.0, 1.0])), x)
    assert info["stop_reason"] == mxl.STOP_BREAKDOWN and info["iterations"] == 0
    B = W.stencil_2d5(4)
    MB = matrix(mxl, ctx, B)
    S = mxl.solver("cg", MB, mxl.jacobi(MB))
    x = torch.ones(16, dtype=torch.float64, device=DEV)
    info = S.solve(torch.zeros(16, dtype=torch.float64, device=DEV), x)
    assert info["stop_reason"] == mxl.STOP_CONVERGED and info["iterations"] == 0
    assert not x.any()
    # resume: a second solve from the returned x needs (almost) no work
    b = O.spmv(B, W.uniform_vec(16, 1))
    x = torch.zeros(16, dtype=torch.float64, device=DEV)
    S.solve(dev(b), x)
    info = S.solve(dev(b), x)
    assert info["iterations"] <= 1


def test_time_criterion(mxl, ctx):
    A = W.stencil_2d5(64)
    M = matrix(mxl, ctx, A)
    S = mxl.solver("cg", M, mxl.jacobi(M), max_iters=100_000, reduction=0.0, time_limit=1e-9,
                   check_every=5)
    x = torch.zeros(A.nrows, dtype=torch.float64, device=DEV)
    info = S.solve(dev(W.uniform_vec(A.nrows, 1)), x)
    assert info["stop_reason"] == mxl.STOP_TIME and info["iterations"] == 5


@pytest.mark.parametrize("A", [W.convdiff_2d5(40), W.stencil_2d5(40), W.aniso_3d7(14)],
                         ids=lambda a: a.name)
def test_bicgstab(mxl, ctx, A):
    b = O.spmv(A, W.uniform_vec(A.nrows, 5))
    d, _ = O.jacobi_dinv(A)
    ref = O.bicgstab(A, b, dinv=d, reduction=1e-10)
    M = matrix(mxl, ctx, A)
    S = mxl.solver("bicgstab", M, mxl.jacobi(M), max_iters=10_000, reduction=1e-10)
    x = torch.zeros(A.nrows, dtype=torch.float64, device=DEV)
    info = S.solve(dev(b), x)
    print(f"[bicgstab {A.name}] gpu {info['iterations']} oracle {ref['iterations']}", flush=True)
    assert info["stop_reason"] == mxl.STOP_CONVERGED
    assert _close_iters(info["iterations"], ref["iterations"])
    assert _true_rel(A, b, x.cpu().numpy()) <= 2e-10


def test_bicgstab_diagonal_half_step(mxl, ctx):
    n = 17
    dvals = np.linspace(1, 5, n)
    A = W.Csr(n, n, np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32), dvals)
    M = matrix(mxl, ctx, A)
    S = mxl.solver("bicgstab", M, mxl.jacobi(M), reduction=1e-14)
    x = torch.zeros(n, dtype=torch.float64, device=DEV)
    info = S.solve(torch.ones(n, dtype=torch.float64, device=DEV), x)
    assert info["stop_reason"] == mxl.STOP_CONVERGED and info["iterations"] == 1
    assert np.allclose(x.cpu().numpy(), 1 / dvals, rtol=1e-15)


def test_ir_mixed_precision(mxl, ctx):
    A = W.aniso_3d7(28)
    b = W.uniform_vec(A.nrows, 4)
    ref = O.ir(A, b, outer_reduction=1e-12, inner_reduction=1e-4)
    M = matrix(mxl, ctx, A)
    S = mxl.ir(M, outer=dict(max_iters=50, reduction=1e-12), inner=dict(reduction=1e-4, max_iters=10_000))
    x = torch.zeros(A.nrows, dtype=torch.float64, device=DEV)
    info = S.solve(dev(b), x, history=60)
    print(f"[ir] gpu outer {info['iterations']} inner {info['inner_iterations']} | oracle "
          f"{ref['outer']} {ref['inner_iterations']}", flush=True)
    assert info["stop_reason"] == mxl.STOP_CONVERGED
    assert abs(info["iterations"] - ref["outer"]) <= 1
    assert abs(info["inner_iterations"] - ref["inner_iterations"]) <= max(4, 0.05 * ref["inner_iterations"])
    assert _true_rel(A, b, x.cpu().numpy()) <= 1e-12


def test_solver_deterministic(mxl, ctx):
    A = W.stencil_3d27(20)
    b = dev(W.uniform_vec(A.nrows, 9))
    M = matrix(mxl, ctx, A).convert("csr", variant=2)
    S = mxl.solver("cg", M, mxl.jacobi(M), reduction=1e-10)
    x1 = torch.zeros(A.nrows, dtype=torch.float64, device=DEV)
    x2 = torch.zeros_like(x1)
    S.solve(b, x1)
    S.solve(b, x2)
    assert torch.equal(x1, x2)


def test_full_size_pcg_stencil27(mxl, ctx):
    """Jacobi-PCG to 1e-10 on the 128^3 27-point system at full size: the
    iteration count against the oracle's stored count, the residual recomputed
    in FP64 on the CPU."""
    g = json.load(open(os.path.join(GOLD, "solver_counts.json")))["stencil27_128_pcg_1e-10"]
    A = W.stencil_3d27(128)
    b = O.spmv(A, W.uniform_vec(A.nrows, 2))
    M = matrix(mxl, ctx, A)
    S = mxl.solver("cg", M, mxl.jacobi(M), max_iters=5000, reduction=1e-10, check_every=8)
    x = torch.zeros(A.nrows, dtype=torch.float64, device=DEV)
    info = S.solve(dev(b), x)
    print(f"[pcg full27] gpu {info['iterations']} oracle {g['iterations']} {info['seconds']:.3f}s", flush=True)
    assert info["stop_reason"] == mxl.STOP_CONVERGED
    assert _close_iters(info["iterations"], g["iterations"])
    assert _true_rel(A, b, x.cpu().numpy()) <= 1.01e-10


def _golden(key):
    return json.load(open(os.path.join(GOLD, "solver_counts.json")))[key]


@pytest.fixture(scope="module")
def aniso160(mxl, ctx):
    """The 160^3 anisotropic system on the ELL operator with 16-bit column
    offsets (the operator the benchmark picks for it), b = U[-1,1) seed 4."""
    A = W.aniso_3d7(160)
    b = W.uniform_vec(A.nrows, 4)
    M = matrix(mxl, ctx, A).convert("ell", variant=2)
    return A, b, M


@pytest.mark.parametrize("red,key", [(1e-10, "aniso7_160_pcg_1e-10"), (1e-12, "aniso7_160_pcg_1e-12")])
def test_full_size_pcg_aniso160(mxl, ctx, aniso160, red, key):
    """FP64 Jacobi-PCG on the 160^3 anisotropic system at full size, in the
    benchmark's launch configuration (ELL16, check_every 16): iteration count
    within 2 of the oracle's stored count, residual recomputed in FP64."""
    A, b, M = aniso160
    g = _golden(key)
    S = mxl.solver("cg", M, mxl.jacobi(M), max_iters=5000, reduction=red, check_every=16)
    x = torch.zeros(A.nrows, dtype=torch.float64, device=DEV)
    info = S.solve(dev(b), x)
    print(f"[pcg aniso160 {red:g}] gpu {info['iterations']} oracle {g['iterations']}", flush=True)
    assert info["stop_reason"] == mxl.STOP_CONVERGED
    assert abs(info["iterations"] - g["iterations"]) <= 2
    assert _true_rel(A, b, x.cpu().numpy()) <= 1.01 * red


def test_full_size_ir_aniso160(mxl, ctx, aniso160):
    """Refinement with the FP32 point-Jacobi inner CG (inner reduction 1e-4)
    to 1e-12 on the 160^3 anisotropic system: corrections within 1 and
    inner iterations within 5 % of the oracle's stored counts; the FP64
    residual recomputed on the CPU."""
    A, b, M = aniso160
    g = _golden("aniso7_160_ir_1e-12_inner_1e-4")
    S = mxl.ir(M, outer=dict(max_iters=60, reduction=1e-12),
               inner=dict(reduction=1e-4, max_iters=10_000, check_every=16))
    x = torch.zeros(A.nrows, dtype=torch.float64, device=DEV)
    info = S.solve(dev(b), x)
    print(f"[ir aniso160] gpu {info['iterations']}/{info['inner_iterations']} oracle "
          f"{g['outer']}/{g['inner_iterations']}", flush=True)
    assert info["stop_reason"] == mxl.STOP_CONVERGED
    assert abs(info["iterations"] - g["outer"]) <= 1
    assert abs(info["inner_iterations"] - g["inner_iterations"]) <= 0.05 * g["inner_iterations"]
    assert _true_rel(A, b, x.cpu().numpy()) <= 1e-12


@pytest.fixture(scope="module")
def stencil128(mxl, ctx):
    A = W.stencil_3d27(128)
    b = O.spmv(A, W.uniform_vec(A.nrows, 2))
    return A, b


def test_full_size_pcg_bench_path(mxl, ctx, stencil128):
    """The benchmark's CG exactly as it is timed: ELL with 16-bit offsets
    (SpMV with the fused p.q), point Jacobi, check_every 16, on the 128^3
    27-point system; count within 2 of the oracle's, FP64 residual."""
    A, b = stencil128
    g = _golden("stencil27_128_pcg_1e-10")
    M = matrix(mxl, ctx, A).convert("ell", variant=2)
    S = mxl.solver("cg", M, mxl.jacobi(M), max_iters=5000, reduction=1e-10, check_every=16)
    x = torch.zeros(A.nrows, dtype=torch.float64, device=DEV)
    info = S.solve(dev(b), x)
    print(f"[pcg bench path] gpu {info['iterations']} oracle {g['iterations']}", flush=True)
    assert info["stop_reason"] == mxl.STOP_CONVERGED
    assert abs(info["iterations"] - g["iterations"]) <= 2
    assert _true_rel(A, b, x.cpu().numpy()) <= 1.01e-10


def test_full_size_bicgstab_stencil27(mxl, ctx, stencil128):
    """Jacobi-BiCGSTAB to 1e-10 on the 128^3 27-point system, ELL16 and
    check_every 16 as benchmarked (the many-workgroup reductions): the first
    ten residuals match the oracle's, the count lies within the oracle's own
    rounding spread widened by 2, FP64 residual."""
    A, b = stencil128
    g = _golden("stencil27_128_bicgstab_1e-10")
    M = matrix(mxl, ctx, A).convert("ell", variant=2)
    S = mxl.solver("bicgstab", M, mxl.jacobi(M), max_iters=5000, reduction=1e-10, check_every=16)
    x = torch.zeros(A.nrows, dtype=torch.float64, device=DEV)
    info = S.solve(dev(b), x, history=5001)
    print(f"[bicgstab full27] gpu {info['iterations']} oracle {g['iterations']} "
          f"perturbed oracle {g['perturbed_counts']}", flush=True)
    assert info["stop_reason"] == mxl.STOP_CONVERGED
    assert_bicgstab_tracks_oracle(info, g)
    assert _true_rel(A, b, x.cpu().numpy()) <= 2e-10
