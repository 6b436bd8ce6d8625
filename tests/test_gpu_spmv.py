"""SpMV parity: every (format, variant, dtype) of the HIP library against the
FP64 CPU oracle, through the C ABI.

Tolerance per row (FP64 1e-12, FP32 1e-5) relative to
|alpha| sum_j |a_ij||x_j| + |beta||y_i|; integer-exact inputs must agree
bitwise in every variant; format arrays must equal the oracle's bitwise.
"""
import math

import numpy as np
import pytest
import torch

import oracle as O
import workloads as W
from tests._gpu import DEV, assert_rows_close, dev, matrix, spmv_reference

pytestmark = pytest.mark.gpu

VARIANTS = [
    ("csr", 0, 0, 0.0, "csr_scalar"),
    ("csr", 1, 2, 0.0, "csr_vec2"),
    ("csr", 1, 4, 0.0, "csr_vec4"),
    ("csr", 1, 16, 0.0, "csr_vec16"),
    ("csr", 1, 32, 0.0, "csr_vec32"),
    ("csr", 1, 64, 0.0, "csr_vec64"),
    ("csr", 2, 0, 0.0, "csr_merge"),
    ("csr", 3, 0, 0.0, "csr_stream"),
    ("coo", 0, 0, 0.0, "coo"),
    ("ell", 0, 0, 0.0, "ell"),
    ("ell", 1, 0, 0.0, "ell_lds"),
    ("ell", 2, 0, 0.0, "ell16"),
    ("hyb", 0, 0, 0.66, "hyb66"),
    ("hyb", 1, 0, 0.9, "hyb90_lds"),
]


def _matrices():
    ms = [W.stencil_2d5(64), W.stencil_3d27(22), W.aniso_3d7(17), W.convdiff_2d5(31)]
    for m in (3, 11, 58):
        A = W.zipf_suite_matrix(m, scale_n=0.01)
        ms.append(A)
    ms += W.edge_matrices()
    return ms


MATS = _matrices()


@pytest.fixture(scope="module")
def mxl():
    import paper_2006_16852_amd as m
    return m


@pytest.fixture(scope="module")
def ctx(mxl):
    return mxl.Context(0)


def _convert(base, fmt, var, vw, q):
    if fmt == "csr":
        return base.convert("csr", variant=var, vector_width=vw)
    return base.convert(fmt, variant=var, hyb_quantile=q)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
@pytest.mark.parametrize("fmt,var,vw,q,name", VARIANTS, ids=[v[-1] for v in VARIANTS])
@pytest.mark.parametrize("A", MATS, ids=[a.name for a in MATS])
def test_spmv_parity(mxl, ctx, A, fmt, var, vw, q, name, dtype):
    print(f"[spmv] {A.name} {name} {dtype}", flush=True)
    base = matrix(mxl, ctx, A, dtype)
    try:
        op = _convert(base, fmt, var, vw, q)
    except mxl.MxlError as e:
        assert e.status == mxl.ERR_INFEASIBLE_FORMAT and fmt == "ell", e
        return
    rng = np.random.default_rng(7)
    x = rng.uniform(-1, 1, A.ncols)
    y0 = rng.uniform(-1, 1, A.nrows)
    fp32 = dtype == torch.float32
    tau = 1e-5 if fp32 else 1e-12
    for alpha, beta in [(1.0, 0.0), (-1.0, 1.0), (0.5, -2.0)]:
        xd = dev(x, dtype)
        yd = dev(y0, dtype) if beta != 0 else torch.full((A.nrows,), float("nan"), dtype=dtype, device=DEV)
        op.apply(xd, yd, alpha, beta)
        torch.cuda.synchronize()
        want, bound = spmv_reference(A, x, alpha, beta, y0, fp32)
        if fp32 and fmt == "csr" and var == 0:
            # one lane sums a whole row sequentially: charge the classical
            # FP32 bound gamma_k for rows longer than the 1e-5 budget allows
            k = A.row_lengths().astype(float) + 2
            u = 2.0 ** -24
            tau_rows = np.maximum(tau, k * u / (1 - k * u))
            assert_rows_close(yd.cpu().numpy(), want, bound * tau_rows / tau, tau, f"{name} a={alpha} b={beta}")
        else:
            assert_rows_close(yd.cpu().numpy(), want, bound, tau, f"{name} a={alpha} b={beta}")


@pytest.mark.parametrize("fmt,var,vw,q,name", VARIANTS, ids=[v[-1] for v in VARIANTS])
def test_spmv_integer_exact_bitwise(mxl, ctx, fmt, var, vw, q, name):
    """Integer values with partial sums < 2^24: every summation order is exact,
    so FP64 and FP32 results must equal the oracle bitwise."""
    A = W.random_sparse(777, 901, 0.02, 21, integer=True, int_range=9, empty_row_frac=0.1)
    rng = np.random.default_rng(3)
    x = rng.integers(-50, 51, A.ncols).astype(np.float64)
    want = O.spmv(A, x)
    assert np.abs(want).max() < 2 ** 24
    for dtype in (torch.float64, torch.float32):
        op = _convert(matrix(mxl, ctx, A, dtype), fmt, var, vw, q)
        y = torch.zeros(A.nrows, dtype=dtype, device=DEV)
        op.apply(dev(x, dtype), y)
        got = y.cpu().numpy().astype(np.float64)
        assert np.array_equal(got, want), name


@pytest.mark.parametrize("fmt,var,vw,q,name", VARIANTS, ids=[v[-1] for v in VARIANTS])
def test_spmv_nan_propagation(mxl, ctx, fmt, var, vw, q, name):
    """x_j = NaN makes exactly the rows that store column j NaN (padding never
    multiplies x), including rows whose stored value is an explicit zero."""
    A = W.random_sparse(300, 300, 0.03, 5)
    j = int(A.col[10])
    A.val[10] = 0.0
    x = np.ones(300)
    x[j] = np.nan
    op = _convert(matrix(mxl, ctx, A), fmt, var, vw, q)
    y = torch.zeros(300, dtype=torch.float64, device=DEV)
    op.apply(dev(x), y)
    stores = np.zeros(300, bool)
    rows = np.repeat(np.arange(300), A.row_lengths())
    stores[rows[A.col == j]] = True
    assert np.array_equal(np.isnan(y.cpu().numpy()), stores)


@pytest.mark.parametrize("A", [MATS[0], MATS[4], MATS[8], MATS[9]], ids=lambda a: a.name)
def test_format_arrays_bitwise(mxl, ctx, A):
    base = matrix(mxl, ctx, A)
    coo = base.convert("coo")
    assert np.array_equal(coo.export("coo_row").cpu().numpy(), O.csr_to_coo(A))
    try:
        ell = base.convert("ell")
        w, n_pad, ec, ev = O.csr_to_ell(A)
        d = ell.describe()
        assert (d["ell_width"], d["n_pad"]) == (w, n_pad)
        assert np.array_equal(ell.export("ell_col").cpu().numpy(), ec)
        assert np.array_equal(ell.export("ell_val").cpu().numpy(), ev)
        # 16-bit offsets: slot s of row i holds col - i, padding -32768
        rows = np.arange(ec.size) % n_pad
        off = np.where(ec >= 0, ec.astype(np.int64) - rows, -32768)
        if np.all(np.abs(off[ec >= 0]) <= 32767):
            e16 = base.convert("ell", variant=mxl.ELL_DELTA16)
            assert e16.export("ell_col").dtype == torch.int16
            assert np.array_equal(e16.export("ell_col").cpu().numpy().astype(np.int64), off)
            assert np.array_equal(e16.export("ell_val").cpu().numpy(), ev)
            assert e16.describe()["stored_bytes"] == ec.size * (8 + 2)
    except mxl.MxlError as e:
        assert e.status == mxl.ERR_INFEASIBLE_FORMAT
    for q in (0.66, 0.9):
        hyb = base.convert("hyb", hyb_quantile=q)
        H = O.csr_to_hyb(A, q=q)
        d = hyb.describe()
        assert d["ell_width"] == H["k"] and d["tail_nnz"] == H["tail_row"].size
        for key in ("ell_col", "ell_val", "tail_row", "tail_col", "tail_val"):
            got = hyb.export(key).cpu().numpy()
            assert np.array_equal(got, H[key]), key


def test_ell16_offset_range(mxl, ctx):
    """16-bit offsets hold |col - row| <= 32767 exactly; one entry further
    out makes the layout infeasible (the 32-bit layout still converts), and
    a HYB request for it is not provided."""
    n = 40000
    for far, ok in ((32767, True), (32768, False)):
        rp = np.concatenate([[0], np.cumsum(np.r_[2, np.ones(n - 1, np.int64)])]).astype(np.int32)
        col = np.concatenate([[0, far], np.arange(1, n)]).astype(np.int32)
        val = np.arange(1, n + 2, dtype=np.float64)
        A = W.Csr(n, n, rp, col, val, f"far{far}")
        base = matrix(mxl, ctx, A)
        base.convert("ell")
        if ok:
            e16 = base.convert("ell", variant=mxl.ELL_DELTA16)
            x = W.uniform_vec(n, 3)
            y = torch.zeros(n, dtype=torch.float64, device=DEV)
            e16.apply(dev(x), y)
            want, bound = spmv_reference(A, x, 1.0, 0.0, np.zeros(n), False)
            assert_rows_close(y.cpu().numpy(), want, bound, 1e-12, "ell16")
        else:
            with pytest.raises(mxl.MxlError) as e:
                base.convert("ell", variant=mxl.ELL_DELTA16)
            assert e.value.status == mxl.ERR_INFEASIBLE_FORMAT
    with pytest.raises(mxl.MxlError) as e:
        base.convert("hyb", variant=mxl.ELL_DELTA16)
    assert e.value.status == mxl.ERR_NOT_IMPLEMENTED


def test_spmv_deterministic(mxl, ctx):
    A = W.zipf_suite_matrix(17, scale_n=0.02)
    x = dev(np.random.default_rng(1).standard_normal(A.ncols))
    for fmt, var, vw, q, name in VARIANTS:
        try:
            op = _convert(matrix(mxl, ctx, A), fmt, var, vw, q)
        except mxl.MxlError as e:
            assert e.status == mxl.ERR_INFEASIBLE_FORMAT
            continue
        y1 = torch.zeros(A.nrows, dtype=torch.float64, device=DEV)
        y2 = torch.zeros_like(y1)
        op.apply(x, y1)
        op.apply(x, y2)
        assert torch.equal(y1, y2), name


def test_full_size_stencil27_sampled(mxl, ctx):
    """The 128^3 27-point operator (n = 2,097,152, nnz = 55,742,968) in every
    format, at the launch configuration the benchmark times; rows sampled and
    checked one by one against the oracle, plus the exact row-sum identity."""
    A = W.stencil_3d27(128)
    assert A.nnz == 55_742_968
    x = W.uniform_vec(A.nrows, 2)
    rng = np.random.default_rng(0)
    rows = np.unique(np.concatenate([rng.integers(0, A.nrows, 4000), [0, A.nrows - 1]]))
    sub = W.Csr(rows.size, A.ncols, np.concatenate([[0], np.cumsum(A.row_lengths()[rows])]).astype(np.int32),
                np.concatenate([A.col[A.row_ptr[r]:A.row_ptr[r + 1]] for r in rows]),
                np.concatenate([A.val[A.row_ptr[r]:A.row_ptr[r + 1]] for r in rows]))
    want, bound = spmv_reference(sub, x, 1.0, 0.0, np.zeros(rows.size), False)
    base = matrix(mxl, ctx, A)
    xd = dev(x)
    ones = torch.ones(A.nrows, dtype=torch.float64, device=DEV)
    idx = np.arange(A.nrows)
    N = 128
    c = [np.where((t == 0) | (t == N - 1), 2, 3) for t in (idx % N, (idx // N) % N, idx // N ** 2)]
    rowsum = (27 - c[0] * c[1] * c[2]).astype(np.float64)
    for fmt, var, vw, q, name in [v for v in VARIANTS if v[-1] in
                                  ("csr_vec32", "csr_merge", "csr_stream", "csr_scalar", "coo", "ell",
                                   "ell16", "hyb90_lds")]:
        print(f"[full27] {name}", flush=True)
        op = _convert(base, fmt, var, vw, q)
        y = torch.empty(A.nrows, dtype=torch.float64, device=DEV)
        op.apply(xd, y)
        assert_rows_close(y.cpu().numpy()[rows], want, bound, 1e-12, name)
        op.apply(ones, y)
        assert np.array_equal(y.cpu().numpy(), rowsum), name
        del op
    torch.cuda.empty_cache()


def _cast_values(n, seed):
    """FP64 values that exercise FP32 rounding: random magnitudes from the
    FP32 subnormal range to beyond its largest finite value, exact halfway
    cases (ties to even), signed zeros, infinities and NaN."""
    rng = np.random.default_rng(seed)
    v = rng.standard_normal(n) * 10.0 ** rng.uniform(-47, 40, n)
    k = np.arange(n)
    ties = (1.0 + np.ldexp(1.0, -24) * (2 * (k % 7) + 1)) * np.ldexp(1.0, (k % 40) - 20)
    v[::5] = ties[::5]                       # halfway between two FP32 neighbours
    v[1::97] = -0.0
    v[2::101] = np.inf
    v[3::103] = -np.inf
    v[4::107] = np.nan
    v[6::109] = np.ldexp(1.0, -149) * 1.5    # halfway above the smallest subnormal
    v[7::113] = np.finfo(np.float32).max * (1 + 2.0 ** -25)   # rounds down to FLT_MAX
    return v


@pytest.mark.parametrize("fmt,kw", [("csr", {}), ("coo", {}), ("ell", {}), ("ell", dict(variant=2)),
                                    ("hyb", dict(hyb_quantile=0.66))],
                         ids=["csr", "coo", "ell", "ell16", "hyb"])
def test_cast_bitwise(mxl, ctx, fmt, kw):
    """mxl_cast to FP32 rounds every stored value to nearest even exactly as
    numpy's float64 -> float32 conversion does (bit patterns compared; NaN
    stays NaN), keeps the index arrays, and the cast back to FP64 is exact."""
    A = W.random_sparse(700, 700, 0.02, 8)
    A = W.Csr(A.nrows, A.ncols, A.row_ptr, A.col, _cast_values(A.nnz, 9))
    M = matrix(mxl, ctx, A).convert(fmt, **kw)
    M32 = M.cast(torch.float32)
    keys = {"csr": ["val"], "coo": ["val"], "ell": ["ell_val"], "hyb": ["ell_val", "tail_val"]}[fmt]
    with np.errstate(over="ignore"):
        for key in keys:
            v64 = M.export(key).cpu().numpy()
            v32 = M32.export(key).cpu().numpy()
            want = v64.astype(np.float32)
            nan = np.isnan(want)
            assert np.array_equal(np.isnan(v32), nan), key
            assert np.array_equal(v32[~nan].view(np.uint32), want[~nan].view(np.uint32)), key
            back = M32.cast(torch.float64).export(key).cpu().numpy()
            assert np.array_equal(back[~nan], want[~nan].astype(np.float64)), key
    idx = {"csr": ["row_ptr", "col"], "coo": ["coo_row"], "ell": ["ell_col"], "hyb": ["ell_col", "tail_col"]}[fmt]
    for key in idx:
        assert torch.equal(M.export(key), M32.export(key)), key


def _long_rows(seed):
    """Rows of every length class of the row-block CSR kernel: long rows
    (> 512 entries, several 512-entry sweeps), exactly 512 and 513, runs of
    long rows, long first and last rows, and short rows."""
    rng = np.random.default_rng(seed)
    n = 6000
    lens = rng.integers(0, 40, n)
    for i, L in [(0, 5000), (1, 4097), (2, 4096), (7, 2048), (8, 2049), (9, 513), (10, 512),
                 (3000, 6000), (3001, 6000), (3002, 100), (4500, 1500), (n - 1, 3333)]:
        lens[i] = L
    rp = np.zeros(n + 1, np.int64)
    rp[1:] = np.cumsum(lens)
    col = np.concatenate([np.sort(rng.choice(n, size=L, replace=False)) for L in lens]).astype(np.int32)
    val = rng.standard_normal(int(rp[-1]))
    return W.Csr(n, n, rp.astype(np.int32), col, val, f"long_rows_{seed}")


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
def test_csr_stream_long_rows(mxl, ctx, dtype):
    """Rows in every length class of the row-block CSR kernel (long rows are
    swept by a whole wave): every row within the oracle's bound, for beta = 0
    and beta != 0."""
    A = _long_rows(1)
    op = matrix(mxl, ctx, A, dtype).convert("csr", variant=mxl.CSR_STREAM)
    rng = np.random.default_rng(2)
    x = rng.uniform(-1, 1, A.ncols)
    y0 = rng.uniform(-1, 1, A.nrows)
    fp32 = dtype == torch.float32
    for alpha, beta in [(1.0, 0.0), (-0.7, 1.3)]:
        yd = dev(y0, dtype)
        op.apply(dev(x, dtype), yd, alpha, beta)
        want, bound = spmv_reference(A, x, alpha, beta, y0, fp32)
        assert_rows_close(yd.cpu().numpy(), want, bound, 1e-5 if fp32 else 1e-12, f"a={alpha} b={beta}")


def test_csr_stream_long_rows_cg(mxl, ctx):
    """The fused dot with a long row: an arrow matrix (row and column 0 dense,
    5,000 entries) made SPD by its diagonal (spread over
    [1, 100], so plain CG needs many iterations) on the row-block CSR
    operator, against the oracle's count and residual."""
    n = 5000
    rng = np.random.default_rng(4)
    u = rng.uniform(0.1, 1.0, n - 1) / np.sqrt(n)
    d = 1.0 + 99.0 * rng.random(n - 1)
    rows = [np.arange(n)] + [np.array([0, i]) for i in range(1, n)]
    vals = [np.concatenate([[2.0 + u @ (u / d)], u])] + [np.array([u[i - 1], d[i - 1]]) for i in range(1, n)]
    lens = np.array([len(r) for r in rows])
    rp = np.zeros(n + 1, np.int64)
    rp[1:] = np.cumsum(lens)
    A = W.Csr(n, n, rp.astype(np.int32), np.concatenate(rows).astype(np.int32), np.concatenate(vals), "arrow5000")
    b = rng.uniform(-1, 1, n)
    ref = O.pcg(A, b, reduction=1e-10)
    assert ref["iterations"] > 20
    op = matrix(mxl, ctx, A).convert("csr", variant=mxl.CSR_STREAM)
    S = mxl.solver("cg", op, None, max_iters=1000, reduction=1e-10, check_every=4, launch_mode=1)
    x = torch.zeros(n, dtype=torch.float64, device=DEV)
    info = S.solve(dev(b), x)
    assert info["stop_reason"] == mxl.STOP_CONVERGED
    assert abs(info["iterations"] - ref["iterations"]) <= 2
    r = b - O.spmv(A, x.cpu().numpy())
    assert np.linalg.norm(r) <= 1e-9 * np.linalg.norm(b)
