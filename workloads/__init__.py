"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the bench.

This module only *builds inputs*: sparsity structures, coefficient values and
random vectors drawn from numpy's PCG64 (``default_rng(seed)``).  It holds none
of the method's arithmetic (no products, no solves, no format conversions), so
the oracle and the HIP path can both consume it without sharing any code that
the parity tests are meant to check.

Every matrix is returned as a canonical CSR triple (int32 row pointers, int32
column indices sorted and unique within each row, float64 values), which is
the compressed-row format the paper's operator examples store their system
matrices in (Sec. 2.2.4).

Workload recipes (all seeds are explicit arguments):

* ``stencil_2d5(N)``       -- 2D 5-point Poisson, lexicographic i + N*j,
                              4 on the diagonal and -1 off it (Dirichlet
                              boundary eliminated).
* ``stencil_3d27(N)``      -- 3D 27-point stencil, 26 / -1.
* ``aniso_3d7(N)``         -- 3D 7-point anisotropic diffusion, coefficient
                              1 / 1e-2 / 1e-4 along the i / j / k index, plus
                              a diagonal shift 1e-3.
* ``zipf_suite_matrix(m)`` -- member m of the 200-matrix row-length-skewed
                              suite (scaled truncated Zipf row lengths,
                              banded-random columns, N(0,1) values).
* ``batch_systems(...)``   -- thousands of small banded, diagonally dominant
                              SPD systems packed in one CSR.
* ``node_block_3d7(N)``    -- 3D 7-point grid of nodes with 1..6 unknowns
                              each, dense coupling within and between
                              neighbouring nodes (variable-size blocks).
* ``random_sparse(...)``, ``edge_matrices()``, ``convdiff_2d5(N)`` -- small
                              cases for parity and edge tests.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

__all__ = [
    "Csr", "stencil_2d5", "stencil_3d27", "aniso_3d7", "convdiff_2d5",
    "uniform_vec", "zipf_suite_params", "zipf_suite_matrix", "batch_systems",
    "random_sparse", "edge_matrices", "spd_integer_small", "node_block_3d7",
]


@dataclass
class Csr:
    nrows: int
    ncols: int
    row_ptr: np.ndarray  # int32[nrows+1]
    col: np.ndarray      # int32[nnz]
    val: np.ndarray      # float64[nnz]
    name: str = ""

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def row_lengths(self) -> np.ndarray:
        return np.diff(self.row_ptr.astype(np.int64))

    def dense(self) -> np.ndarray:
        """Densify (small matrices only; used for brute-force checks)."""
        d = np.zeros((self.nrows, self.ncols), dtype=np.float64)
        rows = np.repeat(np.arange(self.nrows), self.row_lengths())
        d[rows, self.col] = self.val
        return d


def _from_offset_stencil(n, offsets, valid_masks, values, name):
    """Assemble CSR from per-row stencil offsets given in ascending order.

    ``valid_masks[k]`` says which rows own the k-th neighbour; ``values[k]`` is
    its coefficient (scalar or per-row array).  Offsets ascend, so columns come
    out sorted within each row.
    """
    nk = len(offsets)
    counts = np.zeros(n, dtype=np.int64)
    for m in valid_masks:
        counts += m
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    nnz = int(row_ptr[-1])
    col = np.empty(nnz, dtype=np.int32)
    val = np.empty(nnz, dtype=np.float64)
    # position of the k-th neighbour inside its row = number of valid
    # neighbours with a smaller offset
    seen = np.zeros(n, dtype=np.int64)
    rows = np.arange(n, dtype=np.int64)
    for k in range(nk):
        m = valid_masks[k]
        r = rows[m]
        pos = row_ptr[:-1][m] + seen[m]
        col[pos] = (r + offsets[k]).astype(np.int32)
        v = values[k]
        val[pos] = v if np.isscalar(v) else np.asarray(v)[m]
        seen += m
        del r, pos
    assert nnz < 2**31
    return Csr(n, n, row_ptr.astype(np.int32), col, val, name)


def stencil_2d5(N: int) -> Csr:
    """2D 5-point Laplacian on an N x N grid (diag 4, neighbours -1)."""
    n = N * N
    idx = np.arange(n, dtype=np.int64)
    i, j = idx % N, idx // N
    offs = [-N, -1, 0, 1, N]
    masks = [j > 0, i > 0, np.ones(n, bool), i < N - 1, j < N - 1]
    vals = [-1.0, -1.0, 4.0, -1.0, -1.0]
    return _from_offset_stencil(n, offs, masks, vals, f"stencil2d5_{N}")


def stencil_3d27(N: int, diag: float = 26.0, off: float = -1.0) -> Csr:
    """3D 27-point stencil on an N^3 grid, lexicographic i + N*j + N^2*k."""
    n = N ** 3
    idx = np.arange(n, dtype=np.int64)
    i, j, k = idx % N, (idx // N) % N, idx // (N * N)
    lo = [i > 0, j > 0, k > 0]
    hi = [i < N - 1, j < N - 1, k < N - 1]
    offs, masks, vals = [], [], []
    ones = np.ones(n, bool)
    for dk in (-1, 0, 1):
        mk = lo[2] if dk < 0 else (hi[2] if dk > 0 else ones)
        for dj in (-1, 0, 1):
            mj = lo[1] if dj < 0 else (hi[1] if dj > 0 else ones)
            mkj = mk & mj
            for di in (-1, 0, 1):
                mi = lo[0] if di < 0 else (hi[0] if di > 0 else ones)
                offs.append(di + N * dj + N * N * dk)
                masks.append(mkj & mi)
                vals.append(diag if (di, dj, dk) == (0, 0, 0) else off)
    del i, j, k, idx
    return _from_offset_stencil(n, offs, masks, vals, f"stencil3d27_{N}")


def aniso_3d7(N: int, coef=(1.0, 1e-2, 1e-4), shift: float = 1e-3) -> Csr:
    """3D 7-point anisotropic diffusion: sum_d a_d * tridiag(-1,2,-1)_d + shift*I.

    a_0 acts along the unit-stride index i, a_1 along j, a_2 along k.
    """
    ax, ay, az = coef
    n = N ** 3
    idx = np.arange(n, dtype=np.int64)
    i, j, k = idx % N, (idx // N) % N, idx // (N * N)
    d = 2.0 * (ax + ay + az) + shift
    offs = [-N * N, -N, -1, 0, 1, N, N * N]
    masks = [k > 0, j > 0, i > 0, np.ones(n, bool), i < N - 1, j < N - 1, k < N - 1]
    vals = [-az, -ay, -ax, d, -ax, -ay, -az]
    return _from_offset_stencil(n, offs, masks, vals, f"aniso3d7_{N}")


def convdiff_2d5(N: int, peclet: float = 0.5) -> Csr:
    """Nonsymmetric 2D convection-diffusion, 5-point, first-order upwind in x.

    Diffusion gives 4 / -1; convection with cell Peclet number ``peclet`` in
    the +i direction adds +peclet to the diagonal and -peclet to the west
    neighbour.  Diagonally dominant, nonsymmetric.
    """
    n = N * N
    idx = np.arange(n, dtype=np.int64)
    i, j = idx % N, idx // N
    offs = [-N, -1, 0, 1, N]
    masks = [j > 0, i > 0, np.ones(n, bool), i < N - 1, j < N - 1]
    vals = [-1.0, -1.0 - peclet, 4.0 + peclet, -1.0, -1.0]
    return _from_offset_stencil(n, offs, masks, vals, f"convdiff2d5_{N}")


def stencil_grid(nx: int, ny: int, nz: int, points, coefs, name: str = None) -> Csr:
    """CSR of a constant-coefficient stencil on an nx x ny x nz grid (i
    fastest), neighbours outside the grid omitted; points must be given in
    (dk, dj, di) lexicographic order so the columns come out sorted."""
    n = nx * ny * nz
    idx = np.arange(n, dtype=np.int64)
    i, j, k = idx % nx, (idx // nx) % ny, idx // (nx * ny)
    offs, masks = [], []
    for di, dj, dk in points:
        offs.append(di + nx * (dj + ny * dk))
        masks.append((i + di >= 0) & (i + di < nx) & (j + dj >= 0) & (j + dj < ny) & (k + dk >= 0) & (k + dk < nz))
    # points in (dk, dj, di) lexicographic order give every row's in-grid
    # neighbours in ascending column order (an in-grid |di| step is < nx)
    return _from_offset_stencil(n, offs, masks, list(coefs), name or f"grid{nx}x{ny}x{nz}_{len(points)}pt")


# Point lists of the same operators for a matrix-free stencil: (di, dj, dk)
# offsets and coefficients, in the column order the CSR generators use.
def points_2d5():
    return [(0, -1, 0), (-1, 0, 0), (0, 0, 0), (1, 0, 0), (0, 1, 0)], [-1.0, -1.0, 4.0, -1.0, -1.0]


def points_3d27(diag: float = 26.0, off: float = -1.0):
    pts = [(di, dj, dk) for dk in (-1, 0, 1) for dj in (-1, 0, 1) for di in (-1, 0, 1)]
    return pts, [diag if p == (0, 0, 0) else off for p in pts]


def points_aniso7(coef=(1.0, 1e-2, 1e-4), shift: float = 1e-3):
    ax, ay, az = coef
    pts = [(0, 0, -1), (0, -1, 0), (-1, 0, 0), (0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1)]
    return pts, [-az, -ay, -ax, 2.0 * (ax + ay + az) + shift, -ax, -ay, -az]


def points_convdiff(peclet: float = 0.5):
    return ([(0, -1, 0), (-1, 0, 0), (0, 0, 0), (1, 0, 0), (0, 1, 0)],
            [-1.0, -1.0 - peclet, 4.0 + peclet, -1.0, -1.0])


def points_convdiff3d(peclet=(0.5, 0.25, 0.125)):
    """3D 7-point convection-diffusion: diffusion 6 / -1 plus first-order
    upwind convection with cell Peclet numbers (px, py, pz) along +i, +j,
    +k (adds p_d to the diagonal and -p_d to the upwind neighbour).
    Nonsymmetric, diagonally dominant."""
    px, py, pz = peclet
    pts = [(0, 0, -1), (0, -1, 0), (-1, 0, 0), (0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1)]
    return pts, [-1.0 - pz, -1.0 - py, -1.0 - px, 6.0 + px + py + pz, -1.0, -1.0, -1.0]


def convdiff_3d7(N: int, peclet=(0.5, 0.25, 0.125)) -> Csr:
    """CSR of points_convdiff3d on an N^3 grid."""
    pts, cf = points_convdiff3d(peclet)
    return stencil_grid(N, N, N, pts, cf, f"convdiff3d7_{N}")


def uniform_vec(n: int, seed: int, dtype=np.float64) -> np.ndarray:
    """x ~ U[-1, 1) from PCG64(seed)."""
    return np.random.default_rng(seed).uniform(-1.0, 1.0, n).astype(dtype)


# ---------------------------------------------------------------- Zipf suite
@dataclass
class ZipfParams:
    m: int
    n: int
    a: float
    mu: float
    K: int
    bw: int


def zipf_suite_params(m: int) -> ZipfParams:
    rng = np.random.default_rng(1000 + m)
    n = int(round(math.exp(rng.uniform(math.log(1e5), math.log(2e6)))))
    a = float(rng.uniform(1.5, 3.0))
    mu = float(math.exp(rng.uniform(math.log(8.0), math.log(64.0))))
    K = int(min(10_000, n))
    bw = int(round(math.exp(rng.uniform(math.log(1e2), math.log(n)))))
    return ZipfParams(m, n, a, mu, K, bw)


def _zipf_lengths(rng, n, a, mu, K):
    ks = np.arange(1, K + 1, dtype=np.float64)
    pmf = ks ** (-a)
    pmf /= pmf.sum()
    cdf = np.cumsum(pmf)
    cdf[-1] = 1.0
    ez = float((ks * pmf).sum())
    z = np.searchsorted(cdf, rng.random(n), side="right") + 1
    z = np.minimum(z, K)
    lens = np.ceil(z * (mu / ez)).astype(np.int64)
    return np.clip(lens, 1, K)


def zipf_suite_matrix(m: int, scale_n: float = 1.0) -> Csr:
    """Member m (0..199) of the skewed-row-length suite.

    n log-uniform in [1e5, 2e6]; exponent a ~ U[1.5, 3]; target mean row
    length mu log-uniform in [8, 64]; row length = clamp(ceil(Z*mu/E[Z]), 1, K)
    with Z ~ Zipf(a) truncated to [1, K], K = min(1e4, n); column window
    [i-bw, i+bw] with bw log-uniform in [1e2, n], widened (and shifted inside
    [0, n)) when a row is longer than its window.  Columns are drawn uniformly
    with replacement and de-duplicated, so realised row lengths can fall a
    little below the drawn ones (statistics are always measured, never
    assumed).  Values N(0, 1).  ``scale_n`` < 1 shrinks n (tests only).
    """
    p = zipf_suite_params(m)
    n = max(64, int(p.n * scale_n))
    K = min(p.K, n)
    bw = min(p.bw, n)
    rng = np.random.default_rng(10_000 + m)
    lens = _zipf_lengths(rng, n, p.a, p.mu, K)
    rows = np.arange(n, dtype=np.int64)
    lo = np.maximum(rows - bw, 0)
    hi = np.minimum(rows + bw, n - 1)
    width = hi - lo + 1
    wide = lens > width
    # widen: a window of exactly len columns, centred on i and kept in range
    lo = np.where(wide, np.clip(rows - lens // 2, 0, n - lens), lo)
    width = np.where(wide, lens, width)
    total = int(lens.sum())
    r_of = np.repeat(rows, lens)
    off = (rng.random(total) * np.repeat(width, lens)).astype(np.int64)
    colw = np.repeat(lo, lens) + off
    # rows whose sample is dense in its window: take a full permutation prefix
    dense = np.nonzero(lens * 2 > width)[0]
    if dense.size:
        starts = np.concatenate([[0], np.cumsum(lens)])
        for r in dense:
            s, L, w0 = starts[r], lens[r], width[r]
            colw[s:s + L] = lo[r] + rng.permutation(w0)[:L]
    key = np.unique(r_of * n + colw)
    del r_of, colw, off
    rr = key // n
    cc = (key - rr * n).astype(np.int32)
    counts = np.bincount(rr, minlength=n)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    assert row_ptr[-1] < 2**31
    val = rng.standard_normal(cc.size)
    return Csr(n, n, row_ptr.astype(np.int32), cc, val, f"zipf_{m}")


# ------------------------------------------------------- structured suite
def structured_suite() -> list:
    """Regular stencil matrices for the selector's training set, as
    (name, builder, held_out): 2D 5-point, 3D 27-point, anisotropic 3D
    7-point and 3D convection-diffusion at several sizes.  The held-out ones
    (including the 128^3 27-point and 160^3 anisotropic benchmark systems)
    are never trained on."""
    out = []
    for N in (256, 724, 1448):
        out.append((f"stencil2d5_{N}", lambda N=N: stencil_2d5(N), False))
    out.append(("stencil2d5_1024", lambda: stencil_2d5(1024), True))
    for N in (48, 80, 112, 144):
        out.append((f"stencil3d27_{N}", lambda N=N: stencil_3d27(N), False))
    out.append(("stencil3d27_128", lambda: stencil_3d27(128), True))
    for N in (64, 100, 140):
        out.append((f"aniso3d7_{N}", lambda N=N: aniso_3d7(N), False))
    out.append(("aniso3d7_160", lambda: aniso_3d7(160), True))
    for N in (64, 100, 150):
        out.append((f"convdiff3d7_{N}", lambda N=N: convdiff_3d7(N), False))
    out.append(("convdiff3d7_128", lambda: convdiff_3d7(128), True))
    return out


# ------------------------------------------------------------ batched systems
@dataclass
class Batch:
    nsys: int
    sys_ptr: np.ndarray   # int32[nsys+1] row offsets of each system
    row_ptr: np.ndarray   # int32[total_rows+1] global nnz offsets
    col: np.ndarray       # int32[nnz] column index local to its system
    val: np.ndarray       # float64[nnz]
    b: np.ndarray         # float64[total_rows]

    def system(self, s: int) -> Csr:
        r0, r1 = int(self.sys_ptr[s]), int(self.sys_ptr[s + 1])
        k0, k1 = int(self.row_ptr[r0]), int(self.row_ptr[r1])
        rp = (self.row_ptr[r0:r1 + 1].astype(np.int64) - k0).astype(np.int32)
        return Csr(r1 - r0, r1 - r0, rp, self.col[k0:k1].copy(),
                   self.val[k0:k1].copy(), f"sys{s}")


def batch_systems(nsys: int = 10_000, seed: int = 5000, nmin: int = 32,
                  nmax: int = 1024) -> Batch:
    """Independent banded SPD systems: n_s log-uniform in [nmin, nmax], full
    band of odd width w_s ~ U{5,7,...,27}, symmetric N(0,1) off-diagonals,
    diagonal = row absolute sum + 1 (strict diagonal dominance), b ~ U[-1,1).
    """
    rng = np.random.default_rng(seed)
    sizes = np.rint(np.exp(rng.uniform(math.log(nmin), math.log(nmax), nsys))).astype(np.int64)
    widths = rng.choice(np.arange(5, 28, 2), size=nsys)
    rps, cols, vals = [], [], []
    sys_ptr = np.zeros(nsys + 1, dtype=np.int64)
    np.cumsum(sizes, out=sys_ptr[1:])
    nnz_base = 0
    for s in range(nsys):
        n, h = int(sizes[s]), int(widths[s]) // 2
        h = min(h, n - 1)
        band = np.zeros((n, 2 * h + 1))
        for d in range(1, h + 1):
            v = rng.standard_normal(n - d)
            band[:n - d, h + d] = v      # A[i, i+d]
            band[d:, h - d] = v          # A[i+d, i]
        band[:, h] = np.abs(band).sum(axis=1) + 1.0
        ii = np.arange(n)[:, None] + np.arange(-h, h + 1)[None, :]
        mask = (ii >= 0) & (ii < n)
        cnt = mask.sum(axis=1)
        rp = np.zeros(n, dtype=np.int64)
        np.cumsum(cnt[:-1], out=rp[1:])
        rps.append(rp + nnz_base)
        cols.append(ii[mask].astype(np.int32))
        vals.append(band[mask])
        nnz_base += int(cnt.sum())
    row_ptr = np.concatenate(rps + [np.array([nnz_base])]).astype(np.int64)
    assert nnz_base < 2**31
    b = rng.uniform(-1.0, 1.0, int(sys_ptr[-1]))
    return Batch(nsys, sys_ptr.astype(np.int32), row_ptr.astype(np.int32),
                 np.concatenate(cols), np.concatenate(vals), b)


# ------------------------------------------------------ variable node blocks
def node_block_3d7(N: int, kmax: int = 6, seed: int = 7) -> Csr:
    """A 3D 7-point grid of N^3 nodes carrying k_v ~ U{1..kmax} unknowns each
    (seeded), numbered node after node in lexicographic node order.  Every
    unknown couples to all unknowns of its own node and of the (up to six)
    neighbouring nodes, so the rows of one node share one column set (a
    supervariable of k_v rows).  Symmetric values: within a node -U[1, 10),
    between nodes -U[0.1, 1), drawn once per unordered pair; diagonal = the
    row's off-diagonal absolute sum + 1e-2 (symmetric, strictly diagonally
    dominant with a positive diagonal, hence SPD)."""
    rng = np.random.default_rng(seed)
    nn = N ** 3
    k = rng.integers(1, kmax + 1, nn).astype(np.int64)
    start = np.zeros(nn + 1, np.int64)
    np.cumsum(k, out=start[1:])
    n = int(start[-1])
    node = np.repeat(np.arange(nn), k)                      # node of each unknown
    ii, jj, kk = node % N, (node // N) % N, node // (N * N)
    # neighbour nodes in ascending node order: -N^2, -N, -1, 0, +1, +N, +N^2
    offs = [(-N * N, kk > 0), (-N, jj > 0), (-1, ii > 0), (0, np.ones(n, bool)),
            (1, ii < N - 1), (N, jj < N - 1), (N * N, kk < N - 1)]
    cnt = np.zeros(n, np.int64)
    for o, m in offs:
        cnt += np.where(m, k[np.clip(node + o, 0, nn - 1)], 0)
    rp = np.zeros(n + 1, np.int64)
    np.cumsum(cnt, out=rp[1:])
    nnz = int(rp[-1])
    assert nnz < 2**31
    col = np.empty(nnz, np.int64)
    pos = rp[:-1].copy()
    for o, m in offs:
        rows = np.nonzero(m)[0]
        nb = node[rows] + o
        kn = k[nb]
        tot = int(kn.sum())
        r_rep = np.repeat(rows, kn)
        local = np.arange(tot) - np.repeat(np.cumsum(kn) - kn, kn)
        col[np.repeat(pos[rows], kn) + local] = np.repeat(start[nb], kn) + local
        pos[rows] += kn
        del r_rep
    row = np.repeat(np.arange(n), cnt)
    lo, hi = np.minimum(row, col), np.maximum(row, col)
    key = lo * n + hi
    uniq, inv = np.unique(key, return_inverse=True)
    same = node[uniq // n] == node[uniq % n]
    w = np.where(same, rng.uniform(1.0, 10.0, uniq.size), rng.uniform(0.1, 1.0, uniq.size))
    val = -w[inv]
    diag = row == col
    val[diag] = 0.0
    absum = np.bincount(row, weights=np.abs(val), minlength=n)
    val[diag] = absum + 1e-2
    return Csr(n, n, rp.astype(np.int32), col.astype(np.int32), val, f"nodeblock3d7_{N}_k{kmax}")


# ------------------------------------------------------------- small / edge
def random_sparse(nrows: int, ncols: int, density: float, seed: int,
                  integer: bool = False, empty_row_frac: float = 0.0,
                  int_range: int = 8) -> Csr:
    """Uniformly random sparsity; optional integer values in [-int_range, int_range]."""
    rng = np.random.default_rng(seed)
    mask = rng.random((nrows, ncols)) < density
    if empty_row_frac > 0:
        mask[rng.random(nrows) < empty_row_frac, :] = False
    r, c = np.nonzero(mask)
    counts = np.bincount(r, minlength=nrows)
    rp = np.zeros(nrows + 1, dtype=np.int64)
    np.cumsum(counts, out=rp[1:])
    if integer:
        v = rng.integers(-int_range, int_range + 1, r.size).astype(np.float64)
    else:
        v = rng.standard_normal(r.size)
    return Csr(nrows, ncols, rp.astype(np.int32), c.astype(np.int32), v,
               f"rand_{nrows}x{ncols}_{seed}")


def _csr_from_rows(nrows, ncols, rows, name):
    """rows: list of (cols list ascending, vals list)."""
    rp = [0]
    cols, vals = [], []
    for cs, vs in rows:
        cols.extend(cs)
        vals.extend(vs)
        rp.append(len(cols))
    return Csr(nrows, ncols, np.array(rp, np.int32), np.array(cols, np.int32),
               np.array(vals, np.float64), name)


def edge_matrices(seed: int = 11) -> list[Csr]:
    """Degenerate shapes every SpMV variant must handle."""
    rng = np.random.default_rng(seed)
    out = []
    out.append(_csr_from_rows(1, 1, [([0], [3.0])], "one_by_one"))
    out.append(Csr(5, 7, np.zeros(6, np.int32), np.zeros(0, np.int32),
                   np.zeros(0), "all_empty"))
    m = random_sparse(133, 97, 0.08, seed, empty_row_frac=0.3)
    m.name = "empty_rows_ragged"
    out.append(m)
    # one dense row of 10,000 entries among short rows
    n = 10_050
    rows = []
    for i in range(n):
        if i == 17:
            rows.append((list(range(10_000)), list(rng.standard_normal(10_000))))
        else:
            cs = sorted(set(rng.integers(0, n, 3).tolist()))
            rows.append((cs, list(rng.standard_normal(len(cs)))))
    out.append(_csr_from_rows(n, n, rows, "dense_row_1e4"))
    m = random_sparse(64 * 37 + 13, 64 * 37 + 13, 0.004, seed + 1)
    m.name = "ragged_tail"
    out.append(m)
    # long rows everywhere (several carries per workgroup boundary)
    m = random_sparse(40, 6000, 0.6, seed + 2)
    m.name = "wide_rows"
    out.append(m)
    return out


def spd_integer_small(n: int, seed: int) -> np.ndarray:
    """Dense integer SPD matrix A = B^T B + I with small integer B (exact tests)."""
    rng = np.random.default_rng(seed)
    B = rng.integers(-3, 4, (n, n)).astype(np.int64)
    return B.T @ B + np.eye(n, dtype=np.int64)
