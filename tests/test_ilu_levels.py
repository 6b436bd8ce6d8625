"""The host schedule of the exact triangular solves (csrc/ilu_levels.hpp),
compiled with g++ and run on the CPU.

Pins:
- on an N^3 7-point grid (lexicographic order) the level of point (i, j, k)
  is i + j + k in the lower factor and 3(N-1) - (i + j + k) in the upper, so
  there are 3N - 2 levels and level l holds the points with that index sum
  (382 levels at N = 128, the convection-diffusion benchmark grid);
- on random patterns: ptr runs from 0 to n without decreasing, perm is a
  permutation, every dependency of a row sits in an earlier level, and each
  row's level is one more than its deepest dependency;
- solving L y = r and U z = y row by row in the schedule's order gives
  exactly the oracle's sequential substitution (bitwise), and starting from
  NaN shows that no row reads an entry before it is computed;
- the validity check rejects planted faults (a row moved one level early,
  a repeated row, a short last offset).
"""
import os
import subprocess

import numpy as np
import pytest

import oracle as O
import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2006_16852_amd", "csrc")

DRIVER = r"""
#include <cstdio>
#include <cstdlib>
#include <string>
#include <vector>
#include "ilu_levels.hpp"

// usage: levels <n> <nnz> <rp.bin> <col.bin> <lower 0|1> <out-prefix>
// writes <prefix>.perm (int32) and <prefix>.ptr (int64); prints "valid <0|1>".
// With a 7th argument "plant" the schedule read from <prefix>.perm/.ptr is
// checked instead of computed.
int main(int argc, char **argv) {
    long n = atol(argv[1]), nnz = atol(argv[2]);
    std::vector<int> rp(n + 1), col(nnz);
    FILE *f = fopen(argv[3], "rb"); if (fread(rp.data(), 4, n + 1, f) != (size_t)(n + 1)) return 2; fclose(f);
    f = fopen(argv[4], "rb"); if (nnz && fread(col.data(), 4, nnz, f) != (size_t)nnz) return 2; fclose(f);
    const bool lower = atoi(argv[5]) != 0;
    std::string pre = argv[6];
    std::vector<int> perm;
    std::vector<int64_t> ptr;
    if (argc > 7) {
        f = fopen((pre + ".perm").c_str(), "rb"); perm.resize(n);
        if (n && fread(perm.data(), 4, n, f) != (size_t)n) return 2; fclose(f);
        f = fopen((pre + ".ptr").c_str(), "rb"); fseek(f, 0, SEEK_END); long b = ftell(f); fseek(f, 0, SEEK_SET);
        ptr.resize(b / 8); if (fread(ptr.data(), 8, ptr.size(), f) != ptr.size()) return 2; fclose(f);
    } else {
        mxl::ilu_levels_host(rp, col, lower, perm, ptr);
        f = fopen((pre + ".perm").c_str(), "wb"); fwrite(perm.data(), 4, perm.size(), f); fclose(f);
        f = fopen((pre + ".ptr").c_str(), "wb"); fwrite(ptr.data(), 8, ptr.size(), f); fclose(f);
    }
    std::printf("valid %d\n", (int)mxl::ilu_levels_valid(rp, col, lower, perm, ptr));
    return 0;
}
"""


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    d = tmp_path_factory.mktemp("levels")
    src = d / "levels.cpp"
    src.write_text(DRIVER)
    exe = d / "levels"
    subprocess.check_call(["g++", "-std=c++17", "-O2", "-Wall", "-I", CSRC, str(src), "-o", str(exe)])

    def run(A, lower, plant=None):
        rp, col = d / "rp.bin", d / "col.bin"
        A.row_ptr.astype(np.int32).tofile(rp)
        A.col.astype(np.int32).tofile(col)
        pre = str(d / "sched")
        args = [str(exe), str(A.nrows), str(A.nnz), str(rp), str(col), str(int(lower)), pre]
        if plant is not None:
            plant[0].astype(np.int32).tofile(pre + ".perm")
            plant[1].astype(np.int64).tofile(pre + ".ptr")
            args.append("plant")
        out = subprocess.run(args, capture_output=True, text=True, check=True).stdout
        perm = np.fromfile(pre + ".perm", np.int32)
        ptr = np.fromfile(pre + ".ptr", np.int64)
        return perm, ptr, out.strip() == "valid 1"
    return run


def _levels_of(perm, ptr, n):
    lev = np.full(n, -1)
    for l in range(ptr.size - 1):
        lev[perm[ptr[l]:ptr[l + 1]]] = l
    return lev


@pytest.mark.parametrize("N", [5, 17, 128])
def test_grid_levels_closed_form(driver, N):
    A = W.convdiff_3d7(N)
    n = A.nrows
    idx = np.arange(n)
    s = idx % N + (idx // N) % N + idx // (N * N)
    for lower, want in ((True, s), (False, 3 * (N - 1) - s)):
        perm, ptr, valid = driver(A, lower)
        assert valid
        assert ptr.size - 1 == 3 * N - 2                     # 382 at N = 128
        assert np.array_equal(_levels_of(perm, ptr, n), want)
        assert np.array_equal(np.diff(ptr), np.bincount(want, minlength=3 * N - 2))
        # rows ascend within each level (stable order)
        for l in (0, ptr.size // 2, ptr.size - 2):
            assert np.all(np.diff(perm[ptr[l]:ptr[l + 1]]) > 0)


def _deps(A, i, lower):
    c = A.col[A.row_ptr[i]:A.row_ptr[i + 1]]
    return c[c < i] if lower else c[c > i]


@pytest.mark.parametrize("seed", [1, 2, 3])
@pytest.mark.parametrize("lower", [True, False])
def test_random_pattern_schedule(driver, seed, lower):
    A = W.random_sparse(400, 400, 0.01 * seed, seed)
    n = A.nrows
    perm, ptr, valid = driver(A, lower)
    assert valid
    assert ptr[0] == 0 and ptr[-1] == n and np.all(np.diff(ptr) > 0)
    assert np.array_equal(np.sort(perm), np.arange(n))
    lev = _levels_of(perm, ptr, n)
    for i in range(n):
        d = _deps(A, i, lower)
        assert lev[i] == (lev[d].max() + 1 if d.size else 0)


def test_empty_and_diagonal(driver):
    D = W.Csr(6, 6, np.arange(7, dtype=np.int32), np.arange(6, dtype=np.int32), np.ones(6))
    perm, ptr, valid = driver(D, True)
    assert valid and list(ptr) == [0, 6] and list(perm) == list(range(6))
    E = W.Csr(0, 0, np.zeros(1, np.int32), np.zeros(0, np.int32), np.zeros(0))
    perm, ptr, valid = driver(E, True)
    assert valid and list(ptr) == [0] and perm.size == 0


def _with_diag(A):
    """A plus a dominant diagonal (so ILU(0) exists), on the joint pattern."""
    n = A.nrows
    D = np.zeros((n, n))
    rows = np.repeat(np.arange(n), A.row_lengths())
    D[rows, A.col] = A.val
    D += np.eye(n) * (np.abs(D).sum(1).max() + 1)
    r, c = np.nonzero(D)
    rp = np.concatenate([[0], np.cumsum(np.bincount(r, minlength=n))]).astype(np.int32)
    return W.Csr(n, n, rp, c.astype(np.int32), D[r, c])


@pytest.mark.parametrize("seed", [4, 5])
def test_schedule_order_reproduces_oracle_solve(driver, seed):
    """Forward and backward substitution evaluated row by row in the
    schedule's order (each row's sum in ascending column order, as the
    level kernels and the oracle form it) equals the oracle's exact
    ILU application bit for bit; unset entries start as NaN."""
    A = _with_diag(W.random_sparse(300, 300, 0.03, seed))
    lu, bad = O.ilu0(A)
    assert bad == -1
    r = W.uniform_vec(A.nrows, seed)
    want = O.ilu_apply(A, lu, r, mode=0)
    pl, tl, _ = driver(A, True)
    pu, tu, _ = driver(A, False)
    y = np.full(A.nrows, np.nan)
    for i in pl:
        s = r[i]
        for q in range(A.row_ptr[i], A.row_ptr[i + 1]):
            if A.col[q] < i:
                s -= lu[q] * y[A.col[q]]
        y[i] = s
    z = np.full(A.nrows, np.nan)
    for i in pu:
        s, d = y[i], 0.0
        for q in range(A.row_ptr[i], A.row_ptr[i + 1]):
            if A.col[q] > i:
                s -= lu[q] * z[A.col[q]]
            elif A.col[q] == i:
                d = lu[q]
        z[i] = s / d
    assert np.array_equal(z, want)


def test_validity_rejects_planted_faults(driver):
    A = W.convdiff_3d7(6)
    perm, ptr, valid = driver(A, True)
    assert valid
    early = perm.copy()                       # a level-1 row swapped into level 0
    early[ptr[0]], early[ptr[1]] = early[ptr[1]], early[ptr[0]]
    assert not driver(A, True, (early, ptr))[2]
    dup = perm.copy(); dup[5] = dup[4]
    assert not driver(A, True, (dup, ptr))[2]
    short = ptr.copy(); short[-1] -= 1
    assert not driver(A, True, (perm, short))[2]
