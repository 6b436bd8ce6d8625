"""Input generators (no GPU): the point lists of the matrix-free stencils
describe exactly the CSR operators the generators build."""
import numpy as np
import pytest

import workloads as W


@pytest.mark.parametrize("N", [2, 5, 9])
def test_point_lists_match_generators(N):
    cases = [(W.stencil_3d27(N), W.points_3d27(), (N, N, N)),
             (W.aniso_3d7(N), W.points_aniso7(), (N, N, N)),
             (W.stencil_2d5(N), W.points_2d5(), (N, N, 1)),
             (W.convdiff_2d5(N), W.points_convdiff(), (N, N, 1))]
    for A, (pts, cf), shape in cases:
        B = W.stencil_grid(*shape, pts, cf)
        assert np.array_equal(A.row_ptr, B.row_ptr), A.name
        assert np.array_equal(A.col, B.col), A.name
        assert np.array_equal(A.val, B.val), A.name


def test_stencil_grid_ragged_counts():
    """nnz of a ragged grid equals the per-point in-grid neighbour counts."""
    pts, cf = W.points_3d27()
    nx, ny, nz = 13, 7, 5
    A = W.stencil_grid(nx, ny, nz, pts, cf)
    want = sum((nx - abs(di)) * (ny - abs(dj)) * (nz - abs(dk)) for di, dj, dk in pts)
    assert A.nnz == want and A.nrows == nx * ny * nz


def test_structured_suite_holds_out_the_benchmark_systems():
    suite = W.structured_suite()
    names = [s[0] for s in suite]
    assert len(names) == len(set(names))
    held = {s[0] for s in suite if s[2]}
    assert {"stencil3d27_128", "aniso3d7_160"} <= held
    assert all(not s[2] for s in suite if s[0] not in held)
