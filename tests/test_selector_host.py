"""Host logic of the selector (no GPU): labels, the ELL feasibility mirror,
regret and the performance profile."""
import math

import numpy as np
import pytest

import oracle as O
import workloads as W


@pytest.fixture(scope="module")
def S():
    from paper_2006_16852_amd import selector
    return selector


def test_labels_from_times(S):
    T = np.array([[2.0, 1.0, np.inf, 4.0] + [8.0] * (len(S.CLASSES) - 4)])
    Y, M = S.labels_from_times(T)
    assert M[0, 2] == 0 and M.sum() == len(S.CLASSES) - 1
    assert Y[0, 1] == 0.0 and math.isclose(Y[0, 0], math.log(2.0)) and Y[0, 2] == 0.0


@pytest.mark.parametrize("A", [W.stencil_3d27(12), W.zipf_suite_matrix(3, scale_n=0.01),
                               W.edge_matrices()[3]], ids=lambda a: a.name)
def test_ell_feasibility_mirror(S, A):
    """The feature-based mirror agrees with the budget the library applies
    (min(max(4 x CSR bytes, 1 MiB), 32 GiB) for n_pad * w * 12 bytes)."""
    f = O.features(A)
    n_pad = ((A.nrows + 63) // 64) * 64
    w = int(A.row_lengths().max())
    csr = A.nnz * 12 + (A.nrows + 1) * 4
    want = n_pad * w * 12 <= min(max(4 * csr, 1 << 20), 32 << 30)
    assert S.ell_feasible(f) == want


@pytest.mark.parametrize("A", [W.stencil_3d27(12), W.aniso_3d7(40), W.zipf_suite_matrix(3, scale_n=0.01),
                               W.edge_matrices()[3]], ids=lambda a: a.name)
def test_ell16_feasibility_mirror(S, A):
    """16-bit offsets: the feature-based mirror agrees with the exact
    condition max |col - row| <= 32767 plus the storage budget."""
    f = O.features(A)
    rows = np.repeat(np.arange(A.nrows), A.row_lengths())
    maxoff = int(np.abs(A.col.astype(np.int64) - rows).max())
    assert S.ell16_feasible(f) == (S.ell_feasible(f) and maxoff <= 32767)
    k = S.CLASSES.index("ell16")
    assert S.feasible_mask(f)[k] == S.ell16_feasible(f)


def test_regret_and_profile(S):
    T = np.array([[1.0, 2.0, 3.0] + [9.0] * (len(S.CLASSES) - 3),
                  [4.0, 2.0, 1.0] + [9.0] * (len(S.CLASSES) - 3)])
    r = S.regret(T, np.array([0, 1]))
    assert np.allclose(r, [0.0, 1.0])
    prof = S.performance_profile(T, {"p": np.array([0, 1])}, taus=(1.0, 2.0))
    assert prof["p"] == {"1": 0.5, "2": 1.0}


def test_transform_and_init(S):
    F = np.arange(32, dtype=float).reshape(2, 16)
    G = S.transform(F)
    assert np.allclose(G[:, S.LOG_FEATS], np.log1p(F[:, S.LOG_FEATS]))
    th = S.he_init(S.dims_for(len(S.CLASSES)), 0)
    assert th.size == O.mlp_param_count(S.dims_for(len(S.CLASSES)))
