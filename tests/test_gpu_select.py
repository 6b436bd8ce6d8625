"""Selector device work against the oracle: the 16 features (integer ones
bitwise, the rest within 1e-12), the FP32 MLP's outputs, loss and gradients
against the FP64 oracle (1e-4 relative), the Adam step, and GPU training."""
import numpy as np
import pytest
import torch

import oracle as O
import workloads as W
from tests._gpu import DEV, matrix

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mxl():
    import paper_2006_16852_amd as m
    return m


@pytest.fixture(scope="module")
def ctx(mxl):
    return mxl.Context(0)


FEAT_MATS = ([W.zipf_suite_matrix(m, scale_n=0.02) for m in (0, 5, 33, 71)]
             + [W.stencil_2d5(64), W.stencil_3d27(16), W.aniso_3d7(12)]
             + [W.edge_matrices()[i] for i in (0, 2, 3, 4)])


@pytest.mark.parametrize("A", FEAT_MATS, ids=[a.name for a in FEAT_MATS])
def test_features_parity(mxl, ctx, A):
    got = matrix(mxl, ctx, A).features()
    want = O.features(A)
    ints = [5, 6, 7, 8, 9]
    assert np.array_equal(got[ints], want[ints])
    assert np.allclose(got, want, rtol=1e-12, atol=1e-13), np.abs(got - want).max()


def _data(seed, ns=37, dims=(16, 32, 32, 10)):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((ns, dims[0])).astype(np.float32)
    Y = rng.standard_normal((ns, dims[-1])).astype(np.float32)
    M = (rng.random((ns, dims[-1])) < 0.8).astype(np.float32)
    th = (rng.standard_normal(O.mlp_param_count(list(dims))) * 0.3).astype(np.float32)
    return X, Y, M, th


@pytest.mark.parametrize("dims", [(16, 32, 32, 10), (16, 10), (16, 8, 4)], ids=str)
def test_mlp_forward_grad_parity(mxl, ctx, dims):
    X, Y, M, th = _data(1, dims=dims)
    net = mxl.Mlp(ctx, list(dims), th)
    Xd, Yd, Md = (torch.from_numpy(a).to(DEV) for a in (X, Y, M))
    pred = net.forward(Xd).cpu().numpy()
    loss = net.loss_grad(Xd, Yd, Md, 1e-3)
    g = net.grad()
    lo, go, po = O.mlp_loss_grad(list(dims), th.astype(np.float64), X, Y, M, 1e-3, True, True)
    assert np.allclose(pred, po, rtol=1e-4, atol=1e-5)
    assert abs(loss - lo) <= 1e-4 * abs(lo)
    assert np.allclose(g, go, rtol=1e-4, atol=1e-5 * np.abs(go).max())


def test_adam_step_parity(mxl, ctx):
    X, Y, M, th = _data(2)
    dims = [16, 32, 32, 10]
    net = mxl.Mlp(ctx, dims, th)
    Xd, Yd, Md = (torch.from_numpy(a).to(DEV) for a in (X, Y, M))
    t64 = th.astype(np.float64)
    m = np.zeros_like(t64)
    v = np.zeros_like(t64)
    for t in (1, 2, 3):
        net.loss_grad(Xd, Yd, Md, 1e-4)
        g = net.grad().astype(np.float64)
        net.adam_step(t, lr=1e-2)
        O.adam_step(t64, g, m, v, t, lr=1e-2)
        assert np.allclose(net.params(), t64, rtol=1e-5, atol=1e-6)
        net.set_params(t64.astype(np.float32))


def test_training_reduces_loss(mxl, ctx):
    from paper_2006_16852_amd import selector as S
    rng = np.random.default_rng(4)
    F = np.abs(rng.standard_normal((120, 16))) * 3
    nc = len(S.CLASSES)
    T = np.exp(rng.standard_normal((120, nc)) * 0.3 + F[:, :1] * np.linspace(-0.2, 0.2, nc))
    T[::7, 6:8] = np.inf
    sel0 = S.train(ctx, F, T, epochs=1)
    sel = S.train(ctx, F, T, epochs=1500)
    Y, Mk = S.labels_from_times(T)

    def mse(s):
        P = s.scores(ctx, F)
        return float(((P - Y) ** 2 * Mk).sum() / Mk.sum())
    assert mse(sel) < 0.5 * mse(sel0)


def test_trained_selector_gain(mxl, ctx):
    """What the trained network gains over the library without it: on the
    50 held-out matrices of the skewed suite (timings measured by this
    library, stored with the package), the network's choices (forward pass
    on the GPU) have a far lower time regret than the library's default
    (CSR vector with the width from the mean row length) and than a hand
    rule, and with the timing fallback it beats the best single fixed class."""
    import json
    import os
    from paper_2006_16852_amd import selector as S
    from paper_2006_16852_amd.train_selector import hand_rule, default_vector
    d = json.load(open(os.path.join(os.path.dirname(S.__file__), "data", "selector_timings_zipf200.json")))
    F = np.array(d["features"])
    T = np.array(d["times_ms"], dtype=float)
    T[T < 0] = np.inf
    classes = list(d["classes"])
    perm = np.random.default_rng(7).permutation(len(F))
    test = np.sort(perm[:len(F) // 4])
    sel = S.Selector.load()
    assert sel.classes == classes
    Ft, Tt = F[test], T[test]
    P = np.where([sel.feasible(f) for f in Ft], sel.scores(ctx, Ft), np.inf)
    net = P.argmin(axis=1)
    default = np.array([classes.index(default_vector(f)) for f in Ft])
    hand = np.array([classes.index(hand_rule(f)) for f in Ft])
    r_net, r_def, r_hand = S.regret(Tt, net), S.regret(Tt, default), S.regret(Tt, hand)
    print(f"[selector gain] regret net {r_net.mean():.4f} default {r_def.mean():.4f} hand {r_hand.mean():.4f}")
    assert np.all(np.isfinite(r_net))
    assert r_net.mean() < 0.1 * r_def.mean()
    assert r_net.mean() < 0.5 * r_hand.mean()
    fb = []
    for p, t in zip(P, Tt):
        order = np.argsort(p)
        top = [k for k in order[:3] if np.isfinite(p[k])]
        fb.append(top[int(np.argmin(t[top]))] if p[order[1]] - p[order[0]] < sel.delta else order[0])
    Ttr = T[np.sort(perm[len(F) // 4:])]
    slow = Ttr / Ttr.min(axis=1, keepdims=True)
    fixed = int(np.argmin([np.exp(np.mean(np.log(np.where(np.isfinite(slow[:, k]), slow[:, k], 1e3))))
                           for k in range(len(classes))]))
    assert S.regret(Tt, np.array(fb)).mean() <= S.regret(Tt, np.full(len(test), fixed)).mean()


def test_structured_held_out_choices(ctx):
    """The regular stencil systems kept out of training (including the
    128^3 27-point and 160^3 anisotropic benchmark systems): from the stored
    timings of that suite, the shipped network's choice (forward pass on the
    GPU) is within 5 % of the fastest class on every one."""
    import json
    import os
    from paper_2006_16852_amd import selector as S
    d = json.load(open(os.path.join(os.path.dirname(S.__file__), "data", "selector_timings_structured.json")))
    sel = S.Selector.load()
    assert list(d["classes"]) == sel.classes
    F = np.array(d["features"])
    T = np.array(d["times_ms"], dtype=float)
    T[T < 0] = np.inf
    held = np.array(d["held_out"], bool)
    assert held.sum() >= 4 and "stencil3d27_128" in [n for n, h in zip(d["names"], held) if h]
    P = np.where([sel.feasible(f) for f in F[held]], sel.scores(ctx, F[held]), np.inf)
    r = S.regret(T[held], P.argmin(axis=1))
    print(f"[selector structured held-out] regret {r}", flush=True)
    assert np.all(r <= 0.05)


# --------------------------------------------------------------- mxl_select
SEL_MATS = ([W.zipf_suite_matrix(m, scale_n=0.02) for m in (1, 8, 40, 77, 150)]
            + [W.stencil_3d27(16), W.aniso_3d7(12), W.edge_matrices()[3], W.edge_matrices()[0]])


def _oracle_choice(S, sel, A):
    """Expected model choice: oracle features, the standardisation written
    out in numpy, the oracle's FP64 forward pass, argmin over the classes
    whose padded storage fits the conversion budget (widths from the
    oracle's own layout routines)."""
    f = O.features(A)
    z = (S.transform(f) - sel.mean) / sel.std
    nc = len(sel.classes)
    _, _, pred = O.mlp_loss_grad(sel.dims, sel.theta, z[None, :], np.zeros((1, nc)),
                                 np.ones((1, nc)), 0.0, want_grad=False, want_pred=True)
    pred = pred[0]
    n_pad = O.pad_rows(A.nrows)
    csr = A.nnz * 12 + (A.nrows + 1) * 4
    budget = min(max(4 * csr, 1 << 20), 32 << 30)
    rows = np.repeat(np.arange(A.nrows), A.row_lengths())
    maxoff = int(np.abs(A.col.astype(np.int64) - rows).max()) if A.nnz else 0
    feas = np.ones(nc, bool)
    for k, c in enumerate(sel.classes):
        fmt, kw = S.CATALOG[c]
        if fmt == "ell":
            w = int(A.row_lengths().max()) if A.nrows else 0
        elif fmt == "hyb":
            w = O.hyb_width(A, kw["hyb_quantile"])
        else:
            continue
        feas[k] = n_pad * w * 12 <= budget and (kw.get("variant", 0) != 2 or maxoff <= 32767)
    return np.where(feas, pred, np.inf), np.abs(z).max()


@pytest.mark.parametrize("A", SEL_MATS, ids=[a.name for a in SEL_MATS])
def test_select_model_parity(mxl, ctx, A):
    """mxl_select (model mode) takes the oracle's choice: same masked
    scores within the FP32 network's tolerance, same argmin whenever the
    oracle's top-2 margin exceeds that tolerance."""
    from paper_2006_16852_amd import selector as S
    sel = S.Selector.load()
    want, maxz = _oracle_choice(S, sel, A)
    k, info = sel.choose(ctx, matrix(mxl, ctx, A), fallback=False)
    got = info["scores"]
    assert np.array_equal(np.isinf(got), np.isinf(want))
    fin = np.isfinite(want)
    assert np.allclose(got[fin], want[fin], rtol=1e-4, atol=1e-4)
    assert abs(info["max_z"] - maxz) <= 1e-7 * max(1.0, maxz)
    srt = np.sort(want[fin])
    if len(srt) < 2 or srt[1] - srt[0] > 1e-3:
        assert k == int(np.argmin(want))
    assert not info["fallback"] and info["ntimed"] == 0


@pytest.mark.parametrize("A", [W.zipf_suite_matrix(12, scale_n=0.05), W.edge_matrices()[3]],
                         ids=lambda a: a.name)
def test_select_exhaustive_and_fallback(mxl, ctx, A):
    """Exhaustive mode times exactly the feasible classes and returns the
    fastest; a selector that is always unsure times its top 3 and returns
    the fastest of those; without vectors it never times."""
    from paper_2006_16852_amd import selector as S
    base = S.Selector.load()
    want, _ = _oracle_choice(S, base, A)
    M = matrix(mxl, ctx, A)
    x = torch.from_numpy(W.uniform_vec(A.ncols, 3)).to(DEV)
    y = torch.empty(A.nrows, dtype=torch.float64, device=DEV)
    k, t = S.exhaustive(ctx, M, x, y, reps=3, classes=base.classes)
    assert np.array_equal(np.isfinite(t), np.isfinite(want))
    assert k == int(np.argmin(t))
    unsure = S.Selector(base.theta, base.mean, base.std, delta=1e9, zmax=base.zmax)
    k2, info = unsure.choose(ctx, M, x, y, reps=3)
    order = np.argsort(info["scores"], kind="stable")
    top = [int(c) for c in order[:3] if np.isfinite(info["scores"][c])]
    timed = np.flatnonzero(~np.isnan(info["times_ms"]))
    assert info["fallback"] and sorted(timed.tolist()) == sorted(top) and info["ntimed"] == len(top)
    assert k2 == top[int(np.argmin(info["times_ms"][top]))]
    assert info["best_ms"] == info["times_ms"][k2]
    k3, info3 = unsure.choose(ctx, M, None, None)
    assert not info3["fallback"] and k3 == top[0]


def test_select_errors(mxl, ctx):
    from paper_2006_16852_amd import selector as S
    sel = S.Selector.load()
    M = matrix(mxl, ctx, W.stencil_2d5(8))
    h = sel.handle(ctx)
    with pytest.raises(mxl.MxlError) as e:
        h.select(M, mxl.SELECT_EXHAUSTIVE)
    assert e.value.status == mxl.ERR_INVALID_ARG
    with pytest.raises(mxl.MxlError) as e:
        h.select(M, 7)
    assert e.value.status == mxl.ERR_INVALID_ARG
    with pytest.raises(mxl.MxlError) as e:
        mxl.SelectorHandle(ctx, [("csr", {})], sel.dims, sel.theta, sel.mean, sel.std, S.LOG_FEATS)
    assert e.value.status == mxl.ERR_DIM_MISMATCH
    with pytest.raises(mxl.MxlError) as e:
        mxl.SelectorHandle(ctx, [S.CATALOG[c] for c in sel.classes], sel.dims, sel.theta, sel.mean,
                           np.zeros(16), S.LOG_FEATS)
    assert e.value.status == mxl.ERR_INVALID_ARG
