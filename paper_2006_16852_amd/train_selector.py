"""Train and evaluate the format/kernel selector on the 200-matrix
row-length-skewed suite (on one GPU).

For every matrix m (generated from its seed, never stored): the 16 features
on the GPU, then the median time of every feasible (format, variant) class
(20 repetitions, last-level cache flushed before each).  Matrices 0..199 are
split 150 train / 50 test (seed 7).  The MLP is trained on the GPU by the
library's kernels; the test set reports the time regret of the selector,
the selector with its timing fallback, the best single fixed class and a
hand rule, plus their performance profiles.

    python -m paper_2006_16852_amd.train_selector --out DIR [--count 200] [--scale 1.0]
        [--timings FILE] [--structured | --structured-timings FILE]

Writes DIR/selector_timings.json (features + times), DIR/selector_eval.json
and DIR/selector_weights.json.  With --structured the regular stencil suite
(2D 5-point, 3D 27-point, anisotropic 7-point, convection-diffusion at
several sizes) joins the training set except its held-out matrices, which
are reported separately.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import paper_2006_16852_amd as mxl  # noqa: E402
from paper_2006_16852_amd import selector as S  # noqa: E402
import workloads as W  # noqa: E402


def hand_rule(f: np.ndarray) -> str:
    """No-network baseline: a fixed rule on mean and spread of row lengths."""
    mu, cv = f[2], f[4]
    if cv < 0.3 and S.ell_feasible(f):
        return "ell"
    if cv > 1.5:
        return "csr_merge"
    return "csr_vec16" if mu <= 16 else "csr_vec64"


def default_vector(f: np.ndarray) -> str:
    """The library's default CSR kernel: vector width from the mean row length."""
    return "csr_vec4" if f[2] <= 6 else ("csr_vec16" if f[2] <= 24 else "csr_vec64")


def collect(ctx, idx, scale, reps, log, classes=S.CLASSES):
    feats, times, meta = [], [], []
    dev = f"cuda:{ctx.device}"
    for m in idx:
        t0 = time.time()
        A = W.zipf_suite_matrix(m, scale_n=scale)
        rp = torch.from_numpy(A.row_ptr).to(dev)
        col = torch.from_numpy(A.col).to(dev)
        val = torch.from_numpy(A.val).to(dev)
        base = mxl.csr(ctx, rp, col, val)
        x = torch.from_numpy(W.uniform_vec(A.ncols, 2000 + m)).to(dev)
        y = torch.empty(A.nrows, dtype=torch.float64, device=dev)
        f = base.features()
        ws = A.nnz * 12 + A.nrows * 20
        t = S.time_classes(base, x, y, reps=reps, flush=ws < (512 << 20), classes=classes)
        feats.append(f)
        times.append(t)
        meta.append(dict(m=int(m), n=int(A.nrows), nnz=int(A.nnz)))
        log(f"[collect] m={m} n={A.nrows} nnz={A.nnz} best={classes[int(np.argmin(t))]} "
            f"{time.time() - t0:.1f}s")
        del base, rp, col, val, x, y, A
        torch.cuda.empty_cache()
    return np.array(feats), np.array(times), meta


def collect_structured(ctx, reps, log, classes=S.CLASSES):
    """Features and class times of the regular stencil suite
    (workloads.structured_suite); returns F, T, names, held_out flags."""
    feats, times, names, held = [], [], [], []
    dev = f"cuda:{ctx.device}"
    for name, build, ho in W.structured_suite():
        t0 = time.time()
        A = build()
        base = mxl.csr(ctx, torch.from_numpy(A.row_ptr).to(dev), torch.from_numpy(A.col).to(dev),
                       torch.from_numpy(A.val).to(dev))
        x = torch.from_numpy(W.uniform_vec(A.ncols, 2)).to(dev)
        y = torch.empty(A.nrows, dtype=torch.float64, device=dev)
        f = base.features()
        ws = A.nnz * 12 + A.nrows * 20
        t = S.time_classes(base, x, y, reps=reps, flush=ws < (512 << 20), classes=classes)
        feats.append(f)
        times.append(t)
        names.append(name)
        held.append(bool(ho))
        log(f"[collect] {name} n={A.nrows} nnz={A.nnz} best={classes[int(np.argmin(t))]} {time.time() - t0:.1f}s")
        del base, x, y, A
        torch.cuda.empty_cache()
    return np.array(feats), np.array(times), names, np.array(held)


def evaluate(ctx, sel, F, T, fallback_times=None):
    pred = np.array([int(np.argmin(np.where(sel.feasible(f), s, np.inf)))
                     for f, s in zip(F, sel.scores(ctx, F))])
    return pred


def suite_bandwidth(T, meta, test, choice_test, classes):
    """SpMV bandwidth over the suite in CSR-equivalent GB/s (the bytes a CSR
    product must move: nnz (8+4) + (n+1) 4 + 2 n 8, divided by the measured
    time), so that formats compare on the same work: quartiles per class,
    for the fastest class of every matrix, and for the network's choices on
    the held-out matrices."""
    n = np.array([m["n"] for m in meta], float)
    nnz = np.array([m["nnz"] for m in meta], float)
    byts = nnz * 12 + (n + 1) * 4 + 16 * n
    G = np.where(np.isfinite(T), byts[:, None] / (T * 1e-3) / 1e9, np.nan)

    def q(v):
        v = v[np.isfinite(v)]
        return dict(p25=round(float(np.quantile(v, 0.25)), 1), median=round(float(np.median(v)), 1),
                    p75=round(float(np.quantile(v, 0.75)), 1), count=int(v.size)) if v.size else None
    out = {c: q(G[:, k]) for k, c in enumerate(classes)}
    out["best_class"] = q(np.nanmax(G, axis=1))
    out["selector_test"] = q(G[test, choice_test] if len(test) else np.array([]))
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", required=True)
    ap.add_argument("--count", type=int, default=200)
    ap.add_argument("--scale", type=float, default=1.0)
    ap.add_argument("--reps", type=int, default=20)
    ap.add_argument("--epochs", type=int, default=4000)
    ap.add_argument("--lr", type=float, default=3e-3)
    ap.add_argument("--lam", type=float, default=1e-3)
    ap.add_argument("--timings", default=None, help="reuse a timings file instead of measuring")
    ap.add_argument("--structured", action="store_true",
                    help="add the regular stencil suite (its non-held-out part) to the training set")
    ap.add_argument("--structured-timings", default=None, help="reuse a structured-suite timings file")
    args = ap.parse_args()
    os.makedirs(args.out, exist_ok=True)

    def log(s):
        print(s, flush=True)

    ctx = mxl.Context(0)
    if args.timings:
        d = json.load(open(args.timings))
        F, T, meta = np.array(d["features"]), np.array(d["times_ms"]), d["meta"]
        T = np.where(np.array(T) < 0, np.inf, T)
        classes = list(d["classes"])
    else:
        classes = list(S.CLASSES)
        F, T, meta = collect(ctx, range(args.count), args.scale, args.reps, log, classes)
        json.dump(dict(classes=classes, features=F.tolist(),
                       times_ms=np.where(np.isfinite(T), T, -1.0).tolist(), meta=meta,
                       reps=args.reps, scale=args.scale),
                  open(os.path.join(args.out, "selector_timings.json"), "w"))
    n = len(F)
    perm = np.random.default_rng(7).permutation(n)
    ntest = max(1, n // 4)
    test, train_idx = np.sort(perm[:ntest]), np.sort(perm[ntest:])
    Fs = Ts = None
    if args.structured or args.structured_timings:
        if args.structured_timings:
            d = json.load(open(args.structured_timings))
            assert list(d["classes"]) == classes
            Fs, Ts = np.array(d["features"]), np.array(d["times_ms"], dtype=float)
            Ts = np.where(Ts < 0, np.inf, Ts)
            snames, sheld = d["names"], np.array(d["held_out"], bool)
        else:
            Fs, Ts, snames, sheld = collect_structured(ctx, args.reps, log, classes)
            json.dump(dict(classes=classes, features=Fs.tolist(), times_ms=np.where(np.isfinite(Ts), Ts, -1.0).tolist(),
                           names=snames, held_out=sheld.tolist(), reps=args.reps),
                      open(os.path.join(args.out, "selector_structured_timings.json"), "w"))
    Ftrain, Ttrain = F[train_idx], T[train_idx]
    if Fs is not None:
        Ftrain = np.concatenate([Ftrain, Fs[~sheld]])
        Ttrain = np.concatenate([Ttrain, Ts[~sheld]])
    t0 = time.time()
    sel = S.train(ctx, Ftrain, Ttrain, classes, epochs=args.epochs, lr=args.lr, lam=args.lam)
    train_s = time.time() - t0
    sel.save(os.path.join(args.out, "selector_weights.json"))
    Ft, Tt = F[test], T[test]
    choice_net = evaluate(ctx, sel, Ft, Tt)
    # fallback uses the measured test times of the top-3 (the same labels the regret is scored on)
    scores = sel.scores(ctx, Ft)
    choice_fb = []
    nfb = 0
    for f, s, t in zip(Ft, scores, Tt):
        s = np.where(sel.feasible(f), s, np.inf)
        order = np.argsort(s)
        z = np.abs(sel.standardise(f))
        unsure = (s[order[1]] - s[order[0]] < sel.delta) or np.any(z > sel.zmax)
        if unsure:
            nfb += 1
            top = [k for k in order[:3] if np.isfinite(s[k])]
            choice_fb.append(int(top[int(np.argmin(t[top]))]))
        else:
            choice_fb.append(int(order[0]))
    choice_fb = np.array(choice_fb)
    # best single fixed class on the training set (by geometric-mean slowdown)
    Ttr = T[train_idx]
    slow = Ttr / Ttr.min(axis=1, keepdims=True)
    gm = [np.exp(np.mean(np.log(np.where(np.isfinite(slow[:, k]), slow[:, k], 1e3))))
          for k in range(len(classes))]
    fixed = int(np.argmin(gm))
    merge = classes.index("csr_merge")  # always feasible
    choice_fixed = np.array([fixed if np.isfinite(t[fixed]) else merge for t in Tt])
    choice_hand = np.array([classes.index(hand_rule(f)) if np.isfinite(t[classes.index(hand_rule(f))]) else merge
                            for f, t in zip(Ft, Tt)])
    choice_default = np.array([classes.index(default_vector(f)) for f in Ft])

    def stats(ch):
        r = S.regret(Tt, ch)
        return dict(mean=float(r.mean()), geomean=float(np.exp(np.mean(np.log1p(r))) - 1),
                    p90=float(np.quantile(r, 0.9)), max=float(r.max()),
                    exact=float(np.mean(r <= 1e-12)))

    ev = dict(n_train=int(len(train_idx)), n_test=int(len(test)), train_seconds=train_s,
              epochs=args.epochs, lr=args.lr, weight_decay=args.lam, fixed_class=classes[fixed], fallback_used=int(nfb),
              regret=dict(selector=stats(choice_net), selector_fallback=stats(choice_fb),
                          best_fixed=stats(choice_fixed), hand_rule=stats(choice_hand),
                          default_vector=stats(choice_default)),
              profile=S.performance_profile(Tt, dict(selector=choice_net, selector_fallback=choice_fb,
                                                     best_fixed=choice_fixed, hand_rule=choice_hand,
                                                     default_vector=choice_default)),
              classes=classes,
              class_wins={c: int(np.sum(np.argmin(T, axis=1) == k)) for k, c in enumerate(classes)})
    ev["suite_bandwidth"] = suite_bandwidth(T, meta, test, choice_net, classes)
    if Fs is not None:
        sc = sel.scores(ctx, Fs)
        rows = {}
        for k, (f, s_, t) in enumerate(zip(Fs, sc, Ts)):
            s_ = np.where(sel.feasible(f), s_, np.inf)
            order = np.argsort(s_)
            z = np.abs(sel.standardise(f))
            unsure = (s_[order[1]] - s_[order[0]] < sel.delta) or bool(np.any(z > sel.zmax))
            top = [j for j in order[:3] if np.isfinite(s_[j])]
            fbk = int(top[int(np.argmin(t[top]))]) if unsure else int(order[0])
            rows[snames[k]] = dict(held_out=bool(sheld[k]), best=classes[int(np.argmin(t))],
                                   network=classes[int(order[0])], network_regret=float(t[order[0]] / t.min() - 1.0),
                                   fallback_used=bool(unsure), with_fallback=classes[fbk],
                                   with_fallback_regret=float(t[fbk] / t.min() - 1.0))
        ev["structured"] = dict(n_train=int((~sheld).sum()), n_held_out=int(sheld.sum()), matrices=rows)
        ev["n_train"] = int(len(Ftrain))
    json.dump(ev, open(os.path.join(args.out, "selector_eval.json"), "w"), indent=1)
    log(json.dumps(ev["regret"]))


if __name__ == "__main__":
    main()
