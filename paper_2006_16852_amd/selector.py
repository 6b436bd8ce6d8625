"""Learned format/kernel selector.

The paper forks at run time over matrix format and kernel variant (Sec. 7.2)
and compares kernels with a performance profile (Sec. 7.3).  This module
learns that fork: 16 structural features of a CSR matrix (computed on the GPU
by ``mxl_features``) go through a small MLP (trained on the GPU by the
library's own forward/backward/Adam kernels) that predicts, for each
(format, variant) class, s_c ~ log(t_c / t_best).  The choice is the argmin
over feasible classes; when the network is unsure (top-2 margin below
``delta``) or the matrix lies outside the training distribution (a
standardised feature beyond ``zmax``) it falls back to timing the top-3
candidates.  Exhaustive timing (``mxl_time_apply``) produces the labels and
scores the choice (time regret = t_choice / t_best - 1).

A trained selector carries the names of its classes, so weights trained on
one set of classes stay valid when the catalog grows.
"""
from __future__ import annotations

import json
import math
import os

import numpy as np
import torch

from . import Mlp, MxlError, ERR_INFEASIBLE_FORMAT, SelectorHandle, SELECT_MODEL, \
    SELECT_EXHAUSTIVE, SELECT_MODEL_FALLBACK

HERE = os.path.dirname(os.path.abspath(__file__))
WEIGHTS = os.path.join(HERE, "selector_weights.json")

# name -> (format, convert kwargs)
CATALOG = {
    "csr_scalar": ("csr", dict(variant=0)),
    "csr_vec4": ("csr", dict(variant=1, vector_width=4)),
    "csr_vec16": ("csr", dict(variant=1, vector_width=16)),
    "csr_vec64": ("csr", dict(variant=1, vector_width=64)),
    "csr_merge": ("csr", dict(variant=2)),
    "coo": ("coo", {}),
    "ell": ("ell", {}),
    "ell_lds": ("ell", dict(variant=1)),
    "hyb66": ("hyb", dict(hyb_quantile=0.66)),
    "hyb90": ("hyb", dict(hyb_quantile=0.9)),
    "csr_stream": ("csr", dict(variant=3)),
    "ell16": ("ell", dict(variant=2)),
}
CLASSES = list(CATALOG)  # the classes a new selector is trained on
HIDDEN = [32, 32]
# heavy-tailed features enter through log1p before standardisation
LOG_FEATS = [5, 6, 7, 8, 9, 11]


def dims_for(nclasses: int):
    return [16] + HIDDEN + [nclasses]


def transform(F: np.ndarray) -> np.ndarray:
    F = np.array(F, dtype=np.float64, copy=True)
    F[..., LOG_FEATS] = np.log1p(np.maximum(F[..., LOG_FEATS], 0.0))
    return F


def _n_nnz(f):
    n = int(round(10 ** f[0]))
    nnz = int(round(10 ** f[1])) if f[2] > 0 else 0
    return n, nnz


def ell_feasible(f: np.ndarray, vt: int = 8) -> bool:
    """Mirror of the library's padded-storage budget from the features (n,
    nnz, max row length): n_pad * w * (vt + 4) <= min(max(4 CSR, 1 MiB),
    32 GiB); the budget is the same for every ELL index width."""
    n, nnz = _n_nnz(f)
    n_pad = math.ceil(n / 64) * 64
    ell = n_pad * f[5] * (vt + 4)
    csr = nnz * (vt + 4) + (n + 1) * 4
    return ell <= min(max(4 * csr, 1 << 20), 32 * (1 << 30))


def ell16_feasible(f: np.ndarray) -> bool:
    """16-bit offsets also need max |col - row| <= 32767 (feature 12 is that
    maximum divided by n)."""
    n, _ = _n_nnz(f)
    return ell_feasible(f) and round(f[12] * n) <= 32767


def feasible_mask(f: np.ndarray, classes=CLASSES) -> np.ndarray:
    m = np.ones(len(classes), bool)
    for k, c in enumerate(classes):
        if c in ("ell", "ell_lds"):
            m[k] = ell_feasible(f)
        elif c == "ell16":
            m[k] = ell16_feasible(f)
    return m


def convert(base, name: str):
    fmt, kw = CATALOG[name]
    return base.convert(fmt, **kw)


def time_classes(base, x, y, reps: int = 20, flush: bool = True, classes=CLASSES):
    """Median ms of every class (inf when the format is infeasible)."""
    t = np.full(len(classes), np.inf)
    for k, c in enumerate(classes):
        try:
            op = convert(base, c)
        except MxlError as e:
            if e.status == ERR_INFEASIBLE_FORMAT:
                continue
            raise
        t[k] = op.time_apply(x, y, reps=reps, flush=flush)
        del op
    return t


def labels_from_times(T: np.ndarray):
    """y_c = log(t_c / t_best), mask 0 for infeasible classes."""
    best = np.min(T, axis=1, keepdims=True)
    M = np.isfinite(T).astype(np.float64)
    Y = np.where(M > 0, np.log(np.where(M > 0, T, 1.0) / best), 0.0)
    return Y, M


def he_init(dims, seed: int = 0) -> np.ndarray:
    rng = np.random.default_rng(seed)
    parts = []
    for i in range(len(dims) - 1):
        parts.append(rng.standard_normal(dims[i + 1] * dims[i]) * math.sqrt(2.0 / dims[i]))
        parts.append(np.zeros(dims[i + 1]))
    return np.concatenate(parts)


class Selector:
    def __init__(self, theta, mean, std, classes=CLASSES, delta=0.05, zmax=4.0):
        self.classes = list(classes)
        self.dims = dims_for(len(self.classes))
        self.theta = np.asarray(theta, np.float64)
        self.mean = np.asarray(mean, np.float64)
        self.std = np.asarray(std, np.float64)
        self.delta = delta
        self.zmax = zmax
        self._mlp = None
        self._handle = None

    # ---------------------------------------------------------------- io
    def to_json(self) -> dict:
        return dict(dims=self.dims, classes=self.classes, theta=self.theta.tolist(),
                    mean=self.mean.tolist(), std=self.std.tolist(), delta=self.delta,
                    zmax=self.zmax, log_features=LOG_FEATS)

    def save(self, path: str = WEIGHTS):
        json.dump(self.to_json(), open(path, "w"))

    @classmethod
    def load(cls, path: str = WEIGHTS) -> "Selector":
        d = json.load(open(path))
        return cls(d["theta"], d["mean"], d["std"], d["classes"], d.get("delta", 0.05), d.get("zmax", 4.0))

    # ----------------------------------------------------------- predict
    def standardise(self, F) -> np.ndarray:
        return (transform(F) - self.mean) / self.std

    def feasible(self, f) -> np.ndarray:
        return feasible_mask(f, self.classes)

    def scores(self, ctx, F) -> np.ndarray:
        """Predicted log(t_c / t_best) per class, computed on the GPU."""
        Z = np.atleast_2d(self.standardise(F)).astype(np.float32)
        if self._mlp is None or self._mlp.ctx is not ctx:
            self._mlp = Mlp(ctx, self.dims, self.theta.astype(np.float32))
        X = torch.from_numpy(Z).to(f"cuda:{ctx.device}")
        return self._mlp.forward(X).cpu().numpy().astype(np.float64)

    def handle(self, ctx) -> SelectorHandle:
        """The selector as a library object (features, standardisation, MLP
        and fallback timing all run inside mxl_select)."""
        if self._handle is None or self._handle.ctx is not ctx:
            self._handle = SelectorHandle(ctx, [CATALOG[c] for c in self.classes], self.dims,
                                          self.theta.astype(np.float32), self.mean, self.std,
                                          LOG_FEATS, self.delta, self.zmax)
        return self._handle

    def choose(self, ctx, base, x=None, y=None, fallback: bool = True, reps: int = 5):
        """Returns (class index into self.classes, info dict) from mxl_select."""
        mode = SELECT_MODEL_FALLBACK if fallback else SELECT_MODEL
        return self.handle(ctx).select(base, mode, x, y, reps=reps)


def exhaustive(ctx, base, x, y, reps: int = 20, classes=CLASSES):
    """Time every feasible class inside the library; returns (class, times_ms)."""
    d = dims_for(len(classes))
    n = sum(d[i + 1] * d[i] + d[i + 1] for i in range(len(d) - 1))
    sel = Selector(np.zeros(n), np.zeros(16), np.ones(16), classes)
    k, info = sel.handle(ctx).select(base, SELECT_EXHAUSTIVE, x, y, reps=reps)
    return k, np.where(np.isnan(info["times_ms"]), np.inf, info["times_ms"])


def train(ctx, F: np.ndarray, T: np.ndarray, classes=CLASSES, epochs: int = 4000, lr: float = 3e-3,
          lam: float = 1e-3, seed: int = 0) -> Selector:
    """Fit the MLP on the GPU (full batch, Adam) to log time ratios; T has
    one column per entry of `classes`.

    Defaults chosen by 5-fold cross-validation of the mean time regret on the
    training split of the skewed suite (epochs in {2000, 4000}, lr in
    {1e-3, 3e-3}, weight decay in {1e-4, 1e-3, 1e-2}, widths 32 and 64)."""
    classes = list(classes)
    assert T.shape[1] == len(classes)
    dims = dims_for(len(classes))
    Ft = transform(F)
    mean = Ft.mean(axis=0)
    std = Ft.std(axis=0)
    std[std == 0] = 1.0
    Z = ((Ft - mean) / std).astype(np.float32)
    Y, M = labels_from_times(T)
    dev = f"cuda:{ctx.device}"
    X = torch.from_numpy(Z).to(dev)
    Yd = torch.from_numpy(Y.astype(np.float32)).to(dev)
    Md = torch.from_numpy(M.astype(np.float32)).to(dev)
    net = Mlp(ctx, dims, he_init(dims, seed).astype(np.float32))
    for t in range(1, epochs + 1):
        net.loss_grad(X, Yd, Md, lam)
        net.adam_step(t, lr=lr)
    return Selector(net.params().astype(np.float64), mean, std, classes)


def regret(T: np.ndarray, choice: np.ndarray) -> np.ndarray:
    best = np.min(T, axis=1)
    return T[np.arange(len(choice)), choice] / best - 1.0


def performance_profile(T: np.ndarray, choices: dict, taus=(1.0, 1.05, 1.1, 1.25, 1.5, 2.0, 3.0)):
    """Fraction of matrices a policy solves within slowdown tau of the best
    (the performance-profile view of Sec. 7.3)."""
    best = np.min(T, axis=1)
    out = {}
    for name, ch in choices.items():
        r = T[np.arange(len(ch)), ch] / best
        out[name] = {f"{tau:g}": float(np.mean(r <= tau + 1e-12)) for tau in taus}
    return out
