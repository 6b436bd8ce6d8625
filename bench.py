#!/usr/bin/env python
"""Benchmark of the sparse-operator hot path on one MI355X.

Workload: the 3D 27-point stencil on a 128^3 grid (n = 2,097,152,
nnz = 55,742,968), FP64 values 26 / -1, x* ~ U[-1,1) (seed 2), b = A x*.
One step = one pass of the whole hot path over the HBM-resident system:
y = A x once in every storage format (CSR in the selected kernel variant,
COO, ELL, HYB) and one Jacobi-preconditioned CG solve from x0 = 0 to
||r|| <= 1e-10 ||b|| (fused SpMV+dot, fused update kernels, device-side
criterion).  `value` is the step's algorithmic bytes divided by its time
(GB/s).  The roofline block reports the dominant kernel -- the SpMV inside
the CG loop -- timed live with HIP events on the solver's stream.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "SpMV GB/s (% HBM peak); CG time-to-1e-10 residual, FP64 vs mixed/learned"
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_stencil27_128.json")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def spmv_bytes(fmt, n, nnz, desc, vt=8, it=4, beta_nonzero=False):
    """Algorithmic bytes of one y = A x: matrix arrays once, x once, y once."""
    extra = n * vt if beta_nonzero else 0
    if fmt == "csr":
        return nnz * (vt + it) + (n + 1) * it + 2 * n * vt + extra
    if fmt == "coo":
        return nnz * (vt + 2 * it) + 2 * n * vt + extra
    if fmt == "ell":
        return n * desc["ell_width"] * (vt + it) + 2 * n * vt + extra
    if fmt == "ell16":  # 16-bit column offsets
        return n * desc["ell_width"] * (vt + 2) + 2 * n * vt + extra
    if fmt == "hyb":
        return n * desc["ell_width"] * (vt + it) + desc["tail_nnz"] * (vt + 2 * it) + 2 * n * vt + extra
    raise ValueError(fmt)


def source_digest():
    h = hashlib.sha256()
    for f in ("spmv.hip", "device_common.hpp"):
        h.update(open(os.path.join(ROOT, "paper_2006_16852_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def cpu_baseline(A, x, b, sel_fmt):
    """The oracle as it stands (plain FP64 C, one thread) on a bounded sample
    of the same step: one SpMV per format and 25 Jacobi-PCG iterations."""
    import oracle as O
    O.build(force=False)
    n, nnz = A.nrows, A.nnz
    coo_row = O.csr_to_coo(A)
    w, n_pad, ec, ev = O.csr_to_ell(A)
    H = O.csr_to_hyb(A, q=0.9)
    d, _ = O.jacobi_dinv(A)
    iters = 25
    t0 = time.perf_counter()
    O.spmv(A, x)
    O.coo_spmv(n, coo_row, A.col, A.val, x)
    O.ell_spmv(n, n_pad, w, ec, ev, x)
    O.hyb_spmv(n, H, x)
    r = O.pcg(A, b, dinv=d, max_iters=iters, reduction=0.0)
    dt = time.perf_counter() - t0
    byts = (spmv_bytes("csr", n, nnz, {}) + spmv_bytes("coo", n, nnz, {})
            + spmv_bytes("ell", n, nnz, {"ell_width": w})
            + spmv_bytes("hyb", n, nnz, {"ell_width": H["k"], "tail_nnz": H["tail_row"].size})
            + (spmv_bytes("csr", n, nnz, {}, beta_nonzero=True) + 5 * n * 8)
            + r["iterations"] * (spmv_bytes("csr", n, nnz, {}) + 10 * n * 8))
    return {"value": round(byts / dt / 1e9, 3), "unit": "GB/s", "cores": 1, "kind": "oracle",
            "sample": f"4 SpMVs (csr, coo, ell, hyb) + {r['iterations']} Jacobi-PCG iterations "
                      f"(CSR) on the 128^3 27-point system, {dt:.2f} s on the host"}


def mxl_catalog(name):
    from paper_2006_16852_amd.selector import CATALOG
    return CATALOG[name]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--grid", type=int, default=128)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--workload", default="stencil27",
                    choices=["stencil27", "aniso_ir", "poisson2d", "batch", "overhead", "stream", "bicgstab", "stencil_mf",
                             "gmres"])
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on exactly one GPU: the library has no multi-GPU path (a sharded solve "
              "would split rows into contiguous slabs, exchange halo entries of the SpMV input and "
              "all-reduce the scalar dot products).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2006_16852_amd as mxl
    import workloads as W

    if args.workload != "stencil27":
        import bench_extra
        return bench_extra.run(args)

    dev = "cuda:0"
    N = args.grid
    log(f"[bench] generating 27-point stencil {N}^3")
    A = W.stencil_3d27(N)
    n, nnz = A.nrows, A.nnz
    xs = W.uniform_vec(n, 2)
    ctx = mxl.Context(0)
    rp = torch.from_numpy(A.row_ptr).to(dev)
    col = torch.from_numpy(A.col).to(dev)
    val = torch.from_numpy(A.val).to(dev)
    def setup_ms(fn):
        torch.cuda.synchronize()
        t = time.perf_counter()
        out = fn()
        torch.cuda.synchronize()
        return out, round((time.perf_counter() - t) * 1e3, 3)

    base, t_validate = setup_ms(lambda: mxl.csr(ctx, rp, col, val, validate=True))
    xd = torch.from_numpy(xs).to(dev)
    bd = torch.empty(n, dtype=torch.float64, device=dev)
    base.apply(xd, bd)                      # b = A x* on the GPU
    yd = torch.empty(n, dtype=torch.float64, device=dev)

    log("[bench] building formats")
    builds = {
        "csr_vec32": lambda: base.convert("csr", variant=mxl.CSR_VECTOR, vector_width=32),
        "csr_merge": lambda: base.convert("csr", variant=mxl.CSR_MERGE),
        "csr_stream": lambda: base.convert("csr", variant=mxl.CSR_STREAM),
        "coo": lambda: base.convert("coo"),
        "ell": lambda: base.convert("ell"),
        "ell16": lambda: base.convert("ell", variant=mxl.ELL_DELTA16),
        "hyb": lambda: base.convert("hyb", hyb_quantile=0.9),
    }
    ops, t_setup = {}, {"validate_csr": t_validate}
    for k, fn in builds.items():
        ops[k], t_setup[k] = setup_ms(fn)
    fmt_of = {"csr_vec32": "csr", "csr_merge": "csr", "csr_stream": "csr", "coo": "coo", "ell": "ell",
              "ell16": "ell16", "hyb": "hyb"}
    descs = {k: v.describe() for k, v in ops.items()}
    # exhaustive timing picks the operator used inside CG
    t_sel = {k: ops[k].time_apply(xd, yd, reps=20)
             for k in ("csr_vec32", "csr_merge", "csr_stream", "ell", "ell16")}
    sel = min(t_sel, key=t_sel.get)
    log(f"[bench] selection times (ms): {t_sel} -> {sel}")
    csr_best = min(("csr_vec32", "csr_merge", "csr_stream"), key=t_sel.get)
    ell_best = min(("ell", "ell16"), key=t_sel.get)
    spmv_set = [csr_best, "coo", ell_best, "hyb"]
    # achievable-bandwidth references on this GPU (STREAM-style, 2^26 doubles)
    sa = torch.rand(1 << 26, dtype=torch.float64, device=dev)
    sb = torch.rand(1 << 26, dtype=torch.float64, device=dev)
    sc = torch.empty(1 << 26, dtype=torch.float64, device=dev)
    ref_gbs = {op: round(nb / mxl.stream_bench(ctx, op, sa, sb, sc, reps=10) / 1e6, 1)
               for op, nb in (("triad", 24 << 26), ("dot", 16 << 26))}
    del sa, sb, sc
    M = ops[sel]
    P, t_setup["jacobi"] = setup_ms(lambda: mxl.jacobi(M))
    S = mxl.solver("cg", M, P, max_iters=5000, reduction=1e-10, check_every=16)
    x = torch.zeros(n, dtype=torch.float64, device=dev)

    evs = {k: [] for k in spmv_set}
    infos = []

    def step(record):
        for k in spmv_set:
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            ops[k].apply(xd, yd)
            e1.record()
            if record:
                evs[k].append((e0, e1))
        x.zero_()
        info = S.solve(bd, x, time_spmv=16)  # events on every 16th product
        if record:
            infos.append(info)

    for _ in range(args.warmup):
        step(False)
    torch.cuda.synchronize()
    log(f"[bench] timing {args.steps} steps")
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step(True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    step_s = (t1 - t0) / args.steps

    # correctness guard of the timed result (recomputed in FP64 on the GPU)
    r = bd.clone()
    base.apply(x, r, -1.0, 1.0)
    true_rel = float(torch.linalg.norm(r) / torch.linalg.norm(bd))

    # Outside the timed step: the metric's comparisons on the same system.
    # Mixed precision: FP32-inner / FP64-outer refinement on the same operator.
    # Learned: the trained selector's choice against the exhaustive timing.
    log("[bench] comparisons: mixed-precision refinement and the learned selector")
    comp = {"fp64_cg_ms": None}
    ir_runs = {}
    for tin in (1e-2, 1e-3):
        I = mxl.ir(M, outer=dict(max_iters=60, reduction=1e-10),
                   inner=dict(reduction=tin, max_iters=10_000, check_every=16))
        ts = []
        for _ in range(3):
            x.zero_()
            torch.cuda.synchronize()
            t = time.perf_counter()
            iinfo = I.solve(bd, x)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t)
        rr = bd.clone()
        base.apply(x, rr, -1.0, 1.0)
        ir_runs[f"inner{tin:g}"] = {"ms": round(float(np.median(ts)) * 1e3, 3), "corrections": iinfo["iterations"],
                                    "inner_iterations": iinfo["inner_iterations"],
                                    "true_rel_residual": float(torch.linalg.norm(rr) / torch.linalg.norm(bd))}
        del I
    comp["mixed_ir"] = ir_runs
    from paper_2006_16852_amd.selector import Selector
    learned = Selector.load()
    k_model, _ = learned.choose(ctx, base, xd, yd, fallback=False)
    k_fb, _ = learned.choose(ctx, base, xd, yd, fallback=True)
    pick = {"model": learned.classes[k_model], "model_with_fallback": learned.classes[k_fb]}
    t_pick = {}
    for name in set(pick.values()):
        fmt, kw = mxl_catalog(name)
        op = base.convert(fmt, **kw)
        t_pick[name] = op.time_apply(xd, yd, reps=20)
        del op
    best_t = min(t_sel.values())
    comp["learned_selector"] = {"choice": pick, "exhaustive_choice": sel,
                                "regret": {k: round(t_pick[v] / best_t - 1.0, 4) for k, v in pick.items()}}

    spmv_detail = {}
    step_bytes = 0
    for k in spmv_set:
        ms = float(np.median([a.elapsed_time(b) for a, b in evs[k]]))
        byts = spmv_bytes(fmt_of[k], n, nnz, descs[k])
        step_bytes += byts
        spmv_detail[k] = {"us": round(ms * 1e3, 2), "GBs": round(byts / ms / 1e6, 1),
                          "frac_hbm": round(byts / ms / 1e6 / HBM_PEAK_GBS, 4),
                          "alg_MB": round(byts / 1e6, 2), "stored_MB": round(descs[k]["stored_bytes"] / 1e6, 2)}
    its = [i["iterations"] for i in infos]
    cg_spmv = spmv_bytes(fmt_of[sel], n, nnz, descs[sel])
    cg_iter_bytes = cg_spmv + 10 * n * 8
    cg_setup_bytes = spmv_bytes(fmt_of[sel], n, nnz, descs[sel], beta_nonzero=True) + 5 * n * 8
    cg_bytes = float(np.mean(its)) * cg_iter_bytes + cg_setup_bytes
    step_bytes += cg_bytes
    cg_ms = float(np.median([i["seconds"] for i in infos])) * 1e3
    comp["fp64_cg_ms"] = round(cg_ms, 3)
    best_ir = min(v["ms"] for v in comp["mixed_ir"].values())
    comp["ir_speedup_vs_fp64"] = round(cg_ms / best_ir, 3)
    launch_ms = sum(i["spmv_ms"] for i in infos) / max(1, sum(i["spmv_timed"] for i in infos))
    achieved = cg_spmv / (launch_ms * 1e-3) / 1e9

    traffic = None
    if os.path.exists(TRAFFIC_FILE):
        tf = json.load(open(TRAFFIC_FILE))
        if tf.get("source_digest") == source_digest() and tf.get("variant") == sel:
            traffic = tf.get("bytes_per_launch")

    out = {
        "metric": METRIC,
        "value": round(step_bytes / step_s / 1e9, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(step_s * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"stencil27_{N}^3_fp64: spmv csr/coo/ell/hyb + jacobi-pcg to 1e-10",
                   "n": n, "nnz": nnz, "cg_operator": sel, "step_alg_GB": round(step_bytes / 1e9, 4)},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "kernel": f"{sel} SpMV with fused p.q inside the CG loop",
                     "stream_GBs": ref_gbs, "frac_of_dot": round(achieved / ref_gbs["dot"], 4),
                     # the same product's work in format-independent terms: the
                     # CSR-minimal bytes of y = A x over this kernel's time
                     "csr_equiv_GBs": round(spmv_bytes("csr", n, nnz, None) / (launch_ms * 1e-3) / 1e9, 1),
                     "alg_bytes_per_launch": cg_spmv, "avg_launch_us": round(launch_ms * 1e3, 2)},
        "cg": {"iterations": its[0], "time_to_1e-10_ms": round(cg_ms, 3), "true_rel_residual": true_rel,
               "alg_GBs": round(cg_bytes / (cg_ms * 1e-3) / 1e9, 1),
               "us_per_iteration": round(cg_ms * 1e3 / its[0], 2)},
        "spmv": spmv_detail,
        "selection_ms": {k: round(v, 4) for k, v in t_sel.items()},
        "setup_ms": t_setup,
        "comparisons": comp,
    }
    if not args.no_cpu_baseline:
        log("[bench] oracle CPU baseline (bounded sample)")
        out["cpu_baseline"] = cpu_baseline(A, xs, bd.cpu().numpy(), sel)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
