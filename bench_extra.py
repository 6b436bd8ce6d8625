"""Secondary benchmark workloads of bench.py (--workload ...), one JSON line each.

aniso_ir  : 160^3 anisotropic 7-point diffusion, FP64 Jacobi-PCG vs FP64-outer /
            FP32-inner-CG iterative refinement vs block-Jacobi CG (32-row
            blocks, binary64 or adaptive storage): time to 1e-10 and 1e-12.
poisson2d : 64x64 Poisson, Jacobi-PCG to 1e-10: one kernel per step vs the whole
            solve in one persistent workgroup (latency-bound case).
batch     : 10,000 banded SPD systems, batched Jacobi-PCG in one persistent
            launch: default schedule vs autotuned schedule.
overhead  : the size-1, b = NaN protocol of the paper's Table 1 (per-iteration cost).
stream    : copy / triad / dot bandwidth, the achievable-peak calibration.
bicgstab  : 128^3 27-point system, Jacobi-BiCGSTAB to 1e-10.
stencil_mf: the same operator matrix-free: SpMV and Jacobi-PCG to 1e-10.
gmres     : 128^3 3D convection-diffusion (nonsymmetric), Jacobi-GMRES(100) to
            1e-10, with the solve's algorithmic GB/s and the GB/s the paper's
            memory model (Table 2) assigns to the same run.
suite     : SpMV per stored-format class on members of the skewed suite
            (--matrices, e.g. 74,79,60) and the 128^3 27-point system
            (--with-stencil); the workload the SpMV counter passes profile.

Each line carries a cpu_baseline: the oracle on a bounded sample of the same
work (one host core), unless --no-cpu-baseline.
"""
from __future__ import annotations

import json
import sys
import time


def _sync():
    import torch
    torch.cuda.synchronize()


def _timed(fn, steps, warmup):
    for _ in range(warmup):
        fn()
    _sync()
    t0 = time.perf_counter()
    out = None
    for _ in range(steps):
        out = fn()
    _sync()
    return (time.perf_counter() - t0) / steps, out


def _oracle():
    """The oracle as it stands (plain FP64 C, one thread): test
    infrastructure, used here only for the cpu_baseline leg."""
    import oracle as O
    O.build(force=False)
    return O


def aniso_ir(args):
    import numpy as np
    import torch
    import paper_2006_16852_amd as mxl
    import workloads as W
    dev = "cuda:0"
    A = W.aniso_3d7(160)
    n = A.nrows
    ctx = mxl.Context(0)
    base = mxl.csr(ctx, torch.from_numpy(A.row_ptr).to(dev), torch.from_numpy(A.col).to(dev),
                   torch.from_numpy(A.val).to(dev))
    b = torch.from_numpy(W.uniform_vec(n, 4)).to(dev)
    x = torch.zeros_like(b)
    y = torch.empty_like(b)
    cands = {"ell": base.convert("ell"), "ell16": base.convert("ell", variant=mxl.ELL_DELTA16),
             "csr_vec8": base.convert("csr", variant=1, vector_width=8)}
    t_sel = {k: v.time_apply(b, y, reps=20) for k, v in cands.items()}
    M = cands[min(t_sel, key=t_sel.get)]
    P = mxl.jacobi(M)
    out = {"metric": "CG time-to-1e-10 residual, FP64 vs mixed", "unit": "ms", "n_gpus": 1,
           "higher_is_better": False, "dtype": "f64+f32", "data": "synthetic",
           "config": {"workload": "aniso7_160^3: jacobi-pcg fp64 vs ir(fp32 inner cg, point or block jacobi)", "n": n,
                      "nnz": A.nnz, "operator": min(t_sel, key=t_sel.get)}}
    res = {}
    for red in (1e-10, 1e-12):
        S = mxl.solver("cg", M, P, max_iters=5000, reduction=red, check_every=16)

        def f64():
            x.zero_()
            return S.solve(b, x)
        dt, info = _timed(f64, args.steps, args.warmup)
        r = b.clone(); base.apply(x, r, -1.0, 1.0)
        res[f"fp64_{red:g}"] = dict(ms=round(dt * 1e3, 3), iterations=info["iterations"],
                                    true_rel=float(torch.linalg.norm(r) / torch.linalg.norm(b)))
        for tin in (1e-2, 1e-3, 1e-4):
            I = mxl.ir(M, outer=dict(max_iters=60, reduction=red),
                       inner=dict(reduction=tin, max_iters=10_000, check_every=16))

            def irf():
                x.zero_()
                return I.solve(b, x)
            dt, info = _timed(irf, args.steps, args.warmup)
            r = b.clone(); base.apply(x, r, -1.0, 1.0)
            res[f"ir_{red:g}_in{tin:g}"] = dict(ms=round(dt * 1e3, 3), outer=info["iterations"],
                                               inner=info["inner_iterations"],
                                               true_rel=float(torch.linalg.norm(r) / torch.linalg.norm(b)))
    # block-Jacobi CG (32-row blocks): binary64 storage and adaptive storage
    for red in (1e-10, 1e-12):
        for adaptive in (False, True):
            torch.cuda.synchronize()
            tg = time.perf_counter()
            Pb = mxl.bjacobi(M, 32, adaptive, 0.1)
            torch.cuda.synchronize()
            gen_ms = (time.perf_counter() - tg) * 1e3
            Sb = mxl.solver("cg", M, Pb, max_iters=5000, reduction=red, check_every=16)

            def fb():
                x.zero_()
                return Sb.solve(b, x)
            dt, info = _timed(fb, args.steps, args.warmup)
            r = b.clone(); base.apply(x, r, -1.0, 1.0)
            bi = Pb.info()
            res[f"bjacobi32_{'adaptive' if adaptive else 'fp64'}_{red:g}"] = dict(
                ms=round(dt * 1e3, 3), iterations=info["iterations"],
                true_rel=float(torch.linalg.norm(r) / torch.linalg.norm(b)),
                storage_MB=round(bi["storage_bytes"] / 1e6, 2), generate_ms=round(gen_ms, 3),
                blocks_by_precision=[int((bi["precision"] == k).sum()) for k in (0, 1, 2)])
    # refinement whose FP32 inner CG uses the 32-row adaptive block Jacobi
    for red in (1e-10, 1e-12):
        for tin in (1e-2, 1e-3, 1e-4):
            Ib = mxl.ir(M, outer=dict(max_iters=60, reduction=red),
                        inner=dict(reduction=tin, max_iters=10_000, check_every=16), block_size=32,
                        block_accuracy=0.1)

            def irb():
                x.zero_()
                return Ib.solve(b, x)
            dt, info = _timed(irb, args.steps, args.warmup)
            r = b.clone(); base.apply(x, r, -1.0, 1.0)
            res[f"ir_bjacobi32_{red:g}_in{tin:g}"] = dict(ms=round(dt * 1e3, 3), outer=info["iterations"],
                                                         inner=info["inner_iterations"],
                                                         true_rel=float(torch.linalg.norm(r) / torch.linalg.norm(b)))
    best_irb = min((v["ms"], k) for k, v in res.items() if k.startswith("ir_bjacobi32_1e-10"))
    out["ir_bjacobi32_ms_1e-10"] = best_irb[0]
    out["best_ir_bjacobi32"] = best_irb[1]
    out["speedup_ir_bjacobi_vs_fp64_point_1e-10"] = round(res["fp64_1e-10"]["ms"] / best_irb[0], 3)
    best_ir = min((v["ms"], k) for k, v in res.items() if k.startswith("ir_1e-10"))
    out["value"] = best_ir[0]
    out["fp64_ms_1e-10"] = res["fp64_1e-10"]["ms"]
    out["speedup_vs_fp64_1e-10"] = round(res["fp64_1e-10"]["ms"] / best_ir[0], 3)
    out["best_ir"] = best_ir[1]
    out["bjacobi32_adaptive_ms_1e-10"] = res["bjacobi32_adaptive_1e-10"]["ms"]
    out["speedup_bjacobi_vs_fp64_point_1e-10"] = round(res["fp64_1e-10"]["ms"] / res["bjacobi32_adaptive_1e-10"]["ms"], 3)
    out["runs"] = res
    out["steps"], out["warmup"] = args.steps, args.warmup
    if not args.no_cpu_baseline:
        O = _oracle()
        d, _ = O.jacobi_dinv(A)
        bh = W.uniform_vec(n, 4)
        k = 20
        t0 = time.perf_counter()
        O.pcg(A, bh, dinv=d, max_iters=k, reduction=0.0)
        per_it = (time.perf_counter() - t0) / k
        its = res["fp64_1e-10"]["iterations"]
        out["cpu_baseline"] = {"value": round(per_it * its * 1e3, 1), "unit": "ms", "cores": 1, "kind": "oracle",
                               "sample": f"{k} FP64 Jacobi-PCG iterations on the 160^3 system "
                                         f"({per_it * 1e3:.1f} ms each), scaled to the {its} iterations to 1e-10"}
    print(json.dumps(out), flush=True)


def poisson2d(args):
    import numpy as np
    import torch
    import paper_2006_16852_amd as mxl
    import workloads as W
    dev = "cuda:0"
    A = W.stencil_2d5(64)
    ctx = mxl.Context(0)
    M = mxl.csr(ctx, torch.from_numpy(A.row_ptr).to(dev), torch.from_numpy(A.col).to(dev),
                torch.from_numpy(A.val).to(dev))
    xs = torch.from_numpy(W.uniform_vec(A.nrows, 1)).to(dev)
    b = torch.empty_like(xs)
    M.apply(xs, b)
    P = mxl.jacobi(M)
    x = torch.zeros_like(b)
    res = {}
    for kind, mode, name in (("cg", 1, "per_step_kernels"), ("cg", 2, "one_workgroup"),
                             ("bicgstab", 1, "bicgstab_per_step_kernels"), ("bicgstab", 2, "bicgstab_one_workgroup")):
        S = mxl.solver(kind, M, P, max_iters=5000, reduction=1e-10, check_every=32, launch_mode=mode)

        def f():
            x.zero_()
            return S.solve(b, x)
        dt, info = _timed(f, max(args.steps, 20), args.warmup + 2)
        res[name] = dict(ms=round(dt * 1e3, 4), iterations=info["iterations"],
                         us_per_iteration=round(dt * 1e6 / info["iterations"], 3))
    out = {"metric": "CG time-to-1e-10 residual (latency-bound 64x64 Poisson)", "unit": "ms",
           "value": res["one_workgroup"]["ms"], "higher_is_better": False, "n_gpus": 1,
           "dtype": "f64", "data": "synthetic",
           "config": {"workload": "stencil2d5_64^2 jacobi-pcg to 1e-10", "n": A.nrows, "nnz": A.nnz},
           "runs": res, "paper_table1_us_per_iteration_cg": 1.28}
    if not args.no_cpu_baseline:
        O = _oracle()
        d, _ = O.jacobi_dinv(A)
        bh = b.cpu().numpy()
        reps = 20
        t0 = time.perf_counter()
        for _ in range(reps):
            r = O.pcg(A, bh, dinv=d, reduction=1e-10)
        dt = (time.perf_counter() - t0) / reps
        out["cpu_baseline"] = {"value": round(dt * 1e3, 3), "unit": "ms", "cores": 1, "kind": "oracle",
                               "sample": f"the whole solve ({r['iterations']} iterations), mean of {reps}"}
    print(json.dumps(out), flush=True)


def batch(args):
    import numpy as np
    import torch
    import paper_2006_16852_amd as mxl
    import workloads as W
    dev = "cuda:0"
    B = W.batch_systems()
    ctx = mxl.Context(0)
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    dsp, drp, dcol, dval = d(B.sys_ptr), d(B.row_ptr), d(B.col), d(B.val)
    mxl.batch(ctx, B.sys_ptr, dsp, drp, dcol, dval)  # first creation warms the allocator
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    op = mxl.batch(ctx, B.sys_ptr, dsp, drp, dcol, dval)
    torch.cuda.synchronize()
    create_ms = (time.perf_counter() - t0) * 1e3
    b = d(B.b)
    x = torch.zeros_like(b)
    it = torch.zeros(B.nsys, dtype=torch.int32, device=dev)
    rel = torch.zeros(B.nsys, dtype=torch.float64, device=dev)
    st = torch.zeros(B.nsys, dtype=torch.uint8, device=dev)
    res = {}
    dt, _ = _timed(lambda: op.solve(b, x, it, rel, st, tuning=(256, 2, 0), reduction=1e-10),
                   args.steps, args.warmup)
    res["default_256x2_input"] = round(dt * 1e3, 3)
    t0 = time.perf_counter()
    best, best_ms = op.autotune(b, torch.zeros_like(b), reps=2, reduction=1e-10)
    tune_s = time.perf_counter() - t0
    dt, _ = _timed(lambda: op.solve(b, x, it, rel, st, reduction=1e-10), args.steps, args.warmup)
    res["autotuned"] = round(dt * 1e3, 3)
    ok = int((st.cpu().numpy() == 1).sum())
    bytes_once = B.row_ptr[-1] * 12 + B.sys_ptr[-1] * (4 + 8 * 3)
    # no-reuse model: every iteration of system s moves its matrix and 11 n_s values
    ns = np.diff(B.sys_ptr).astype(np.int64)
    nz = np.diff(B.row_ptr[B.sys_ptr]).astype(np.int64)
    iters = it.cpu().numpy().astype(np.int64)
    bytes_noreuse = int((iters * (nz * 12 + (ns + 1) * 4 + 11 * ns * 8)).sum())
    # denominators: HBM peak and the measured read bandwidth of the caches
    # the systems' working sets live in between iterations
    sa = torch.rand(1 << 24, dtype=torch.float64, device=dev)
    sc = torch.empty(1 << 12, dtype=torch.float64, device=dev)
    cached = cached_read_bandwidth(mxl, ctx, sa, sc)
    del sa, sc
    noreuse_gbs = bytes_noreuse / dt / 1e9
    print(json.dumps({"metric": "batched Jacobi-CG systems/s (10,000 systems to 1e-10)", "unit": "systems/s",
                      "value": round(B.nsys / (dt), 1), "higher_is_better": True, "n_gpus": 1,
                      "dtype": "f64", "data": "synthetic",
                      "config": {"workload": "10k banded spd systems n in [32,1024]", "rows": int(B.sys_ptr[-1]),
                                 "nnz": int(B.row_ptr[-1])},
                      "ms": res, "create_ms": round(create_ms, 3), "autotuned_schedule": best,
                      "autotune_seconds": round(tune_s, 3),
                      "converged": ok, "total_iterations": int(it.sum()),
                      "read_once_GBs": round(bytes_once / dt / 1e9, 1),
                      "noreuse_GBs": round(noreuse_gbs, 1),
                      "noreuse_frac_hbm": round(noreuse_gbs / 8000.0, 3),
                      "cached_read_GBs": cached,
                      "noreuse_frac_llc": round(noreuse_gbs / cached["llc_128MiB"], 3),
                      **({} if args.no_cpu_baseline else {"cpu_baseline": _batch_cpu(B)})}), flush=True)


def _batch_cpu(B, count=500):
    """The oracle's batched PCG on the first `count` systems, in systems/s."""
    import numpy as np
    import workloads as W
    O = _oracle()
    rows = int(B.sys_ptr[count])
    sub = W.Batch(count, B.sys_ptr[:count + 1].copy(), B.row_ptr[:rows + 1].copy(),
                  B.col[:B.row_ptr[rows]].copy(), B.val[:B.row_ptr[rows]].copy(), B.b[:rows].copy())
    t0 = time.perf_counter()
    O.batch_pcg(sub, reduction=1e-10)
    dt = time.perf_counter() - t0
    return {"value": round(count / dt, 1), "unit": "systems/s", "cores": 1, "kind": "oracle",
            "sample": f"the first {count} of the 10,000 systems to 1e-10, {dt:.2f} s"}


def overhead(args):
    """The per-iteration cost protocol of the paper's Table 1: a size-1
    matrix, x = 0, b = NaN, 1,000 iterations (no early stop), averaged."""
    import numpy as np
    import torch
    import paper_2006_16852_amd as mxl
    dev = "cuda:0"
    ctx = mxl.Context(0)
    M = mxl.csr(ctx, torch.tensor([0, 1], dtype=torch.int32, device=dev),
                torch.tensor([0], dtype=torch.int32, device=dev),
                torch.tensor([2.0], dtype=torch.float64, device=dev))
    b = torch.full((1,), float("nan"), dtype=torch.float64, device=dev)
    x = torch.zeros(1, dtype=torch.float64, device=dev)
    iters = 1000
    res = {}
    for kind, mode, name in (("cg", 2, "cg_one_workgroup"), ("cg", 1, "cg_per_step_kernels"),
                             ("bicgstab", 2, "bicgstab_one_workgroup"),
                             ("bicgstab", 1, "bicgstab_per_step_kernels"),
                             ("gmres", 0, "gmres100_one_workgroup"),
                             ("gmres", 1, "gmres100_per_step_kernels")):
        S = mxl.solver(kind, M, None, max_iters=iters, nonfinite_check=0, check_every=iters,
                       launch_mode=mode)

        def f():
            x.zero_()
            return S.solve(b, x)
        dt, info = _timed(f, max(3, args.steps), 1)
        assert info["iterations"] == iters
        res[name] = round(dt * 1e6 / iters, 3)
    out = {"metric": "solver overhead per iteration (size-1 system, b = NaN, 1,000 iterations)",
           "unit": "us/iteration", "value": res["cg_one_workgroup"], "higher_is_better": False,
           "n_gpus": 1, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "n=1 nan-rhs protocol"}, "runs": res,
           "paper_table1_us": {"CG": 1.28, "BiCGSTAB": 1.26, "GMRES": 1.51}}
    if not args.no_cpu_baseline:
        import workloads as W
        O = _oracle()
        A1 = W.Csr(1, 1, np.array([0, 1], np.int32), np.array([0], np.int32), np.array([2.0]))
        reps = 200
        t0 = time.perf_counter()
        for _ in range(reps):
            O.pcg(A1, np.array([np.nan]), max_iters=iters, nonfinite_check=0)
        dt = (time.perf_counter() - t0) / reps
        out["cpu_baseline"] = {"value": round(dt * 1e6 / iters, 4), "unit": "us/iteration", "cores": 1,
                               "kind": "oracle", "sample": f"{reps} solves of {iters} iterations"}
    print(json.dumps(out), flush=True)


def gmres_table2_bytes(n, nnz, iters, k, VT=8, IT=4):
    """Read + write volume of a GMRES(k) run by the paper's memory model
    (Table 2), r = iters mod k and the triangular inner-step count
    iter_r = floor(iters/k) (k-1) k / 2 + (r-1) r / 2."""
    r = iters % k
    q = iters // k
    iter_r = q * (k - 1) * k / 2 + (r - 1) * r / 2
    rd = ((11 * n + 2 * nnz + 2.5 * r + n * r + r * r / 2 + 1) * VT + 2 * nnz * IT
          + q * ((1 + 2.5 * k + 10 * n + 2 * nnz + k * k / 2 + k * n) * VT + 2 * nnz * IT)
          + iters * ((7 * n + 5 + 2 * nnz) * VT + 2 * nnz * IT + 8) + iter_r * ((4 * n + 4) * VT))
    wr = ((6 * n + r + 2 * k + 3) * VT + 8 + q * ((k + 6 * n + 2) * VT + 8)
          + iters * ((4 * n + 8) * VT + 8) + iter_r * ((n + 2) * VT))
    return rd + wr


def gmres_alg_bytes(n, spmv, iters, k, restarts, extra_spmv=0):
    """Algorithmic bytes of this implementation's GMRES(k) run: step j (of
    a cycle) moves its SpMV plus (2 j + 8) n values (multi-dot over the j
    final basis vectors, the candidate t_j and u; multi-axpy over the same
    plus dinv, writing v_j, t_{j+1} and z); a cycle of J steps ends with one
    more multi-dot, (J + 1) n, and the closing combination, (J + 3) n; the
    start and every restart move a residual SpMV and 6 n (b copy, norm, z).
    extra_spmv: products of steps whose column the criterion did not need."""
    total = extra_spmv * spmv
    left = iters
    for _ in range(restarts + 1):
        J = min(k, left)
        left -= J
        total += J * spmv + sum((2 * j + 8) * n * 8 for j in range(J))
        total += (J + 1) * n * 8 + (J + 3) * n * 8 + spmv + 6 * n * 8
    return total


def gmres(args):
    """Jacobi-GMRES(100) on the 128^3 3D convection-diffusion system to 1e-10
    (ELL with 16-bit column offsets)."""
    import numpy as np
    import torch
    import paper_2006_16852_amd as mxl
    import workloads as W
    dev = "cuda:0"
    N = 128
    A = W.convdiff_3d7(N)
    n = A.nrows
    ctx = mxl.Context(0)
    base = mxl.csr(ctx, torch.from_numpy(A.row_ptr).to(dev), torch.from_numpy(A.col).to(dev),
                   torch.from_numpy(A.val).to(dev))
    b = torch.from_numpy(W.uniform_vec(n, 5)).to(dev)
    M = base.convert("ell", variant=mxl.ELL_DELTA16)
    d = M.describe()
    spmv = n * d["ell_width"] * (8 + 2) + 2 * n * 8
    k = 100
    S = mxl.solver("gmres", M, mxl.jacobi(M), krylov_dim=k, max_iters=5000, reduction=1e-10, check_every=25)
    x = torch.zeros_like(b)

    def f():
        x.zero_()
        return S.solve(b, x)
    dt, info = _timed(f, args.steps, args.warmup)
    r = b.clone()
    base.apply(x, r, -1.0, 1.0)
    its = info["iterations"]
    alg = gmres_alg_bytes(n, spmv, its, k, info["restarts"], info["spmv_count"] - 1 - its - info["restarts"])
    t2 = gmres_table2_bytes(n, A.nnz, its, k)
    out = {"metric": "GMRES(100) time-to-1e-10 residual", "unit": "ms", "value": round(dt * 1e3, 3),
           "higher_is_better": False, "n_gpus": 1, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "convdiff3d7_128^3 jacobi-gmres(100) to 1e-10", "n": n, "nnz": A.nnz,
                      "operator": "ell16", "krylov_dim": k},
           "iterations": its, "restarts": info["restarts"], "spmv_count": info["spmv_count"],
           "stop": info["stop"], "true_rel_residual": float(torch.linalg.norm(r) / torch.linalg.norm(b)),
           "alg_GB": round(alg / 1e9, 3), "alg_GBs": round(alg / dt / 1e9, 1),
           "table2_model_GB": round(t2 / 1e9, 3), "table2_model_GBs": round(t2 / dt / 1e9, 1),
           "us_per_iteration": round(dt * 1e6 / max(its, 1), 2),
           "steps": args.steps, "warmup": args.warmup}
    # the same solve preconditioned by ParILU(3) factors, with Jacobi-sweep
    # (4 per triangle) or exact level-scheduled triangular solves
    ilu_runs = {}
    for name, mode, ts in (("parilu3_jacobi4", "jacobi", 4), ("parilu3_exact", "exact", 0)):
        t0 = time.perf_counter()
        Pi = mxl.ilu(M, sweeps=3, trisolve=mode, trs_sweeps=ts)
        _sync()
        gen_ms = (time.perf_counter() - t0) * 1e3
        Si = mxl.solver("gmres", M, Pi, krylov_dim=k, max_iters=5000, reduction=1e-10, check_every=25)

        def fi():
            x.zero_()
            return Si.solve(b, x)
        dti, infoi = _timed(fi, max(1, args.steps if mode == "jacobi" else 1), 1 if mode == "jacobi" else 0)
        ri = b.clone()
        base.apply(x, ri, -1.0, 1.0)
        lv = Pi.info()
        ilu_runs[name] = {"ms": round(dti * 1e3, 3), "iterations": infoi["iterations"],
                          "restarts": infoi["restarts"], "stop": infoi["stop"],
                          "true_rel_residual": float(torch.linalg.norm(ri) / torch.linalg.norm(b)),
                          "generate_ms": round(gen_ms, 2),
                          "levels": [lv["levels_lower"], lv["levels_upper"]]}
    out["ilu"] = ilu_runs
    if not args.no_cpu_baseline:
        O = _oracle()
        dh, _ = O.jacobi_dinv(A)
        kk = 20
        bh = b.cpu().numpy()
        t0 = time.perf_counter()
        O.gmres(A, bh, dinv=dh, krylov_dim=k, max_iters=kk, reduction=0.0)
        first = time.perf_counter() - t0
        # step j of a cycle costs about (j + 1) basis passes: scale the first
        # kk steps' time by the ratio of the full run's basis work
        def work(m):
            return sum(j + 2 for j in range(m))
        full = sum(work(min(k, its - c * k)) for c in range(info["restarts"] + 1))
        est = first * full / work(kk)
        out["cpu_baseline"] = {"value": round(est * 1e3, 1), "unit": "ms", "cores": 1, "kind": "oracle",
                               "sample": f"the first {kk} Jacobi-GMRES(100) steps ({first:.2f} s), scaled by "
                                         f"the basis work of the {its} steps to 1e-10"}
    print(json.dumps(out), flush=True)


def stream(args):
    """STREAM-style bandwidth of copy, triad and dot on 2^28 doubles (2 GiB
    per array; the calibration the paper uses for solver bandwidth, Sec. 7.4
    and Table 3)."""
    import torch
    import paper_2006_16852_amd as mxl
    dev = "cuda:0"
    ctx = mxl.Context(0)
    n = 1 << 28
    torch.manual_seed(11)
    a = torch.rand(n, dtype=torch.float64, device=dev)
    b = torch.rand(n, dtype=torch.float64, device=dev)
    c = torch.empty(n, dtype=torch.float64, device=dev)
    reps = max(5, args.steps)
    res = {}
    for op, nbytes in (("copy", 16 * n), ("triad", 24 * n), ("dot", 16 * n), ("read", 8 * n)):
        ms = mxl.stream_bench(ctx, op, a, b, c, reps=reps)
        res[op] = {"ms": round(ms, 4), "GBs": round(nbytes / ms / 1e6, 1), "bytes": nbytes}
    print(json.dumps({"metric": "STREAM triad bandwidth", "unit": "GB/s", "value": res["triad"]["GBs"],
                      "higher_is_better": True, "n_gpus": 1, "dtype": "f64", "data": "synthetic",
                      "config": {"workload": "stream 2^28 doubles", "n": n}, "runs": res,
                      "cached_read_GBs": cached_read_bandwidth(mxl, ctx, a, c, reps),
                      "peak_GBs": 8000.0}), flush=True)


def cached_read_bandwidth(mxl, ctx, a, c, reps=10):
    """Read bandwidth (GB/s) of the cached read-only kernel over arrays that
    fit the caches; one launch sweeps the array until 2^28 values are read
    (the first sweep fills the cache): 2^24 doubles (128 MiB: in the 256 MB
    last-level cache, but 16 MiB per XCD, beyond its 4 MB L2) and 2^21
    doubles (16 MiB: each XCD sweeps a 2 MiB band inside its L2)."""
    out = {}
    for tag, m in (("llc_128MiB", 1 << 24), ("l2_16MiB", 1 << 21)):
        v = a[:m]
        sweeps = -(-(1 << 28) // m)
        ms = mxl.stream_bench(ctx, "read", v, None, c, reps=reps)
        out[tag] = round(8 * m * sweeps / ms / 1e6, 1)
    return out


def bicgstab(args):
    """Jacobi-BiCGSTAB on the 128^3 27-point system to 1e-10 (the operator
    chosen by timing among ELL layouts), with algorithmic GB/s: per
    iteration two SpMVs plus 21 n value words of vector traffic (p pass 6n,
    s pass 5n, t dots 2n, x/r pass 8n)."""
    import numpy as np
    import torch
    import paper_2006_16852_amd as mxl
    import workloads as W
    dev = "cuda:0"
    A = W.stencil_3d27(128)
    n = A.nrows
    ctx = mxl.Context(0)
    base = mxl.csr(ctx, torch.from_numpy(A.row_ptr).to(dev), torch.from_numpy(A.col).to(dev),
                   torch.from_numpy(A.val).to(dev))
    xs = torch.from_numpy(W.uniform_vec(n, 2)).to(dev)
    b = torch.empty_like(xs)
    base.apply(xs, b)
    y = torch.empty_like(b)
    cands = {"ell": base.convert("ell"), "ell16": base.convert("ell", variant=mxl.ELL_DELTA16)}
    t_sel = {k: v.time_apply(b, y, reps=20) for k, v in cands.items()}
    name = min(t_sel, key=t_sel.get)
    M = cands[name]
    d = M.describe()
    it_b = 2 if name == "ell16" else 4
    spmv = n * d["ell_width"] * (8 + it_b) + 2 * n * 8
    S = mxl.solver("bicgstab", M, mxl.jacobi(M), max_iters=5000, reduction=1e-10, check_every=16)
    x = torch.zeros_like(b)

    def f():
        x.zero_()
        return S.solve(b, x)
    dt, info = _timed(f, args.steps, args.warmup)
    r = b.clone()
    base.apply(x, r, -1.0, 1.0)
    its = info["iterations"]
    byts = its * (2 * spmv + 21 * n * 8)
    out = {"metric": "BiCGSTAB time-to-1e-10 residual", "unit": "ms", "value": round(dt * 1e3, 3),
           "higher_is_better": False, "n_gpus": 1, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "stencil27_128^3 jacobi-bicgstab to 1e-10", "n": n, "nnz": A.nnz,
                      "operator": name},
           "iterations": its, "stop": info["stop"],
           "true_rel_residual": float(torch.linalg.norm(r) / torch.linalg.norm(b)),
           "alg_GBs": round(byts / dt / 1e9, 1), "us_per_iteration": round(dt * 1e6 / max(its, 1), 2),
           "steps": args.steps, "warmup": args.warmup}
    # a nonsymmetric system: 128^3 convection-diffusion, point vs block Jacobi
    C3 = W.convdiff_3d7(128)
    cb = mxl.csr(ctx, torch.from_numpy(C3.row_ptr).to(dev), torch.from_numpy(C3.col).to(dev),
                 torch.from_numpy(C3.val).to(dev))
    Mc = cb.convert("ell", variant=mxl.ELL_DELTA16)
    bc = torch.from_numpy(W.uniform_vec(C3.nrows, 5)).to(dev)
    xc = torch.zeros_like(bc)
    conv = {}
    for pname, Pc in (("jacobi", mxl.jacobi(Mc)), ("bjacobi8", mxl.bjacobi(cb, 8, True)),
                      ("bjacobi32", mxl.bjacobi(cb, 32, True))):
        Sc = mxl.solver("bicgstab", Mc, Pc, max_iters=5000, reduction=1e-10, check_every=16)

        def fc():
            xc.zero_()
            return Sc.solve(bc, xc)
        dtc, infc = _timed(fc, args.steps, args.warmup)
        rc = bc.clone()
        cb.apply(xc, rc, -1.0, 1.0)
        conv[pname] = {"ms": round(dtc * 1e3, 3), "iterations": infc["iterations"], "stop": infc["stop"],
                       "true_rel_residual": float(torch.linalg.norm(rc) / torch.linalg.norm(bc))}
    out["convdiff3d7_128"] = conv
    if not args.no_cpu_baseline:
        O = _oracle()
        dh, _ = O.jacobi_dinv(A)
        k = 5
        t0 = time.perf_counter()
        O.bicgstab(A, b.cpu().numpy(), dinv=dh, max_iters=k, reduction=0.0)
        per_it = (time.perf_counter() - t0) / k
        out["cpu_baseline"] = {"value": round(per_it * its * 1e3, 1), "unit": "ms", "cores": 1,
                               "kind": "oracle",
                               "sample": f"{k} Jacobi-BiCGSTAB iterations ({per_it * 1e3:.0f} ms each), "
                                         f"scaled to the {its} iterations to 1e-10"}
    print(json.dumps(out), flush=True)


def stencil_mf(args):
    """Matrix-free 27-point operator on the 128^3 grid (the user-defined
    operator of the paper's Sec. 4): SpMV time and Jacobi-PCG to 1e-10,
    next to the stored-matrix path (ELL with 16-bit offsets).  A
    matrix-free product moves x and y only: 2 n 8 bytes."""
    import numpy as np
    import torch
    import paper_2006_16852_amd as mxl
    import workloads as W
    dev = "cuda:0"
    N = 128
    A = W.stencil_3d27(N)
    n = A.nrows
    ctx = mxl.Context(0)
    pts, cf = W.points_3d27()
    op = mxl.stencil(ctx, (N, N, N), pts, cf)
    base = mxl.csr(ctx, torch.from_numpy(A.row_ptr).to(dev), torch.from_numpy(A.col).to(dev),
                   torch.from_numpy(A.val).to(dev))
    ell = base.convert("ell", variant=mxl.ELL_DELTA16)
    xs = torch.from_numpy(W.uniform_vec(n, 2)).to(dev)
    b = torch.empty_like(xs)
    op.apply(xs, b)
    y = torch.empty_like(b)
    t_mf = op.time_apply(xs, y, reps=50)
    t_ell = ell.time_apply(xs, y, reps=20)
    res = {}
    for name, M in (("matrix_free", op), ("ell16", ell)):
        S = mxl.solver("cg", M, mxl.jacobi(M), max_iters=5000, reduction=1e-10, check_every=16)
        x = torch.zeros_like(b)

        def f():
            x.zero_()
            return S.solve(b, x, time_spmv=16)
        dt, info = _timed(f, args.steps, args.warmup)
        r = b.clone()
        op.apply(x, r, -1.0, 1.0)
        res[name] = dict(ms=round(dt * 1e3, 3), iterations=info["iterations"],
                         us_per_iteration=round(dt * 1e6 / info["iterations"], 2),
                         spmv_us_in_loop=round(info["spmv_ms"] * 1e3 / max(info["spmv_timed"], 1), 2),
                         true_rel=float(torch.linalg.norm(r) / torch.linalg.norm(b)))
    mf_bytes = 2 * n * 8
    out = {"metric": "CG time-to-1e-10 residual, matrix-free stencil", "unit": "ms",
           "value": res["matrix_free"]["ms"], "higher_is_better": False, "n_gpus": 1, "dtype": "f64",
           "data": "synthetic", "config": {"workload": "stencil27_128^3 matrix-free jacobi-pcg to 1e-10", "n": n},
           "spmv": {"matrix_free_us": round(t_mf * 1e3, 2), "matrix_free_GBs": round(mf_bytes / t_mf / 1e6, 1),
                    "ell16_us": round(t_ell * 1e3, 2)},
           "runs": res, "steps": args.steps, "warmup": args.warmup}
    print(json.dumps(out), flush=True)


def suite(args):
    """SpMV of every stored-format class on members of the skewed suite (row
    lengths Zipf-distributed, banded-random columns) and on the 128^3
    27-point system: the per-class GB/s (CSR-minimal bytes and the class's
    own bytes) that the counter passes are read against."""
    import numpy as np
    import torch
    import paper_2006_16852_amd as mxl
    import workloads as W
    from paper_2006_16852_amd.selector import convert
    dev = "cuda:0"
    ctx = mxl.Context(0)
    classes = ["csr_stream", "csr_merge", "csr_vec64", "coo", "hyb66", "ell16"]
    mats = [int(m) for m in args.matrices.split(",")] if args.matrices else []
    out = {"metric": "SpMV GB/s per class, skewed suite members and the 128^3 27-point system",
           "unit": "GB/s", "n_gpus": 1, "higher_is_better": True, "dtype": "f64", "data": "synthetic",
           "reps": args.steps, "matrices": {}}
    todo = [(f"zipf{m}", lambda m=m: W.zipf_suite_matrix(m)) for m in mats]
    if args.with_stencil:
        todo.append(("stencil27_128", lambda: W.stencil_3d27(128)))
    for name, gen in todo:
        A = gen()
        n, nnz = A.nrows, A.nnz
        base = mxl.csr(ctx, torch.from_numpy(A.row_ptr).to(dev), torch.from_numpy(A.col).to(dev),
                       torch.from_numpy(A.val).to(dev))
        x = torch.from_numpy(W.uniform_vec(A.ncols, 2)).to(dev)
        y = torch.empty(n, dtype=torch.float64, device=dev)
        csr_b = nnz * 12 + (n + 1) * 4 + 2 * n * 8
        rec = {"n": n, "nnz": nnz, "max_row": int(np.diff(A.row_ptr).max()), "csr_MB": round(csr_b / 1e6, 1)}
        if name.startswith("zipf"):
            p = W.zipf_suite_params(int(name[4:]))
            rec.update(zipf_a=round(p.a, 3), bandwidth=p.bw)
        for c in classes:
            try:
                op = convert(base, c)
            except mxl.MxlError as e:
                if e.status == mxl.ERR_INFEASIBLE_FORMAT:
                    rec[c] = None
                    continue
                raise
            ms = op.time_apply(x, y, reps=args.steps, flush=True)
            d = op.describe()
            rec[c] = {"us": round(ms * 1e3, 2), "csr_GBs": round(csr_b / ms / 1e6, 1),
                      "stored_MB": round(d["stored_bytes"] / 1e6, 1)}
            log(f"[suite] {name} {c}: {ms * 1e3:.1f} us, {csr_b / ms / 1e6:.0f} GB/s (CSR bytes)")
            del op
        out["matrices"][name] = rec
        del base, A
    print(json.dumps(out), flush=True)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def run(args):
    {"aniso_ir": aniso_ir, "poisson2d": poisson2d, "batch": batch, "overhead": overhead,
     "stream": stream, "bicgstab": bicgstab, "stencil_mf": stencil_mf, "gmres": gmres,
     "suite": suite}[args.workload](args)
