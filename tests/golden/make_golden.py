"""Write the oracle's iteration counts at the full workload sizes.

Calls only the CPU oracle and the seeded input generators; the GPU tests
compare the HIP solvers' counts against these stored values because the
oracle needs minutes at these sizes.  Run from the repository root:
    python tests/golden/make_golden.py            # everything
    python tests/golden/make_golden.py bjacobi    # only the block-Jacobi entry
    python tests/golden/make_golden.py gmres      # only the GMRES entry
    python tests/golden/make_golden.py ilu        # only the ILU-GMRES entry
    python tests/golden/make_golden.py bicgstab   # only the BiCGSTAB entries
    python tests/golden/make_golden.py bicgstab_spread  # their rounding spread
"""
import json
import os
import sys
import time

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__)))))

import oracle as O  # noqa: E402
import workloads as W  # noqa: E402


def bjacobi(out):
    """Block-Jacobi-PCG (32-row blocks, adaptive storage) on the 160^3
    anisotropic system."""
    A = W.aniso_3d7(160)
    b = W.uniform_vec(A.nrows, 4)
    t = time.time()
    bp = O.uniform_blocks(A.nrows, 32)
    inv, cond, prec = O.bj_generate(A, bp, adaptive=True, accuracy=0.1)
    r = O.pcg_block(A, b, bp, inv, reduction=1e-10, max_iters=5000)
    out["aniso7_160_bjacobi32_pcg_1e-10"] = dict(
        recipe="b = U[-1,1) seed 4, x0 = 0; blocks of 32 rows, adaptive storage, accuracy 0.1",
        iterations=r["iterations"], stop=r["stop_reason"], rel_residual=r["rel_residual"],
        precision_counts=[int((prec == k).sum()) for k in (0, 1, 2)],
        cond_max=float(cond.max()))
    print("bjacobi", r["iterations"], time.time() - t, flush=True)


def gmres(out):
    """Jacobi-GMRES(100) on the 128^3 convection-diffusion system."""
    A = W.convdiff_3d7(128)
    b = W.uniform_vec(A.nrows, 5)
    t = time.time()
    d, _ = O.jacobi_dinv(A)
    r = O.gmres(A, b, dinv=d, krylov_dim=100, reduction=1e-10, max_iters=5000)
    out["convdiff3d7_128_gmres100_jacobi_1e-10"] = dict(
        recipe="peclet (0.5, 0.25, 0.125); b = U[-1,1) seed 5, x0 = 0",
        iterations=r["iterations"], spmv_count=r["spmv_count"], stop=r["stop_reason"],
        rel_residual=r["rel_residual"])
    print("gmres", r["iterations"], time.time() - t, flush=True)


def ilu(out):
    """GMRES(100) with ParILU (3 sweeps) and Jacobi-sweep triangular solves
    (4 sweeps) on the 128^3 convection-diffusion system."""
    A = W.convdiff_3d7(128)
    b = W.uniform_vec(A.nrows, 5)
    t = time.time()
    lu, _ = O.parilu(A, 3)
    r = O.gmres_ilu(A, b, lu, trs_mode=1, trs_sweeps=4, krylov_dim=100, reduction=1e-10, max_iters=5000)
    out["convdiff3d7_128_gmres100_parilu3_jacobi4_1e-10"] = dict(
        recipe="peclet (0.5, 0.25, 0.125); b = U[-1,1) seed 5, x0 = 0; ParILU 3 sweeps, 4 Jacobi sweeps per triangle",
        iterations=r["iterations"], spmv_count=r["spmv_count"], stop=r["stop_reason"],
        rel_residual=r["rel_residual"])
    print("ilu", r["iterations"], time.time() - t, flush=True)


def bicgstab(out):
    """Jacobi-BiCGSTAB to 1e-10 on the 128^3 27-point system (b = A x*), and
    on the 128^3 convection-diffusion system with point Jacobi and with
    block Jacobi of 8- and 32-row blocks (adaptive storage)."""
    A = W.stencil_3d27(128)
    b = O.spmv(A, W.uniform_vec(A.nrows, 2))
    t = time.time()
    d, _ = O.jacobi_dinv(A)
    r = O.bicgstab(A, b, dinv=d, reduction=1e-10, max_iters=5000)
    out["stencil27_128_bicgstab_1e-10"] = dict(
        recipe="x* = U[-1,1) seed 2, b = A x*, x0 = 0; point Jacobi",
        iterations=r["iterations"], spmv_count=r["spmv_count"], stop=r["stop_reason"],
        rel_residual=r["rel_residual"])
    print("bicgstab 27pt", r["iterations"], time.time() - t, flush=True)
    del A, b, d
    A = W.convdiff_3d7(128)
    b = W.uniform_vec(A.nrows, 5)
    t = time.time()
    d, _ = O.jacobi_dinv(A)
    r = O.bicgstab(A, b, dinv=d, reduction=1e-10, max_iters=5000)
    out["convdiff3d7_128_bicgstab_jacobi_1e-10"] = dict(
        recipe="peclet (0.5, 0.25, 0.125); b = U[-1,1) seed 5, x0 = 0; point Jacobi",
        iterations=r["iterations"], spmv_count=r["spmv_count"], stop=r["stop_reason"],
        rel_residual=r["rel_residual"])
    print("bicgstab convdiff jacobi", r["iterations"], time.time() - t, flush=True)
    for bs in (8, 32):
        t = time.time()
        bp = O.uniform_blocks(A.nrows, bs)
        inv, cond, prec = O.bj_generate(A, bp, adaptive=True, accuracy=0.1)
        r = O.bicgstab_block(A, b, bp, inv, reduction=1e-10, max_iters=5000)
        out[f"convdiff3d7_128_bicgstab_bjacobi{bs}_1e-10"] = dict(
            recipe=f"peclet (0.5, 0.25, 0.125); b = U[-1,1) seed 5, x0 = 0; blocks of {bs} rows, "
                   "adaptive storage, accuracy 0.1",
            iterations=r["iterations"], spmv_count=r["spmv_count"], stop=r["stop_reason"],
            rel_residual=r["rel_residual"],
            precision_counts=[int((prec == k).sum()) for k in (0, 1, 2)])
        print("bicgstab convdiff bjacobi", bs, r["iterations"], time.time() - t, flush=True)


def bicgstab_spread(out, nperturb=6):
    """How far rounding alone moves BiCGSTAB's iteration count on the four
    128^3 systems above: the oracle's counts when b is perturbed at rounding
    level, b_i (1 + 4e-16 g_i) with g ~ N(0,1) (seeds 1..nperturb), and the
    first 31 entries of the unperturbed residual history (relative
    recurrence-residual norms), which rounding has not yet amplified."""
    import numpy as np

    def runs(key, solve, b):
        t = time.time()
        r = solve(b, True)
        counts = []
        for seed in range(1, nperturb + 1):
            g = np.random.default_rng(seed).standard_normal(b.size)
            counts.append(int(solve(b * (1.0 + 4e-16 * g), False)["iterations"]))
        out[key]["history_head"] = [float(v) for v in r["history"][:31]]
        out[key]["perturbed_counts"] = counts
        out[key]["perturbation"] = "b_i (1 + 4e-16 g_i), g ~ N(0,1) seeds 1..%d" % nperturb
        print(key, r["iterations"], counts, time.time() - t, flush=True)

    A = W.stencil_3d27(128)
    b = O.spmv(A, W.uniform_vec(A.nrows, 2))
    d, _ = O.jacobi_dinv(A)
    runs("stencil27_128_bicgstab_1e-10",
         lambda bb, h: O.bicgstab(A, bb, dinv=d, reduction=1e-10, max_iters=5000, history=h), b)
    del A, b, d
    A = W.convdiff_3d7(128)
    b = W.uniform_vec(A.nrows, 5)
    d, _ = O.jacobi_dinv(A)
    runs("convdiff3d7_128_bicgstab_jacobi_1e-10",
         lambda bb, h: O.bicgstab(A, bb, dinv=d, reduction=1e-10, max_iters=5000, history=h), b)
    for bs in (8, 32):
        bp = O.uniform_blocks(A.nrows, bs)
        inv, _, _ = O.bj_generate(A, bp, adaptive=True, accuracy=0.1)
        runs(f"convdiff3d7_128_bicgstab_bjacobi{bs}_1e-10",
             lambda bb, h: O.bicgstab_block(A, bb, bp, inv, reduction=1e-10, max_iters=5000, history=h), b)


ONLY = {"bjacobi": bjacobi, "gmres": gmres, "ilu": ilu, "bicgstab": bicgstab, "bicgstab_spread": bicgstab_spread}


def main():
    O.build(force=False)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "solver_counts.json")
    if len(sys.argv) == 2 and sys.argv[1] in ONLY:
        out = json.load(open(path))
        ONLY[sys.argv[1]](out)
        json.dump(out, open(path, "w"), indent=1)
        print("wrote", path)
        return
    out = {"note": "oracle (plain FP64 C) counts; inputs from workloads with the seeds below"}
    t = time.time()
    A = W.stencil_3d27(128)
    b = O.spmv(A, W.uniform_vec(A.nrows, 2))
    d, _ = O.jacobi_dinv(A)
    r = O.pcg(A, b, dinv=d, reduction=1e-10, max_iters=5000)
    out["stencil27_128_pcg_1e-10"] = dict(recipe="x* = U[-1,1) seed 2, b = A x*, x0 = 0",
                                          iterations=r["iterations"], stop=r["stop_reason"],
                                          rel_residual=r["rel_residual"])
    print("27pt", r["iterations"], time.time() - t, flush=True)
    del A, b, d
    A = W.aniso_3d7(160)
    b = W.uniform_vec(A.nrows, 4)
    d, _ = O.jacobi_dinv(A)
    for red in (1e-10, 1e-12):
        t = time.time()
        r = O.pcg(A, b, dinv=d, reduction=red, max_iters=5000)
        out[f"aniso7_160_pcg_{red:g}"] = dict(recipe="b = U[-1,1) seed 4, x0 = 0",
                                             iterations=r["iterations"], stop=r["stop_reason"],
                                             rel_residual=r["rel_residual"])
        print("aniso", red, r["iterations"], time.time() - t, flush=True)
    t = time.time()
    r = O.ir(A, b, outer_reduction=1e-12, inner_reduction=1e-4)
    out["aniso7_160_ir_1e-12_inner_1e-4"] = dict(recipe="b = U[-1,1) seed 4, x0 = 0",
                                                 outer=r["outer"], inner_iterations=r["inner_iterations"],
                                                 stop=r["stop_reason"], history=list(r["history"]))
    print("ir", r["outer"], r["inner_iterations"], time.time() - t, flush=True)
    bjacobi(out)
    gmres(out)
    ilu(out)
    bicgstab(out)
    bicgstab_spread(out)
    json.dump(out, open(path, "w"), indent=1)
    print("wrote", path)


if __name__ == "__main__":
    main()
