"""Python binding of libmxl, the MI355X (gfx950) sparse linear-operator library.

Argument marshalling only: every step of SpMV, Jacobi, the Krylov solvers,
iterative refinement, the batched solver, the features and the MLP runs in
the HIP kernels of ``libmxl.so`` behind the C ABI of ``include/mxl.h``.
PyTorch provides device memory and the current HIP stream.  There is no CPU
fallback: if ``libmxl.so`` is missing, importing this package raises.
"""
from __future__ import annotations

import atexit
import ctypes as C
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmxl.so")

# ----------------------------------------------------------------- constants
F64, F32 = 0, 1
CSR, COO, ELL, HYB, STENCIL = 0, 1, 2, 3, 4
CSR_SCALAR, CSR_VECTOR, CSR_MERGE, CSR_STREAM = 0, 1, 2, 3
COO_SEGRED = 0
ELL_PLAIN, ELL_LDS, ELL_DELTA16 = 0, 1, 2
OP_MATRIX, OP_JACOBI, OP_SOLVER, OP_BATCH, OP_ILU = 0, 1, 2, 3, 4
SOLVER_CG, SOLVER_BICGSTAB, SOLVER_IR, SOLVER_GMRES = 0, 1, 2, 3
STOP_NONE, STOP_CONVERGED, STOP_MAX_ITERS, STOP_TIME, STOP_BREAKDOWN, STOP_NONFINITE = range(6)
OK, ERR_INVALID_ARG, ERR_DIM_MISMATCH, ERR_DTYPE, ERR_NOT_IMPLEMENTED, ERR_INVALID_MATRIX, \
    ERR_ZERO_DIAG, ERR_OUT_OF_MEMORY, ERR_INFEASIBLE_FORMAT, ERR_DEVICE, ERR_INTERNAL = range(11)
STATUS_NAMES = ["OK", "INVALID_ARG", "DIM_MISMATCH", "DTYPE", "NOT_IMPLEMENTED",
                "INVALID_MATRIX", "ZERO_DIAG", "OUT_OF_MEMORY", "INFEASIBLE_FORMAT", "DEVICE",
                "INTERNAL"]
STOP_NAMES = ["none", "converged", "max_iters", "time", "breakdown", "nonfinite"]
FORMATS = {"csr": CSR, "coo": COO, "ell": ELL, "hyb": HYB}
EXPORT_IDS = {"row_ptr": 0, "col": 1, "val": 2, "coo_row": 3, "ell_col": 4, "ell_val": 5,
              "tail_row": 6, "tail_col": 7, "tail_val": 8, "dinv": 9}


class MxlError(RuntimeError):
    def __init__(self, status: int, msg: str):
        self.status = status
        name = STATUS_NAMES[status] if 0 <= status < len(STATUS_NAMES) else str(status)
        super().__init__(f"mxl {name}: {msg}")


class Criteria(C.Structure):
    _fields_ = [("max_iters", C.c_int64), ("reduction", C.c_double),
                ("time_limit_s", C.c_double), ("check_every", C.c_int32),
                ("nonfinite_check", C.c_int32), ("launch_mode", C.c_int32)]


class SolveInfo(C.Structure):
    _fields_ = [("iterations", C.c_int64), ("spmv_count", C.c_int64),
                ("rel_residual", C.c_double), ("stop_reason", C.c_int32),
                ("seconds", C.c_double), ("history", C.POINTER(C.c_double)),
                ("history_cap", C.c_int64), ("inner_iterations", C.c_int64),
                ("time_spmv", C.c_int32), ("spmv_ms", C.c_double), ("spmv_timed", C.c_int64),
                ("restarts", C.c_int64), ("reorth", C.c_int64)]


class FormatParams(C.Structure):
    _fields_ = [("variant", C.c_int32), ("vector_width", C.c_int32),
                ("hyb_quantile", C.c_double)]


class OpDesc(C.Structure):
    _fields_ = [("kind", C.c_int32), ("format", C.c_int32), ("variant", C.c_int32),
                ("dtype", C.c_int32), ("nrows", C.c_int64), ("ncols", C.c_int64),
                ("nnz", C.c_int64), ("vector_width", C.c_int32), ("ell_width", C.c_int32),
                ("n_pad", C.c_int64), ("tail_nnz", C.c_int64), ("stored_bytes", C.c_int64),
                ("ell_reuse", C.c_int32)]


class IrParams(C.Structure):
    _fields_ = [("outer", Criteria), ("inner", Criteria), ("inner_block_size", C.c_int32),
                ("inner_block_accuracy", C.c_double), ("inner_block_mode", C.c_int32)]


class Tuning(C.Structure):
    _fields_ = [("wg_size", C.c_int32), ("wgs_per_cu", C.c_int32), ("order", C.c_int32), ("format", C.c_int32)]


class KernelClass(C.Structure):
    _fields_ = [("format", C.c_int32), ("params", FormatParams)]


class SelectInfo(C.Structure):
    _fields_ = [("margin", C.c_double), ("max_z", C.c_double), ("fallback", C.c_int32),
                ("ntimed", C.c_int32), ("best_ms", C.c_double)]


SELECT_MODEL, SELECT_EXHAUSTIVE, SELECT_MODEL_FALLBACK = 0, 1, 2


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; "
            f"g.build()'` (hipcc, gfx950). There is no CPU fallback.")
    L = C.CDLL(LIB_PATH)
    vp, i64, i32, f64, st = C.c_void_p, C.c_int64, C.c_int32, C.c_double, C.c_int
    pp = C.POINTER(C.c_void_p)
    sig = {
        "mxl_ctx_create": [C.c_int, vp, pp],
        "mxl_ctx_set_stream": [vp, vp],
        "mxl_ctx_destroy": [vp],
        "mxl_csr_create": [vp, C.c_int, i64, i64, i64, vp, vp, vp, C.c_int, pp],
        "mxl_convert": [vp, C.c_int, C.POINTER(FormatParams), pp],
        "mxl_cast": [vp, C.c_int, pp],
        "mxl_apply": [vp, vp, vp],
        "mxl_apply_adv": [vp, f64, vp, f64, vp],
        "mxl_op_describe": [vp, C.POINTER(OpDesc)],
        "mxl_op_export": [vp, i32, vp, i64],
        "mxl_op_destroy": [vp],
        "mxl_jacobi_generate": [vp, pp],
        "mxl_solver_generate": [C.c_int, vp, vp, C.POINTER(Criteria), pp],
        "mxl_gmres_generate": [vp, vp, C.POINTER(Criteria), C.c_int32, pp],
        "mxl_solve": [vp, vp, vp, C.POINTER(SolveInfo)],
        "mxl_ir_generate": [vp, C.POINTER(IrParams), pp],
        "mxl_batch_csr_create": [vp, i64, vp, vp, vp, vp, vp, C.c_int, pp],
        "mxl_batch_solve": [vp, C.POINTER(Criteria), C.POINTER(Tuning), vp, vp, vp, vp, vp],
        "mxl_batch_solve_noalloc": [vp, C.POINTER(Criteria), C.POINTER(Tuning), vp, vp, vp, vp, vp],
        "mxl_batch_autotune": [vp, C.POINTER(Criteria), vp, vp, C.c_int, C.POINTER(Tuning),
                               C.POINTER(C.c_double)],
        "mxl_features": [vp, vp],
        "mxl_time_apply": [vp, vp, vp, C.c_int, C.c_int, C.POINTER(C.c_double)],
        "mxl_stream_bench": [vp, C.c_int, i64, vp, vp, vp, C.c_int, C.POINTER(C.c_double)],
        "mxl_mlp_create": [vp, i32, vp, vp, pp],
        "mxl_mlp_get_params": [vp, vp, i64],
        "mxl_mlp_set_params": [vp, vp, i64],
        "mxl_mlp_forward": [vp, i64, vp, vp],
        "mxl_mlp_loss_grad": [vp, i64, vp, vp, vp, C.c_float, vp],
        "mxl_mlp_get_grad": [vp, vp, i64],
        "mxl_mlp_adam_step": [vp, i64, C.c_float, C.c_float, C.c_float, C.c_float],
        "mxl_mlp_destroy": [vp],
        "mxl_selector_create": [vp, i32, vp, i32, vp, vp, vp, vp, C.c_uint32, f64, f64, pp],
        "mxl_stencil_create": [vp, C.c_int, i64, i64, i64, i32, vp, vp, pp],
        "mxl_bjacobi_generate": [vp, i32, i32, f64, pp],
        "mxl_bjacobi_info": [vp, C.POINTER(C.c_int64), vp, vp, vp, C.POINTER(C.c_int64)],
        "mxl_bjacobi_generate_var": [vp, i64, vp, i32, i32, f64, pp],
        "mxl_bjacobi_blocks": [vp, vp],
        "mxl_ilu_generate": [vp, i32, i32, i32, pp],
        "mxl_ilu_info": [vp, vp, vp],
        "mxl_selector_destroy": [vp],
        "mxl_select": [vp, vp, i32, vp, vp, i32, C.POINTER(C.c_int32), vp, vp,
                       C.POINTER(SelectInfo)],
    }
    for name, args in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = st
    L.mxl_last_error.restype = C.c_char_p
    L.mxl_last_error.argtypes = []
    L.mxl_version.restype = C.c_char_p
    L.mxl_version.argtypes = []
    return L


lib = _load()
_alive = [True]


@atexit.register
def _shutdown():
    # handles still referenced at interpreter exit are reclaimed by the
    # process teardown; calling into HIP from finalizers then is unsafe
    _alive[0] = False


def _check(status: int):
    if status != OK:
        raise MxlError(status, lib.mxl_last_error().decode(errors="replace"))


def _ptr(t):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        raise TypeError("expected a torch tensor")
    return C.c_void_p(t.data_ptr())


def _dtype_code(t: torch.Tensor) -> int:
    if t.dtype == torch.float64:
        return F64
    if t.dtype == torch.float32:
        return F32
    raise MxlError(ERR_DTYPE, f"unsupported value dtype {t.dtype}")


def _torch_dtype(code: int):
    return torch.float64 if code == F64 else torch.float32


def _need_cuda(*ts):
    for t in ts:
        if t is not None and (not t.is_cuda or not t.is_contiguous()):
            raise MxlError(ERR_INVALID_ARG, "tensors must be contiguous and on the GPU")


def version() -> str:
    return lib.mxl_version().decode()


class Context:
    """Executor: one device plus torch's current HIP stream."""

    def __init__(self, device: int = 0):
        self.device = device
        h = C.c_void_p()
        with torch.cuda.device(device):
            stream = torch.cuda.current_stream(device).cuda_stream
        _check(lib.mxl_ctx_create(device, C.c_void_p(stream), C.byref(h)))
        self.h = h

    def use_current_stream(self):
        s = torch.cuda.current_stream(self.device).cuda_stream
        _check(lib.mxl_ctx_set_stream(self.h, C.c_void_p(s)))

    def __del__(self):
        if getattr(self, "h", None) and _alive and _alive[0]:
            lib.mxl_ctx_destroy(self.h)
            self.h = None


class Op:
    """Reference-counted operator handle (matrix, Jacobi, solver)."""

    def __init__(self, h, ctx, keep=(), parents=()):
        self.h = h
        self.ctx = ctx
        self._keep = tuple(keep)      # borrowed tensors must outlive the handle
        self._parents = tuple(parents)

    def describe(self) -> dict:
        d = OpDesc()
        _check(lib.mxl_op_describe(self.h, C.byref(d)))
        return {f: getattr(d, f) for f, _ in OpDesc._fields_}

    @property
    def nrows(self):
        return self.describe()["nrows"]

    @property
    def dtype(self):
        return _torch_dtype(self.describe()["dtype"])

    def export(self, which: str) -> torch.Tensor:
        d = self.describe()
        n, nnz, w, npad, tail = d["nrows"], d["nnz"], d["ell_width"], d["n_pad"], d["tail_nnz"]
        vt = _torch_dtype(d["dtype"])
        shape = {"row_ptr": (n + 1, torch.int32), "col": (nnz, torch.int32), "val": (nnz, vt),
                 "coo_row": (nnz, torch.int32),
                 "ell_col": (w * npad, torch.int16 if (d["format"] == ELL and d["variant"] == ELL_DELTA16)
                             else torch.int32),
                 "ell_val": (w * npad, vt), "tail_row": (tail, torch.int32),
                 "tail_col": (tail, torch.int32), "tail_val": (tail, vt), "dinv": (n, vt)}[which]
        out = torch.empty(max(shape[0], 1), dtype=shape[1], device=f"cuda:{self.ctx.device}")
        self.ctx.use_current_stream()
        _check(lib.mxl_op_export(self.h, EXPORT_IDS[which], _ptr(out),
                                 out.numel() * out.element_size()))
        return out[:shape[0]]

    def apply(self, b: torch.Tensor, x: torch.Tensor, alpha: float = 1.0, beta: float = 0.0):
        """x = alpha * L(b) + beta * x (stream-ordered)."""
        _need_cuda(b, x)
        self.ctx.use_current_stream()
        _check(lib.mxl_apply_adv(self.h, alpha, _ptr(b), beta, _ptr(x)))
        return x

    def convert(self, fmt: str, variant: int = 0, vector_width: int = 0,
                hyb_quantile: float = 0.0) -> "Op":
        p = FormatParams(variant, vector_width, hyb_quantile)
        h = C.c_void_p()
        self.ctx.use_current_stream()
        _check(lib.mxl_convert(self.h, FORMATS[fmt], C.byref(p), C.byref(h)))
        return Op(h, self.ctx, parents=(self,))

    def cast(self, dtype) -> "Op":
        code = F64 if dtype == torch.float64 else F32
        h = C.c_void_p()
        self.ctx.use_current_stream()
        _check(lib.mxl_cast(self.h, code, C.byref(h)))
        return Op(h, self.ctx, parents=(self,))

    def time_apply(self, x, y, reps=20, flush=False) -> float:
        _need_cuda(x, y)
        ms = C.c_double()
        self.ctx.use_current_stream()
        _check(lib.mxl_time_apply(self.h, _ptr(x), _ptr(y), reps, int(flush), C.byref(ms)))
        return ms.value

    def features(self):
        import numpy as np
        out = np.zeros(16)
        self.ctx.use_current_stream()
        _check(lib.mxl_features(self.h, out.ctypes.data_as(C.c_void_p)))
        return out

    def __del__(self):
        if getattr(self, "h", None) and _alive and _alive[0]:
            lib.mxl_op_destroy(self.h)
            self.h = None


def csr(ctx: Context, row_ptr, col, val, ncols=None, copy=False, validate=False) -> Op:
    """Wrap device CSR arrays (int32 row_ptr/col, float64/float32 values)."""
    _need_cuda(row_ptr, col, val)
    if row_ptr.dtype != torch.int32 or col.dtype != torch.int32:
        raise MxlError(ERR_INVALID_ARG, "row_ptr and col must be int32")
    n = row_ptr.numel() - 1
    ncols = n if ncols is None else ncols
    flags = (1 if copy else 0) | (2 if validate else 0)
    h = C.c_void_p()
    ctx.use_current_stream()
    _check(lib.mxl_csr_create(ctx.h, _dtype_code(val), n, ncols, col.numel(), _ptr(row_ptr),
                              _ptr(col), _ptr(val), flags, C.byref(h)))
    return Op(h, ctx, keep=() if copy else (row_ptr, col, val))


def stencil(ctx: Context, shape, points, coefs, dtype=torch.float64) -> Op:
    """Matrix-free constant-coefficient stencil on an (nx, ny, nz) grid:
    points = [(di, dj, dk), ...] with entries in {-1, 0, 1}, coefs the
    matching coefficients (Dirichlet boundary)."""
    import numpy as np
    nx, ny, nz = (tuple(shape) + (1, 1))[:3]
    off = np.ascontiguousarray(np.asarray(points, np.int32).reshape(-1, 3))
    cf = np.ascontiguousarray(np.asarray(coefs, np.float64))
    if off.shape[0] != cf.size:
        raise MxlError(ERR_DIM_MISMATCH, "one coefficient per point")
    code = F64 if dtype == torch.float64 else F32
    h = C.c_void_p()
    ctx.use_current_stream()
    _check(lib.mxl_stencil_create(ctx.h, code, nx, ny, nz, cf.size, off.ctypes.data_as(C.c_void_p),
                                  cf.ctypes.data_as(C.c_void_p), C.byref(h)))
    return Op(h, ctx)


def stream_bench(ctx: Context, op: str, a, b=None, c=None, reps: int = 10) -> float:
    """Median ms of a STREAM-style kernel: 'copy' c = a, 'triad' c = a + 0.5 b,
    'dot' a.b (c receives per-workgroup partials), 'read' sum of a with
    ordinary (caching) loads (c receives partials)."""
    code = {"copy": 0, "triad": 1, "dot": 2, "read": 3}[op]
    ms = C.c_double()
    ctx.use_current_stream()
    _check(lib.mxl_stream_bench(ctx.h, code, a.numel(), _ptr(a), _ptr(b), _ptr(c), reps,
                                C.byref(ms)))
    return ms.value


def jacobi(A: Op) -> Op:
    h = C.c_void_p()
    A.ctx.use_current_stream()
    _check(lib.mxl_jacobi_generate(A.h, C.byref(h)))
    return Op(h, A.ctx, parents=(A,))


class BlockJacobi(Op):
    """Block-Jacobi preconditioner (inverted diagonal blocks, adaptive
    storage precision)."""

    def info(self, inverses: bool = False) -> dict:
        import numpy as np
        nb = C.c_int64()
        nbytes = C.c_int64()
        _check(lib.mxl_bjacobi_info(self.h, C.byref(nb), None, None, None, C.byref(nbytes)))
        cond = np.zeros(max(nb.value, 1))
        prec = np.zeros(max(nb.value, 1), np.int32)
        inv = None
        ptr_inv = None
        if inverses:
            sizes = np.diff(self.blocks()).astype(np.int64)
            inv = np.zeros(max(int((sizes ** 2).sum()), 1))
            ptr_inv = inv.ctypes.data_as(C.c_void_p)
        _check(lib.mxl_bjacobi_info(self.h, C.byref(nb), cond.ctypes.data_as(C.c_void_p),
                                    prec.ctypes.data_as(C.c_void_p), ptr_inv, C.byref(nbytes)))
        out = dict(nblocks=nb.value, cond=cond[:nb.value], precision=prec[:nb.value],
                   storage_bytes=nbytes.value)
        if inverses:
            out["inv"] = inv
        return out

    def blocks(self):
        """Block boundaries (int32, nblocks + 1 entries)."""
        import numpy as np
        nb = C.c_int64()
        _check(lib.mxl_bjacobi_info(self.h, C.byref(nb), None, None, None, None))
        bp = np.zeros(nb.value + 1, np.int32)
        _check(lib.mxl_bjacobi_blocks(self.h, bp.ctypes.data_as(C.c_void_p)))
        return bp


class Ilu(Op):
    """ILU-type preconditioner: ParILU factors on A's pattern, applied by two
    triangular solves (exact or Jacobi sweeps)."""

    def info(self, factors: bool = False) -> dict:
        import numpy as np
        lev = (C.c_int32 * 2)()
        lu = np.zeros(max(self.describe()["nnz"], 1)) if factors else None
        _check(lib.mxl_ilu_info(self.h, lu.ctypes.data_as(C.c_void_p) if factors else None,
                                C.cast(lev, C.c_void_p)))
        out = dict(levels_lower=lev[0], levels_upper=lev[1])
        if factors:
            out["lu"] = lu[:self.describe()["nnz"]]
        return out


def ilu(A: Op, sweeps: int = 5, trisolve: str = "exact", trs_sweeps: int = 0) -> Ilu:
    """ParILU(sweeps) factors; trisolve "exact" (level-scheduled
    substitution) or "jacobi" (trs_sweeps Jacobi sweeps per triangle)."""
    h = C.c_void_p()
    A.ctx.use_current_stream()
    mode = {"exact": 0, "jacobi": 1}[trisolve]
    _check(lib.mxl_ilu_generate(A.h, int(sweeps), mode, int(trs_sweeps), C.byref(h)))
    return Ilu(h, A.ctx, parents=(A,))


def bjacobi(A: Op, block_size: int = 8, adaptive: bool = True, accuracy: float = 0.1) -> BlockJacobi:
    h = C.c_void_p()
    A.ctx.use_current_stream()
    _check(lib.mxl_bjacobi_generate(A.h, block_size, int(adaptive), accuracy, C.byref(h)))
    return BlockJacobi(h, A.ctx, parents=(A,))


def bjacobi_var(A: Op, bptr=None, max_block_size: int = 32, adaptive: bool = True,
                accuracy: float = 0.1) -> BlockJacobi:
    """Block Jacobi with blocks of varying size: the given boundaries (int32
    host array, nblocks + 1 entries) or, with bptr None, supervariable
    agglomeration with at most max_block_size rows per block."""
    import numpy as np
    h = C.c_void_p()
    A.ctx.use_current_stream()
    if bptr is None:
        _check(lib.mxl_bjacobi_generate_var(A.h, 0, None, max_block_size, int(adaptive), accuracy, C.byref(h)))
    else:
        bp = np.ascontiguousarray(bptr, np.int32)
        _check(lib.mxl_bjacobi_generate_var(A.h, bp.size - 1, bp.ctypes.data_as(C.c_void_p), max_block_size,
                                            int(adaptive), accuracy, C.byref(h)))
    return BlockJacobi(h, A.ctx, parents=(A,))


def criteria(max_iters=10_000, reduction=1e-10, time_limit=0.0, check_every=1,
             nonfinite_check=1, launch_mode=0) -> Criteria:
    """launch_mode (CG, BiCGSTAB): 0 auto, 1 one kernel per step, 2 one persistent workgroup."""
    return Criteria(max_iters, reduction, time_limit, check_every, nonfinite_check, launch_mode)


class Solver(Op):
    def solve(self, b: torch.Tensor, x: torch.Tensor, history: int = 0,
              time_spmv: int = 0) -> dict:
        """Solve A x = b in place (x = initial guess on entry).  time_spmv = k > 0
        times every k-th SpMV launch of the CG loop with HIP events (True = 1)."""
        _need_cuda(b, x)
        info = SolveInfo()
        info.time_spmv = int(time_spmv)
        hbuf = None
        if history:
            hbuf = (C.c_double * history)()
            info.history = C.cast(hbuf, C.POINTER(C.c_double))
            info.history_cap = history
        self.ctx.use_current_stream()
        _check(lib.mxl_solve(self.h, _ptr(b), _ptr(x), C.byref(info)))
        out = dict(iterations=info.iterations, spmv_count=info.spmv_count,
                   rel_residual=info.rel_residual, stop_reason=info.stop_reason,
                   stop=STOP_NAMES[info.stop_reason], seconds=info.seconds,
                   inner_iterations=info.inner_iterations, spmv_ms=info.spmv_ms,
                   spmv_timed=info.spmv_timed, restarts=info.restarts, reorth=info.reorth)
        if history:
            cnt = min(history, (info.iterations + 1))
            out["history"] = list(hbuf[:cnt])
        return out


def solver(kind: str, A: Op, P: Op = None, krylov_dim: int = None, **crit) -> Solver:
    """kind: "cg", "bicgstab" or "gmres" (GMRES(krylov_dim), default 100)."""
    k = {"cg": SOLVER_CG, "bicgstab": SOLVER_BICGSTAB, "gmres": SOLVER_GMRES}[kind]
    c = criteria(**crit)
    h = C.c_void_p()
    A.ctx.use_current_stream()
    Ph = P.h if P is not None else None
    if kind == "gmres" and krylov_dim is not None:
        _check(lib.mxl_gmres_generate(A.h, Ph, C.byref(c), int(krylov_dim), C.byref(h)))
    else:
        _check(lib.mxl_solver_generate(k, A.h, Ph, C.byref(c), C.byref(h)))
    return Solver(h, A.ctx, parents=(A,) + ((P,) if P is not None else ()))


class Batch(Op):
    """Independent small systems solved by batched Jacobi-PCG in one launch."""

    def solve(self, b, x, iters, rel_res, status, tuning=None, **crit) -> None:
        _need_cuda(b, x, iters, rel_res, status)
        c = criteria(**({"max_iters": 0} | crit))
        t = Tuning(*tuning) if tuning is not None else None
        self.ctx.use_current_stream()
        _check(lib.mxl_batch_solve(self.h, C.byref(c), C.byref(t) if t is not None else None,
                                   _ptr(b), _ptr(x), _ptr(iters), _ptr(rel_res), _ptr(status)))

    def solve_noalloc(self, b, x, iters, rel_res, status, tuning=None, **crit) -> None:
        """mxl_batch_solve_noalloc: enqueued on the stream, no allocation, no host wait."""
        _need_cuda(b, x, iters, rel_res, status)
        c = criteria(**({"max_iters": 0} | crit))
        t = Tuning(*tuning) if tuning is not None else None
        self.ctx.use_current_stream()
        _check(lib.mxl_batch_solve_noalloc(self.h, C.byref(c), C.byref(t) if t is not None else None,
                                           _ptr(b), _ptr(x), _ptr(iters), _ptr(rel_res), _ptr(status)))

    def autotune(self, b, x_scratch, reps: int = 2, **crit):
        """Time every schedule on this batch; returns ((wg_size, wgs_per_cu, order, format), ms)."""
        _need_cuda(b, x_scratch)
        c = criteria(**({"max_iters": 0} | crit))
        t = Tuning()
        ms = C.c_double()
        self.ctx.use_current_stream()
        _check(lib.mxl_batch_autotune(self.h, C.byref(c), _ptr(b), _ptr(x_scratch), reps,
                                      C.byref(t), C.byref(ms)))
        return (t.wg_size, t.wgs_per_cu, t.order, t.format), ms.value


def batch(ctx: Context, sys_ptr_host, sys_ptr, row_ptr, col, val) -> Batch:
    """sys_ptr_host: numpy int32 row offsets of the systems; the rest device tensors."""
    import numpy as np
    sp = np.ascontiguousarray(sys_ptr_host, dtype=np.int32)
    _need_cuda(sys_ptr, row_ptr, col, val)
    h = C.c_void_p()
    ctx.use_current_stream()
    _check(lib.mxl_batch_csr_create(ctx.h, sp.size - 1, sp.ctypes.data_as(C.c_void_p),
                                    _ptr(sys_ptr), _ptr(row_ptr), _ptr(col), _ptr(val), 0,
                                    C.byref(h)))
    return Batch(h, ctx, keep=(sys_ptr, row_ptr, col, val))


class Mlp:
    """FP32 MLP whose forward pass, gradient and Adam step run on the GPU."""

    def __init__(self, ctx: Context, dims, theta=None):
        import numpy as np
        self.ctx = ctx
        self.dims = list(dims)
        self.nparams = sum(self.dims[i + 1] * self.dims[i] + self.dims[i + 1]
                           for i in range(len(self.dims) - 1))
        d = np.asarray(self.dims, np.int32)
        th = None if theta is None else np.ascontiguousarray(theta, np.float32)
        if th is not None and th.size != self.nparams:
            raise MxlError(ERR_DIM_MISMATCH, "theta size")
        h = C.c_void_p()
        ctx.use_current_stream()
        _check(lib.mxl_mlp_create(ctx.h, len(self.dims) - 1, d.ctypes.data_as(C.c_void_p),
                                  th.ctypes.data_as(C.c_void_p) if th is not None else None,
                                  C.byref(h)))
        self.h = h

    def params(self):
        import numpy as np
        out = np.zeros(self.nparams, np.float32)
        _check(lib.mxl_mlp_get_params(self.h, out.ctypes.data_as(C.c_void_p), self.nparams))
        return out

    def set_params(self, theta):
        import numpy as np
        th = np.ascontiguousarray(theta, np.float32)
        _check(lib.mxl_mlp_set_params(self.h, th.ctypes.data_as(C.c_void_p), th.size))

    def grad(self):
        import numpy as np
        out = np.zeros(self.nparams, np.float32)
        _check(lib.mxl_mlp_get_grad(self.h, out.ctypes.data_as(C.c_void_p), self.nparams))
        return out

    def forward(self, X: torch.Tensor) -> torch.Tensor:
        _need_cuda(X)
        Y = torch.empty((X.shape[0], self.dims[-1]), dtype=torch.float32, device=X.device)
        self.ctx.use_current_stream()
        _check(lib.mxl_mlp_forward(self.h, X.shape[0], _ptr(X), _ptr(Y)))
        return Y

    def loss_grad(self, X, T, M, lam: float = 1e-4) -> float:
        _need_cuda(X, T, M)
        loss = C.c_float()
        self.ctx.use_current_stream()
        _check(lib.mxl_mlp_loss_grad(self.h, X.shape[0], _ptr(X), _ptr(T), _ptr(M), lam,
                                     C.byref(loss)))
        return loss.value

    def adam_step(self, t: int, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        self.ctx.use_current_stream()
        _check(lib.mxl_mlp_adam_step(self.h, t, lr, beta1, beta2, eps))

    def __del__(self):
        if getattr(self, "h", None) and _alive and _alive[0]:
            lib.mxl_mlp_destroy(self.h)
            self.h = None


class SelectorHandle:
    """A trained format/kernel selector living in the library (mxl_select).

    classes: list of (format name, convert kwargs) as for Op.convert."""

    def __init__(self, ctx: Context, classes, dims, theta, mean, std, log_features,
                 delta: float = 0.05, zmax: float = 4.0):
        import numpy as np
        self.ctx = ctx
        self.classes = list(classes)
        k = (KernelClass * len(self.classes))()
        for i, (fmt, kw) in enumerate(self.classes):
            k[i].format = FORMATS[fmt]
            k[i].params = FormatParams(kw.get("variant", 0), kw.get("vector_width", 0),
                                       kw.get("hyb_quantile", 0.0))
        d = np.asarray(dims, np.int32)
        th = np.ascontiguousarray(theta, np.float32)
        mu = np.ascontiguousarray(mean, np.float64)
        sd = np.ascontiguousarray(std, np.float64)
        mask = 0
        for j in log_features:
            mask |= 1 << int(j)
        h = C.c_void_p()
        ctx.use_current_stream()
        _check(lib.mxl_selector_create(ctx.h, len(self.classes), C.cast(k, C.c_void_p), len(d) - 1,
                                       d.ctypes.data_as(C.c_void_p), th.ctypes.data_as(C.c_void_p),
                                       mu.ctypes.data_as(C.c_void_p), sd.ctypes.data_as(C.c_void_p),
                                       mask, delta, zmax, C.byref(h)))
        self.h = h

    def select(self, A: Op, mode: int = SELECT_MODEL_FALLBACK, x: torch.Tensor = None,
               y: torch.Tensor = None, reps: int = 5):
        """Returns (class index, info dict with scores, times_ms, margin, ...)."""
        import numpy as np
        if x is not None or y is not None:
            _need_cuda(x, y)
        n = len(self.classes)
        sc = np.zeros(n)
        tm = np.zeros(n)
        out = C.c_int32()
        info = SelectInfo()
        self.ctx.use_current_stream()
        _check(lib.mxl_select(self.h, A.h, mode, _ptr(x) if x is not None else None,
                              _ptr(y) if y is not None else None, reps, C.byref(out),
                              sc.ctypes.data_as(C.c_void_p), tm.ctypes.data_as(C.c_void_p),
                              C.byref(info)))
        return int(out.value), dict(scores=sc, times_ms=tm, margin=info.margin, max_z=info.max_z,
                                    fallback=bool(info.fallback), ntimed=info.ntimed,
                                    best_ms=info.best_ms)

    def __del__(self):
        if getattr(self, "h", None) and _alive and _alive[0]:
            lib.mxl_selector_destroy(self.h)
            self.h = None


def ir(A: Op, outer: dict = None, inner: dict = None, block_size: int = 0,
       block_accuracy: float = 0.1, block_mode: int = 0) -> Solver:
    """FP64-outer / FP32-inner-CG iterative refinement operator; block_size > 0
    preconditions the inner CG with adaptive block Jacobi (block_mode 0:
    uniform blocks, 1: supervariable blocks of at most block_size rows)."""
    o = criteria(**({"max_iters": 50, "reduction": 1e-12} | (outer or {})))
    i = criteria(**({"max_iters": 10_000, "reduction": 1e-4} | (inner or {})))
    prm = IrParams(o, i, block_size, block_accuracy, block_mode)
    h = C.c_void_p()
    A.ctx.use_current_stream()
    _check(lib.mxl_ir_generate(A.h, C.byref(prm), C.byref(h)))
    return Solver(h, A.ctx, parents=(A,))
