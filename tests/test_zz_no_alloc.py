"""mxl_batch_solve_noalloc against mxl_batch_solve.

The allocation-free entry point runs the same kernels with the work counter
and spill region in the library's fixed device array, so on the same batch
and schedule its outputs (x, iteration counts, residuals, stop reasons) must
equal mxl_batch_solve's bit for bit.  Two calls in a row, the second on a
smaller batch, check that the array's leftover contents from one call do not
leak into the next; a schedule whose spill region exceeds the array is
refused; and the device's free memory does not move across a call that
spills (where mxl_batch_solve allocates its spill region)."""
import ctypes as C

import numpy as np
import pytest
import torch

import oracle as O
import workloads as W
from tests._gpu import DEV, dev

pytestmark = pytest.mark.gpu

LIMIT = 96 << 20


@pytest.fixture(scope="module")
def mxl():
    import paper_2006_16852_amd as m
    return m


@pytest.fixture(scope="module")
def ctx(mxl):
    return mxl.Context(0)


def _big_batch():
    """The 64x64 Poisson system (4,096 rows: more than a workgroup's LDS
    holds at 2 workgroups per CU, so it runs from the spill region) among
    small banded systems."""
    A = W.stencil_2d5(64)
    b1 = O.spmv(A, W.uniform_vec(A.nrows, 1))
    S = W.batch_systems(nsys=40, seed=21)
    rp = np.concatenate([A.row_ptr[:-1], S.row_ptr + A.nnz]).astype(np.int32)
    sp = np.concatenate([[0], S.sys_ptr + A.nrows]).astype(np.int32)
    return W.Batch(41, sp, rp, np.concatenate([A.col, S.col]), np.concatenate([A.val, S.val]),
                   np.concatenate([b1, S.b]))


def _outputs(B):
    b = dev(B.b)
    return (b, torch.zeros_like(b), torch.zeros(B.nsys, dtype=torch.int32, device=DEV),
            torch.zeros(B.nsys, dtype=torch.float64, device=DEV),
            torch.zeros(B.nsys, dtype=torch.uint8, device=DEV))


def _handle(mxl, ctx, B):
    return mxl.batch(ctx, B.sys_ptr, dev(B.sys_ptr), dev(B.row_ptr), dev(B.col), dev(B.val))


def _solve(op, B, noalloc, tuning):
    b, x, it, rel, st = _outputs(B)
    if noalloc:
        op.solve_noalloc(b, x, it, rel, st, tuning=tuning, reduction=1e-10)
        torch.cuda.synchronize()
    else:
        op.solve(b, x, it, rel, st, tuning=tuning, reduction=1e-10)
    return [t.cpu().numpy() for t in (x, it, rel, st)]


def _check_solution(B, x, st):
    assert np.all(st == 1)
    for s in range(B.nsys):
        r0, r1 = B.sys_ptr[s], B.sys_ptr[s + 1]
        r = B.b[r0:r1] - O.spmv(B.system(s), x[r0:r1])
        assert np.linalg.norm(r) <= 1.01e-10 * np.linalg.norm(B.b[r0:r1]), s


@pytest.mark.parametrize("fmt", [1, 2], ids=["csr", "ell"])
def test_noalloc_equals_batch_solve_two_calls(mxl, ctx, fmt):
    big = _big_batch()
    small = W.batch_systems(nsys=200, seed=77)
    cases = [(big, (256, 2, 0, fmt)), (small, None)]  # the second call: fewer, smaller systems
    for B, tuning in cases:
        print(f"[noalloc] nsys {B.nsys} max rows {int(np.diff(B.sys_ptr).max())} tuning {tuning}",
              flush=True)
        op = _handle(mxl, ctx, B)
        got = _solve(op, B, True, tuning)
        want = _solve(_handle(mxl, ctx, B), B, False, tuning)
        for g, w, name in zip(got, want, ("x", "iters", "rel_res", "status")):
            assert np.array_equal(g, w), name
        _check_solution(B, got[0], got[3])


def test_noalloc_refuses_oversized_schedule(mxl, ctx):
    B = _big_batch()
    op = _handle(mxl, ctx, B)
    b, x, it, rel, st = _outputs(B)
    ncu = torch.cuda.get_device_properties(0).multi_processor_count
    need = 256 + 8 * ncu * 5 * 4096 * 8
    assert need > LIMIT
    with pytest.raises(mxl.MxlError) as e:
        op.solve_noalloc(b, x, it, rel, st, tuning=(256, 8, 0, 2), reduction=1e-10)
    assert e.value.status == mxl.ERR_INVALID_ARG
    assert "static limit" in str(e.value)


def test_noalloc_call_leaves_free_memory_unchanged(mxl, ctx):
    B = _big_batch()
    tuning = (256, 2, 0, 2)  # spills: mxl_batch_solve would allocate about 84 MB here
    op = _handle(mxl, ctx, B)
    b, x, it, rel, st = _outputs(B)
    op.solve_noalloc(b, x, it, rel, st, tuning=tuning, reduction=1e-10)  # loads the kernels
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info(0)[0]
    op.solve_noalloc(b, x, it, rel, st, tuning=tuning, reduction=1e-10)
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info(0)[0]
    assert free1 == free0
    # the allocating entry point on a fresh handle does take memory: the
    # measurement can see an allocation of this size
    op2 = _handle(mxl, ctx, B)
    torch.cuda.synchronize()
    free2 = torch.cuda.mem_get_info(0)[0]
    op2.solve(b, x, it, rel, st, tuning=tuning, reduction=1e-10)
    free3 = torch.cuda.mem_get_info(0)[0]
    assert free2 - free3 >= 80 << 20
    _check_solution(B, x.cpu().numpy(), st.cpu().numpy())
