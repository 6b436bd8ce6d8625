// runtime.hip -- host runtime behind the C ABI of include/mxl.h: context,
// reference-counted operator handles, argument validation, format
// conversion, and the host side of the Krylov solvers (kernel sequencing,
// criterion checks, convergence records).
//
// The solver loops keep every scalar on the device: a kernel publishes one
// partial per workgroup and the kernel that needs the scalar reduces all of
// them in its prologue; the host only reads the solver state every
// check_every iterations to evaluate the Time criterion and to stop
// launching.  Kernels enqueued after a device-side stop
// return immediately, so the result does not depend on check_every.
#include <algorithm>
#include <chrono>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "device_common.hpp"
#include "internal.hpp"

using namespace mxl;

namespace {

mxl_status fail(mxl_status st, const std::string &msg) { return mxl::record_error(st, msg.c_str()); }

mxl_status hip_fail(hipError_t e, const char *where) {
    return fail(e == hipErrorOutOfMemory ? MXL_ERR_OUT_OF_MEMORY : MXL_ERR_DEVICE,
                std::string(where) + ": " + hipGetErrorString(e));
}

#define HIP_TRY(expr)                                      \
    do {                                                   \
        hipError_t _e = (expr);                            \
        if (_e != hipSuccess) return hip_fail(_e, #expr);  \
    } while (0)

BufPtr alloc(size_t bytes, hipError_t *err) {
    auto b = std::make_shared<DevBuf>();
    b->bytes = bytes;
    b->owned = true;
    *err = hipMalloc(&b->p, bytes > 0 ? bytes : 16);
    if (*err != hipSuccess) {
        b->p = nullptr;
        b->owned = false;
        return nullptr;
    }
    return b;
}

BufPtr borrow(const void *p, size_t bytes) {
    auto b = std::make_shared<DevBuf>();
    b->p = const_cast<void *>(p);
    b->bytes = bytes;
    b->owned = false;
    return b;
}

}  // namespace
namespace mxl {
size_t vt_size(int dtype) { return dtype == MXL_F64 ? 8 : 4; }
}  // namespace mxl
namespace {

// Device pointer on ctx's device whose allocation covers `bytes` from p.
mxl_status check_dev(const mxl_ctx *ctx, const void *p, size_t bytes, const char *what) {
    if (bytes == 0) return MXL_OK;
    if (!p) return fail(MXL_ERR_INVALID_ARG, std::string(what) + " is NULL");
    hipPointerAttribute_t attr;
    if (hipPointerGetAttributes(&attr, p) != hipSuccess) {
        (void)hipGetLastError();
        return fail(MXL_ERR_INVALID_ARG, std::string(what) + " is not device memory");
    }
    if (attr.type != hipMemoryTypeDevice || attr.device != ctx->device)
        return fail(MXL_ERR_INVALID_ARG, std::string(what) + " is not device memory of the context's device");
    void *base = nullptr;
    size_t size = 0;
    if (hipMemGetAddressRange(&base, &size, const_cast<void *>(p)) == hipSuccess && base) {
        size_t off = (size_t)((const char *)p - (const char *)base);
        if (off + bytes > size)
            return fail(MXL_ERR_DIM_MISMATCH, std::string(what) + " is shorter than the operator needs");
    } else {
        (void)hipGetLastError();
    }
    return MXL_OK;
}

template <typename T>
mxl_status to_host(const mxl_ctx *ctx, const BufPtr &b, std::vector<T> &out, size_t count) {
    out.resize(count);
    if (count == 0) return MXL_OK;
    HIP_TRY(hipMemcpyAsync(out.data(), b->p, count * sizeof(T), hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    return MXL_OK;
}

int auto_vector_width(int64_t n, int64_t nnz) {
    double mean = n > 0 ? (double)nnz / (double)n : 1.0;
    int w = 2;
    while (w < 64 && w < mean) w <<= 1;
    return w;
}

mxl_status finish_matrix(MatrixImpl &A) {
    spmv_plan(A);
    return MXL_OK;
}

}  // namespace
namespace mxl {
int64_t csr_bytes(const MatrixImpl &A) {
    return A.nnz * (int64_t)(vt_size(A.dtype) + 4) + (A.nrows + 1) * 4;
}

bool ell_fits(const MatrixImpl &S, int64_t w) {
    const int64_t n_pad = ((S.nrows + 63) / 64) * 64;
    const double ell_bytes = (double)w * (double)n_pad * (double)(vt_size(S.dtype) + 4);
    const double budget = std::min(std::max(4.0 * (double)csr_bytes(S), (double)(1 << 20)),
                                   32.0 * (double)(1ull << 30));
    return ell_bytes <= budget || ell_bytes <= 0;
}

int64_t quantile_rank(double q, int64_t n) {
    const int64_t rank = (int64_t)std::ceil(q * (double)n);
    return std::min<int64_t>(std::max<int64_t>(rank, 1), n);
}
}  // namespace mxl
namespace {

void compute_stored_bytes(MatrixImpl &A) {
    const int64_t vt = (int64_t)vt_size(A.dtype);
    switch (A.format) {
    case MXL_FMT_STENCIL: A.stored_bytes = 0; break;
    case MXL_FMT_CSR: A.stored_bytes = csr_bytes(A); break;
    case MXL_FMT_COO: A.stored_bytes = A.nnz * (vt + 8); break;
    case MXL_FMT_ELL:
        A.stored_bytes = (int64_t)A.ell_w * A.n_pad * (vt + (A.variant == MXL_ELL_DELTA16 ? 2 : 4));
        break;
    case MXL_FMT_HYB:
        A.stored_bytes = (int64_t)A.ell_w * A.n_pad * (vt + 4) + A.tail_nnz * (vt + 8);
        break;
    }
}

mxl_op *wrap_matrix(std::shared_ptr<MatrixImpl> m) {
    auto *op = new mxl_op;
    op->kind = MXL_OP_MATRIX;
    op->mat = std::move(m);
    return op;
}

// Merge-path partition and carry buffers of a CSR merge operator.
mxl_status build_merge(MatrixImpl &A) {
    hipError_t e;
    A.ntiles = merge_tiles(A.nrows, A.nnz);
    A.part = alloc((size_t)(A.ntiles + 1) * sizeof(int2), &e);
    if (!A.part) return hip_fail(e, "alloc merge partition");
    A.carries = alloc((size_t)carry_bytes(A.ntiles), &e);
    if (!A.carries) return hip_fail(e, "alloc carries");
    HIP_TRY(merge_partition(A, A.ctx->stream));
    return MXL_OK;
}

mxl_status build_ell_windows(MatrixImpl &A) {
    hipError_t e;
    int64_t nt = (A.nrows + kWG * A.ell_rpt - 1) / (kWG * A.ell_rpt);
    A.ell_win = alloc((size_t)(nt > 0 ? nt : 1) * sizeof(int2), &e);
    if (!A.ell_win) return hip_fail(e, "alloc ell windows");
    HIP_TRY(launch_ell_windows(A, (int2 *)A.ell_win->p, A.ctx->stream));
    return MXL_OK;
}

double elapsed_s(std::chrono::steady_clock::time_point t0) {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace

namespace mxl {
void ctx_release(mxl_ctx *c) {
    if (c->refs.fetch_sub(1) != 1) return;
    DeviceScope ds(c->device);
    c->flush_buf.reset();
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    if (c->pinned) (void)hipHostFree(c->pinned);
    delete c;
}

mxl_status set_error(mxl_status st, const std::string &msg) { return fail(st, msg); }
mxl_status check_device_ptr(const mxl_ctx *ctx, const void *p, size_t bytes, const char *what) {
    return check_dev(ctx, p, bytes, what);
}
}  // namespace mxl

// ================================================================== ABI

extern "C" {

const char *mxl_last_error(void) { return mxl::last_error(); }

const char *mxl_version(void) { return "mxl 0.1 gfx950"; }

mxl_status mxl_ctx_create(int device, void *hip_stream, mxl_ctx **out) try {
    if (!out) return fail(MXL_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev)
        return fail(MXL_ERR_DEVICE, "no such HIP device");
    DeviceScope ds(device);
    hipDeviceProp_t prop;
    HIP_TRY(hipGetDeviceProperties(&prop, device));
    std::string arch = prop.gcnArchName;
    if (arch.rfind("gfx950", 0) != 0)
        return fail(MXL_ERR_DEVICE, "device is " + arch + ", this library is built for gfx950");
    auto *c = new mxl_ctx;
    c->device = device;
    c->stream = (hipStream_t)hip_stream;
    c->num_cu = prop.multiProcessorCount;
    c->arch = arch;
    c->pinned_bytes = 4096;
    if (hipHostMalloc(&c->pinned, c->pinned_bytes, hipHostMallocDefault) != hipSuccess) {
        delete c;
        return fail(MXL_ERR_OUT_OF_MEMORY, "pinned host staging");
    }
    // the static scratch of mxl_batch_solve_noalloc: a failed lookup leaves
    // NULL, and only that entry point reports it
    if (mxl::noalloc_scratch_init(device, &c->noalloc_scratch) != hipSuccess) c->noalloc_scratch = nullptr;
    *out = c;
    return MXL_OK;
} catch (...) {
    return mxl::abi_exception(__func__);
}

mxl_status mxl_ctx_set_stream(mxl_ctx *ctx, void *hip_stream) try {
    if (!ctx) return fail(MXL_ERR_INVALID_ARG, "ctx is NULL");
    ctx->stream = (hipStream_t)hip_stream;
    return MXL_OK;
} catch (...) {
    return mxl::abi_exception(__func__);
}

mxl_status mxl_ctx_destroy(mxl_ctx *ctx) try {
    if (!ctx) return MXL_OK;
    {
        DeviceScope ds(ctx->device);
        (void)hipStreamSynchronize(ctx->stream);
    }
    ctx_release(ctx);  // objects still using the context keep it alive
    return MXL_OK;
} catch (...) {
    return mxl::abi_exception(__func__);
}

mxl_status mxl_csr_create(mxl_ctx *ctx, mxl_dtype dtype, int64_t nrows, int64_t ncols, int64_t nnz,
                          const int32_t *row_ptr, const int32_t *col, const void *val, int flags,
                          mxl_op **Aout) try {
    if (!ctx || !Aout) return fail(MXL_ERR_INVALID_ARG, "ctx/out is NULL");
    *Aout = nullptr;
    if (dtype != MXL_F64 && dtype != MXL_F32) return fail(MXL_ERR_DTYPE, "unknown dtype");
    if (nrows < 0 || ncols < 0 || nnz < 0) return fail(MXL_ERR_INVALID_ARG, "negative size");
    if (nnz >= (int64_t)INT_MAX || nrows >= (int64_t)INT_MAX || ncols >= (int64_t)INT_MAX)
        return fail(MXL_ERR_INVALID_ARG, "sizes must be below 2^31 (int32 indices)");
    DeviceScope ds(ctx->device);
    const size_t vt = vt_size(dtype);
    mxl_status st;
    if ((st = check_dev(ctx, row_ptr, (size_t)(nrows + 1) * 4, "row_ptr")) != MXL_OK) return st;
    if ((st = check_dev(ctx, col, (size_t)nnz * 4, "col")) != MXL_OK) return st;
    if ((st = check_dev(ctx, val, (size_t)nnz * vt, "val")) != MXL_OK) return st;
    auto A = std::make_shared<MatrixImpl>();
    A->ctx = ctx;
    A->dtype = dtype;
    A->nrows = nrows;
    A->ncols = ncols;
    A->nnz = nnz;
    const bool copy = flags & MXL_COPY;
    hipError_t e;
    if (copy) {
        A->row_ptr = alloc((size_t)(nrows + 1) * 4, &e);
        A->col = alloc((size_t)nnz * 4, &e);
        A->val = alloc((size_t)nnz * vt, &e);
        if (!A->row_ptr || !A->col || !A->val) return hip_fail(hipErrorOutOfMemory, "csr copy");
        HIP_TRY(hipMemcpyAsync(A->row_ptr->p, row_ptr, (nrows + 1) * 4, hipMemcpyDeviceToDevice, ctx->stream));
        if (nnz) {
            HIP_TRY(hipMemcpyAsync(A->col->p, col, nnz * 4, hipMemcpyDeviceToDevice, ctx->stream));
            HIP_TRY(hipMemcpyAsync(A->val->p, val, nnz * vt, hipMemcpyDeviceToDevice, ctx->stream));
        }
    } else {
        A->row_ptr = borrow(row_ptr, (nrows + 1) * 4);
        A->col = borrow(col, nnz * 4);
        A->val = borrow(val, nnz * vt);
    }
    if (flags & MXL_VALIDATE) {
        auto fl = alloc(sizeof(int), &e);
        if (!fl) return hip_fail(e, "alloc flags");
        HIP_TRY(launch_fill(MXL_F32, 1, 0.0, fl->p, ctx->stream));  // 0.0f has the bit pattern of int 0
        HIP_TRY(launch_validate(*A, (int *)fl->p, ctx->stream));
        int h = 0;
        HIP_TRY(hipMemcpyAsync(&h, fl->p, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
        HIP_TRY(hipStreamSynchronize(ctx->stream));
        if (h) {
            // mask bits in the order the rules are checked: the lowest set bit
            // names the first violated rule
            static const char *const rule[5] = {"row_ptr[0] != 0", "row_ptr decreases",
                                                "row_ptr[n] != nnz", "column out of range",
                                                "columns not strictly increasing"};
            int first = 0;
            while (first < 4 && !(h & (1 << first))) ++first;
            char msg[160];
            snprintf(msg, sizeof msg, "CSR arrays are not canonical (violation mask 0x%x; first: %s)", h,
                     rule[first]);
            return fail(MXL_ERR_INVALID_MATRIX, msg);
        }
    }
    A->format = MXL_FMT_CSR;
    A->variant = MXL_CSR_VECTOR;
    A->vw = auto_vector_width(nrows, nnz);
    compute_stored_bytes(*A);
    finish_matrix(*A);
    *Aout = wrap_matrix(A);
    return MXL_OK;
} catch (...) {
    return mxl::abi_exception(__func__);
}

mxl_status mxl_stencil_create(mxl_ctx *ctx, mxl_dtype dtype, int64_t nx, int64_t ny, int64_t nz,
                              int32_t npts, const int32_t *offsets, const double *coef, mxl_op **Aout) try {
    if (!ctx || !offsets || !coef || !Aout) return fail(MXL_ERR_INVALID_ARG, "NULL argument");
    *Aout = nullptr;
    if (dtype != MXL_F64 && dtype != MXL_F32) return fail(MXL_ERR_DTYPE, "dtype must be F64 or F32");
    if (nx < 1 || ny < 1 || nz < 1 || npts < 1 || npts > 27)
        return fail(MXL_ERR_INVALID_ARG, "grid sizes >= 1 and 1 <= npts <= 27 required");
    if ((double)nx * (double)ny * (double)nz >= 2147483647.0)
        return fail(MXL_ERR_INVALID_ARG, "the grid must have fewer than 2^31 points");
    auto A = std::make_shared<MatrixImpl>();
    A->ctx = ctx;
    A->dtype = dtype;
    A->nx = nx;
    A->ny = ny;
    A->nz = nz;
    A->nrows = A->ncols = nx * ny * nz;
    A->st_npts = npts;
    int64_t nnz = 0;
    for (int q = 0; q < npts; ++q) {
        for (int d = 0; d < 3; ++d) {
            const int32_t v = offsets[3 * q + d];
            if (v < -1 || v > 1) return fail(MXL_ERR_INVALID_ARG, "stencil offsets must be -1, 0 or 1");
            A->st_off[q][d] = (int8_t)v;
        }
        for (int r = 0; r < q; ++r)
            if (A->st_off[r][0] == A->st_off[q][0] && A->st_off[r][1] == A->st_off[q][1] &&
                A->st_off[r][2] == A->st_off[q][2])
                return fail(MXL_ERR_INVALID_ARG, "stencil points must be distinct");
        if (!std::isfinite(coef[q])) return fail(MXL_ERR_INVALID_ARG, "stencil coefficients must be finite");
        A->st_coef[q] = coef[q];
        nnz += (nx - std::abs((int)A->st_off[q][0])) * (ny - std::abs((int)A->st_off[q][1])) *
               (nz - std::abs((int)A->st_off[q][2]));
    }
    A->nnz = nnz;  // entries of the equivalent matrix
    A->format = MXL_FMT_STENCIL;
    A->variant = 0;
    compute_stored_bytes(*A);
    finish_matrix(*A);
    *Aout = wrap_matrix(A);
    return MXL_OK;
} catch (...) {
    return mxl::abi_exception(__func__);
}

mxl_status mxl_convert(const mxl_op *Aop, mxl_format fmt, const mxl_format_params *params,
                       mxl_op **out) try {
    if (!Aop || !out || Aop->kind != MXL_OP_MATRIX) return fail(MXL_ERR_INVALID_ARG, "not a matrix operator");
    *out = nullptr;
    const MatrixImpl &S = *Aop->mat;
    if (S.format == MXL_FMT_STENCIL) return fail(MXL_ERR_NOT_IMPLEMENTED, "a matrix-free stencil has no arrays to convert");
    mxl_ctx *ctx = S.ctx;
    DeviceScope ds(ctx->device);
    mxl_format_params prm{};
    if (params) prm = *params;
    auto A = std::make_shared<MatrixImpl>();
    A->ctx = ctx;
    A->dtype = S.dtype;
    A->nrows = S.nrows;
    A->ncols = S.ncols;
    A->nnz = S.nnz;
    A->row_ptr = S.row_ptr;
    A->col = S.col;
    A->val = S.val;
    A->format = fmt;
    A->variant = prm.variant;
    const size_t vt = vt_size(S.dtype);
    hipError_t e;
    mxl_status st;
    switch (fmt) {
    case MXL_FMT_CSR:
        if (prm.variant == MXL_CSR_SCALAR) {
        } else if (prm.variant == MXL_CSR_VECTOR) {
            int w = prm.vector_width > 0 ? prm.vector_width : auto_vector_width(S.nrows, S.nnz);
            if (w != 2 && w != 4 && w != 8 && w != 16 && w != 32 && w != 64)
                return fail(MXL_ERR_INVALID_ARG, "vector_width must be 2, 4, 8, 16, 32 or 64");
            A->vw = w;
        } else if (prm.variant == MXL_CSR_MERGE) {
            if ((st = build_merge(*A)) != MXL_OK) return st;
        } else if (prm.variant == MXL_CSR_STREAM) {
            std::vector<int32_t> rp, bk;
            if ((st = to_host(ctx, S.row_ptr, rp, (size_t)S.nrows + 1)) != MXL_OK) return st;
            stream_blocks(rp, bk);
            A->ntiles = (int64_t)bk.size() / 2 - 1;
            A->part = alloc(bk.size() * 4, &e);
            if (!A->part) return hip_fail(e, "alloc row blocks");
            HIP_TRY(hipMemcpyAsync(A->part->p, bk.data(), bk.size() * 4, hipMemcpyHostToDevice, ctx->stream));
            HIP_TRY(hipStreamSynchronize(ctx->stream));  // bk lifetime
        } else {
            return fail(MXL_ERR_NOT_IMPLEMENTED, "unknown CSR variant");
        }
        break;
    case MXL_FMT_COO:
        if (prm.variant != MXL_COO_SEGRED) return fail(MXL_ERR_NOT_IMPLEMENTED, "unknown COO variant");
        A->coo_row = alloc((size_t)S.nnz * 4, &e);
        if (!A->coo_row) return hip_fail(e, "alloc coo rows");
        HIP_TRY(launch_csr_to_coo(*A, (int *)A->coo_row->p, ctx->stream));
        A->ntiles = coo_tiles(S.nnz);
        A->carries = alloc((size_t)carry_bytes(A->ntiles), &e);
        if (!A->carries) return hip_fail(e, "alloc carries");
        break;
    case MXL_FMT_ELL:
    case MXL_FMT_HYB: {
        if (prm.variant != MXL_ELL_PLAIN && prm.variant != MXL_ELL_LDS &&
            !(fmt == MXL_FMT_ELL && prm.variant == MXL_ELL_DELTA16))
            return fail(MXL_ERR_NOT_IMPLEMENTED, "unknown ELL variant");
        std::vector<int32_t> rp;
        if ((st = to_host(ctx, S.row_ptr, rp, (size_t)S.nrows + 1)) != MXL_OK) return st;
        std::vector<int32_t> len((size_t)S.nrows);
        for (int64_t i = 0; i < S.nrows; ++i) len[i] = rp[i + 1] - rp[i];
        int w = 0;
        if (fmt == MXL_FMT_ELL) {
            for (int32_t l : len) w = std::max(w, l);
        } else {
            double q = prm.hyb_quantile > 0 ? prm.hyb_quantile : 0.9;
            if (q > 1.0) return fail(MXL_ERR_INVALID_ARG, "hyb_quantile must be in (0, 1]");
            A->hyb_q = q;
            if (S.nrows > 0) {
                std::vector<int32_t> srt(len);
                const int64_t rank = quantile_rank(q, S.nrows);
                std::nth_element(srt.begin(), srt.begin() + (rank - 1), srt.end());
                w = srt[rank - 1];
            }
        }
        const int64_t n_pad = ((S.nrows + 63) / 64) * 64;
        const bool d16 = fmt == MXL_FMT_ELL && prm.variant == MXL_ELL_DELTA16;
        if (!ell_fits(S, w))
            return fail(MXL_ERR_INFEASIBLE_FORMAT, "ELL storage would exceed min(4x CSR bytes, 32 GiB)");
        A->ell_w = w;
        A->n_pad = n_pad;
        A->ell_rpt = prm.vector_width > 0 ? prm.vector_width : 2;
        if (A->ell_rpt != 1 && A->ell_rpt != 2 && A->ell_rpt != 4)
            return fail(MXL_ERR_INVALID_ARG, "ELL rows per thread (vector_width) must be 1, 2 or 4");
        A->ell_col = alloc((size_t)w * n_pad * (d16 ? 2 : 4), &e);
        A->ell_val = alloc((size_t)w * n_pad * vt, &e);
        if (!A->ell_col || !A->ell_val) return hip_fail(hipErrorOutOfMemory, "alloc ell");
        if (d16) {
            auto flag = alloc(4, &e);
            if (!flag) return hip_fail(e, "alloc overflow flag");
            int32_t over = 0;
            HIP_TRY(hipMemcpyAsync(flag->p, &over, 4, hipMemcpyHostToDevice, ctx->stream));
            HIP_TRY(launch_csr_to_ell16(*A, w, n_pad, (short *)A->ell_col->p, A->ell_val->p, (int *)flag->p,
                                        ctx->stream));
            HIP_TRY(hipMemcpyAsync(&over, flag->p, 4, hipMemcpyDeviceToHost, ctx->stream));
            HIP_TRY(hipStreamSynchronize(ctx->stream));
            if (over)
                return fail(MXL_ERR_INFEASIBLE_FORMAT, "a column offset |col - row| exceeds 32767 (16-bit ELL)");
        } else {
            HIP_TRY(launch_csr_to_ell(*A, w, n_pad, (int *)A->ell_col->p, A->ell_val->p, ctx->stream));
        }
        if (prm.variant == MXL_ELL_LDS)
            if ((st = build_ell_windows(*A)) != MXL_OK) return st;
        if (prm.variant != MXL_ELL_LDS && S.nnz > 0) {
            // neighbour reuse pays where at least a quarter of the ELL
            // entries can take x from the row below (stencils: runs of
            // consecutive columns); elsewhere its shuffles are overhead
            unsigned long long stored = 0;  // entries in the ELL slots
            for (int64_t i = 0; i < S.nrows; ++i) stored += (unsigned long long)std::min(len[i], w);
            auto cnt = alloc(8, &e);
            if (!cnt) return hip_fail(e, "alloc reuse count");
            unsigned long long hits = 0;
            HIP_TRY(hipMemcpyAsync(cnt->p, &hits, 8, hipMemcpyHostToDevice, ctx->stream));
            HIP_TRY(launch_ell_reuse_count(*A, w, (unsigned long long *)cnt->p, ctx->stream));
            HIP_TRY(hipMemcpyAsync(&hits, cnt->p, 8, hipMemcpyDeviceToHost, ctx->stream));
            HIP_TRY(hipStreamSynchronize(ctx->stream));
            A->ell_nb = stored > 0 && 4 * hits >= stored ? 1 : 0;
        }
        if (fmt == MXL_FMT_HYB) {
            std::vector<int64_t> toff((size_t)S.nrows + 1, 0);
            for (int64_t i = 0; i < S.nrows; ++i) toff[i + 1] = toff[i] + std::max(0, len[i] - w);
            A->tail_nnz = toff[S.nrows];
            A->tail_row = alloc((size_t)A->tail_nnz * 4, &e);
            A->tail_col = alloc((size_t)A->tail_nnz * 4, &e);
            A->tail_val = alloc((size_t)A->tail_nnz * vt, &e);
            auto dtoff = alloc(toff.size() * 8, &e);
            if (!A->tail_row || !A->tail_col || !A->tail_val || !dtoff)
                return hip_fail(hipErrorOutOfMemory, "alloc hyb tail");
            HIP_TRY(hipMemcpyAsync(dtoff->p, toff.data(), toff.size() * 8, hipMemcpyHostToDevice, ctx->stream));
            HIP_TRY(launch_hyb_tail(*A, w, (const int64_t *)dtoff->p, (int *)A->tail_row->p,
                                    (int *)A->tail_col->p, A->tail_val->p, ctx->stream));
            HIP_TRY(hipStreamSynchronize(ctx->stream));  // toff host vector lifetime
            A->ntiles = coo_tiles(A->tail_nnz);
            A->carries = alloc((size_t)carry_bytes(A->ntiles), &e);
            if (!A->carries) return hip_fail(e, "alloc carries");
        }
        break;
    }
    default:
        return fail(MXL_ERR_NOT_IMPLEMENTED, "unknown format");
    }
    compute_stored_bytes(*A);
    finish_matrix(*A);
    *out = wrap_matrix(A);
    return MXL_OK;
} catch (...) {
    return mxl::abi_exception(__func__);
}

mxl_status mxl_cast(const mxl_op *Aop, mxl_dtype dtype, mxl_op **out) try {
    if (!Aop || !out || Aop->kind != MXL_OP_MATRIX) return fail(MXL_ERR_INVALID_ARG, "not a matrix operator");
    if (dtype != MXL_F64 && dtype != MXL_F32) return fail(MXL_ERR_DTYPE, "unknown dtype");
    *out = nullptr;
    const MatrixImpl &S = *Aop->mat;
    DeviceScope ds(S.ctx->device);
    auto A = std::make_shared<MatrixImpl>(S);  // shares every array
    A->dtype = dtype;
    if (S.format == MXL_FMT_STENCIL) {
        // coefficients are kept in FP64 and rounded to the dtype by the kernel
    } else if (dtype != S.dtype) {
        hipError_t e;
        const size_t vt = vt_size(dtype);
        auto conv = [&](const BufPtr &src, int64_t count) -> BufPtr {
            if (!src) return nullptr;
            BufPtr d = alloc((size_t)count * vt, &e);
            if (d) e = launch_convert_vals(count, S.dtype, src->p, d->p, S.ctx->stream);
            return d;
        };
        A->val = conv(S.val, S.nnz);
        if (S.ell_val) A->ell_val = conv(S.ell_val, (int64_t)S.ell_w * S.n_pad);
        if (S.tail_val) A->tail_val = conv(S.tail_val, S.tail_nnz);
        if (!A->val || (S.ell_val && !A->ell_val) || (S.tail_val && !A->tail_val))
            return hip_fail(hipErrorOutOfMemory, "cast values");
        // carries are per operator (written during apply)
        if (S.carries) {
            A->carries = alloc((size_t)carry_bytes(S.ntiles), &e);
            if (!A->carries) return hip_fail(e, "alloc carries");
        }
    } else if (S.carries) {
        hipError_t e;
        A->carries = alloc((size_t)carry_bytes(S.ntiles), &e);
        if (!A->carries) return hip_fail(e, "alloc carries");
    }
    compute_stored_bytes(*A);
    finish_matrix(*A);
    *out = wrap_matrix(A);
    return MXL_OK;
} catch (...) {
    return mxl::abi_exception(__func__);
}

static mxl_status apply_matrix(const MatrixImpl &A, double alpha, const void *b, double beta,
                               void *x) {
    const size_t vt = vt_size(A.dtype);
    mxl_status st;
    if ((st = check_dev(A.ctx, b, (size_t)A.ncols * vt, "b")) != MXL_OK) return st;
    if ((st = check_dev(A.ctx, x, (size_t)A.nrows * vt, "x")) != MXL_OK) return st;
    SpmvArgs a;
    a.alpha = alpha;
    a.beta = beta;
    a.x = b;
    a.y = x;
    HIP_TRY(spmv_launch(A, a, A.ctx->stream));
    return MXL_OK;
}

mxl_status mxl_apply_adv(const mxl_op *L, double alpha, const void *b, double beta, void *x) try {
    if (!L) return fail(MXL_ERR_INVALID_ARG, "operator is NULL");
    if (!b || !x) return fail(MXL_ERR_INVALID_ARG, "vector is NULL");
    if (b == x) return fail(MXL_ERR_INVALID_ARG, "input and output alias");
    switch (L->kind) {
    case MXL_OP_MATRIX: {
        DeviceScope ds(L->mat->ctx->device);
        return apply_matrix(*L->mat, alpha, b, beta, x);
    }
    case MXL_OP_JACOBI: {
        const MatrixImpl &A = *L->jac->A;
        DeviceScope ds(A.ctx->device);
        const size_t vt = vt_size(A.dtype);
        mxl_status st;
        if ((st = check_dev(A.ctx, b, (size_t)A.nrows * vt, "b")) != MXL_OK) return st;
        if ((st = check_dev(A.ctx, x, (size_t)A.nrows * vt, "x")) != MXL_OK) return st;
        if (L->jac->block) HIP_TRY(bj_apply(A.ctx, *L->jac, A.nrows, alpha, b, beta, x, A.ctx->stream));
        else HIP_TRY(launch_jacobi_apply(A.dtype, A.nrows, alpha, L->jac->dinv->p, b, beta, x, A.ctx->stream));
        return MXL_OK;
    }
    case MXL_OP_ILU: {
        const MatrixImpl &A = *L->ilu->A;
        DeviceScope ds(A.ctx->device);
        mxl_status st;
        if ((st = check_dev(A.ctx, b, (size_t)A.nrows * 8, "b")) != MXL_OK) return st;
        if ((st = check_dev(A.ctx, x, (size_t)A.nrows * 8, "x")) != MXL_OK) return st;
        HIP_TRY(ilu_apply(*L->ilu, alpha, b, beta, x, A.ctx->stream));
        return MXL_OK;
    }
    case MXL_OP_SOLVER:
        if (alpha == 1.0 && beta == 0.0) return mxl_solve(L, b, x, nullptr);
        return fail(MXL_ERR_NOT_IMPLEMENTED, "advanced apply of a solver");
    default:
        return fail(MXL_ERR_NOT_IMPLEMENTED, "apply of this operator kind");
    }
} catch (...) {
    return mxl::abi_exception(__func__);
}

mxl_status mxl_apply(const mxl_op *L, const void *b, void *x) try { return mxl_apply_adv(L, 1.0, b, 0.0, x); } catch (...) {
    return mxl::abi_exception(__func__);
}

mxl_status mxl_op_describe(const mxl_op *op, mxl_op_desc *out) try {
    if (!op || !out) return fail(MXL_ERR_INVALID_ARG, "NULL argument");
    memset(out, 0, sizeof(*out));
    out->kind = op->kind;
    const MatrixImpl *A = nullptr;
    if (op->kind == MXL_OP_MATRIX) A = op->mat.get();
    else if (op->kind == MXL_OP_JACOBI) A = op->jac->A.get();
    else if (op->kind == MXL_OP_SOLVER) A = op->sol->A.get();
    else if (op->kind == MXL_OP_ILU) A = op->ilu->A.get();
    if (!A) return MXL_OK;
    out->format = A->format;
    out->variant = A->variant;
    out->dtype = A->dtype;
    out->nrows = A->nrows;
    out->ncols = A->ncols;
    out->nnz = A->nnz;
    out->vector_width = A->vw;
    out->ell_width = A->ell_w;
    out->n_pad = A->n_pad;
    out->tail_nnz = A->tail_nnz;
    out->stored_bytes = A->stored_bytes;
    out->ell_reuse = A->ell_nb;
    return MXL_OK;
} catch (...) {
    return mxl::abi_exception(__func__);
}

mxl_status mxl_op_export(const mxl_op *op, int32_t which, void *dst, int64_t dst_bytes) try {
    if (!op || !dst) return fail(MXL_ERR_INVALID_ARG, "NULL argument");
    const MatrixImpl *A = op->kind == MXL_OP_MATRIX ? op->mat.get()
                          : op->kind == MXL_OP_JACOBI ? op->jac->A.get() : nullptr;
    if (!A) return fail(MXL_ERR_INVALID_ARG, "operator has no arrays");
    DeviceScope ds(A->ctx->device);
    const size_t vt = vt_size(A->dtype);
    BufPtr b;
    size_t bytes = 0;
    switch (which) {
    case 0: b = A->row_ptr; bytes = (A->nrows + 1) * 4; break;
    case 1: b = A->col; bytes = A->nnz * 4; break;
    case 2: b = A->val; bytes = A->nnz * vt; break;
    case 3: b = A->coo_row; bytes = A->nnz * 4; break;
    case 4:
        b = A->ell_col;
        bytes = (size_t)A->ell_w * A->n_pad *
                (A->format == MXL_FMT_ELL && A->variant == MXL_ELL_DELTA16 ? 2 : 4);
        break;
    case 5: b = A->ell_val; bytes = (size_t)A->ell_w * A->n_pad * vt; break;
    case 6: b = A->tail_row; bytes = A->tail_nnz * 4; break;
    case 7: b = A->tail_col; bytes = A->tail_nnz * 4; break;
    case 8: b = A->tail_val; bytes = A->tail_nnz * vt; break;
    case 9:
        if (op->kind == MXL_OP_JACOBI) { b = op->jac->dinv; bytes = A->nrows * vt; }
        break;
    default: return fail(MXL_ERR_INVALID_ARG, "unknown array id");
    }
    if (!b) return fail(MXL_ERR_INVALID_ARG, "array not present in this format");
    if ((int64_t)bytes > dst_bytes) return fail(MXL_ERR_DIM_MISMATCH, "destination too small");
    mxl_status st;
    if ((st = check_dev(A->ctx, dst, bytes, "dst")) != MXL_OK) return st;
    if (bytes) HIP_TRY(hipMemcpyAsync(dst, b->p, bytes, hipMemcpyDeviceToDevice, A->ctx->stream));
    return MXL_OK;
} catch (...) {
    return mxl::abi_exception(__func__);
}

mxl_status mxl_op_destroy(mxl_op *op) try {
    if (!op) return MXL_OK;
    const MatrixImpl *A = op->kind == MXL_OP_MATRIX ? op->mat.get()
                          : op->kind == MXL_OP_JACOBI ? op->jac->A.get()
                          : op->kind == MXL_OP_SOLVER ? op->sol->A.get()
                          : op->kind == MXL_OP_ILU ? op->ilu->A.get() : nullptr;
    mxl_ctx *ctx = A ? A->ctx : op->kind == MXL_OP_BATCH ? batch_ctx(*op->bat) : nullptr;
    if (ctx) {  // queued work may still use the arrays
        DeviceScope ds(ctx->device);
        (void)hipStreamSynchronize(ctx->stream);
    }
    delete op;
    return MXL_OK;
} catch (...) {
    return mxl::abi_exception(__func__);
}

mxl_status mxl_jacobi_generate(const mxl_op *Aop, mxl_op **P) try {
    if (!Aop || !P || Aop->kind != MXL_OP_MATRIX) return fail(MXL_ERR_INVALID_ARG, "not a matrix operator");
    *P = nullptr;
    const auto &A = Aop->mat;
    if (A->nrows != A->ncols) return fail(MXL_ERR_NOT_IMPLEMENTED, "Jacobi needs a square matrix");
    DeviceScope ds(A->ctx->device);
    hipError_t e;
    auto J = std::make_shared<JacobiImpl>();
    J->A = A;
    J->dinv = alloc((size_t)A->nrows * vt_size(A->dtype), &e);
    if (!J->dinv) return hip_fail(hipErrorOutOfMemory, "alloc jacobi");
    if (A->format == MXL_FMT_STENCIL) {  // constant diagonal: the point (0,0,0)
        double diag = 0.0;
        for (int q = 0; q < A->st_npts; ++q)
            if (A->st_off[q][0] == 0 && A->st_off[q][1] == 0 && A->st_off[q][2] == 0) diag = A->st_coef[q];
        if (A->dtype == MXL_F32) diag = (double)(float)diag;
        if (diag == 0.0) return fail(MXL_ERR_ZERO_DIAG, "the stencil has no nonzero centre point");
        HIP_TRY(launch_fill(A->dtype, A->nrows, 1.0 / diag, J->dinv->p, A->ctx->stream));
        auto *op = new mxl_op;
        op->kind = MXL_OP_JACOBI;
        op->jac = J;
        *P = op;
        return MXL_OK;
    }
    auto bad = alloc(sizeof(int), &e);
    if (!J->dinv || !bad) return hip_fail(hipErrorOutOfMemory, "alloc jacobi");
    int init = INT_MAX;
    HIP_TRY(hipMemcpyAsync(bad->p, &init, sizeof(int), hipMemcpyHostToDevice, A->ctx->stream));
    HIP_TRY(launch_jacobi(*A, J->dinv->p, (int *)bad->p, A->ctx->stream));
    int h = INT_MAX;
    HIP_TRY(hipMemcpyAsync(&h, bad->p, sizeof(int), hipMemcpyDeviceToHost, A->ctx->stream));
    HIP_TRY(hipStreamSynchronize(A->ctx->stream));
    if (h != INT_MAX) {
        char msg[96];
        snprintf(msg, sizeof msg, "row %d has a missing or zero diagonal entry", h);
        return fail(MXL_ERR_ZERO_DIAG, msg);
    }
    auto *op = new mxl_op;
    op->kind = MXL_OP_JACOBI;
    op->jac = J;
    *P = op;
    return MXL_OK;
} catch (...) {
    return mxl::abi_exception(__func__);
}

static mxl_status make_solver(int kind, const std::shared_ptr<MatrixImpl> &A,
                              const std::shared_ptr<JacobiImpl> &P, const mxl_criteria &crit,
                              std::shared_ptr<SolverImpl> &out, int krylov = 0,
                              const std::shared_ptr<IluImpl> &ilu = nullptr) {
    if (crit.max_iters < 0) return fail(MXL_ERR_INVALID_ARG, "max_iters < 0");
    if (crit.max_iters >= INT_MAX) return fail(MXL_ERR_INVALID_ARG, "max_iters too large");
    if (!(crit.reduction >= 0.0)) return fail(MXL_ERR_INVALID_ARG, "reduction must be >= 0");
    if (A->nrows != A->ncols) return fail(MXL_ERR_DIM_MISMATCH, "solver needs a square matrix");
    if (A->nrows == 0) return fail(MXL_ERR_INVALID_ARG, "empty system");
    // Block-Jacobi inverses keep their own storage precision and are applied
    // in FP64, so they conform to vectors of either type; point Jacobi's
    // dinv has the matrix's value type.
    if (P && (P->A->nrows != A->nrows || (!P->block && P->A->dtype != A->dtype)))
        return fail(P->A->nrows != A->nrows ? MXL_ERR_DIM_MISMATCH : MXL_ERR_DTYPE,
                    "preconditioner does not conform to the matrix");
    auto S = std::make_shared<SolverImpl>();
    S->kind = kind;
    S->A = A;
    S->P = P;
    S->crit = crit;
    if (S->crit.check_every < 1) S->crit.check_every = 1;
    hipError_t e;
    const size_t vb = (size_t)A->nrows * vt_size(A->dtype);
    auto need = [&](BufPtr &b, size_t bytes) {
        b = alloc(bytes, &e);
        return b != nullptr;
    };
    bool ok = need(S->r, vb) && need(S->p, vb) && need(S->q, vb) && need(S->state, sizeof(SolverState)) &&
              need(S->partials, (size_t)kRegions * kSolverSlots * 3 * sizeof(double));
    if (ok && kind == MXL_SOLVER_BICGSTAB)
        ok = need(S->rhat, vb) && need(S->v, vb) && need(S->s, vb) && need(S->t, vb) && need(S->z, vb);
    if (ok && P && P->block) ok = need(S->z, vb);  // z = M r is kept in memory
    if (ok && P && P->var && kind == MXL_SOLVER_CG) ok = need(S->r2, vb);
    if (ok && kind == MXL_SOLVER_GMRES) {
        // basis of krylov+1 vectors (ld rounded to 64 rows), z = M^{-1} v,
        // multi-dot partials, norm partials, Hessenberg/rotation workspace
        S->krylov = krylov;
        S->ld = (A->nrows + 63) / 64 * 64;
        const int G = gm_grid(A->nrows);
        ok = need(S->V, (size_t)(krylov + 1) * (size_t)S->ld * sizeof(double)) &&
             need(S->gmws, gm_ws_bytes(krylov)) &&
             need(S->gdots, (size_t)(2 * krylov + 2) * (size_t)G * sizeof(double)) &&
             need(S->gnorm, (size_t)std::max(G, 2 * kMaxGrid) * sizeof(double)) &&
             (!(P || ilu) || need(S->z, vb));
        S->ilu = ilu;
    }
    S->hist_len = crit.max_iters + 1;
    if (ok) ok = need(S->hist, (size_t)S->hist_len * sizeof(double));
    if (!ok) return hip_fail(hipErrorOutOfMemory, "solver workspace");
    if (spmv_slots(*A) > kSolverSlots) return fail(MXL_ERR_NOT_IMPLEMENTED, "too many reduction slots");
    out = S;
    return MXL_OK;
}

mxl_status mxl_solver_generate(mxl_solver_kind kind, const mxl_op *Aop, const mxl_op *Pop,
                               const mxl_criteria *crit, mxl_op **Sout) try {
    if (!Aop || !Sout || !crit || Aop->kind != MXL_OP_MATRIX)
        return fail(MXL_ERR_INVALID_ARG, "matrix operator and criteria required");
    if (kind != MXL_SOLVER_CG && kind != MXL_SOLVER_BICGSTAB && kind != MXL_SOLVER_GMRES)
        return fail(MXL_ERR_NOT_IMPLEMENTED, "unknown solver kind");
    return mxl_gmres_generate(Aop, Pop, crit, kind == MXL_SOLVER_GMRES ? 100 : -(int)kind - 1, Sout);
} catch (...) {
    return mxl::abi_exception(__func__);
}

// kdim >= 1: GMRES(kdim); kdim = -kind-1 routes the other Krylov kinds here.
mxl_status mxl_gmres_generate(const mxl_op *Aop, const mxl_op *Pop, const mxl_criteria *crit, int32_t kdim,
                              mxl_op **Sout) try {
    if (!Aop || !Sout || !crit || Aop->kind != MXL_OP_MATRIX)
        return fail(MXL_ERR_INVALID_ARG, "matrix operator and criteria required");
    const int kind = kdim < 0 ? -kdim - 1 : MXL_SOLVER_GMRES;
    if (kind == MXL_SOLVER_GMRES && (kdim < 1 || kdim > kGmMaxKrylov))
        return fail(MXL_ERR_INVALID_ARG, "krylov_dim must be in [1, 1024]");
    if (kind == MXL_SOLVER_GMRES && Aop->mat->dtype != MXL_F64)
        return fail(MXL_ERR_NOT_IMPLEMENTED, "GMRES needs an FP64 operator");
    const bool ilu = Pop && Pop->kind == MXL_OP_ILU;
    if (Pop && Pop->kind != MXL_OP_JACOBI && !ilu)
        return fail(MXL_ERR_NOT_IMPLEMENTED, "only Jacobi or ILU preconditioning");
    if (Pop && !ilu && Pop->jac->block && kind == MXL_SOLVER_BICGSTAB && Aop->mat->dtype != MXL_F64)
        return fail(MXL_ERR_NOT_IMPLEMENTED, "block-Jacobi BiCGSTAB needs an FP64 operator");
    if (ilu && kind != MXL_SOLVER_GMRES) return fail(MXL_ERR_NOT_IMPLEMENTED, "ILU preconditions GMRES");
    if (ilu && Pop->ilu->A->nrows != Aop->mat->nrows)
        return fail(MXL_ERR_DIM_MISMATCH, "preconditioner does not conform to the matrix");
    *Sout = nullptr;
    DeviceScope ds(Aop->mat->ctx->device);
    std::shared_ptr<SolverImpl> S;
    mxl_status st = make_solver(kind, Aop->mat, Pop && !ilu ? Pop->jac : nullptr, *crit, S,
                                kind == MXL_SOLVER_GMRES ? kdim : 0, ilu ? Pop->ilu : nullptr);
    if (st != MXL_OK) return st;
    auto *op = new mxl_op;
    op->kind = MXL_OP_SOLVER;
    op->sol = S;
    *Sout = op;
    return MXL_OK;
} catch (...) {
    return mxl::abi_exception(__func__);
}

}  // extern "C"

// ----------------------------------------------------------- solve loops
namespace {

// Optional per-iteration HIP-event timing of the SpMV launches of a Krylov
// loop (events recorded on the solver's stream around each launch).
// HIP events around every `every`-th SpMV launch of a Krylov loop (the
// first kCap samples): each recorded event is a packet in the stream, so
// timing every launch would itself slow the loop it measures.  The events
// belong to the solver and are reused by later solves.
struct EventTimer {
    static constexpr int64_t kCap = 4096;
    bool on;
    int64_t every;
    hipStream_t s;
    std::vector<hipEvent_t> &ev;
    EventTimer(int32_t period, hipStream_t st, std::vector<hipEvent_t> &events)
        : on(period > 0), every(period > 0 ? period : 1), s(st), ev(events) {}
    bool sampled(int64_t k) const { return on && k % every == 0 && k / every <= kCap; }
    void begin(int64_t k) {
        if (!sampled(k)) return;
        const int64_t j = k / every;
        if ((int64_t)ev.size() < 2 * j) ev.resize(2 * j, nullptr);
        if (!ev[2 * j - 2]) (void)hipEventCreate(&ev[2 * j - 2]);
        if (!ev[2 * j - 1]) (void)hipEventCreate(&ev[2 * j - 1]);
        (void)hipEventRecord(ev[2 * j - 2], s);
    }
    void end(int64_t k) {
        if (!sampled(k)) return;
        (void)hipEventRecord(ev[2 * (k / every) - 1], s);
    }
    void collect(int64_t iters, double *ms, int64_t *count) {
        *ms = 0.0;
        *count = 0;
        (void)hipStreamSynchronize(s);
        for (int64_t j = 1; j * every <= iters && j <= kCap && 2 * j <= (int64_t)ev.size(); ++j) {
            float t = 0.f;
            if (ev[2 * j - 2] && ev[2 * j - 1] && hipEventElapsedTime(&t, ev[2 * j - 2], ev[2 * j - 1]) == hipSuccess) {
                *ms += t;
                ++*count;
            }
        }
    }
};

mxl_status read_state(const SolverImpl &S, SolverState &out) {
    mxl_ctx *ctx = S.A->ctx;
    HIP_TRY(hipMemcpyAsync(ctx->pinned, S.state->p, sizeof(SolverState), hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    memcpy(&out, ctx->pinned, sizeof(SolverState));
    return MXL_OK;
}

// Host checks that trail the device by one chunk of iterations.  After each
// chunk the state is copied to one of two pinned slots; the host then waits
// for the copy made after the chunk before, so the next chunk is already
// queued while it reads (the GPU does not idle for the host's round trip).
// A chunk queued after a device-side stop returns at once in every kernel.
struct TrailingCheck {
    const SolverImpl &S;
    int next = 0;
    bool pending = false;
    static constexpr size_t kSlot0 = 1024, kSlotBytes = 512;  // offsets in ctx->pinned
    static_assert(sizeof(SolverState) <= kSlotBytes, "state snapshot slot");
    explicit TrailingCheck(const SolverImpl &s) : S(s) {}
    // Snapshot the state after the work queued so far; if an earlier
    // snapshot is in flight, wait for it and return it in out (have = true).
    mxl_status step(SolverState &out, bool &have) {
        mxl_ctx *ctx = S.A->ctx;
        hipStream_t s = ctx->stream;
        have = false;
        if (ctx->pinned_bytes < kSlot0 + 2 * kSlotBytes) return fail(MXL_ERR_INTERNAL, "pinned staging too small");
        for (int i = 0; i < 2; ++i)
            if (!S.chk_ev[i]) HIP_TRY(hipEventCreateWithFlags(&S.chk_ev[i], hipEventDisableTiming));
        char *base = (char *)ctx->pinned + kSlot0;
        const int slot = next, prev = next ^ 1;
        HIP_TRY(hipMemcpyAsync(base + slot * kSlotBytes, S.state->p, sizeof(SolverState), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipEventRecord(S.chk_ev[slot], s));
        if (pending) {
            HIP_TRY(hipEventSynchronize(S.chk_ev[prev]));
            memcpy(&out, base + prev * kSlotBytes, sizeof(SolverState));
            have = true;
        }
        pending = true;
        next = prev;
        return MXL_OK;
    }
};

// r = b - A x into S.r
mxl_status residual(const SolverImpl &S, const void *b, const void *x) {
    const MatrixImpl &A = *S.A;
    HIP_TRY(launch_copy(A.dtype, A.nrows, b, S.r->p, A.ctx->stream));
    SpmvArgs a;
    a.alpha = -1.0;
    a.beta = 1.0;
    a.x = x;
    a.y = S.r->p;
    HIP_TRY(spmv_launch(A, a, A.ctx->stream));
    return MXL_OK;
}

void fill_info(mxl_solve_info *info, const SolverImpl &S, const SolverState &h, int64_t iters,
               int stop, int64_t spmvs, double secs) {
    if (!info) return;
    info->iterations = iters;
    info->spmv_count = spmvs;
    info->rel_residual = h.nb2 > 0 ? std::sqrt(h.rr / h.nb2) : 0.0;
    info->stop_reason = stop;
    info->seconds = secs;
    info->inner_iterations = 0;
    info->restarts = 0;
    info->reorth = 0;
    if (info->history && info->history_cap > 0) {
        int64_t cnt = std::min<int64_t>(iters + 1, std::min<int64_t>(info->history_cap, S.hist_len));
        if (cnt > 0) {
            (void)hipMemcpyAsync(info->history, S.hist->p, cnt * sizeof(double), hipMemcpyDeviceToHost,
                                 S.A->ctx->stream);
            (void)hipStreamSynchronize(S.A->ctx->stream);
        }
    }
}

int map_stop(int s) {
    switch (s) {
    case ST_CONVERGED:
    case ST_HALF: return MXL_STOP_CONVERGED;
    case ST_BREAKDOWN: return MXL_STOP_BREAKDOWN;
    case ST_NONFINITE: return MXL_STOP_NONFINITE;
    default: return MXL_STOP_NONE;
    }
}

double *region(const SolverImpl &S, int r) { return (double *)S.partials->p + (size_t)r * kSolverSlots * 3; }

constexpr int64_t kSingleAutoN = 8192;   // auto: one persistent workgroup up to this size
constexpr int64_t kSingleMaxN = 16384;

bool single_launch_ok(const SolverImpl &S, const mxl_solve_info *info) {
    const mxl_criteria &c = S.crit;
    if ((S.kind != MXL_SOLVER_CG && S.kind != MXL_SOLVER_BICGSTAB) || S.A->dtype != MXL_F64 || c.launch_mode == 1)
        return false;
    if (S.A->format == MXL_FMT_STENCIL) return false;  // the one-launch path reads CSR arrays
    if (S.P && S.P->block) return false;                // and point-Jacobi scaling only
    if (c.max_iters < 1 || c.time_limit_s > 0 || S.A->nrows > kSingleMaxN) return false;
    if (info && ((info->history && info->history_cap > 0) || info->time_spmv)) return false;
    return c.launch_mode == 2 || S.A->nrows <= kSingleAutoN;
}

mxl_status solve_cg_single(SolverImpl &S, const void *b, void *x, mxl_solve_info *info) {
    auto t0 = std::chrono::steady_clock::now();
    if (!S.single) {
        S.single = batch_from_matrix(*S.A, S.P ? S.P->dinv->p : nullptr);
        hipError_t e;
        S.single_out = alloc(64, &e);
        if (!S.single || !S.single_out) return fail(MXL_ERR_OUT_OF_MEMORY, "single-launch workspace");
    }
    int64_t iters = 0;
    double rel = 0.0;
    int stop = 0;
    mxl_status st = batch_single_solve(*S.single, S.crit, (const double *)b, (double *)x, S.single_out->p,
                                       &iters, &rel, &stop);
    if (st != MXL_OK) return st;
    if (info) {
        info->iterations = iters;
        info->spmv_count = 1 + iters;
        info->rel_residual = rel;
        info->stop_reason = stop == ST_MAX_ITERS ? MXL_STOP_MAX_ITERS : map_stop(stop);
        info->seconds = elapsed_s(t0);
        info->inner_iterations = 0;
    }
    return MXL_OK;
}

// x_zero: x is known to be zero (the inner solve of iterative refinement),
// so r = b needs no product and the host does not wait for the initial
// state: a zero b or an initial residual below the criterion stops on the
// device, and the trailing check sees it.
mxl_status solve_cg(const SolverImpl &S, const void *b, void *x, mxl_solve_info *info, bool x_zero = false) {
    if (single_launch_ok(S, info)) return solve_cg_single(const_cast<SolverImpl &>(S), b, x, info);
    auto t0 = std::chrono::steady_clock::now();
    const MatrixImpl &A = *S.A;
    mxl_ctx *ctx = A.ctx;
    hipStream_t s = ctx->stream;
    const int dt = A.dtype;
    const int64_t n = A.nrows;
    auto *st = (SolverState *)S.state->p;
    double *pA = region(S, 0), *pB = region(S, 1), *pC = region(S, 2);
    const int gv = vec_grid(ctx, n), gs = spmv_slots(A);
    double *hist = (double *)S.hist->p;
    const void *dinv = S.P && S.P->dinv ? S.P->dinv->p : nullptr;
    const mxl_criteria &c = S.crit;
    mxl_status rs;
    HIP_TRY(launch_state_init(st, c.reduction, c.nonfinite_check, s));
    if (x_zero) HIP_TRY(launch_copy(dt, n, b, S.r->p, s));
    else if ((rs = residual(S, b, x)) != MXL_OK) return rs;
    const bool blockp = S.P && S.P->block;
    if (blockp) HIP_TRY(bj_cg_init(ctx, *S.P, dt, n, b, S.r->p, S.p->p, pC, s));
    else HIP_TRY(cg_init(ctx, dt, n, b, S.r->p, S.p->p, dinv, pC, s));
    HIP_TRY(launch_finalize(3, pC, gv, st, FIN_CG_INIT, 0, 0, hist, s));
    SolverState h{};
    if (!x_zero) {
        if ((rs = read_state(S, h)) != MXL_OK) return rs;
        if (h.nb2 == 0.0) {
            HIP_TRY(launch_fill(dt, n, 0.0, x, s));
            HIP_TRY(hipStreamSynchronize(s));
            fill_info(info, S, h, 0, MXL_STOP_CONVERGED, 1, elapsed_s(t0));
            return MXL_OK;
        }
    }
    int64_t k = 0;
    int stop = h.stop ? map_stop(h.stop) : MXL_STOP_NONE;
    int64_t iters = 0;
    EventTimer timer(info ? info->time_spmv : 0, s, const_cast<SolverImpl &>(S).spmv_events);
    TrailingCheck chk(S);
    while (stop == MXL_STOP_NONE && k < c.max_iters) {
        ++k;
        timer.begin(k);
        SpmvArgs a;
        a.x = S.p->p;
        a.y = S.q->p;
        a.stop = &st->stop;
        a.w = S.p->p;
        a.partials = pA;
        HIP_TRY(spmv_launch(A, a, s));
        timer.end(k);
        if (blockp) {  // r update fused with z = M r; then p = z + beta p (z passed as "r", no scaling)
            // variable-size blocks: iteration k reads r from rb[(k-1)&1] and writes rb[k&1]
            void *rin = S.P->var && !(k & 1) ? S.r2->p : S.r->p;
            void *rout = S.P->var && (k & 1) ? S.r2->p : S.r->p;
            HIP_TRY(bj_cg_update(ctx, *S.P, dt, n, rin, rout, S.q->p, S.z->p, st, pA, gs, pB, (int)k, s));
            HIP_TRY(cg_pupdate(ctx, dt, n, x, S.z->p, S.p->p, nullptr, st, pB, gv, (int)k, hist, s));
        } else {
            HIP_TRY(cg_update(ctx, dt, n, S.r->p, S.q->p, dinv, st, pA, gs, pB, (int)k, s));
            HIP_TRY(cg_pupdate(ctx, dt, n, x, S.r->p, S.p->p, dinv, st, pB, cg_update_grid(ctx, n), (int)k, hist,
                               s));
        }
        if (k % c.check_every == 0 || k == c.max_iters) {
            bool have = false;
            if ((rs = chk.step(h, have)) != MXL_OK) return rs;
            if (have && h.stop) {
                stop = map_stop(h.stop);
                break;
            }
            if (c.time_limit_s > 0 && elapsed_s(t0) >= c.time_limit_s) {
                stop = MXL_STOP_TIME;
                break;
            }
        }
    }
    if ((rs = read_state(S, h)) != MXL_OK) return rs;
    // a stop the trailing check had not seen yet decides over max_iters and time
    if ((stop == MXL_STOP_NONE || stop == MXL_STOP_TIME) && h.stop) stop = map_stop(h.stop);
    if (stop == MXL_STOP_NONE) {
        stop = MXL_STOP_MAX_ITERS;
        iters = k;
    } else if (stop == MXL_STOP_TIME) {
        iters = k;
    } else {
        iters = h.iters;
    }
    int64_t spmvs = (x_zero ? 0 : 1) + iters + (stop == MXL_STOP_BREAKDOWN || stop == MXL_STOP_NONFINITE ? 1 : 0);
    fill_info(info, S, h, iters, stop, spmvs, elapsed_s(t0));
    if (info && info->time_spmv) timer.collect(iters, &info->spmv_ms, &info->spmv_timed);
    return MXL_OK;
}

// The whole BiCGSTAB in one workgroup for small systems (false: no register
// shape holds the system; the caller runs the per-step solver).
bool solve_bicgstab_single(SolverImpl &S, const void *b, void *x, mxl_solve_info *info, mxl_status *st) {
    auto t0 = std::chrono::steady_clock::now();
    *st = MXL_OK;
    if (!S.single) {
        S.single = batch_from_matrix(*S.A, S.P ? S.P->dinv->p : nullptr);
        hipError_t e;
        S.single_out = alloc(64, &e);
        if (!S.single || !S.single_out) {
            *st = fail(MXL_ERR_OUT_OF_MEMORY, "single-launch workspace");
            return true;
        }
    }
    int64_t iters = 0;
    double rel = 0.0;
    int stop = 0, half = 0;
    if (!batch_single_bicgstab(*S.single, S.crit, (const double *)b, (double *)x, S.single_out->p, &iters, &rel,
                               &stop, &half, st))
        return false;
    if (*st != MXL_OK) return true;
    if (info) {
        info->iterations = iters;
        info->spmv_count = 1 + 2 * iters - half;
        info->rel_residual = rel;
        info->stop_reason = stop == ST_MAX_ITERS ? MXL_STOP_MAX_ITERS : map_stop(stop);
        info->seconds = elapsed_s(t0);
        info->inner_iterations = 0;
        info->restarts = 0;
        info->reorth = 0;
    }
    return true;
}

mxl_status solve_bicgstab(const SolverImpl &S, const void *b, void *x, mxl_solve_info *info) {
    if (single_launch_ok(S, info)) {
        mxl_status st;
        if (solve_bicgstab_single(const_cast<SolverImpl &>(S), b, x, info, &st)) return st;
    }
    auto t0 = std::chrono::steady_clock::now();
    const MatrixImpl &A = *S.A;
    mxl_ctx *ctx = A.ctx;
    hipStream_t s = ctx->stream;
    const int dt = A.dtype;
    const int64_t n = A.nrows;
    auto *st = (SolverState *)S.state->p;
    double *pA = region(S, 0), *pB = region(S, 1), *pC = region(S, 2), *pD = region(S, 3);
    const int gv = vec_grid(ctx, n), gs = spmv_slots(A);
    double *hist = (double *)S.hist->p;
    const void *dinv = S.P && S.P->dinv ? S.P->dinv->p : nullptr;
    const mxl_criteria &c = S.crit;
    const int mi = (int)c.max_iters;
    void *phat = S.z->p;
    void *shat = S.q->p;
    mxl_status rs;
    HIP_TRY(launch_state_init(st, c.reduction, c.nonfinite_check, s));
    if ((rs = residual(S, b, x)) != MXL_OK) return rs;
    HIP_TRY(bi_init(ctx, dt, n, b, S.r->p, S.rhat->p, S.p->p, S.v->p, pC, s));
    HIP_TRY(launch_finalize(3, pC, gv, st, FIN_BI_INIT, 0, mi, hist, s));
    SolverState h;
    if ((rs = read_state(S, h)) != MXL_OK) return rs;
    if (h.nb2 == 0.0) {
        HIP_TRY(launch_fill(dt, n, 0.0, x, s));
        HIP_TRY(hipStreamSynchronize(s));
        fill_info(info, S, h, 0, MXL_STOP_CONVERGED, 1, elapsed_s(t0));
        return MXL_OK;
    }
    int64_t k = 0;
    int stop = h.stop ? map_stop(h.stop) : MXL_STOP_NONE;
    // block Jacobi: the block products p_hat = M p, s_hat = M s follow the
    // fused kernels as kernels of their own
    const bool blockp = S.P && S.P->block;
    TrailingCheck chk(S);
    while (stop == MXL_STOP_NONE && k < c.max_iters) {
        ++k;
        // with block Jacobi the fused kernels store no p_hat / s_hat (NULL):
        // the block products write them
        HIP_TRY(bi_pupdate(ctx, dt, n, S.r->p, S.p->p, S.v->p, blockp ? nullptr : phat, dinv, st, pC, gv, (int)k,
                           hist, s));
        if (blockp) HIP_TRY(bj_apply(ctx, *S.P, n, 1.0, S.p->p, 0.0, phat, s, &st->stop));
        SpmvArgs a;
        a.x = phat;
        a.y = S.v->p;
        a.stop = &st->stop;
        a.w = S.rhat->p;
        a.partials = pA;
        HIP_TRY(spmv_launch(A, a, s));
        HIP_TRY(bi_supdate(ctx, dt, n, S.r->p, S.v->p, S.s->p, blockp ? nullptr : shat, dinv, st, pA, gs, pB,
                           (int)k, s));
        if (blockp) HIP_TRY(bj_apply(ctx, *S.P, n, 1.0, S.s->p, 0.0, shat, s, &st->stop));
        SpmvArgs t;
        t.x = shat;
        t.y = S.t->p;
        t.stop = &st->stop;
        HIP_TRY(spmv_launch(A, t, s));
        HIP_TRY(bi_tdots(ctx, dt, n, S.t->p, S.s->p, st, pB, gv, pD, (int)k, hist, s));
        HIP_TRY(bi_xupdate(ctx, dt, n, x, S.r->p, phat, shat, S.s->p, S.t->p, S.rhat->p, st, pD, gv, pC,
                           (int)k, s));
        if (k % c.check_every == 0 || k == c.max_iters) {
            bool have = false;
            if ((rs = chk.step(h, have)) != MXL_OK) return rs;
            if (have && h.stop) {
                stop = map_stop(h.stop);
                break;
            }
            if (c.time_limit_s > 0 && elapsed_s(t0) >= c.time_limit_s) {
                stop = MXL_STOP_TIME;
                break;
            }
        }
    }
    if (stop == MXL_STOP_NONE && k > 0)  // criterion of the last iteration
        HIP_TRY(launch_finalize(3, pC, gv, st, FIN_BI_LAST, (int)k, mi, hist, s));
    if ((rs = read_state(S, h)) != MXL_OK) return rs;
    // a stop the trailing check had not seen yet decides over max_iters and time
    if ((stop == MXL_STOP_NONE || stop == MXL_STOP_TIME) && h.stop) stop = map_stop(h.stop);
    int64_t iters;
    if (stop == MXL_STOP_NONE) {
        stop = MXL_STOP_MAX_ITERS;
        iters = k;
    } else if (stop == MXL_STOP_TIME) {
        iters = k;
    } else {
        iters = h.iters;
    }
    fill_info(info, S, h, iters, stop, 1 + 2 * iters - (h.half ? 1 : 0), elapsed_s(t0));
    return MXL_OK;
}

// Restarted GMRES(m): the cycle's steps are enqueued without reading the
// state (each kernel returns at once after a device-side stop); the host
// reads it every check_every steps and at the end of every cycle, where it
// closes the cycle (x update) and restarts from the recomputed residual.
mxl_status solve_gmres(const SolverImpl &S, const void *b, void *xv, mxl_solve_info *info) {
    auto t0 = std::chrono::steady_clock::now();
    const MatrixImpl &A = *S.A;
    mxl_ctx *ctx = A.ctx;
    hipStream_t s = ctx->stream;
    const int64_t n = A.nrows, ld = S.ld;
    const int m = S.krylov;
    auto *st = (SolverState *)S.state->p;
    double *V = (double *)S.V->p, *dp = (double *)S.gdots->p, *np = (double *)S.gnorm->p;
    void *ws = S.gmws->p;
    double *x = (double *)xv, *hist = (double *)S.hist->p;
    // point Jacobi is fused into the basis kernels; block Jacobi and ILU
    // are applied by their own kernels (z = M^{-1} v, x += M^{-1} t)
    const bool blockp = (S.P && S.P->block) || S.ilu;
    const double *dinv = S.P && S.P->dinv ? (const double *)S.P->dinv->p : nullptr;
    double *z = S.P || S.ilu ? (double *)S.z->p : nullptr;
    auto apply_M = [&](const double *in, double beta, double *out) -> hipError_t {
        if (S.ilu) return ilu_apply(*S.ilu, 1.0, in, beta, out, s);
        return bj_apply(ctx, *S.P, n, 1.0, in, beta, out, s);
    };
    const mxl_criteria &c = S.crit;
    mxl_status rs;
    // r = b - A x into V_0, ||r||, z = M^{-1} V_0, g = beta e_1, criteria
    auto restart = [&](int first) -> mxl_status {
        HIP_TRY(launch_copy(MXL_F64, n, b, V, s));
        SpmvArgs a;
        a.alpha = -1.0;
        a.beta = 1.0;
        a.x = x;
        a.y = V;
        HIP_TRY(spmv_launch(A, a, s));
        int slots = 0;
        HIP_TRY(gm_prep(ctx, n, V, first ? (const double *)b : nullptr, blockp ? nullptr : dinv,
                        blockp ? nullptr : z, np, &slots, s));
        HIP_TRY(gm_start(np, slots, st, ws, m, hist, first, s));
        if (blockp) HIP_TRY(apply_M(V, 0.0, z));
        return MXL_OK;
    };
    // steps j0 .. j0+cnt-1 of a cycle: the SpMV u = A z (z = M^{-1} t_j, or
    // t_j itself), the basis kernels, and z for the next step
    auto enqueue = [&](int j0, int cnt) -> mxl_status {
        for (int j = j0; j < j0 + cnt; ++j) {
            SpmvArgs a;
            a.x = z ? (const void *)z : (const void *)(V + (int64_t)j * ld);
            a.y = S.q->p;
            a.stop = &st->stop;
            HIP_TRY(spmv_launch(A, a, s));
            HIP_TRY(gm_step(n, ld, V, j, (const double *)S.q->p, blockp ? nullptr : dinv, blockp ? nullptr : z,
                            dp, st, ws, m, hist, s));
            if (blockp) HIP_TRY(apply_M(V + (int64_t)(j + 1) * ld, 0.0, z));
        }
        return MXL_OK;
    };
    // small systems: the whole solve in one workgroup
    if (c.launch_mode != 1 && n <= 1024 && m <= 128 && !blockp && A.format != MXL_FMT_STENCIL &&
        c.time_limit_s <= 0) {
        HIP_TRY(gm_small((int)n, m, (const int *)A.row_ptr->p, (const int *)A.col->p, (const double *)A.val->p, dinv,
                         (const double *)b, x, V, ld, ws, c.reduction, c.max_iters, c.nonfinite_check, hist,
                         S.gnorm->p, s));
        char o[40];
        HIP_TRY(hipMemcpyAsync(o, S.gnorm->p, 40, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        int64_t it, sp, rs_;
        int32_t stc;
        double rel;
        memcpy(&it, o, 8);
        memcpy(&sp, o + 8, 8);
        memcpy(&rs_, o + 16, 8);
        memcpy(&stc, o + 24, 4);
        memcpy(&rel, o + 32, 8);
        SolverState h0{};
        fill_info(info, S, h0, it, stc == ST_MAX_ITERS ? MXL_STOP_MAX_ITERS : map_stop(stc), sp, elapsed_s(t0));
        if (info) {
            info->rel_residual = rel;
            info->restarts = rs_;
            info->reorth = it;
        }
        return MXL_OK;
    }
    // replay captured chunks unless asked for direct launches, or when the
    // preconditioner is an exact ILU (hundreds of level launches per step)
    const bool use_graph = c.launch_mode != 1 && !(S.ilu && S.ilu->trisolve == 0);
    auto &graphs = const_cast<SolverImpl &>(S).graphs;
    HIP_TRY(launch_state_init(st, c.reduction, c.nonfinite_check, s));
    if ((rs = restart(1)) != MXL_OK) return rs;
    SolverState h;
    if ((rs = read_state(S, h)) != MXL_OK) return rs;
    if (h.nb2 == 0.0) {
        HIP_TRY(launch_fill(MXL_F64, n, 0.0, x, s));
        HIP_TRY(hipStreamSynchronize(s));
        fill_info(info, S, h, 0, MXL_STOP_CONVERGED, 1, elapsed_s(t0));
        return MXL_OK;
    }
    int64_t k = 0, restarts = 0;
    int stop = h.stop ? map_stop(h.stop) : MXL_STOP_NONE;
    while (stop == MXL_STOP_NONE && k < c.max_iters) {
        const int steps = (int)std::min<int64_t>(m, c.max_iters - k);
        int done = 0;
        for (int j0 = 0; j0 < steps;) {
            const int cnt = std::min(c.check_every, steps - j0);
            if (use_graph) {
                const int64_t key = (int64_t)j0 * 65536 + cnt;
                auto &G = graphs[key];
                if (!G) {  // capture the chunk's launches once (on the context's capture stream)
                    if (!ctx->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking));
                    auto hold = std::make_shared<GraphHold>();
                    hipStream_t cs_ = ctx->cap_stream;
                    HIP_TRY(hipStreamBeginCapture(cs_, hipStreamCaptureModeThreadLocal));
                    std::swap(s, cs_);  // enqueue launches on s
                    const mxl_status cs = enqueue(j0, cnt);
                    std::swap(s, cs_);
                    const hipError_t ce = hipStreamEndCapture(ctx->cap_stream, &hold->g);
                    if (cs != MXL_OK) return cs;
                    HIP_TRY(ce);
                    HIP_TRY(hipGraphInstantiate(&hold->e, hold->g, nullptr, nullptr, 0));
                    G = hold;
                }
                HIP_TRY(hipGraphLaunch(G->e, s));
            } else if ((rs = enqueue(j0, cnt)) != MXL_OK) {
                return rs;
            }
            j0 += cnt;
            k += cnt;
            done += cnt;
            if ((rs = read_state(S, h)) != MXL_OK) return rs;
            if (h.stop) break;
            if (c.time_limit_s > 0 && elapsed_s(t0) >= c.time_limit_s) {
                stop = MXL_STOP_TIME;
                break;
            }
        }
        // the cycle's last column becomes final in one more multi-dot pass
        HIP_TRY(gm_step(n, ld, V, done, nullptr, nullptr, nullptr, dp, st, ws, m, hist, s));
        HIP_TRY(gm_close(n, ld, V, blockp ? nullptr : dinv, x, blockp ? (double *)S.r->p : nullptr, st, ws, m, s));
        if (blockp) HIP_TRY(apply_M((const double *)S.r->p, 1.0, x));
        if ((rs = read_state(S, h)) != MXL_OK) return rs;
        if (h.stop) {
            stop = map_stop(h.stop);
            break;
        }
        if (stop != MXL_STOP_NONE || k >= c.max_iters) break;
        if ((rs = restart(0)) != MXL_OK) return rs;
        ++restarts;
        if ((rs = read_state(S, h)) != MXL_OK) return rs;
        if (h.stop) stop = map_stop(h.stop);
    }
    if ((rs = read_state(S, h)) != MXL_OK) return rs;
    if (stop == MXL_STOP_NONE && h.stop) stop = map_stop(h.stop);
    int64_t iters;
    if (stop == MXL_STOP_NONE) {
        stop = MXL_STOP_MAX_ITERS;
        iters = k;
    } else if (stop == MXL_STOP_TIME) {
        iters = k;
    } else {
        iters = h.iters;
    }
    int64_t nspmv = 0;
    HIP_TRY(gm_read(ws, &nspmv, s));
    fill_info(info, S, h, iters, stop, 1 + nspmv + restarts, elapsed_s(t0));
    if (info) {
        info->restarts = restarts;
        info->reorth = iters;  // every basis vector is orthogonalised twice
    }
    return MXL_OK;
}

}  // namespace

// Mixed-precision iterative refinement: an FP64 operator, its FP32 value
// copy with FP32 Jacobi (dinv rounded from the FP64 reciprocal), an FP32
// Jacobi-CG inner solver, and FP64 outer work vectors.
namespace {

mxl_status solve_ir(const SolverImpl &S, const void *bv, void *xv, mxl_solve_info *info) {
    auto t0 = std::chrono::steady_clock::now();
    const IrImpl &ir = *S.ir;
    const SolverImpl &O = *ir.outer;
    const MatrixImpl &A = *ir.A64;
    mxl_ctx *ctx = A.ctx;
    hipStream_t s = ctx->stream;
    const int64_t n = A.nrows;
    const double *b = (const double *)bv;
    double *x = (double *)xv;
    auto *st = (SolverState *)O.state->p;
    auto *part = (double *)O.partials->p;
    const mxl_criteria &oc = ir.prm.outer;
    mxl_status rs;
    std::vector<double> hist;
    HIP_TRY(launch_state_init(st, oc.reduction, 1, s));
    HIP_TRY(ir_norms(ctx, n, b, st, part, s));
    SolverState h;
    if ((rs = read_state(O, h)) != MXL_OK) return rs;
    const double nb = std::sqrt(h.sums[0]);
    int stop = MXL_STOP_NONE;
    int64_t outer = 0, inner_total = 0, spmvs = 0;
    double rel = 0.0;
    if (nb == 0.0) {
        HIP_TRY(launch_fill(MXL_F64, n, 0.0, x, s));
        HIP_TRY(hipStreamSynchronize(s));
        stop = MXL_STOP_CONVERGED;
        hist.push_back(0.0);
    }
    while (stop == MXL_STOP_NONE) {
        if ((rs = residual(O, b, x)) != MXL_OK) return rs;
        ++spmvs;
        HIP_TRY(ir_norms(ctx, n, (const double *)O.r->p, st, part, s));
        if ((rs = read_state(O, h)) != MXL_OK) return rs;
        rel = std::sqrt(h.sums[0]) / nb;
        hist.push_back(rel);
        if (rel <= oc.reduction) { stop = MXL_STOP_CONVERGED; break; }
        if (!std::isfinite(rel)) { stop = MXL_STOP_NONFINITE; break; }
        if (outer >= oc.max_iters) { stop = MXL_STOP_MAX_ITERS; break; }
        if (oc.time_limit_s > 0 && elapsed_s(t0) >= oc.time_limit_s) { stop = MXL_STOP_TIME; break; }
        HIP_TRY(ir_scale_to_f32(n, (const double *)O.r->p, st, (float *)ir.r32->p, s));
        HIP_TRY(launch_fill(MXL_F32, n, 0.0, ir.d32->p, s));
        mxl_solve_info ii{};
        if ((rs = solve_cg(*ir.inner, ir.r32->p, ir.d32->p, &ii, true)) != MXL_OK) return rs;
        inner_total += ii.iterations;
        spmvs += ii.spmv_count;
        HIP_TRY(ir_correct(n, x, (const float *)ir.d32->p, st, s));
        ++outer;
    }
    HIP_TRY(hipStreamSynchronize(s));
    if (info) {
        info->iterations = outer;
        info->inner_iterations = inner_total;
        info->spmv_count = spmvs;
        info->rel_residual = rel;
        info->stop_reason = stop;
        info->seconds = elapsed_s(t0);
        if (info->history && info->history_cap > 0) {
            int64_t cnt = std::min<int64_t>((int64_t)hist.size(), info->history_cap);
            memcpy(info->history, hist.data(), cnt * sizeof(double));
        }
    }
    return MXL_OK;
}

}  // namespace

extern "C" mxl_status mxl_ir_generate(const mxl_op *Aop, const mxl_ir_params *prm, mxl_op **out) try {
    if (!Aop || !prm || !out || Aop->kind != MXL_OP_MATRIX)
        return fail(MXL_ERR_INVALID_ARG, "matrix operator and parameters required");
    *out = nullptr;
    const auto &A = Aop->mat;
    if (A->dtype != MXL_F64) return fail(MXL_ERR_DTYPE, "iterative refinement needs an FP64 matrix");
    DeviceScope ds(A->ctx->device);
    auto ir = std::make_shared<IrImpl>();
    ir->A64 = A;
    ir->prm = *prm;
    mxl_op *a32 = nullptr;
    mxl_status st = mxl_cast(Aop, MXL_F32, &a32);
    if (st != MXL_OK) return st;
    ir->A32 = a32->mat;
    delete a32;
    hipError_t e;
    std::shared_ptr<JacobiImpl> J32;
    if (prm->inner_block_mode != 0 && prm->inner_block_mode != 1)
        return fail(MXL_ERR_INVALID_ARG, "inner_block_mode must be 0 or 1");
    if (prm->inner_block_size > 0) {
        // block Jacobi from the FP64 matrix; usable with the FP32 vectors as is
        mxl_op *bj = nullptr;
        st = prm->inner_block_mode == 1
                 ? mxl_bjacobi_generate_var(Aop, 0, nullptr, prm->inner_block_size, 1, prm->inner_block_accuracy, &bj)
                 : mxl_bjacobi_generate(Aop, prm->inner_block_size, 1, prm->inner_block_accuracy, &bj);
        if (st != MXL_OK) return st;
        J32 = bj->jac;
        delete bj;
    } else {
        if (prm->inner_block_size < 0) return fail(MXL_ERR_INVALID_ARG, "inner_block_size < 0");
        mxl_op *j64 = nullptr;
        if ((st = mxl_jacobi_generate(Aop, &j64)) != MXL_OK) return st;
        J32 = std::make_shared<JacobiImpl>();
        J32->A = ir->A32;
        J32->dinv = alloc((size_t)A->nrows * 4, &e);
        if (!J32->dinv) { delete j64; return hip_fail(e, "alloc dinv32"); }
        e = launch_convert_vals(A->nrows, MXL_F64, j64->jac->dinv->p, J32->dinv->p, A->ctx->stream);
        if (e != hipSuccess) { delete j64; return hip_fail(e, "convert dinv"); }
        HIP_TRY(hipStreamSynchronize(A->ctx->stream));
        delete j64;
    }
    mxl_criteria oc = prm->outer;
    if ((st = make_solver(MXL_SOLVER_CG, ir->A32, J32, prm->inner, ir->inner)) != MXL_OK) return st;
    mxl_criteria o2 = oc;
    o2.max_iters = 0;  // the outer record only needs vectors and state
    if ((st = make_solver(MXL_SOLVER_CG, A, nullptr, o2, ir->outer)) != MXL_OK) return st;
    ir->r32 = alloc((size_t)A->nrows * 4, &e);
    ir->d32 = alloc((size_t)A->nrows * 4, &e);
    if (!ir->r32 || !ir->d32) return hip_fail(hipErrorOutOfMemory, "alloc ir vectors");
    auto S = std::make_shared<SolverImpl>();
    S->kind = MXL_SOLVER_IR;
    S->A = A;
    S->crit = oc;
    S->ir = ir;
    auto *op = new mxl_op;
    op->kind = MXL_OP_SOLVER;
    op->sol = S;
    *out = op;
    return MXL_OK;
} catch (...) {
    return mxl::abi_exception(__func__);
}

extern "C" mxl_status mxl_solve(const mxl_op *Sop, const void *b, void *x, mxl_solve_info *info) try {
    if (!Sop || Sop->kind != MXL_OP_SOLVER) return fail(MXL_ERR_INVALID_ARG, "not a solver operator");
    if (!b || !x) return fail(MXL_ERR_INVALID_ARG, "vector is NULL");
    if (b == x) return fail(MXL_ERR_INVALID_ARG, "right-hand side and solution alias");
    const SolverImpl &S = *Sop->sol;
    const MatrixImpl &A = *S.A;
    DeviceScope ds(A.ctx->device);
    const size_t vt = vt_size(A.dtype);
    mxl_status st;
    if ((st = check_dev(A.ctx, b, (size_t)A.nrows * vt, "b")) != MXL_OK) return st;
    if ((st = check_dev(A.ctx, x, (size_t)A.nrows * vt, "x")) != MXL_OK) return st;
    if (S.kind == MXL_SOLVER_CG) return solve_cg(S, b, x, info);
    if (S.kind == MXL_SOLVER_BICGSTAB) return solve_bicgstab(S, b, x, info);
    if (S.kind == MXL_SOLVER_IR) return solve_ir(S, b, x, info);
    if (S.kind == MXL_SOLVER_GMRES) return solve_gmres(S, b, x, info);
    return fail(MXL_ERR_NOT_IMPLEMENTED, "unknown solver kind");
} catch (...) {
    return mxl::abi_exception(__func__);
}

extern "C" mxl_status mxl_time_apply(const mxl_op *Aop, const void *x, void *y, int reps, int flush,
                                     double *median_ms) try {
    if (!Aop || Aop->kind != MXL_OP_MATRIX || !median_ms || reps < 1)
        return fail(MXL_ERR_INVALID_ARG, "matrix operator, reps >= 1 and output required");
    const MatrixImpl &A = *Aop->mat;
    mxl_ctx *ctx = A.ctx;
    DeviceScope ds(ctx->device);
    const size_t vt = vt_size(A.dtype);
    mxl_status st;
    if ((st = check_dev(ctx, x, (size_t)A.ncols * vt, "x")) != MXL_OK) return st;
    if ((st = check_dev(ctx, y, (size_t)A.nrows * vt, "y")) != MXL_OK) return st;
    if (x == y) return fail(MXL_ERR_INVALID_ARG, "input and output alias");
    hipStream_t s = ctx->stream;
    if (flush && !ctx->flush_buf) {
        hipError_t e;
        ctx->flush_buf = alloc((size_t)1 << 30, &e);
        if (!ctx->flush_buf) return hip_fail(e, "alloc flush buffer");
    }
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    std::vector<double> ts;
    SpmvArgs a;
    a.x = x;
    a.y = y;
    // one untimed launch first: the first launch of a kernel in a process
    // also loads its code and maps the arrays' pages
    hipError_t err = spmv_launch(A, a, s);
    for (int r = 0; r < reps && err == hipSuccess; ++r) {
        if (flush) err = launch_flush(ctx->flush_buf->p, ctx->flush_buf->bytes, s);
        if (err == hipSuccess) err = hipEventRecord(e0, s);
        if (err == hipSuccess) err = spmv_launch(A, a, s);
        if (err == hipSuccess) err = hipEventRecord(e1, s);
        if (err == hipSuccess) err = hipEventSynchronize(e1);
        float ms = 0.f;
        if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
        ts.push_back(ms);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (err != hipSuccess) return hip_fail(err, "time_apply");
    std::sort(ts.begin(), ts.end());
    size_t m = ts.size();
    *median_ms = m % 2 ? ts[m / 2] : 0.5 * (ts[m / 2 - 1] + ts[m / 2]);
    return MXL_OK;
} catch (...) {
    return mxl::abi_exception(__func__);
}

extern "C" mxl_status mxl_stream_bench(mxl_ctx *ctx, int op, int64_t n, const double *a,
                                       const double *b, double *c, int reps, double *median_ms) try {
    if (!ctx || !median_ms || reps < 1 || n < 2 || (n & 1) || op < 0 || op > 3)
        return fail(MXL_ERR_INVALID_ARG, "stream: op in 0..3, even n >= 2, reps >= 1");
    DeviceScope ds(ctx->device);
    mxl_status st;
    const size_t bytes = (size_t)n * 8;
    if ((st = check_dev(ctx, a, bytes, "a")) != MXL_OK) return st;
    if ((op == 1 || op == 2) && (st = check_dev(ctx, b, bytes, "b")) != MXL_OK) return st;
    const size_t cbytes = op >= 2 ? (size_t)ctx->num_cu * 8 * 8 : bytes;
    if ((st = check_dev(ctx, c, cbytes, "c")) != MXL_OK) return st;
    hipStream_t s = ctx->stream;
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    std::vector<double> ts;
    hipError_t err = hipSuccess;
    for (int r = 0; r < reps && err == hipSuccess; ++r) {
        err = hipEventRecord(e0, s);
        if (err == hipSuccess) err = launch_stream(ctx, op, n, a, b, c, s);
        if (err == hipSuccess) err = hipEventRecord(e1, s);
        if (err == hipSuccess) err = hipEventSynchronize(e1);
        float ms = 0.f;
        if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
        ts.push_back(ms);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (err != hipSuccess) return hip_fail(err, "stream");
    std::sort(ts.begin(), ts.end());
    size_t m = ts.size();
    *median_ms = m % 2 ? ts[m / 2] : 0.5 * (ts[m / 2 - 1] + ts[m / 2]);
    return MXL_OK;
} catch (...) {
    return mxl::abi_exception(__func__);
}
