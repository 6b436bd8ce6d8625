// internal.hpp -- host-side objects of the library (context, reference-
// counted device buffers, operator handles) and the launcher interfaces the
// runtime uses to reach the kernels.  Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <atomic>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "../../include/mxl.h"
#include "abi_guard.hpp"

namespace mxl {


struct SolverState;

// A device allocation, freed when the last shared owner lets go.  Borrowed
// views (owned = false) are never freed.
struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
    bool owned = false;
    ~DevBuf() {
        if (owned && p) (void)hipFree(p);
    }
};
using BufPtr = std::shared_ptr<DevBuf>;

}  // namespace mxl

struct mxl_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    int num_cu = 256;
    std::string arch;
    void *pinned = nullptr;     // host-pinned staging for solver state read-back
    size_t pinned_bytes = 0;
    mxl::BufPtr flush_buf;      // lazily allocated 1 GiB buffer for cache flushes
    hipStream_t cap_stream = nullptr;  // lazily created stream that graphs are captured on
                                       // (the caller's stream may be the null stream)
    void *noalloc_scratch = nullptr;   // this device's copy of the static batch scratch
                                       // (NULL if its address could not be looked up)
    // The caller's handle plus one count per library object that uses the
    // context: mxl_ctx_destroy drops the caller's count, and the context is
    // freed with the last object, whatever order handles are destroyed in.
    std::atomic<int> refs{1};
};

namespace mxl {

void ctx_release(mxl_ctx *c);  // frees the context when the count reaches zero

// A counted reference to a context (held by every object that uses one).
struct CtxRef {
    mxl_ctx *p = nullptr;
    CtxRef() = default;
    explicit CtxRef(mxl_ctx *c) : p(c) { retain(); }
    CtxRef(const CtxRef &o) : p(o.p) { retain(); }
    CtxRef &operator=(const CtxRef &o) { return *this = o.p; }
    CtxRef &operator=(mxl_ctx *c) {
        if (c) c->refs.fetch_add(1);
        if (p) ctx_release(p);
        p = c;
        return *this;
    }
    ~CtxRef() {
        if (p) ctx_release(p);
    }
    mxl_ctx *operator->() const { return p; }
    operator mxl_ctx *() const { return p; }

private:
    void retain() {
        if (p) p->refs.fetch_add(1);
    }
};

struct MatrixImpl {
    CtxRef ctx;
    int dtype = MXL_F64;
    int64_t nrows = 0, ncols = 0, nnz = 0;
    int format = MXL_FMT_CSR;
    int variant = MXL_CSR_VECTOR;
    int vw = 32;                       // CSR vector lanes per row
    BufPtr row_ptr, col, val;          // canonical CSR (always present)
    BufPtr coo_row;                    // COO
    BufPtr ell_col, ell_val, ell_win;  // ELL / HYB ELL part
    int ell_w = 0;
    int ell_rpt = 1;                   // ELL rows per thread (1, 2, 4)
    int ell_nb = 0;                    // ELL: neighbour reuse of gathered x values on
    int64_t n_pad = 0;
    double hyb_q = 0.0;
    BufPtr tail_row, tail_col, tail_val;  // HYB COO tail
    int64_t tail_nnz = 0;
    BufPtr part;                       // merge-path tile boundaries / row-block descriptors (int2)
    int64_t ntiles = 0;                // merge / COO / HYB-tail tiles, row blocks
    BufPtr carries;                    // per-tile carries
    // matrix-free stencil: grid and points (host copies, passed by value)
    int64_t nx = 0, ny = 0, nz = 0;
    int st_npts = 0;
    int8_t st_off[27][3] = {};
    double st_coef[27] = {};
    int grid_main = 0, grid_tail = 0;  // workgroups of the chain's kernels
    int grid_dot = 0;                  // ELL: workgroups of fused-dot launches
    int64_t stored_bytes = 0;
};

struct JacobiImpl {
    std::shared_ptr<MatrixImpl> A;
    BufPtr dinv;                 // point Jacobi
    // block Jacobi: inverses of consecutive bs-row diagonal blocks, each
    // stored bs x bs at byte offset boff[b] in precision bprec[b]
    bool block = false;
    int bs = 1;
    int64_t nblocks = 0;
    BufPtr bstore, boff, bprec, bcond;
    int64_t bstore_bytes = 0;
    // variable-size blocks (var): block b holds rows bptr[b] .. bptr[b+1)
    // (at most 32); its m x m inverse is stored row by row, each row padded
    // to a whole number of 16-byte chunks; rblk[i] = block of row i
    bool var = false;
    BufPtr bptr_d, rblk;
    std::vector<int32_t> bptr_h;
};

// ILU-type preconditioner: factors on A's pattern (strict lower = L with
// unit diagonal, the rest = U), diagonal positions, dependency levels of
// both triangles (rows listed level by level) and three work vectors.
struct IluImpl {
    std::shared_ptr<MatrixImpl> A;
    int sweeps = 0, trisolve = 0, trs_sweeps = 0;
    BufPtr lu, dpos, lperm, uperm, y, t, z;
    std::vector<int64_t> lptr, uptr;
    // exact solves: the level offsets on the device (runs of small levels are
    // solved by one workgroup in one launch) and the schedule of launches
    BufPtr lptr_d, uptr_d;
    std::vector<int2> lruns, uruns;  // (first level, end level): a run of small levels, or one level
    // each triangle's strict entries in level order, slot-major [w][n_pad]
    // (position t of the level schedule at slot*n_pad + t; column -1 pads),
    // and diag(U) in upper level order; NULL when the padding would exceed
    // 4x the factor storage (the solves then walk the CSR rows)
    int lw_lv = 0, uw_lv = 0;
    BufPtr lcol_lv, lval_lv, ucol_lv, uval_lv, udiag_lv;
    // slot-major strict triangles and diag(U) for the Jacobi sweeps (optional)
    int wl = 0, wu = 0;
    int64_t n_pad = 0;
    BufPtr lcol, lval, ucol, uval, udiag;
};

struct IrImpl;
struct BatchImpl;

// An instantiated HIP graph (a captured chunk of a solver's launches).
struct GraphHold {
    hipGraph_t g = nullptr;
    hipGraphExec_t e = nullptr;
    GraphHold() = default;
    GraphHold(const GraphHold &) = delete;
    GraphHold &operator=(const GraphHold &) = delete;
    ~GraphHold() {
        if (e) (void)hipGraphExecDestroy(e);
        if (g) (void)hipGraphDestroy(g);
    }
};

struct SolverImpl {
    int kind = MXL_SOLVER_CG;
    std::shared_ptr<MatrixImpl> A;
    std::shared_ptr<JacobiImpl> P;  // may be null
    std::shared_ptr<IluImpl> ilu;   // ILU preconditioner (GMRES), may be null
    mxl_criteria crit{};
    // work vectors (A's value type)
    BufPtr r, p, q, z, rhat, v, s, t, ones;
    BufPtr r2;        // CG with variable-size block Jacobi: r alternates between r and r2
    BufPtr state;     // SolverState
    BufPtr partials;  // 3 doubles per slot
    BufPtr hist;      // max_iters + 1 doubles
    int64_t hist_len = 0;
    std::shared_ptr<IrImpl> ir;  // iterative refinement only
    std::shared_ptr<BatchImpl> single;  // one-launch CG of a small system
    BufPtr single_out;                  // iterations, residual, status
    // GMRES(krylov): basis V (krylov+1 vectors of ld doubles), workspace,
    // multi-dot and norm partials
    int krylov = 0;
    int64_t ld = 0;
    BufPtr V, gmws, gdots, gnorm;
    // GMRES step chunks captured as graphs, keyed by (first step, count);
    // their kernels take only solver-owned pointers and the step index
    std::map<int64_t, std::shared_ptr<GraphHold>> graphs;
    // HIP events of the sampled SpMV timing, kept across solves so that a
    // timed solve creates none
    std::vector<hipEvent_t> spmv_events;
    // events of the two state snapshots of the trailing host check
    mutable hipEvent_t chk_ev[2] = {nullptr, nullptr};
    SolverImpl() = default;
    SolverImpl(const SolverImpl &) = delete;
    SolverImpl &operator=(const SolverImpl &) = delete;
    ~SolverImpl() {
        for (hipEvent_t e : spmv_events)
            if (e) (void)hipEventDestroy(e);
        for (hipEvent_t e : chk_ev)
            if (e) (void)hipEventDestroy(e);
    }
};

struct IrImpl {
    std::shared_ptr<MatrixImpl> A64, A32;
    std::shared_ptr<SolverImpl> outer;  // FP64 residual vector, state, partials
    std::shared_ptr<SolverImpl> inner;  // FP32 Jacobi-CG
    BufPtr r32, d32;
    mxl_ir_params prm{};
};

struct BatchImpl;  // batched.hip
mxl_ctx *batch_ctx(const BatchImpl &B);
// Size of the fixed device scratch behind mxl_batch_solve_noalloc (96 MiB):
// the queue counter plus the spill region of 8 workgroups per CU on 256 CUs
// at 1,024-row systems (80 MiB).
constexpr size_t kNoAllocScratchBytes = (size_t)96 << 20;
// Looks up (once per device, with that device current) the address of the
// device's copy of that scratch.
hipError_t noalloc_scratch_init(int device, void **out);
std::shared_ptr<BatchImpl> batch_from_matrix(const MatrixImpl &A, const void *dinv);
mxl_status batch_single_solve(BatchImpl &Bt, const mxl_criteria &c, const double *b, double *x,
                              void *out3, int64_t *iters, double *rel, int *stop);
// One-workgroup BiCGSTAB; false when no register shape holds the system.
bool batch_single_bicgstab(BatchImpl &Bt, const mxl_criteria &c, const double *b, double *x, void *out3,
                           int64_t *iters, double *rel, int *stop, int *half, mxl_status *st);

struct SpmvArgs {
    double alpha = 1.0, beta = 0.0;
    const void *x = nullptr;
    void *y = nullptr;
    const int *stop = nullptr;  // skip all work when *stop != 0 (device flag)
    const void *w = nullptr;    // fused dot w.y (nullable; never the output y) ...
    double *partials = nullptr; // ... one partial per workgroup, spmv_slots(A) slots
};

// ------------------------------------------------------------- spmv.hip
void spmv_plan(MatrixImpl &A);
int spmv_slots(const MatrixImpl &A);
int64_t merge_tiles(int64_t n, int64_t nnz);
int64_t coo_tiles(int64_t nnz);
int64_t carry_bytes(int64_t ntiles);
// Row blocks of the streaming CSR kernel from host row pointers: (first
// row, first nonzero) of every block plus the terminator (n, nnz).
void stream_blocks(const std::vector<int32_t> &rp, std::vector<int32_t> &out);
int ell_lds_cap();
hipError_t merge_partition(const MatrixImpl &A, hipStream_t s);
hipError_t spmv_launch(const MatrixImpl &A, const SpmvArgs &a, hipStream_t s);
hipError_t launch_validate(const MatrixImpl &A, int *flags, hipStream_t s);
hipError_t launch_csr_to_coo(const MatrixImpl &A, int *row, hipStream_t s);
hipError_t launch_csr_to_ell16(const MatrixImpl &A, int w, int64_t n_pad, short *ecol, void *evals,
                               int *overflow, hipStream_t s);
hipError_t launch_csr_to_ell(const MatrixImpl &A, int w, int64_t n_pad, int *ecol, void *evals,
                             hipStream_t s);
hipError_t launch_ell_reuse_count(const MatrixImpl &A, int w, unsigned long long *count, hipStream_t s);
hipError_t launch_hyb_tail(const MatrixImpl &A, int k, const int64_t *toff, int *trow, int *tcol,
                           void *tval, hipStream_t s);
hipError_t launch_ell_windows(const MatrixImpl &A, int2 *win, hipStream_t s);
hipError_t launch_jacobi(const MatrixImpl &A, void *dinv, int *bad, hipStream_t s);
hipError_t launch_convert_vals(int64_t n, int from, const void *in, void *out, hipStream_t s);

// ------------------------------------------------------------- krylov.hip
constexpr int kSolverSlots = 8192;  // partial slots per reduction region
constexpr int kRegions = 4;         // partial regions A..D, 3 doubles per slot
int vec_grid(const mxl_ctx *ctx, int64_t n);
int cg_update_grid(const mxl_ctx *ctx, int64_t n);  // grid (and partial count) of cg_update / cg_pupdate
hipError_t launch_finalize(int nv, const double *parts, int slots, SolverState *st, int op, int k,
                           int max_iters, double *hist, hipStream_t s);
hipError_t launch_jacobi_apply(int dtype, int64_t n, double alpha, const void *dinv, const void *b,
                               double beta, void *x, hipStream_t s);
hipError_t launch_copy(int dtype, int64_t n, const void *src, void *dst, hipStream_t s);
hipError_t launch_fill(int dtype, int64_t n, double v, void *dst, hipStream_t s);
hipError_t launch_state_init(SolverState *st, double red, int nonfinite_check, hipStream_t s);
hipError_t cg_init(const mxl_ctx *ctx, int dtype, int64_t n, const void *b, const void *r, void *p,
                   const void *dinv, double *parts, hipStream_t s);
hipError_t cg_update(const mxl_ctx *ctx, int dtype, int64_t n, void *r, const void *q, const void *dinv,
                     SolverState *st, const double *pq_parts, int pq_slots, double *parts, int k,
                     hipStream_t s);
hipError_t cg_pupdate(const mxl_ctx *ctx, int dtype, int64_t n, void *x, const void *r, void *p,
                      const void *dinv, SolverState *st, const double *parts, int slots, int k,
                      double *hist, hipStream_t s);
hipError_t bi_init(const mxl_ctx *ctx, int dtype, int64_t n, const void *b, const void *r,
                   void *rhat, void *p, void *v, double *parts, hipStream_t s);
hipError_t bi_pupdate(const mxl_ctx *ctx, int dtype, int64_t n, const void *r, void *p,
                      const void *v, void *phat, const void *dinv, SolverState *st,
                      const double *parts, int slots, int k, double *hist, hipStream_t s);
hipError_t bi_supdate(const mxl_ctx *ctx, int dtype, int64_t n, const void *r, const void *v,
                      void *sv, void *shat, const void *dinv, SolverState *st,
                      const double *rv_parts, int rv_slots, double *parts, int k, hipStream_t s);
hipError_t bi_tdots(const mxl_ctx *ctx, int dtype, int64_t n, const void *t, const void *sv,
                    SolverState *st, const double *ss_parts, int ss_slots, double *parts, int k,
                    double *hist, hipStream_t s);
hipError_t bi_xupdate(const mxl_ctx *ctx, int dtype, int64_t n, void *x, void *r, const void *phat,
                      const void *shat, const void *sv, const void *t, const void *rhat,
                      SolverState *st, const double *ts_parts, int ts_slots, double *parts, int k,
                      hipStream_t s);
hipError_t ir_norms(const mxl_ctx *ctx, int64_t n, const double *r, SolverState *st, double *parts,
                    hipStream_t s);
hipError_t ir_scale_to_f32(int64_t n, const double *r, const SolverState *st, float *r32,
                           hipStream_t s);
hipError_t ir_correct(int64_t n, double *x, const float *d, const SolverState *st, hipStream_t s);
hipError_t launch_flush(void *buf, size_t bytes, hipStream_t s);
hipError_t launch_stream(const mxl_ctx *ctx, int op, int64_t n, const double *a, const double *b,
                         double *c, hipStream_t s);

// ------------------------------------------------------------- bjacobi.hip
hipError_t bj_cg_init(const mxl_ctx *ctx, const JacobiImpl &P, int dtype, int64_t n, const void *b,
                      const void *r, void *p, double *parts, hipStream_t s);
// r_out = r_in - alpha q (r_out == r_in: in place; variable-size blocks
// need distinct buffers, since a workgroup also reads the rows of blocks
// that reach into its neighbours' tiles)
hipError_t bj_cg_update(const mxl_ctx *ctx, const JacobiImpl &P, int dtype, int64_t n, const void *r_in,
                        void *r_out, const void *q, void *z, SolverState *st, const double *pq_parts, int pq_slots,
                        double *parts, int k, hipStream_t s);
// z = alpha M r + beta z; stop (nullable, device) skips the product once a
// solve has stopped.
hipError_t bj_apply(const mxl_ctx *ctx, const JacobiImpl &P, int64_t n, double alpha, const void *r,
                    double beta, void *z, hipStream_t s, const int *stop = nullptr);

// ------------------------------------------------------------- gmres.hip
constexpr int kGmMaxKrylov = 1024;
size_t gm_ws_bytes(int m);
int gm_grid(int64_t n);
hipError_t gm_prep(const mxl_ctx *ctx, int64_t n, const double *v, const double *b, const double *dinv,
                   double *z, double *parts, int *slots, hipStream_t s);
hipError_t gm_start(const double *parts, int slots, SolverState *st, void *ws, int m, double *hist, int first,
                    hipStream_t s);
// Arnoldi step j after u = A M^{-1} t_j (u == nullptr: the cycle's closing pass)
hipError_t gm_step(int64_t n, int64_t ld, double *V, int j, const double *u, const double *dinv, double *z,
                   double *dparts, SolverState *st, void *ws, int m, double *hist, hipStream_t s);
hipError_t gm_close(int64_t n, int64_t ld, const double *V, const double *dinv, double *x, double *t,
                    const SolverState *st, void *ws, int m, hipStream_t s);
hipError_t gm_read(const void *ws, int64_t *nspmv, hipStream_t s);
// The whole solve of a small system (n <= 1024, m <= 128) in one workgroup;
// out: iterations, products, restarts (int64), status (int32 at 24), rel (double at 32)
hipError_t gm_small(int n, int m, const int *rp, const int *col, const double *val, const double *dinv,
                    const double *b, double *x, double *V, int64_t ld, void *ws, double red, int64_t maxit, int chk,
                    double *hist, void *out, hipStream_t s);

// ------------------------------------------------------------- ilu.hip
// out = alpha U^{-1} L^{-1} r + beta out (beta == 0 overwrites)
hipError_t ilu_apply(const IluImpl &P, double alpha, const void *r, double beta, void *out, hipStream_t s);

// ------------------------------------------------------------- runtime.hip
mxl_status set_error(mxl_status st, const std::string &msg);
mxl_status check_device_ptr(const mxl_ctx *ctx, const void *p, size_t bytes, const char *what);

// Makes `dev` current for the scope's lifetime, then restores the caller's device.
struct DeviceScope {
    int prev = -1;
    explicit DeviceScope(int dev) {
        (void)hipGetDevice(&prev);
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~DeviceScope() {
        int cur = -1;
        (void)hipGetDevice(&cur);
        if (prev >= 0 && cur != prev) (void)hipSetDevice(prev);
    }
};

size_t vt_size(int dtype);
int64_t csr_bytes(const MatrixImpl &A);
// Padded ELL storage (w slots of n rounded up to 64 rows) may cost up to 4x
// the CSR bytes, at least 1 MiB (so tiny matrices are never refused for
// their row padding) and at most 32 GiB.
bool ell_fits(const MatrixImpl &S, int64_t w);
// Nearest-rank q-quantile of row lengths, rank = ceil(q n) clamped to [1, n].
int64_t quantile_rank(double q, int64_t n);

// ------------------------------------------------------------- select.hip
// The 16 features; hist (optional) receives the row-length histogram and
// maxbw (optional) the largest |col - row|.
mxl_status features_compute(const MatrixImpl &A, double out[16], std::vector<unsigned> *hist = nullptr,
                            int64_t *maxbw = nullptr);

}  // namespace mxl

// The opaque handle handed out by the ABI.
struct mxl_op {
    int kind = MXL_OP_MATRIX;
    std::shared_ptr<mxl::MatrixImpl> mat;
    std::shared_ptr<mxl::JacobiImpl> jac;
    std::shared_ptr<mxl::SolverImpl> sol;
    std::shared_ptr<mxl::BatchImpl> bat;
    std::shared_ptr<mxl::IluImpl> ilu;
};
