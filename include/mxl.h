/*
 * mxl.h -- C ABI of the MI355X (gfx950) sparse linear-operator library.
 *
 * The library follows the operator view of the paper (Sec. 2.2): a sparse
 * matrix, a preconditioner and a solver are all linear operators with one
 * application call, x = L(b) (Sec. 2.2.2), and an advanced form
 * x = alpha*L(b) + beta*x (Sec. 4.2).  Solvers and preconditioners are
 * produced by binding a system matrix to a factory (Sec. 2.2.3), with the
 * stopping criteria of Sec. 2.5.
 *
 * Conventions for every entry point
 *  - Every call returns mxl_status; MXL_OK is 0.  No C++ exception crosses
 *    this boundary: a host allocation failure inside the library returns
 *    MXL_ERR_OUT_OF_MEMORY, any other unexpected failure MXL_ERR_INTERNAL.
 *    On a non-OK status, mxl_last_error() returns a thread-local,
 *    NUL-terminated description (at most 511 characters) valid until the
 *    next failing call on the same thread.
 *  - Vector and matrix-array arguments are DEVICE pointers on the context's
 *    device unless a parameter says "host".  The library never frees memory
 *    it did not allocate.
 *  - Work is enqueued on the context's HIP stream (borrowed from the caller)
 *    and is stream-ordered: mxl_apply* returns before the result is ready,
 *    exactly like a kernel launch.  mxl_solve and
 *    mxl_batch_solve block until the solve has stopped;
 *    mxl_batch_solve_noalloc does not.
 *  - Index arrays are int32 and must describe canonical CSR: row_ptr[0] = 0,
 *    non-decreasing, row_ptr[nrows] = nnz, column indices in [0, ncols) and
 *    strictly increasing within a row.
 *  - Handles are not thread-safe: do not use one handle from two host
 *    threads at once.
 */
#ifndef MXL_H
#define MXL_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    MXL_OK = 0,
    MXL_ERR_INVALID_ARG = 1,       /* null/unknown argument, aliasing, bad enum */
    MXL_ERR_DIM_MISMATCH = 2,      /* operand sizes do not conform */
    MXL_ERR_DTYPE = 3,             /* operand value type does not match */
    MXL_ERR_NOT_IMPLEMENTED = 4,   /* combination not provided */
    MXL_ERR_INVALID_MATRIX = 5,    /* CSR arrays not canonical */
    MXL_ERR_ZERO_DIAG = 6,         /* missing or zero diagonal entry */
    MXL_ERR_OUT_OF_MEMORY = 7,
    MXL_ERR_INFEASIBLE_FORMAT = 8, /* padded format exceeds its memory budget */
    MXL_ERR_DEVICE = 9,            /* HIP runtime error */
    MXL_ERR_INTERNAL = 10          /* unexpected failure inside the library */
} mxl_status;

typedef enum { MXL_F64 = 0, MXL_F32 = 1 } mxl_dtype;

typedef enum {
    MXL_FMT_CSR = 0, MXL_FMT_COO = 1, MXL_FMT_ELL = 2, MXL_FMT_HYB = 3,
    MXL_FMT_STENCIL = 4  /* matrix-free stencil (mxl_stencil_create); no arrays */
} mxl_format;

/* Kernel variants (the "kernel variant selection" fork of Sec. 7.2). */
enum {
    MXL_CSR_SCALAR = 0,  /* one lane per row */
    MXL_CSR_VECTOR = 1,  /* W lanes per row, W = vector_width in {2..64} */
    MXL_CSR_MERGE = 2,   /* merge-path split of rows+nonzeros */
    MXL_CSR_STREAM = 3,  /* blocks of <= 63 rows / 512 nonzeros per wave,
                            coalesced loads staged in LDS; long rows alone */
    MXL_COO_SEGRED = 0,  /* segmented reduction over row-sorted triplets */
    MXL_ELL_PLAIN = 0,   /* one lane per row, gathers x from memory */
    MXL_ELL_LDS = 1,     /* stages each block's x window in LDS when it fits */
    MXL_ELL_DELTA16 = 2, /* ELL only: 16-bit column offsets col - row (padding
                            -32768), 2 index bytes per slot instead of 4;
                            INFEASIBLE_FORMAT if some |col - row| > 32767 */
    MXL_HYB_DEFAULT = 0
};

typedef struct {
    int32_t variant;       /* MXL_CSR_* / MXL_ELL_* ... */
    int32_t vector_width;  /* CSR vector: lanes per row (0 = from mean row length);
                              ELL/HYB: rows per thread 1, 2 or 4 (0 = 2) */
    double  hyb_quantile;  /* HYB: ELL width = nearest-rank quantile of row lengths (0 = 0.9) */
} mxl_format_params;

typedef enum { MXL_OP_MATRIX = 0, MXL_OP_JACOBI = 1, MXL_OP_SOLVER = 2, MXL_OP_BATCH = 3,
               MXL_OP_ILU = 4 } mxl_op_kind;

typedef enum { MXL_SOLVER_CG = 0, MXL_SOLVER_BICGSTAB = 1, MXL_SOLVER_IR = 2,
               MXL_SOLVER_GMRES = 3 } mxl_solver_kind;

/* Stop reasons: the stopping_status of Sec. 2.5. */
typedef enum {
    MXL_STOP_NONE = 0, MXL_STOP_CONVERGED = 1, MXL_STOP_MAX_ITERS = 2,
    MXL_STOP_TIME = 3, MXL_STOP_BREAKDOWN = 4, MXL_STOP_NONFINITE = 5
} mxl_stop;

/* Stopping criteria (Sec. 2.5), combined by logical OR: the first one met
 * stops the iteration.  Iteration: max_iters.  ResidualNormReduction:
 * ||r_k||_2 <= reduction * ||b||_2 on the recurrence residual.  Time:
 * time_limit_s wall seconds, checked on the host every check_every
 * iterations (<= 0 disables).  check_every >= 1 is how often the host reads
 * the device-side status; iterations after a device-side stop are no-ops, so
 * results do not depend on it.  nonfinite_check = 1 stops with
 * MXL_STOP_NONFINITE when a reduction yields NaN/Inf. */
typedef struct {
    int64_t max_iters;
    double  reduction;
    double  time_limit_s;
    int32_t check_every;
    int32_t nonfinite_check;
    int32_t launch_mode;   /* CG and BiCGSTAB: 0 auto, 1 one kernel per step,
                              2 the whole solve in one persistent workgroup
                              (FP64, point Jacobi or none, max_iters >= 1, no
                              Time criterion and no history; CG n <= 16384,
                              BiCGSTAB n <= 4096 with <= 5 entries per row
                              (<= 8 for n <= 1024), else per step); auto
                              picks 2 for n <= 8192.  GMRES: 1 launches every
                              kernel of every step; otherwise systems with
                              n <= 1024 and krylov_dim <= 128 (point Jacobi or
                              none, no Time criterion) run whole in one
                              workgroup, and larger ones capture each chunk
                              of check_every steps once as a HIP graph and
                              replay it (except with an exact ILU) */
} mxl_criteria;

/* Convergence record (the Convergence logger of Sec. 2.6) plus an optional
 * residual history (the Record logger): if history is a non-null HOST
 * pointer with history_cap > 0 entries, history[k] receives ||r_k||/||b||
 * for k = 0..min(iterations, history_cap-1). */
typedef struct {
    int64_t iterations;
    int64_t spmv_count;
    double  rel_residual;   /* recurrence residual norm / ||b|| at exit */
    int32_t stop_reason;    /* mxl_stop */
    double  seconds;        /* host wall time of the solve */
    double *history;        /* in: host buffer or NULL */
    int64_t history_cap;    /* in */
    int64_t inner_iterations; /* iterative refinement: total inner iterations */
    int32_t time_spmv;      /* in: k > 0 = time every k-th SpMV launch of
                               the CG loop with HIP events (first 4096
                               samples); 0 = no events */
    double  spmv_ms;        /* out: summed SpMV time of the timed launches */
    int64_t spmv_timed;     /* out: number of timed launches */
    int64_t restarts;       /* out, GMRES: restarted cycles */
    int64_t reorth;         /* out, GMRES: basis vectors orthogonalised a second time */
} mxl_solve_info;

typedef struct mxl_ctx mxl_ctx;
typedef struct mxl_op mxl_op;

/* ---------------------------------------------------------------- context */

/* Executor (Sec. 2.3): one gfx950 device plus the caller's HIP stream
 * (borrowed, not destroyed; NULL = the null stream).  Errors: INVALID_ARG
 * for out==NULL, DEVICE if the device cannot be selected or is not gfx950. */
mxl_status mxl_ctx_create(int device, void *hip_stream, mxl_ctx **out);
mxl_status mxl_ctx_set_stream(mxl_ctx *ctx, void *hip_stream);
mxl_status mxl_ctx_destroy(mxl_ctx *ctx);
const char *mxl_last_error(void);
/* Library version string, static storage. */
const char *mxl_version(void);

/* ---------------------------------------------------------------- matrices */

enum { MXL_BORROW = 0, MXL_COPY = 1, MXL_VALIDATE = 2 };

/* Wrap a CSR matrix (Sec. 2.2.4) as an operator.  row_ptr (nrows+1), col
 * (nnz) and val (nnz, dtype) are device arrays.  flags: MXL_BORROW keeps
 * views of the caller's arrays, which must stay alive and unchanged until
 * the handle and everything derived from it are destroyed (the Array views
 * of Sec. 2.4); MXL_COPY makes library-owned copies.  MXL_VALIDATE (or-ed
 * in) checks canonical form on the device and fails with INVALID_MATRIX;
 * mxl_last_error() then gives the mask of violated rules (1 row_ptr[0] != 0,
 * 2 row_ptr decreases, 4 row_ptr[nrows] != nnz, 8 a column outside
 * [0, ncols), 16 columns of a row not strictly increasing) and names the
 * first of them in that order.  Errors: INVALID_ARG (null, negative sizes, nnz >= 2^31), DTYPE,
 * INVALID_MATRIX, OUT_OF_MEMORY. */
mxl_status mxl_csr_create(mxl_ctx *ctx, mxl_dtype dtype, int64_t nrows,
                          int64_t ncols, int64_t nnz, const int32_t *row_ptr,
                          const int32_t *col, const void *val, int flags,
                          mxl_op **A);

/* Matrix-free constant-coefficient stencil operator on an nx x ny x nz grid:
 * a user-defined linear operator in the sense of Sec. 4, which stores no
 * matrix.  Unknown r = i + nx (j + ny k); row r of A x is
 *     sum_p coef[p] * x[(i + di_p) + nx ((j + dj_p) + ny (k + dk_p))]
 * over the points p whose neighbour lies inside the grid (Dirichlet
 * boundary: the others are omitted), summed in (dk, dj, di) lexicographic
 * order (the column order of the equivalent CSR matrix).
 * offsets: HOST int32 [npts][3] = (di, dj, dk), each in {-1, 0, 1}, all
 * distinct; coef: HOST double [npts]; 1 <= npts <= 27; dtype F64 or F32
 * (coefficients rounded to it).  The operator supports mxl_apply*,
 * mxl_cast, mxl_jacobi_generate (the point (0,0,0) is the diagonal;
 * ZERO_DIAG if it is absent or zero), the solvers and mxl_time_apply;
 * mxl_convert, mxl_features and mxl_select return NOT_IMPLEMENTED.
 * Errors: INVALID_ARG, DTYPE. */
mxl_status mxl_stencil_create(mxl_ctx *ctx, mxl_dtype dtype, int64_t nx, int64_t ny,
                              int64_t nz, int32_t npts, const int32_t *offsets,
                              const double *coef, mxl_op **A);

/* New operator with the same values in another format or kernel variant
 * (COO: explicit row of each entry, CSR order; ELL: slot-major [w][n_pad]
 * with n_pad = nrows rounded up to 64, padding column -1 / value 0; HYB:
 * ELL part of width k = nearest-rank quantile of row lengths plus a
 * row-sorted COO tail).  The result shares A's arrays by reference counting
 * and adds its own.  Errors: INFEASIBLE_FORMAT when ELL storage exceeds
 * min(4 x CSR bytes, 32 GiB); NOT_IMPLEMENTED; INVALID_ARG. */
mxl_status mxl_convert(const mxl_op *A, mxl_format fmt,
                       const mxl_format_params *params, mxl_op **out);

/* New operator with values rounded to another precision (same format and
 * variant; index arrays shared).  Memory precision decoupled from
 * arithmetic precision, Sec. 3.2. */
mxl_status mxl_cast(const mxl_op *A, mxl_dtype dtype, mxl_op **out);

/* x = L(b) (Sec. 2.2.2).  Matrix: SpMV.  Jacobi: x = D^{-1} b.  Solver:
 * solve with x as the initial guess (blocks; see mxl_solve).
 * Errors: INVALID_ARG (null, b == x), NOT_IMPLEMENTED. */
mxl_status mxl_apply(const mxl_op *L, const void *b, void *x);

/* x = alpha*L(b) + beta*x (Sec. 4.2).  beta == 0: x is not read (BLAS
 * convention, so NaN in x does not propagate).  Matrices and Jacobi only. */
mxl_status mxl_apply_adv(const mxl_op *L, double alpha, const void *b,
                         double beta, void *x);

/* Describe an operator. */
typedef struct {
    int32_t kind, format, variant, dtype;
    int64_t nrows, ncols, nnz;
    int32_t vector_width, ell_width;
    int64_t n_pad, tail_nnz;
    int64_t stored_bytes;  /* bytes of the format's own arrays */
    int32_t ell_reuse;     /* ELL and HYB (not LDS-staged): 1 when the product takes x
                              values from the neighbouring row instead of gathering
                              them, set at conversion when at least a quarter of the
                              entries (i, s) of the ELL slots share their column
                              with (i+1, s-1) */
} mxl_op_desc;
mxl_status mxl_op_describe(const mxl_op *A, mxl_op_desc *out);

/* Copy one of the format's arrays into dst (device memory, dst_bytes
 * capacity) on the context stream, for inspection.  which: 0 row_ptr, 1 col,
 * 2 val, 3 coo_row, 4 ell_col, 5 ell_val, 6 tail_row, 7 tail_col,
 * 8 tail_val, 9 jacobi dinv.  ell_col is int32 [w][n_pad], or int16
 * offsets col - row for MXL_ELL_DELTA16.  Errors: INVALID_ARG if absent,
 * DIM_MISMATCH if dst is too small. */
mxl_status mxl_op_export(const mxl_op *A, int32_t which, void *dst,
                         int64_t dst_bytes);

/* Decrement the reference count; storage owned by the library is released
 * when no handle refers to it any more.  NULL is accepted. */
mxl_status mxl_op_destroy(mxl_op *op);

/* ---------------------------------------------------- preconditioner/solver */

/* Point Jacobi (block-Jacobi with block size 1, Sec. 3.2):
 * dinv_i = 1/a_ii computed in FP64 and rounded to A's precision.
 * Errors: ZERO_DIAG (a missing or zero a_ii), NOT_IMPLEMENTED (non-square). */
mxl_status mxl_jacobi_generate(const mxl_op *A, mxl_op **P);

/* Block-Jacobi preconditioner (Sec. 3.2): the diagonal blocks of A over
 * consecutive ranges of block_size rows (the last range may be shorter) are
 * inverted by Gauss-Jordan elimination with partial pivoting in FP64.  With
 * adaptive != 0 each inverse is stored in the lowest of binary16, binary32,
 * binary64 for which cond_1(D_b) * u <= accuracy (u = 2^-11, 2^-24) and
 * every nonzero entry lies in that format's normal range (memory precision
 * decoupled from the FP64 arithmetic); otherwise binary64.  accuracy 0
 * means 0.1.  mxl_apply computes z = M r in FP64 from the stored entries.
 * It preconditions CG (per-kernel path, FP64 or FP32 vectors), BiCGSTAB
 * (FP64) and GMRES.  block_size in
 * {1, 2, 4, 8, 16, 32}.  Errors: INVALID_ARG, NOT_IMPLEMENTED (non-square,
 * FP32 or matrix-free operator), ZERO_DIAG (a singular diagonal block),
 * OUT_OF_MEMORY, DEVICE. */
mxl_status mxl_bjacobi_generate(const mxl_op *A, int32_t block_size, int32_t adaptive,
                                double accuracy, mxl_op **P);

/* Block-Jacobi with blocks of varying size (Sec. 3.2: the diagonal blocks
 * are inverted by a batched variable-size Gauss-Jordan elimination).
 * Boundaries: with bptr_host (HOST int32[nblocks + 1], 0 = bptr[0] <
 * bptr[1] < ... < bptr[nblocks] = nrows, every block 1 to 32 rows) block b
 * is rows bptr[b] .. bptr[b+1]-1; with bptr_host == NULL (nblocks ignored)
 * the library finds them by supervariable agglomeration: runs of
 * consecutive rows with identical column index sets, each cut into pieces
 * of at most max_block_size (1..32) rows, are packed in row order into
 * blocks of at most max_block_size rows, a piece that does not fit
 * starting the next block (on a matrix whose rows all differ in pattern
 * this gives uniform blocks of max_block_size rows).  Elimination,
 * condition numbers, the adaptive storage rule, the product and the solvers
 * it preconditions are those of mxl_bjacobi_generate.  Errors: INVALID_ARG
 * (boundaries or max_block_size out of range), NOT_IMPLEMENTED, ZERO_DIAG,
 * OUT_OF_MEMORY, DEVICE. */
mxl_status mxl_bjacobi_generate_var(const mxl_op *A, int64_t nblocks, const int32_t *bptr_host,
                                    int32_t max_block_size, int32_t adaptive, double accuracy,
                                    mxl_op **P);

/* Block boundaries of a block-Jacobi operator: HOST int32[nblocks + 1]
 * (nblocks from mxl_bjacobi_info).  Errors: INVALID_ARG. */
mxl_status mxl_bjacobi_blocks(const mxl_op *P, int32_t *bptr_host);

/* Per-block data of a block-Jacobi operator (HOST outputs, each may be
 * NULL): the number of blocks, cond_1 of every diagonal block, its storage
 * precision (0 binary64, 1 binary32, 2 binary16), the stored inverses as
 * FP64 (block after block, each m x m row-major, m the block's rows) and
 * the bytes the inverses occupy.  Blocks until the copies are done. */
mxl_status mxl_bjacobi_info(const mxl_op *P, int64_t *nblocks, double *cond,
                            int32_t *precision, double *inv, int64_t *storage_bytes);

/* ILU-type preconditioner (Sec. 3.2): incomplete LU factors of A on A's
 * own sparsity pattern (L unit lower, U upper; ILU(0) is their fixed point)
 * generated by `sweeps` synchronous ParILU fixed-point sweeps from
 * l_ij = a_ij / a_jj, u_ij = a_ij (each sweep recomputes every entry from
 * the previous sweep's factors: s = a_ij - sum_{k<min(i,j)} l_ik u_kj,
 * l_ij = s / u_jj or u_ij = s).  mxl_apply(P, r, z) computes
 * z = U^{-1} L^{-1} r by two triangular solves: trisolve 0 exact
 * substitution (level-scheduled: one launch per dependency level of each
 * triangle), 1 iterative, trs_sweeps Jacobi sweeps per triangle from
 * y = r and z = y / u_ii.  P preconditions GMRES.  A FP64, square, stored
 * (not matrix-free); P keeps a reference to A.  Errors: INVALID_ARG
 * (sweeps or trs_sweeps < 0, trisolve not 0/1, empty A), NOT_IMPLEMENTED,
 * ZERO_DIAG (a missing or zero diagonal entry), OUT_OF_MEMORY, DEVICE. */
mxl_status mxl_ilu_generate(const mxl_op *A, int32_t sweeps, int32_t trisolve,
                            int32_t trs_sweeps, mxl_op **P);

/* HOST copies (each may be NULL): the factors in A's CSR order (nnz
 * doubles) and the number of dependency levels of L and of U (levels[2]). */
mxl_status mxl_ilu_info(const mxl_op *P, double *lu, int32_t *levels);

/* Solver factory .generate(A) (Sec. 2.2.3, Sec. 3.1): Krylov solver bound to
 * A with optional preconditioner P (NULL = none).  The solver keeps shared
 * references to A and P and owns its work vectors.  MXL_SOLVER_GMRES is
 * GMRES(100), the restart the paper's solver study uses (Sec. 7.4). */
mxl_status mxl_solver_generate(mxl_solver_kind kind, const mxl_op *A,
                               const mxl_op *P, const mxl_criteria *crit,
                               mxl_op **S);

/* Restarted GMRES(krylov_dim) (Sec. 3.1; memory model and restart of
 * Table 2), preconditioned from the right by P (point or block Jacobi, or
 * NULL): x = x0 + M^{-1} V y minimises ||b - A x|| over the cycle's Krylov
 * space, so the criterion is checked on the residual of A x = b itself
 * (the Givens estimate inside a cycle, the recomputed b - A x at each
 * restart).  P may also be an ILU operator.  One iteration = one Arnoldi
 * step (one product with A);
 * info->restarts counts restarted cycles, info->spmv_count = 1 + iterations
 * + restarts (+ 1 when the criterion stops a cycle early: the product of
 * the step that finalises the converged column).  The basis is
 * orthogonalised twice by classical Gram-Schmidt, the second pass of each
 * vector delayed into the next step so that every step reads the basis
 * twice (info->reorth counts the vectors).  Memory: (krylov_dim + 1) basis
 * vectors of n doubles plus O(krylov_dim^2).  A FP64, krylov_dim in
 * [1, 1024].  Errors: INVALID_ARG, NOT_IMPLEMENTED (FP32 operator, non-Jacobi
 * P), DTYPE / DIM_MISMATCH (P does not conform), OUT_OF_MEMORY. */
mxl_status mxl_gmres_generate(const mxl_op *A, const mxl_op *P,
                              const mxl_criteria *crit, int32_t krylov_dim,
                              mxl_op **S);

/* Solve A x = b; x holds the initial guess on entry and the solution on exit
 * (Sec. 2.1).  Blocks until a criterion stops the iteration.  Not reaching
 * the tolerance is not an error: the status is OK and info->stop_reason
 * tells which criterion stopped it.  info may be NULL. */
mxl_status mxl_solve(const mxl_op *S, const void *b, void *x,
                     mxl_solve_info *info);

/* Mixed-precision iterative refinement (the IR solver with a configurable
 * inner solver of Sec. 2.2.3 and Sec. 3.1, the inner solve in FP32 storage
 * per the precision decoupling of Sec. 3.2).  A must be FP64.  The
 * generated operator holds an FP32 copy of A's values, FP32 Jacobi
 * (dinv rounded from the FP64 reciprocal) and an FP32 Jacobi-CG.  mxl_solve
 * on it repeats: r = b - A x (FP64, on the device); stop if
 * ||r||/||b|| <= outer.reduction (or outer.max_iters corrections applied, or
 * outer.time_limit_s); s = ||r||_inf; solve A32 d = fp32(r/s) from d = 0 to
 * inner.reduction / inner.max_iters; x += s*d (FP64).  info->iterations
 * counts corrections, info->inner_iterations all inner CG iterations,
 * info->history the outer relative residuals.  inner_block_size > 0 (1, 2,
 * 4, 8, 16 or 32) replaces the inner point Jacobi with block Jacobi over
 * uniform blocks of that many rows, generated from the FP64 matrix with the
 * adaptive storage rule at inner_block_accuracy (as mxl_bjacobi_generate
 * with adaptive = 1): the inverses are applied in FP64 and z = M r is
 * rounded to FP32, so the inner solve decouples three precisions
 * (binary16/32/64 inverses, FP32 vectors, FP64 arithmetic).  0 keeps point
 * Jacobi; a zero-initialised tail of this struct is therefore the point
 * Jacobi solver.  inner_block_mode 1 takes variable-size blocks found by
 * supervariable agglomeration with at most inner_block_size rows (as
 * mxl_bjacobi_generate_var with bptr_host == NULL; any size 1..32); 0 the
 * uniform blocks.  Errors: DTYPE (A not FP64), INVALID_ARG (block size or
 * mode not supported), ZERO_DIAG (a singular diagonal block, or a zero
 * diagonal entry for point Jacobi), OUT_OF_MEMORY. */
typedef struct {
    mxl_criteria outer;
    mxl_criteria inner;
    int32_t inner_block_size;
    double inner_block_accuracy;
    int32_t inner_block_mode;
} mxl_ir_params;
mxl_status mxl_ir_generate(const mxl_op *A, const mxl_ir_params *params, mxl_op **S);

/* ----------------------------------------------------------------- batched */

/* nsys independent systems packed in one CSR: system s owns rows
 * sys_ptr[s]..sys_ptr[s+1]-1; row_ptr holds global nonzero offsets; column
 * indices are local to the system.  All arrays are device arrays, FP64
 * values.  flags as in mxl_csr_create. */
mxl_status mxl_batch_csr_create(mxl_ctx *ctx, int64_t nsys,
                                const int32_t *sys_ptr_host,
                                const int32_t *sys_ptr, const int32_t *row_ptr,
                                const int32_t *col, const double *val,
                                int flags, mxl_op **B);

/* Schedule of the persistent batched kernel.  wg_size in {64,128,256,512,
 * 1024}; wgs_per_cu >= 1 resident workgroups per compute unit; order 0 =
 * systems in input order, 1 = largest first; format 0 = the per-system ELL
 * copy when the batch has one, else CSR, 1 = CSR, 2 = ELL (NOT_IMPLEMENTED
 * when the batch has no ELL copy).  mxl_batch_csr_create builds the ELL
 * copy (slot-major per system, int16 local columns) when every system has
 * at most 32767 rows and the padded slots total at most 1.5 x the stored
 * entries (+ 64 per system); the ELL kernel keeps a system's vectors and,
 * when they fit, its matrix in LDS for all of its iterations. */
typedef struct { int32_t wg_size; int32_t wgs_per_cu; int32_t order; int32_t format; } mxl_tuning;

/* Jacobi-PCG on every system independently (per-system stopping status,
 * Sec. 2.5), all in one persistent launch.  crit->max_iters <= 0 means
 * 10*n_s per system.  tuning NULL = the autotuned schedule (cached per
 * handle).  b, x: device FP64 of total rows; iters, rel_res, status: device
 * arrays of nsys entries. */
mxl_status mxl_batch_solve(const mxl_op *B, const mxl_criteria *crit,
                           const mxl_tuning *tuning, const double *b,
                           double *x, int32_t *iters, double *rel_res,
                           uint8_t *status);

/* Autotune the batched schedule: times each candidate (reps launches each)
 * and stores the best on the handle; best may be NULL. */
mxl_status mxl_batch_autotune(const mxl_op *B, const mxl_criteria *crit,
                              const double *b, double *x_scratch, int reps,
                              mxl_tuning *best, double *best_ms);

/* mxl_batch_solve for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same kernels, schedule rules and results, but the work counter and the
 * spill region of systems too large for LDS live in a fixed 96 MiB device
 * array that the library holds on each GPU until the process ends, and the
 * call neither allocates nor synchronises: the solve is enqueued on the
 * context's stream and its outputs are ready when that stream reaches it.
 * Arguments, layout and ownership as for mxl_batch_solve; tuning NULL takes
 * the handle's autotuned schedule if mxl_batch_autotune has run, else the
 * default one (no tuning happens here).  INVALID_ARG when the schedule's
 * spill region (wgs_per_cu * CUs * 5 * the largest system's rows doubles,
 * 0 when every system fits in LDS) plus 256 bytes exceeds 96 MiB; DEVICE
 * when the array's address could not be looked up at mxl_ctx_create.  All
 * calls on one GPU share the array: calls whose solves overlap on the device
 * (other streams, other contexts or threads) race and give wrong results. */
mxl_status mxl_batch_solve_noalloc(const mxl_op *B, const mxl_criteria *crit,
                                   const mxl_tuning *tuning, const double *b,
                                   double *x, int32_t *iters, double *rel_res,
                                   uint8_t *status);

/* ---------------------------------------------------------------- selector */

/* The 16 structural features of a CSR matrix (host output, FP64):
 * log10 n, log10 nnz, mean/std/cv/max/min/median/p90/p99 row length,
 * fraction of rows longer than twice the mean, ELL fill n*max/nnz,
 * max and mean |i-j|/n, fraction of entries with |i-j| <= 64, skewness. */
mxl_status mxl_features(const mxl_op *A, double out_host[16]);

/* Median time in milliseconds of reps applications y = A x (HIP events on
 * the context stream), after one untimed application (the first launch of a
 * kernel also loads its code).  flush != 0 reads a 1 GiB buffer (allocated on first
 * use and kept by the context) before every rep to evict the 256 MB
 * last-level cache without leaving dirty lines; its time is excluded. */
mxl_status mxl_time_apply(const mxl_op *A, const void *x, void *y, int reps,
                          int flush, double *median_ms);

/* Bandwidth reference kernels, the STREAM-style operations the paper uses
 * to calibrate solver bandwidth (Sec. 7.4, Table 3): op 0 copy c = a,
 * op 1 triad c = a + 0.5*b, op 2 dot a.b (partials written to c, which
 * then needs 8*8*num_CU bytes), all with nontemporal loads; op 3 the sum
 * of a with ordinary loads (b unused, partials in c as for op 2), sweeping
 * the array ceil(2^28 / n) times in one launch (once when n >= 2^28; it
 * reads 8 n bytes per sweep): ordinary loads are cached, so over an array
 * that fits L2 or the last-level cache the launch measures that cache's
 * read bandwidth.  FP64, n even.
 * median_ms: median of reps launches timed with HIP events on the context
 * stream. */
mxl_status mxl_stream_bench(mxl_ctx *ctx, int op, int64_t n, const double *a,
                            const double *b, double *c, int reps,
                            double *median_ms);

/* Small FP32 multilayer perceptron dims[0] -> ... -> dims[nlayers] with
 * ReLU between layers (weights live on the device).  theta_host packs
 * W_l (row-major, dims[l+1] x dims[l]) then b_l for each layer. */
typedef struct mxl_mlp mxl_mlp;
mxl_status mxl_mlp_create(mxl_ctx *ctx, int32_t nlayers, const int32_t *dims,
                          const float *theta_host, mxl_mlp **out);
mxl_status mxl_mlp_get_params(const mxl_mlp *m, float *theta_host, int64_t n);
mxl_status mxl_mlp_set_params(mxl_mlp *m, const float *theta_host, int64_t n);
/* Y = f(X): X device FP32 (nsamples x dims[0]) -> Y device (nsamples x dims[L]). */
mxl_status mxl_mlp_forward(const mxl_mlp *m, int64_t nsamples, const float *X,
                           float *Y);
/* loss = sum M (f(X)-T)^2 / sum M + lambda sum ||W||^2; gradient kept on the
 * device (mxl_mlp_get_grad copies it out).  loss_host may be NULL. */
mxl_status mxl_mlp_loss_grad(mxl_mlp *m, int64_t nsamples, const float *X,
                             const float *T, const float *M, float lambda,
                             float *loss_host);
mxl_status mxl_mlp_get_grad(const mxl_mlp *m, float *grad_host, int64_t n);
/* Adam step on the stored gradient (bias-corrected, step t >= 1). */
mxl_status mxl_mlp_adam_step(mxl_mlp *m, int64_t t, float lr, float beta1,
                             float beta2, float eps);
mxl_status mxl_mlp_destroy(mxl_mlp *m);

/* Run-time choice of (format, kernel variant), the fork of Sec. 7.2, learned
 * from timings and scored by time, with performance profiles (Sec. 7.3) as
 * the evaluation.  A selector holds the candidate classes, a trained MLP
 * (16 features -> one score per class, s_c ~ log(t_c / t_best)) and the
 * feature standardisation z_j = (phi_j(f_j) - mean_j) / std_j, where phi_j is
 * log(1 + f) for the features flagged in log_mask (bit j) and the identity
 * otherwise.  All arrays are HOST pointers and are copied. */
typedef struct {
    int32_t format;             /* mxl_format */
    mxl_format_params params;   /* as for mxl_convert */
} mxl_kernel_class;

typedef struct mxl_selector mxl_selector;

/* dims[0] must be 16 and dims[nlayers] = nclasses (1..64).  delta: top-2
 * score margin below which the prediction counts as unsure; zmax: largest
 * |z_j| still inside the training distribution.  Errors: INVALID_ARG,
 * OUT_OF_MEMORY, DEVICE. */
mxl_status mxl_selector_create(mxl_ctx *ctx, int32_t nclasses,
                               const mxl_kernel_class *classes,
                               int32_t nlayers, const int32_t *dims,
                               const float *theta_host, const double *mean16,
                               const double *std16, uint32_t log_mask,
                               double delta, double zmax, mxl_selector **out);
mxl_status mxl_selector_destroy(mxl_selector *s);

enum {
    MXL_SELECT_MODEL = 0,           /* argmin of the predicted scores */
    MXL_SELECT_EXHAUSTIVE = 1,      /* time every feasible class */
    MXL_SELECT_MODEL_FALLBACK = 2   /* model; time the top 3 when unsure */
};

typedef struct {
    double  margin;     /* second-best minus best predicted score (inf if one class) */
    double  max_z;      /* largest |standardised feature| */
    int32_t fallback;   /* 1 if the choice was made by timing */
    int32_t ntimed;     /* classes timed */
    double  best_ms;    /* median time of the chosen class if timed, else 0 */
} mxl_select_info;

/* Choose a class for the CSR matrix A (any matrix operator; its CSR arrays
 * are used).  Classes whose padded storage exceeds the mxl_convert budget
 * are never chosen.  Timing (EXHAUSTIVE, and FALLBACK when unsure) converts
 * each candidate and takes the median of reps applications y = A x with the
 * last-level cache flushed before each (mxl_time_apply), so it needs device
 * vectors x (ncols) and y (nrows, overwritten); with x or y NULL the
 * FALLBACK mode never times and EXHAUSTIVE is INVALID_ARG.  Optional HOST
 * outputs: scores[nclasses] (predicted scores, +inf for infeasible classes;
 * NaN in EXHAUSTIVE mode), times_ms[nclasses] (NaN where not timed), info.
 * Blocks until done.  Errors: INVALID_ARG, DIM_MISMATCH, OUT_OF_MEMORY,
 * DEVICE, or any error of mxl_convert other than INFEASIBLE_FORMAT. */
mxl_status mxl_select(const mxl_selector *s, const mxl_op *A, int32_t mode,
                      const void *x, void *y, int32_t reps, int32_t *class_out,
                      double *scores, double *times_ms, mxl_select_info *info);

#ifdef __cplusplus
}
#endif
#endif /* MXL_H */
