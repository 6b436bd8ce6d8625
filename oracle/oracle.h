/*
 * oracle.h -- plain, slow, obviously-correct CPU reference for the sparse
 * operator hot path (SpMV in CSR/COO/ELL/HYB, point Jacobi, Jacobi-PCG,
 * Jacobi-BiCGSTAB, restarted GMRES, incomplete LU (ILU(0), ParILU,
 * triangular solves), FP32-inner iterative refinement, batched Jacobi-PCG,
 * matrix features and the selector MLP).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or helper with the GPU library; the two agree only through
 * the definitions written out here.
 *
 * Arithmetic: IEEE double, sequential loops in natural index order, built
 * with -ffp-contract=off so no fused multiply-add changes a rounding.  The
 * FP32 inner solver of iterative refinement is the one place where single
 * precision is part of the method's definition.
 *
 * Index type int32, sizes int64.  All pointers are host memory owned by the
 * caller.  Nothing here allocates memory that outlives a call.
 */
#ifndef MXL_ORACLE_H
#define MXL_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* stop reasons (a stopping_status equivalent, Sec. 2.5) */
enum { ORC_RUNNING = 0, ORC_CONVERGED = 1, ORC_MAX_ITERS = 2, ORC_TIME = 3,
       ORC_BREAKDOWN = 4, ORC_NONFINITE = 5 };

/* CSR canonical-form violations */
enum { ORC_CSR_OK = 0, ORC_CSR_BAD_START = 1, ORC_CSR_NOT_MONOTONE = 2,
       ORC_CSR_BAD_END = 3, ORC_CSR_COL_RANGE = 4, ORC_CSR_COL_ORDER = 5 };

typedef struct {
    int64_t max_iters;     /* Iteration criterion */
    double  reduction;     /* ResidualNormReduction: stop when ||r|| <= reduction*||b|| */
    int32_t nonfinite_check; /* 1: stop with NONFINITE when a scalar is NaN/Inf */
} orc_criteria;

typedef struct {
    int64_t iterations;    /* Krylov iterations (CG: number of q = A p products) */
    int64_t spmv_count;
    double  rel_residual;  /* recurrence residual / ||b|| at exit */
    int32_t stop_reason;
    int64_t inner_iterations; /* IR: total inner iterations */
} orc_info;

int  orc_csr_check(int64_t nrows, int64_t ncols, int64_t nnz,
                   const int32_t *row_ptr, const int32_t *col);

void orc_csr_spmv(int64_t nrows, const int32_t *row_ptr, const int32_t *col,
                  const double *val, double alpha, const double *x,
                  double beta, double *y);

void orc_csr_to_coo(int64_t nrows, const int32_t *row_ptr, int32_t *row_out);
void orc_coo_spmv(int64_t nrows, int64_t nnz, const int32_t *row,
                  const int32_t *col, const double *val, double alpha,
                  const double *x, double beta, double *y);

int32_t orc_max_row_len(int64_t nrows, const int32_t *row_ptr);
void orc_csr_to_ell(int64_t nrows, const int32_t *row_ptr, const int32_t *col,
                    const double *val, int32_t width, int64_t n_pad,
                    int32_t *ell_col, double *ell_val);
void orc_ell_spmv(int64_t nrows, int64_t n_pad, int32_t width,
                  const int32_t *ell_col, const double *ell_val, double alpha,
                  const double *x, double beta, double *y);

int32_t orc_hyb_width(int64_t nrows, const int32_t *row_ptr, double q);
int64_t orc_hyb_tail_count(int64_t nrows, const int32_t *row_ptr, int32_t k);
void orc_csr_to_hyb(int64_t nrows, const int32_t *row_ptr, const int32_t *col,
                    const double *val, int32_t k, int64_t n_pad,
                    int32_t *ell_col, double *ell_val, int32_t *tail_row,
                    int32_t *tail_col, double *tail_val);
void orc_hyb_spmv(int64_t nrows, int64_t n_pad, int32_t k,
                  const int32_t *ell_col, const double *ell_val, int64_t ntail,
                  const int32_t *tail_row, const int32_t *tail_col,
                  const double *tail_val, double alpha, const double *x,
                  double beta, double *y);

int64_t orc_jacobi_dinv(int64_t n, const int32_t *row_ptr, const int32_t *col,
                        const double *val, double *dinv);

int orc_pcg(int64_t n, const int32_t *row_ptr, const int32_t *col,
            const double *val, const double *dinv, const double *b, double *x,
            orc_criteria crit, orc_info *info, double *history);

int orc_bicgstab_block(int64_t n, const int32_t *row_ptr, const int32_t *col, const double *val,
                       int64_t nblocks, const int32_t *bptr, const double *inv, const double *b, double *x,
                       orc_criteria crit, orc_info *info, double *history);
int orc_bicgstab(int64_t n, const int32_t *row_ptr, const int32_t *col,
                 const double *val, const double *dinv, const double *b,
                 double *x, orc_criteria crit, orc_info *info, double *history);

/* Restarted right-preconditioned GMRES(krylov_dim), modified Gram-Schmidt
 * Arnoldi with Givens rotations; dinv == NULL means no preconditioner. */
int orc_gmres(int64_t n, const int32_t *row_ptr, const int32_t *col, const double *val,
              const double *dinv, const double *b, double *x, int32_t krylov_dim,
              orc_criteria crit, orc_info *info, double *history);
int orc_gmres_block(int64_t n, const int32_t *row_ptr, const int32_t *col, const double *val,
                    int64_t nblocks, const int32_t *bptr, const double *inv, const double *b,
                    double *x, int32_t krylov_dim, orc_criteria crit, orc_info *info,
                    double *history);

int orc_pcg_f32(int64_t n, const int32_t *row_ptr, const int32_t *col,
                const float *val, const float *dinv, const float *b, float *x,
                orc_criteria crit, orc_info *info);

int orc_pcg_f32_block(int64_t n, const int32_t *row_ptr, const int32_t *col, const float *val,
                      int64_t nblocks, const int32_t *bptr, const double *inv, const float *b, float *x,
                      orc_criteria crit, orc_info *info);
int orc_ir_block_var(int64_t n, const int32_t *row_ptr, const int32_t *col,
                     const double *val, const double *b, double *x,
                     int64_t max_outer, double outer_reduction,
                     int64_t inner_max_iters, double inner_reduction, int64_t nblocks, const int32_t *bptr,
                     double accuracy, orc_info *info, double *outer_history);
int orc_ir_block(int64_t n, const int32_t *row_ptr, const int32_t *col,
                 const double *val, const double *b, double *x,
                 int64_t max_outer, double outer_reduction,
                 int64_t inner_max_iters, double inner_reduction, int32_t block_size, double accuracy,
                 orc_info *info, double *outer_history);
int orc_ir(int64_t n, const int32_t *row_ptr, const int32_t *col,
           const double *val, const double *b, double *x,
           int64_t max_outer, double outer_reduction,
           int64_t inner_max_iters, double inner_reduction,
           orc_info *info, double *outer_history);

void orc_batch_pcg(int64_t nsys, const int32_t *sys_ptr, const int32_t *row_ptr,
                   const int32_t *col, const double *val, const double *b,
                   double *x, double reduction, int64_t iter_factor,
                   int32_t *iters, double *rel_res, uint8_t *status);

void orc_features(int64_t nrows, int64_t ncols, const int32_t *row_ptr,
                  const int32_t *col, double out[16]);

double orc_mlp_loss_grad(int32_t nlayers, const int32_t *dims,
                         const double *theta, int64_t nsamples,
                         const double *X, const double *Y, const double *M,
                         double lambda, double *grad, double *pred);
void orc_adam_step(int64_t nparams, double *theta, const double *grad,
                   double *m, double *v, int64_t t, double lr, double beta1,
                   double beta2, double eps);

/* Block-Jacobi (Sec. 3.2), adaptive storage precision: see oracle.c. */
enum { ORC_P64 = 0, ORC_P32 = 1, ORC_P16 = 2 };
double  orc_round_f16(double x);
int     orc_bj_choose_precision(int m, const double *inv, double cond, double accuracy);
int64_t orc_bj_supervariable_blocks(int64_t n, const int32_t *row_ptr, const int32_t *col, int max_bs,
                                    int32_t *bptr);
int64_t orc_bj_generate(int64_t n, const int32_t *row_ptr, const int32_t *col, const double *val,
                        int64_t nblocks, const int32_t *bptr, int adaptive, double accuracy,
                        double *inv, double *cond, int32_t *prec);
void    orc_bj_apply(int64_t nblocks, const int32_t *bptr, const double *inv, const double *r,
                     double *z);
int     orc_pcg_block(int64_t n, const int32_t *row_ptr, const int32_t *col, const double *val,
                      int64_t nblocks, const int32_t *bptr, const double *inv, const double *b,
                      double *x, orc_criteria crit, orc_info *info, double *history);

/* Incomplete LU on A's pattern (strict lower = L with unit diagonal, the
 * rest = U): exact ILU(0), ParILU synchronous sweeps, the two triangular
 * solves (mode 0 exact, 1 Jacobi sweeps) and right-preconditioned GMRES
 * with it. */
int64_t orc_ilu0(int64_t n, const int32_t *row_ptr, const int32_t *col, const double *val, double *lu);
int64_t orc_parilu(int64_t n, const int32_t *row_ptr, const int32_t *col, const double *val,
                   int32_t sweeps, double *lu);
void orc_ilu_apply(int64_t n, const int32_t *row_ptr, const int32_t *col, const double *lu,
                   int32_t mode, int32_t sweeps, const double *r, double *z);
int orc_gmres_ilu(int64_t n, const int32_t *row_ptr, const int32_t *col, const double *val,
                  const double *lu, int32_t trs_mode, int32_t trs_sweeps, const double *b,
                  double *x, int32_t krylov_dim, orc_criteria crit, orc_info *info, double *history);

#ifdef __cplusplus
}
#endif
#endif
