/*
 * oracle.c -- plain FP64 CPU reference (TEST INFRASTRUCTURE ONLY; see
 * oracle.h).  Single-threaded, sequential, natural-order loops, compiled
 * with -ffp-contract=off.  Every routine cites the passage of the paper it
 * follows; where the paper only names a method (CG, BiCGSTAB, Jacobi,
 * iterative refinement) the textbook definition of the method the paper
 * cites (Saad's book, cited for CSR in Sec. 2.2.4) is written out step by
 * step in the paper's operator notation.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ CSR */

/* Canonical CSR (Sec. 2.2.4 stores system matrices in CSR): row_ptr starts at
 * 0, never decreases, ends at nnz; every column index lies in [0, ncols) and
 * the indices of one row strictly increase (sorted, no duplicates). */
int orc_csr_check(int64_t nrows, int64_t ncols, int64_t nnz,
                  const int32_t *row_ptr, const int32_t *col)
{
    if (row_ptr[0] != 0) return ORC_CSR_BAD_START;
    for (int64_t i = 0; i < nrows; ++i)
        if (row_ptr[i + 1] < row_ptr[i]) return ORC_CSR_NOT_MONOTONE;
    if ((int64_t)row_ptr[nrows] != nnz) return ORC_CSR_BAD_END;
    for (int64_t i = 0; i < nrows; ++i) {
        for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) {
            if (col[k] < 0 || (int64_t)col[k] >= ncols) return ORC_CSR_COL_RANGE;
            if (k > row_ptr[i] && col[k] <= col[k - 1]) return ORC_CSR_COL_ORDER;
        }
    }
    return ORC_CSR_OK;
}

/* Advanced apply y = alpha*A*x + beta*y (Sec. 4.2; the simple apply of
 * Sec. 2.2.2 is alpha = 1, beta = 0).  beta == 0 means y is not read. */
void orc_csr_spmv(int64_t nrows, const int32_t *row_ptr, const int32_t *col,
                  const double *val, double alpha, const double *x,
                  double beta, double *y)
{
    for (int64_t i = 0; i < nrows; ++i) {
        double s = 0.0;
        for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k)
            s += val[k] * x[col[k]];
        y[i] = (beta == 0.0) ? alpha * s : alpha * s + beta * y[i];
    }
}

/* ------------------------------------------------------------------ COO */

/* COO (the format of the solver-bandwidth study, Sec. 7.4): triplets in CSR
 * order, the row of each entry written out explicitly. */
void orc_csr_to_coo(int64_t nrows, const int32_t *row_ptr, int32_t *row_out)
{
    for (int64_t i = 0; i < nrows; ++i)
        for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k)
            row_out[k] = (int32_t)i;
}

/* y = alpha*A*x + beta*y from row-sorted triplets; each row's entries are
 * summed in storage order, rows without entries get alpha*0 + beta*y. */
void orc_coo_spmv(int64_t nrows, int64_t nnz, const int32_t *row,
                  const int32_t *col, const double *val, double alpha,
                  const double *x, double beta, double *y)
{
    double *s = (double *)calloc((size_t)(nrows > 0 ? nrows : 1), sizeof(double));
    for (int64_t k = 0; k < nnz; ++k)
        s[row[k]] += val[k] * x[col[k]];
    for (int64_t i = 0; i < nrows; ++i)
        y[i] = (beta == 0.0) ? alpha * s[i] : alpha * s[i] + beta * y[i];
    free(s);
}

/* ------------------------------------------------------------------ ELL */

int32_t orc_max_row_len(int64_t nrows, const int32_t *row_ptr)
{
    int32_t w = 0;
    for (int64_t i = 0; i < nrows; ++i) {
        int32_t len = row_ptr[i + 1] - row_ptr[i];
        if (len > w) w = len;
    }
    return w;
}

/* ELL: width w slots per row, stored slot-major: slot s of row i sits at
 * s*n_pad + i.  Row i's entries fill its first len_i slots in column order;
 * unused slots hold the sentinel column -1 and value 0 and are skipped by the
 * product (so a NaN/Inf in x never meets a padding zero). */
void orc_csr_to_ell(int64_t nrows, const int32_t *row_ptr, const int32_t *col,
                    const double *val, int32_t width, int64_t n_pad,
                    int32_t *ell_col, double *ell_val)
{
    for (int64_t s = 0; s < width; ++s)
        for (int64_t i = 0; i < n_pad; ++i) {
            ell_col[s * n_pad + i] = -1;
            ell_val[s * n_pad + i] = 0.0;
        }
    for (int64_t i = 0; i < nrows; ++i)
        for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) {
            int64_t s = k - row_ptr[i];
            ell_col[s * n_pad + i] = col[k];
            ell_val[s * n_pad + i] = val[k];
        }
}

void orc_ell_spmv(int64_t nrows, int64_t n_pad, int32_t width,
                  const int32_t *ell_col, const double *ell_val, double alpha,
                  const double *x, double beta, double *y)
{
    for (int64_t i = 0; i < nrows; ++i) {
        double s = 0.0;
        for (int64_t j = 0; j < width; ++j) {
            int32_t c = ell_col[j * n_pad + i];
            if (c >= 0) s += ell_val[j * n_pad + i] * x[c];
        }
        y[i] = (beta == 0.0) ? alpha * s : alpha * s + beta * y[i];
    }
}

/* ------------------------------------------------------------------ HYB */

static int cmp_i32(const void *a, const void *b)
{
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

/* Hybrid split width k = nearest-rank q-quantile of the row lengths:
 * sorted length at 1-based rank ceil(q*n) (q in (0,1]). */
int32_t orc_hyb_width(int64_t nrows, const int32_t *row_ptr, double q)
{
    if (nrows == 0) return 0;
    int32_t *len = (int32_t *)malloc((size_t)nrows * sizeof(int32_t));
    for (int64_t i = 0; i < nrows; ++i) len[i] = row_ptr[i + 1] - row_ptr[i];
    qsort(len, (size_t)nrows, sizeof(int32_t), cmp_i32);
    int64_t rank = (int64_t)ceil(q * (double)nrows);
    if (rank < 1) rank = 1;
    if (rank > nrows) rank = nrows;
    int32_t k = len[rank - 1];
    free(len);
    return k;
}

int64_t orc_hyb_tail_count(int64_t nrows, const int32_t *row_ptr, int32_t k)
{
    int64_t t = 0;
    for (int64_t i = 0; i < nrows; ++i) {
        int64_t len = row_ptr[i + 1] - row_ptr[i];
        if (len > k) t += len - k;
    }
    return t;
}

/* HYB = ELL part holding each row's first min(len, k) entries + a row-sorted
 * COO tail holding the rest, in CSR order. */
void orc_csr_to_hyb(int64_t nrows, const int32_t *row_ptr, const int32_t *col,
                    const double *val, int32_t k, int64_t n_pad,
                    int32_t *ell_col, double *ell_val, int32_t *tail_row,
                    int32_t *tail_col, double *tail_val)
{
    for (int64_t s = 0; s < k; ++s)
        for (int64_t i = 0; i < n_pad; ++i) {
            ell_col[s * n_pad + i] = -1;
            ell_val[s * n_pad + i] = 0.0;
        }
    int64_t t = 0;
    for (int64_t i = 0; i < nrows; ++i)
        for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
            int64_t s = e - row_ptr[i];
            if (s < k) {
                ell_col[s * n_pad + i] = col[e];
                ell_val[s * n_pad + i] = val[e];
            } else {
                tail_row[t] = (int32_t)i;
                tail_col[t] = col[e];
                tail_val[t] = val[e];
                ++t;
            }
        }
}

/* Each row: ELL slots in order, then its tail entries in order. */
void orc_hyb_spmv(int64_t nrows, int64_t n_pad, int32_t k,
                  const int32_t *ell_col, const double *ell_val, int64_t ntail,
                  const int32_t *tail_row, const int32_t *tail_col,
                  const double *tail_val, double alpha, const double *x,
                  double beta, double *y)
{
    double *s = (double *)calloc((size_t)(nrows > 0 ? nrows : 1), sizeof(double));
    for (int64_t i = 0; i < nrows; ++i)
        for (int64_t j = 0; j < k; ++j) {
            int32_t c = ell_col[j * n_pad + i];
            if (c >= 0) s[i] += ell_val[j * n_pad + i] * x[c];
        }
    for (int64_t t = 0; t < ntail; ++t)
        s[tail_row[t]] += tail_val[t] * x[tail_col[t]];
    for (int64_t i = 0; i < nrows; ++i)
        y[i] = (beta == 0.0) ? alpha * s[i] : alpha * s[i] + beta * y[i];
    free(s);
}

/* --------------------------------------------------------------- Jacobi */

/* Point Jacobi (block-Jacobi with block size 1, Sec. 3.2):
 * dinv_i = 1 / a_ii.  Returns -1 on success, else the first row whose
 * diagonal entry is missing or zero. */
int64_t orc_jacobi_dinv(int64_t n, const int32_t *row_ptr, const int32_t *col,
                        const double *val, double *dinv)
{
    for (int64_t i = 0; i < n; ++i) {
        double d = 0.0;
        int found = 0;
        for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k)
            if (col[k] == i) { d = val[k]; found = 1; }
        if (!found || d == 0.0) return i;
        dinv[i] = 1.0 / d;
    }
    return -1;
}

/* ---------------------------------------------------------- vector ops */

static double dot(int64_t n, const double *a, const double *b)
{
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) s += a[i] * b[i];
    return s;
}

static double nrm2(int64_t n, const double *a) { return sqrt(dot(n, a, a)); }

static void prec(int64_t n, const double *dinv, const double *in, double *out)
{
    for (int64_t i = 0; i < n; ++i) out[i] = dinv ? dinv[i] * in[i] : in[i];
}

/* A preconditioner z = M^{-1} r: point Jacobi (dinv, or none), block
 * Jacobi (bptr/inv) or incomplete LU (lu on the pattern rp/col, applied by
 * two triangular solves, exact or trs_sweeps Jacobi sweeps). */
typedef struct {
    const double *dinv;
    int64_t nblocks;
    const int32_t *bptr;
    const double *inv;
    const int32_t *rp, *col;
    const double *lu;
    int32_t trs_mode, trs_sweeps;
} orc_prec;

static void orc_bj_apply_impl(int64_t nb, const int32_t *bptr, const double *inv,
                              const double *r, double *z);
void orc_ilu_apply(int64_t n, const int32_t *row_ptr, const int32_t *col, const double *lu,
                   int32_t mode, int32_t sweeps, const double *r, double *z);

static void apply_prec(int64_t n, const orc_prec *M, const double *in, double *out)
{
    if (M->lu) orc_ilu_apply(n, M->rp, M->col, M->lu, M->trs_mode, M->trs_sweeps, in, out);
    else if (M->bptr) orc_bj_apply_impl(M->nblocks, M->bptr, M->inv, in, out);
    else prec(n, M->dinv, in, out);
}

static int nonfinite(double v) { return !isfinite(v); }

/* ------------------------------------------------------------------- CG */

/* Jacobi-preconditioned CG (CG of Sec. 3.1 with the Jacobi preconditioner of
 * Sec. 3.2, as configured in the introductory example of Sec. 2.1).
 * Criteria (Sec. 2.5): Iteration (max_iters) OR ResidualNormReduction
 * (||r_k|| <= reduction*||b||, the recurrence residual), first one met wins.
 *
 *   r = b - A x ; z = M^{-1} r ; p = z ; rho = r.z
 *   repeat: q = A p ; eta = p.q ; alpha = rho/eta ; x += alpha p ;
 *           r -= alpha q ; stop if ||r|| small ; z = M^{-1} r ;
 *           rho' = r.z ; p = z + (rho'/rho) p ; rho = rho'
 *
 * The iteration count is the number of products q = A p.  eta <= 0 (the
 * operator is not positive definite along p) or rho' == 0 with r != 0 stops
 * with BREAKDOWN.  history[k] (optional, max_iters+1 entries) receives
 * ||r_k||/||b||. */
static int pcg_core(int64_t n, const int32_t *row_ptr, const int32_t *col,
                    const double *val, const orc_prec *M, const double *b, double *x,
                    orc_criteria crit, orc_info *info, double *history);

int orc_pcg(int64_t n, const int32_t *row_ptr, const int32_t *col,
            const double *val, const double *dinv, const double *b, double *x,
            orc_criteria crit, orc_info *info, double *history)
{
    orc_prec M = {dinv, 0, NULL, NULL, NULL, NULL, NULL, 0, 0};
    return pcg_core(n, row_ptr, col, val, &M, b, x, crit, info, history);
}

int orc_pcg_block(int64_t n, const int32_t *row_ptr, const int32_t *col,
                  const double *val, int64_t nblocks, const int32_t *bptr,
                  const double *inv, const double *b, double *x,
                  orc_criteria crit, orc_info *info, double *history)
{
    orc_prec M = {NULL, nblocks, bptr, inv, NULL, NULL, NULL, 0, 0};
    return pcg_core(n, row_ptr, col, val, &M, b, x, crit, info, history);
}

static int pcg_core(int64_t n, const int32_t *row_ptr, const int32_t *col,
                    const double *val, const orc_prec *M, const double *b, double *x,
                    orc_criteria crit, orc_info *info, double *history)
{
    double *r = (double *)malloc((size_t)(n + 1) * sizeof(double));
    double *z = (double *)malloc((size_t)(n + 1) * sizeof(double));
    double *p = (double *)malloc((size_t)(n + 1) * sizeof(double));
    double *q = (double *)malloc((size_t)(n + 1) * sizeof(double));
    memset(info, 0, sizeof(*info));
    double nb = nrm2(n, b);
    int stop = ORC_RUNNING;
    int64_t k = 0;
    double rel = 0.0;
    if (nb == 0.0) {
        for (int64_t i = 0; i < n; ++i) x[i] = 0.0;
        stop = ORC_CONVERGED;
        if (history) history[0] = 0.0;
        goto done;
    }
    for (int64_t i = 0; i < n; ++i) r[i] = b[i];
    orc_csr_spmv(n, row_ptr, col, val, -1.0, x, 1.0, r);
    info->spmv_count = 1;
    double rr = dot(n, r, r);
    rel = sqrt(rr) / nb;
    if (history) history[0] = rel;
    if (sqrt(rr) <= crit.reduction * nb) { stop = ORC_CONVERGED; goto done; }
    apply_prec(n, M, r, z);
    for (int64_t i = 0; i < n; ++i) p[i] = z[i];
    double rho = dot(n, r, z);
    while (k < crit.max_iters) {
        orc_csr_spmv(n, row_ptr, col, val, 1.0, p, 0.0, q);
        info->spmv_count++;
        double eta = dot(n, p, q);
        if (crit.nonfinite_check && nonfinite(eta)) { stop = ORC_NONFINITE; break; }
        if (eta <= 0.0) { stop = ORC_BREAKDOWN; break; }
        double alpha = rho / eta;
        for (int64_t i = 0; i < n; ++i) x[i] += alpha * p[i];
        for (int64_t i = 0; i < n; ++i) r[i] -= alpha * q[i];
        ++k;
        rr = dot(n, r, r);
        rel = sqrt(rr) / nb;
        if (history) history[k] = rel;
        if (crit.nonfinite_check && nonfinite(rr)) { stop = ORC_NONFINITE; break; }
        if (sqrt(rr) <= crit.reduction * nb) { stop = ORC_CONVERGED; break; }
        apply_prec(n, M, r, z);
        double rho_new = dot(n, r, z);
        if (crit.nonfinite_check && nonfinite(rho_new)) { stop = ORC_NONFINITE; break; }
        if (rho_new == 0.0) { stop = ORC_BREAKDOWN; break; }
        double beta = rho_new / rho;
        for (int64_t i = 0; i < n; ++i) p[i] = z[i] + beta * p[i];
        rho = rho_new;
    }
    if (stop == ORC_RUNNING) stop = ORC_MAX_ITERS;
done:
    info->iterations = k;
    info->rel_residual = rel;
    info->stop_reason = stop;
    free(r); free(z); free(p); free(q);
    return stop;
}

/* ------------------------------------------------------------- BiCGSTAB */

/* BiCGSTAB (Sec. 3.1; van der Vorst's method) with right Jacobi
 * preconditioning, same criteria as CG.  One iteration = one pass of the
 * loop (two products with A); the half step exits early with
 * x += alpha*p_hat when ||s|| already meets the criterion.
 *
 *   r = b - A x ; r_hat = r ; rho_old = alpha = omega = 1 ; v = p = 0
 *   repeat: rho = r_hat.r ; beta = (rho/rho_old)(alpha/omega)
 *           p = r + beta (p - omega v) ; p_hat = M^{-1} p ; v = A p_hat
 *           alpha = rho / (r_hat.v) ; s = r - alpha v
 *           [||s|| small: x += alpha p_hat, stop]
 *           s_hat = M^{-1} s ; t = A s_hat ; omega = (t.s)/(t.t)
 *           x += alpha p_hat + omega s_hat ; r = s - omega t
 *           [||r|| small: stop] ; rho_old = rho
 *
 * rho == 0, r_hat.v == 0, t.t == 0 or omega == 0 stops with BREAKDOWN. */
static int bicgstab_core(int64_t n, const int32_t *row_ptr, const int32_t *col, const double *val,
                         const orc_prec *M, const double *b, double *x, orc_criteria crit, orc_info *info,
                         double *history);

int orc_bicgstab(int64_t n, const int32_t *row_ptr, const int32_t *col,
                 const double *val, const double *dinv, const double *b,
                 double *x, orc_criteria crit, orc_info *info, double *history)
{
    orc_prec M = {dinv, 0, NULL, NULL, NULL, NULL, NULL, 0, 0};
    return bicgstab_core(n, row_ptr, col, val, &M, b, x, crit, info, history);
}

/* BiCGSTAB with the block-Jacobi preconditioner: p_hat = blockdiag(inv) p
 * and s_hat = blockdiag(inv) s (right preconditioning, Sec. 3.1 / 3.2). */
int orc_bicgstab_block(int64_t n, const int32_t *row_ptr, const int32_t *col, const double *val,
                       int64_t nblocks, const int32_t *bptr, const double *inv, const double *b, double *x,
                       orc_criteria crit, orc_info *info, double *history)
{
    orc_prec M = {NULL, nblocks, bptr, inv, NULL, NULL, NULL, 0, 0};
    return bicgstab_core(n, row_ptr, col, val, &M, b, x, crit, info, history);
}

static int bicgstab_core(int64_t n, const int32_t *row_ptr, const int32_t *col, const double *val,
                         const orc_prec *M, const double *b, double *x, orc_criteria crit, orc_info *info,
                         double *history)
{
    size_t bytes = (size_t)(n + 1) * sizeof(double);
    double *r = malloc(bytes), *rh = malloc(bytes), *p = calloc(n + 1, sizeof(double));
    double *v = calloc(n + 1, sizeof(double)), *ph = malloc(bytes), *s = malloc(bytes);
    double *sh = malloc(bytes), *t = malloc(bytes);
    memset(info, 0, sizeof(*info));
    int stop = ORC_RUNNING;
    int64_t k = 0;
    double rel = 0.0;
    double nb = nrm2(n, b);
    if (nb == 0.0) {
        for (int64_t i = 0; i < n; ++i) x[i] = 0.0;
        stop = ORC_CONVERGED;
        if (history) history[0] = 0.0;
        goto done;
    }
    for (int64_t i = 0; i < n; ++i) r[i] = b[i];
    orc_csr_spmv(n, row_ptr, col, val, -1.0, x, 1.0, r);
    info->spmv_count = 1;
    for (int64_t i = 0; i < n; ++i) rh[i] = r[i];
    double rn = nrm2(n, r);
    rel = rn / nb;
    if (history) history[0] = rel;
    if (rn <= crit.reduction * nb) { stop = ORC_CONVERGED; goto done; }
    double rho_old = 1.0, alpha = 1.0, omega = 1.0;
    while (k < crit.max_iters) {
        double rho = dot(n, rh, r);
        if (crit.nonfinite_check && nonfinite(rho)) { stop = ORC_NONFINITE; break; }
        if (rho == 0.0) { stop = ORC_BREAKDOWN; break; }
        double beta = (rho / rho_old) * (alpha / omega);
        for (int64_t i = 0; i < n; ++i) p[i] = r[i] + beta * (p[i] - omega * v[i]);
        apply_prec(n, M, p, ph);
        orc_csr_spmv(n, row_ptr, col, val, 1.0, ph, 0.0, v);
        info->spmv_count++;
        double rv = dot(n, rh, v);
        if (crit.nonfinite_check && nonfinite(rv)) { stop = ORC_NONFINITE; break; }
        if (rv == 0.0) { stop = ORC_BREAKDOWN; break; }
        alpha = rho / rv;
        for (int64_t i = 0; i < n; ++i) s[i] = r[i] - alpha * v[i];
        ++k;
        double sn = nrm2(n, s);
        if (sn <= crit.reduction * nb) {
            for (int64_t i = 0; i < n; ++i) x[i] += alpha * ph[i];
            rel = sn / nb;
            if (history) history[k] = rel;
            stop = ORC_CONVERGED;
            break;
        }
        apply_prec(n, M, s, sh);
        orc_csr_spmv(n, row_ptr, col, val, 1.0, sh, 0.0, t);
        info->spmv_count++;
        double tt = dot(n, t, t);
        double ts = dot(n, t, s);
        if (crit.nonfinite_check && (nonfinite(tt) || nonfinite(ts))) { stop = ORC_NONFINITE; break; }
        if (tt == 0.0) { stop = ORC_BREAKDOWN; break; }
        omega = ts / tt;
        for (int64_t i = 0; i < n; ++i) x[i] += alpha * ph[i] + omega * sh[i];
        for (int64_t i = 0; i < n; ++i) r[i] = s[i] - omega * t[i];
        rn = nrm2(n, r);
        rel = rn / nb;
        if (history) history[k] = rel;
        if (crit.nonfinite_check && nonfinite(rn)) { stop = ORC_NONFINITE; break; }
        if (rn <= crit.reduction * nb) { stop = ORC_CONVERGED; break; }
        if (omega == 0.0) { stop = ORC_BREAKDOWN; break; }
        rho_old = rho;
    }
    if (stop == ORC_RUNNING) stop = ORC_MAX_ITERS;
done:
    info->iterations = k;
    info->rel_residual = rel;
    info->stop_reason = stop;
    free(r); free(rh); free(p); free(v); free(ph); free(s); free(sh); free(t);
    return stop;
}

/* --------------------------------------------------------------- GMRES */

/* Restarted GMRES(m) (Sec. 3.1 lists GMRES among the Krylov solvers; the
 * memory-volume model of Table 2 counts one dot and one axpy per basis
 * vector and step, i.e. modified Gram-Schmidt, and a restart parameter),
 * preconditioned from the right (x = x0 + M^{-1} V y, so the minimised
 * residual is the residual of the original system), same criteria as CG.
 *
 *   r = b - A x ; beta = ||r||
 *   cycle: v_0 = r/beta ; g = (beta, 0, ..., 0)
 *     step j = 0, 1, ...: w = A M^{-1} v_j
 *       for i = 0..j: h_ij = w.v_i ; w -= h_ij v_i      (modified G-S)
 *       h_{j+1,j} = ||w||
 *       apply the rotations G_0..G_{j-1} to column j of H, then the
 *       rotation G_j that zeroes h_{j+1,j}; g <- G_j g
 *       |g_{j+1}| is ||b - A x_{j+1}|| ; stop if small (or max_iters)
 *       v_{j+1} = w / h_{j+1,j}    (before the rotation)
 *     y = R^{-1} g (back substitution) ; x += M^{-1} (V y)
 *     restart unless stopped: r = b - A x ; beta = ||r|| ; stop if small.
 *
 * The iteration count is the number of Arnoldi steps (products A M^{-1} v).
 * A zero h_{j+1,j} (happy breakdown) gives g_{j+1} = 0, which meets any
 * reduction.  history[k] receives the residual estimate |g| / ||b|| after
 * step k. */
static int gmres_core(int64_t n, const int32_t *row_ptr, const int32_t *col,
                      const double *val, const orc_prec *M, const double *b, double *x,
                      int32_t m, orc_criteria crit, orc_info *info, double *history)
{
    memset(info, 0, sizeof(*info));
    if (m < 1) m = 1;
    double *V = (double *)malloc((size_t)(m + 1) * (size_t)(n + 1) * sizeof(double));
    double *H = (double *)calloc((size_t)(m + 1) * (size_t)m, sizeof(double)); /* H[i + (m+1) j] */
    double *cs = (double *)malloc((size_t)m * sizeof(double));
    double *sn = (double *)malloc((size_t)m * sizeof(double));
    double *g = (double *)malloc((size_t)(m + 1) * sizeof(double));
    double *y = (double *)malloc((size_t)m * sizeof(double));
    double *r = (double *)malloc((size_t)(n + 1) * sizeof(double));
    double *z = (double *)malloc((size_t)(n + 1) * sizeof(double));
    double *w = (double *)malloc((size_t)(n + 1) * sizeof(double));
#define VV(i) (V + (size_t)(i) * (size_t)(n + 1))
#define HH(i, j) H[(size_t)(i) + (size_t)(m + 1) * (size_t)(j)]
    int stop = ORC_RUNNING;
    int64_t k = 0;
    double rel = 0.0;
    const double nb = nrm2(n, b);
    if (nb == 0.0) {
        for (int64_t i = 0; i < n; ++i) x[i] = 0.0;
        stop = ORC_CONVERGED;
        if (history) history[0] = 0.0;
        goto done;
    }
    for (int64_t i = 0; i < n; ++i) r[i] = b[i];
    orc_csr_spmv(n, row_ptr, col, val, -1.0, x, 1.0, r);
    info->spmv_count = 1;
    double beta = nrm2(n, r);
    rel = beta / nb;
    if (history) history[0] = rel;
    if (crit.nonfinite_check && nonfinite(beta)) { stop = ORC_NONFINITE; goto done; }
    if (beta <= crit.reduction * nb) { stop = ORC_CONVERGED; goto done; }
    for (;;) {
        for (int64_t i = 0; i < n; ++i) VV(0)[i] = r[i] / beta;
        for (int i = 0; i <= m; ++i) g[i] = 0.0;
        g[0] = beta;
        int j = 0;
        while (j < m && k < crit.max_iters) {
            apply_prec(n, M, VV(j), z);
            orc_csr_spmv(n, row_ptr, col, val, 1.0, z, 0.0, w);
            info->spmv_count++;
            for (int i = 0; i <= j; ++i) {
                const double h = dot(n, w, VV(i));
                HH(i, j) = h;
                for (int64_t t = 0; t < n; ++t) w[t] -= h * VV(i)[t];
            }
            const double hn = nrm2(n, w);
            HH(j + 1, j) = hn;
            for (int i = 0; i < j; ++i) {
                const double a = HH(i, j), c = HH(i + 1, j);
                HH(i, j) = cs[i] * a + sn[i] * c;
                HH(i + 1, j) = -sn[i] * a + cs[i] * c;
            }
            const double a = HH(j, j), c = HH(j + 1, j);
            const double d = hypot(a, c);
            cs[j] = d == 0.0 ? 1.0 : a / d;
            sn[j] = d == 0.0 ? 0.0 : c / d;
            HH(j, j) = d;
            HH(j + 1, j) = 0.0;
            g[j + 1] = -sn[j] * g[j];
            g[j] = cs[j] * g[j];
            ++j;
            ++k;
            rel = fabs(g[j]) / nb;
            if (history) history[k] = rel;
            if (crit.nonfinite_check && (nonfinite(rel) || nonfinite(d))) { stop = ORC_NONFINITE; break; }
            if (fabs(g[j]) <= crit.reduction * nb) { stop = ORC_CONVERGED; break; }
            if (hn == 0.0 || d == 0.0) { stop = ORC_BREAKDOWN; break; }
            if (j < m)
                for (int64_t t = 0; t < n; ++t) VV(j)[t] = w[t] / hn;
        }
        if (stop == ORC_NONFINITE) break;
        /* x += M^{-1} V y with R y = g over the j steps of this cycle */
        for (int i = j - 1; i >= 0; --i) {
            double s = g[i];
            for (int l = i + 1; l < j; ++l) s -= HH(i, l) * y[l];
            y[i] = s / HH(i, i);
        }
        for (int64_t t = 0; t < n; ++t) {
            double s = 0.0;
            for (int i = 0; i < j; ++i) s += VV(i)[t] * y[i];
            w[t] = s;
        }
        apply_prec(n, M, w, z);
        for (int64_t t = 0; t < n; ++t) x[t] += z[t];
        if (stop != ORC_RUNNING) break;
        if (k >= crit.max_iters) { stop = ORC_MAX_ITERS; break; }
        for (int64_t i = 0; i < n; ++i) r[i] = b[i];
        orc_csr_spmv(n, row_ptr, col, val, -1.0, x, 1.0, r);
        info->spmv_count++;
        beta = nrm2(n, r);
        rel = beta / nb;
        if (crit.nonfinite_check && nonfinite(beta)) { stop = ORC_NONFINITE; break; }
        if (beta <= crit.reduction * nb) { stop = ORC_CONVERGED; break; }
    }
#undef VV
#undef HH
done:
    info->iterations = k;
    info->rel_residual = rel;
    info->stop_reason = stop;
    free(V); free(H); free(cs); free(sn); free(g); free(y); free(r); free(z); free(w);
    return stop;
}

int orc_gmres(int64_t n, const int32_t *row_ptr, const int32_t *col, const double *val,
              const double *dinv, const double *b, double *x, int32_t krylov_dim,
              orc_criteria crit, orc_info *info, double *history)
{
    orc_prec M = {dinv, 0, NULL, NULL, NULL, NULL, NULL, 0, 0};
    return gmres_core(n, row_ptr, col, val, &M, b, x, krylov_dim, crit, info, history);
}

int orc_gmres_block(int64_t n, const int32_t *row_ptr, const int32_t *col, const double *val,
                    int64_t nblocks, const int32_t *bptr, const double *inv, const double *b,
                    double *x, int32_t krylov_dim, orc_criteria crit, orc_info *info,
                    double *history)
{
    orc_prec M = {NULL, nblocks, bptr, inv, NULL, NULL, NULL, 0, 0};
    return gmres_core(n, row_ptr, col, val, &M, b, x, krylov_dim, crit, info, history);
}

/* ------------------------------------------------------ FP32 inner CG */

/* Jacobi-CG whose matrix values and vectors are stored in FP32 (memory
 * precision decoupled from arithmetic precision, Sec. 3.2):
 *  - SpMV accumulates each row in FP32 in storage order;
 *  - dot products multiply FP32 entries exactly in FP64 and sum in FP64;
 *  - scalars alpha, beta, rho are FP64;
 *  - each vector update is evaluated in FP64 and rounded once to FP32.
 * Criterion: ||r_k|| <= reduction*||b|| or max_iters. */
static void spmv_f32(int64_t n, const int32_t *rp, const int32_t *col,
                     const float *val, const float *x, float *y)
{
    for (int64_t i = 0; i < n; ++i) {
        float s = 0.0f;
        for (int64_t k = rp[i]; k < rp[i + 1]; ++k) {
            float prod = val[k] * x[col[k]];
            s = s + prod;
        }
        y[i] = s;
    }
}

static double dot_f32(int64_t n, const float *a, const float *b)
{
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) s += (double)a[i] * (double)b[i];
    return s;
}

/* z = M r for the FP32 inner solver, evaluated in FP64: point Jacobi
 * (dinv, FP32 entries) or the stored block inverses (bptr/inv), summed over
 * ascending columns; zr32 != 0 rounds z to FP32 (the block variant keeps z
 * as an FP32 vector). */
static void prec_f32(int64_t n, const float *dinv, int64_t nb, const int32_t *bptr, const double *inv,
                     int zr32, const float *r, double *z)
{
    if (bptr) {
        int64_t off = 0;
        for (int64_t b = 0; b < nb; ++b) {
            const int r0 = bptr[b], m = bptr[b + 1] - bptr[b];
            for (int i = 0; i < m; ++i) {
                double s = 0.0;
                for (int j = 0; j < m; ++j) s += inv[off + (int64_t)i * m + j] * (double)r[r0 + j];
                z[r0 + i] = zr32 ? (double)(float)s : s;
            }
            off += (int64_t)m * m;
        }
    } else {
        for (int64_t i = 0; i < n; ++i) z[i] = (double)dinv[i] * (double)r[i];
    }
}

static int pcg_f32_core(int64_t n, const int32_t *row_ptr, const int32_t *col, const float *val,
                        const float *dinv, int64_t nblocks, const int32_t *bptr, const double *inv,
                        const float *b, float *x, orc_criteria crit, orc_info *info);

int orc_pcg_f32(int64_t n, const int32_t *row_ptr, const int32_t *col,
                const float *val, const float *dinv, const float *b, float *x,
                orc_criteria crit, orc_info *info)
{
    return pcg_f32_core(n, row_ptr, col, val, dinv, 0, NULL, NULL, b, x, crit, info);
}

/* The same FP32 CG with the block-Jacobi preconditioner (inverses stored as
 * decided by the adaptive rule, applied in FP64, z rounded to FP32). */
int orc_pcg_f32_block(int64_t n, const int32_t *row_ptr, const int32_t *col, const float *val,
                      int64_t nblocks, const int32_t *bptr, const double *inv, const float *b, float *x,
                      orc_criteria crit, orc_info *info)
{
    return pcg_f32_core(n, row_ptr, col, val, NULL, nblocks, bptr, inv, b, x, crit, info);
}

static int pcg_f32_core(int64_t n, const int32_t *row_ptr, const int32_t *col, const float *val,
                        const float *dinv, int64_t nblocks, const int32_t *bptr, const double *inv,
                        const float *b, float *x, orc_criteria crit, orc_info *info)
{
    size_t bytes = (size_t)(n + 1) * sizeof(float);
    float *r = malloc(bytes), *p = malloc(bytes), *q = malloc(bytes);
    memset(info, 0, sizeof(*info));
    int stop = ORC_RUNNING;
    int64_t k = 0;
    double rel = 0.0;
    double nb = sqrt(dot_f32(n, b, b));
    if (nb == 0.0) {
        for (int64_t i = 0; i < n; ++i) x[i] = 0.0f;
        stop = ORC_CONVERGED;
        goto done;
    }
    spmv_f32(n, row_ptr, col, val, x, q);
    info->spmv_count = 1;
    for (int64_t i = 0; i < n; ++i) r[i] = (float)((double)b[i] - (double)q[i]);
    double rr = dot_f32(n, r, r);
    rel = sqrt(rr) / nb;
    if (sqrt(rr) <= crit.reduction * nb) { stop = ORC_CONVERGED; goto done; }
    double *z = malloc((size_t)(n + 1) * sizeof(double));
    double rho = 0.0;
    prec_f32(n, dinv, nblocks, bptr, inv, bptr != NULL, r, z);
    for (int64_t i = 0; i < n; ++i) {
        p[i] = (float)z[i];
        rho += (double)r[i] * z[i];
    }
    while (k < crit.max_iters) {
        spmv_f32(n, row_ptr, col, val, p, q);
        info->spmv_count++;
        double eta = dot_f32(n, p, q);
        if (crit.nonfinite_check && nonfinite(eta)) { stop = ORC_NONFINITE; break; }
        if (eta <= 0.0) { stop = ORC_BREAKDOWN; break; }
        double alpha = rho / eta;
        for (int64_t i = 0; i < n; ++i) {
            x[i] = (float)((double)x[i] + alpha * (double)p[i]);
            r[i] = (float)((double)r[i] - alpha * (double)q[i]);
        }
        ++k;
        rr = dot_f32(n, r, r);
        rel = sqrt(rr) / nb;
        if (crit.nonfinite_check && nonfinite(rr)) { stop = ORC_NONFINITE; break; }
        if (sqrt(rr) <= crit.reduction * nb) { stop = ORC_CONVERGED; break; }
        prec_f32(n, dinv, nblocks, bptr, inv, bptr != NULL, r, z);
        double rho_new = 0.0;
        for (int64_t i = 0; i < n; ++i) rho_new += (double)r[i] * z[i];
        if (rho_new == 0.0) { stop = ORC_BREAKDOWN; break; }
        double beta = rho_new / rho;
        for (int64_t i = 0; i < n; ++i) p[i] = (float)(z[i] + beta * (double)p[i]);
        rho = rho_new;
    }
    if (stop == ORC_RUNNING) stop = ORC_MAX_ITERS;
    free(z);
done:
    info->iterations = k;
    info->rel_residual = rel;
    info->stop_reason = stop;
    free(r); free(p); free(q);
    return stop;
}

/* --------------------------------------------- iterative refinement */

/* Iterative refinement with an inner Jacobi-CG (the IR solver with a
 * configurable inner solver of Sec. 2.2.3 and Sec. 3.1), the inner solve run
 * in FP32 storage (precision decoupling, Sec. 3.2):
 *
 *   x = x0 ; repeat: r = b - A x (FP64) ; stop if ||r||/||b|| <= outer_red
 *            s = ||r||_inf ; r32 = fp32(r / s)
 *            solve A32 d = r32 by FP32 Jacobi-CG from d = 0 to
 *              ||r_in|| <= inner_red*||r32|| or inner_max_iters
 *            x += s * fp64(d)
 *
 * A32 = fp32(values); dinv32 = fp32(1/a_ii) with the reciprocal taken in
 * FP64.  info->iterations counts outer steps (refinement corrections
 * applied), info->inner_iterations all inner CG iterations. */
static int ir_core(int64_t n, const int32_t *row_ptr, const int32_t *col, const double *val,
                   const double *b, double *x, int64_t max_outer, double outer_reduction,
                   int64_t inner_max_iters, double inner_reduction, int32_t block_size, double accuracy,
                   int64_t nb_given, const int32_t *bptr_given,
                   orc_info *info, double *outer_history);

int orc_ir(int64_t n, const int32_t *row_ptr, const int32_t *col,
           const double *val, const double *b, double *x,
           int64_t max_outer, double outer_reduction,
           int64_t inner_max_iters, double inner_reduction,
           orc_info *info, double *outer_history)
{
    return ir_core(n, row_ptr, col, val, b, x, max_outer, outer_reduction, inner_max_iters, inner_reduction, 0,
                   0.0, 0, NULL, info, outer_history);
}

/* IR whose FP32 inner CG uses block Jacobi: blocks of block_size rows of the
 * FP64 matrix, inverted and stored by the adaptive rule (accuracy), applied
 * in FP64 with z rounded to FP32 (memory precision decoupled from the
 * arithmetic, Sec. 3.2). */
int orc_ir_block(int64_t n, const int32_t *row_ptr, const int32_t *col,
                 const double *val, const double *b, double *x,
                 int64_t max_outer, double outer_reduction,
                 int64_t inner_max_iters, double inner_reduction, int32_t block_size, double accuracy,
                 orc_info *info, double *outer_history)
{
    return ir_core(n, row_ptr, col, val, b, x, max_outer, outer_reduction, inner_max_iters, inner_reduction,
                   block_size, accuracy, 0, NULL, info, outer_history);
}

/* The same with blocks of varying size: the nblocks blocks of bptr. */
int orc_ir_block_var(int64_t n, const int32_t *row_ptr, const int32_t *col,
                     const double *val, const double *b, double *x,
                     int64_t max_outer, double outer_reduction,
                     int64_t inner_max_iters, double inner_reduction, int64_t nblocks, const int32_t *bptr,
                     double accuracy, orc_info *info, double *outer_history)
{
    return ir_core(n, row_ptr, col, val, b, x, max_outer, outer_reduction, inner_max_iters, inner_reduction,
                   1, accuracy, nblocks, bptr, info, outer_history);
}

static int ir_core(int64_t n, const int32_t *row_ptr, const int32_t *col, const double *val,
                   const double *b, double *x, int64_t max_outer, double outer_reduction,
                   int64_t inner_max_iters, double inner_reduction, int32_t block_size, double accuracy,
                   int64_t nb_given, const int32_t *bptr_given, orc_info *info, double *outer_history)
{
    int64_t nnz = row_ptr[n];
    float *v32 = malloc((size_t)(nnz + 1) * sizeof(float));
    float *dinv32 = malloc((size_t)(n + 1) * sizeof(float));
    double *dinv = malloc((size_t)(n + 1) * sizeof(double));
    double *r = malloc((size_t)(n + 1) * sizeof(double));
    float *r32 = malloc((size_t)(n + 1) * sizeof(float));
    float *d32 = malloc((size_t)(n + 1) * sizeof(float));
    memset(info, 0, sizeof(*info));
    int stop = ORC_RUNNING;
    int64_t nblocks = 0;
    int32_t *bptr = NULL;
    double *inv = NULL;
    for (int64_t k = 0; k < nnz; ++k) v32[k] = (float)val[k];
    if (orc_jacobi_dinv(n, row_ptr, col, val, dinv) >= 0) { stop = ORC_BREAKDOWN; goto done; }
    for (int64_t i = 0; i < n; ++i) dinv32[i] = (float)dinv[i];
    if (block_size > 0) {
        nblocks = bptr_given ? nb_given : (n + block_size - 1) / block_size;
        bptr = malloc((size_t)(nblocks + 1) * sizeof(int32_t));
        for (int64_t k = 0; k <= nblocks; ++k)
            bptr[k] = bptr_given ? bptr_given[k] : (int32_t)(k * block_size < n ? k * block_size : n);
        int64_t tot = 0;
        for (int64_t k = 0; k < nblocks; ++k) tot += (int64_t)(bptr[k + 1] - bptr[k]) * (bptr[k + 1] - bptr[k]);
        inv = malloc((size_t)(tot + 1) * sizeof(double));
        double *cond = malloc((size_t)(nblocks + 1) * sizeof(double));
        int32_t *prc = malloc((size_t)(nblocks + 1) * sizeof(int32_t));
        int64_t bad = orc_bj_generate(n, row_ptr, col, val, nblocks, bptr, 1, accuracy, inv, cond, prc);
        free(cond);
        free(prc);
        if (bad >= 0) { stop = ORC_BREAKDOWN; goto done; }
    }
    double nb = nrm2(n, b);
    if (nb == 0.0) {
        for (int64_t i = 0; i < n; ++i) x[i] = 0.0;
        stop = ORC_CONVERGED;
        goto done;
    }
    int64_t outer = 0;
    for (;;) {
        for (int64_t i = 0; i < n; ++i) r[i] = b[i];
        orc_csr_spmv(n, row_ptr, col, val, -1.0, x, 1.0, r);
        info->spmv_count++;
        double rel = nrm2(n, r) / nb;
        info->rel_residual = rel;
        if (outer_history) outer_history[outer] = rel;
        if (rel <= outer_reduction) { stop = ORC_CONVERGED; break; }
        if (nonfinite(rel)) { stop = ORC_NONFINITE; break; }
        if (outer >= max_outer) { stop = ORC_MAX_ITERS; break; }
        double s = 0.0;
        for (int64_t i = 0; i < n; ++i) if (fabs(r[i]) > s) s = fabs(r[i]);
        for (int64_t i = 0; i < n; ++i) { r32[i] = (float)(r[i] / s); d32[i] = 0.0f; }
        orc_criteria ic = { inner_max_iters, inner_reduction, 1 };
        orc_info ii;
        pcg_f32_core(n, row_ptr, col, v32, bptr ? NULL : dinv32, nblocks, bptr, inv, r32, d32, ic, &ii);
        info->inner_iterations += ii.iterations;
        info->spmv_count += ii.spmv_count;
        for (int64_t i = 0; i < n; ++i) x[i] += s * (double)d32[i];
        ++outer;
    }
    info->iterations = outer;
done:
    info->stop_reason = stop;
    free(v32); free(dinv32); free(dinv); free(r); free(r32); free(d32); free(bptr); free(inv);
    return stop;
}

/* ------------------------------------------------------ batched PCG */

/* Independent Jacobi-PCG per system (per-system stopping status,
 * Sec. 2.5): system s owns rows sys_ptr[s]..sys_ptr[s+1]-1 of the packed CSR,
 * its column indices are local to the system.  x0 = 0, criterion
 * ||r|| <= reduction*||b_s|| or iter_factor*n_s iterations. */
void orc_batch_pcg(int64_t nsys, const int32_t *sys_ptr, const int32_t *row_ptr,
                   const int32_t *col, const double *val, const double *b,
                   double *x, double reduction, int64_t iter_factor,
                   int32_t *iters, double *rel_res, uint8_t *status)
{
    for (int64_t s = 0; s < nsys; ++s) {
        int64_t r0 = sys_ptr[s], r1 = sys_ptr[s + 1], n = r1 - r0;
        int64_t k0 = row_ptr[r0];
        int32_t *rp = malloc((size_t)(n + 1) * sizeof(int32_t));
        for (int64_t i = 0; i <= n; ++i) rp[i] = (int32_t)(row_ptr[r0 + i] - k0);
        double *dinv = malloc((size_t)(n + 1) * sizeof(double));
        const int32_t *c = col + k0;
        const double *v = val + k0;
        double *xs = x + r0;
        for (int64_t i = 0; i < n; ++i) xs[i] = 0.0;
        orc_info info;
        if (orc_jacobi_dinv(n, rp, c, v, dinv) >= 0) {
            iters[s] = 0; rel_res[s] = NAN; status[s] = ORC_BREAKDOWN;
        } else {
            orc_criteria crit = { iter_factor * n, reduction, 1 };
            orc_pcg(n, rp, c, v, dinv, b + r0, xs, crit, &info, NULL);
            iters[s] = (int32_t)info.iterations;
            rel_res[s] = info.rel_residual;
            status[s] = (uint8_t)info.stop_reason;
        }
        free(rp); free(dinv);
    }
}

/* ------------------------------------------------------------ features */

static int cmp_i64(const void *a, const void *b)
{
    int64_t x = *(const int64_t *)a, y = *(const int64_t *)b;
    return (x > y) - (x < y);
}

/* Sixteen structural statistics of a sparse matrix, the input of the
 * format/kernel selector (the paper's runtime "kernel variant selection"
 * fork, Sec. 7.2):
 *  0 log10 n          1 log10 max(nnz,1)   2 mean row length mu
 *  3 std sigma        4 sigma/mu            5 max length
 *  6 min length       7 median (nearest rank 50%)
 *  8 p90              9 p99 (nearest rank: sorted[ceil(P*n/100)-1])
 * 10 fraction of rows with len > 2 mu   11 n*max/nnz (ELL fill)
 * 12 max|i-j|/n      13 mean|i-j|/n over entries
 * 14 fraction of entries with |i-j| <= 64
 * 15 skewness m3/m2^1.5 of the row lengths (0 when m2 == 0)
 * Moments are population moments, computed in two passes in FP64. */
void orc_features(int64_t nrows, int64_t ncols, const int32_t *row_ptr,
                  const int32_t *col, double out[16])
{
    (void)ncols;
    for (int j = 0; j < 16; ++j) out[j] = 0.0;
    if (nrows <= 0) return;
    int64_t nnz = row_ptr[nrows];
    int64_t *len = malloc((size_t)nrows * sizeof(int64_t));
    for (int64_t i = 0; i < nrows; ++i) len[i] = row_ptr[i + 1] - row_ptr[i];
    double n = (double)nrows;
    double mu = (double)nnz / n;
    double m2 = 0.0, m3 = 0.0;
    for (int64_t i = 0; i < nrows; ++i) {
        double d = (double)len[i] - mu;
        m2 += d * d;
        m3 += d * d * d;
    }
    m2 /= n;
    m3 /= n;
    int64_t above = 0;
    for (int64_t i = 0; i < nrows; ++i) if (len[i] * nrows > 2 * nnz) ++above;
    int64_t maxbw = 0, near = 0;
    double sumbw = 0.0;
    for (int64_t i = 0; i < nrows; ++i)
        for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) {
            int64_t d = (int64_t)col[k] - i;
            if (d < 0) d = -d;
            if (d > maxbw) maxbw = d;
            sumbw += (double)d;
            if (d <= 64) ++near;
        }
    qsort(len, (size_t)nrows, sizeof(int64_t), cmp_i64);
    int64_t r50 = (50 * nrows + 99) / 100, r90 = (90 * nrows + 99) / 100;
    int64_t r99 = (99 * nrows + 99) / 100;
    double sigma = sqrt(m2);
    out[0] = log10(n);
    out[1] = log10(nnz > 0 ? (double)nnz : 1.0);
    out[2] = mu;
    out[3] = sigma;
    out[4] = mu > 0.0 ? sigma / mu : 0.0;
    out[5] = (double)len[nrows - 1];
    out[6] = (double)len[0];
    out[7] = (double)len[r50 - 1];
    out[8] = (double)len[r90 - 1];
    out[9] = (double)len[r99 - 1];
    out[10] = (double)above / n;
    out[11] = nnz > 0 ? n * (double)len[nrows - 1] / (double)nnz : 0.0;
    out[12] = (double)maxbw / n;
    out[13] = nnz > 0 ? sumbw / (double)nnz / n : 0.0;
    out[14] = nnz > 0 ? (double)near / (double)nnz : 0.0;
    out[15] = m2 > 0.0 ? m3 / pow(m2, 1.5) : 0.0;
    free(len);
}

/* ----------------------------------------------------------------- MLP */

/* Fully connected network dims[0] -> dims[1] -> ... -> dims[nlayers], ReLU
 * after every layer but the last.  theta packs, layer by layer, W_l
 * (dims[l+1] x dims[l], row-major) followed by b_l (dims[l+1]).
 *
 * loss = sum_{i,c} M_ic (yhat_ic - Y_ic)^2 / sum M  +  lambda * sum_l ||W_l||_F^2
 *
 * grad (optional) receives d loss / d theta by reverse-mode differentiation
 * of exactly this expression; pred (optional) receives yhat (N x dims[L]). */
double orc_mlp_loss_grad(int32_t nlayers, const int32_t *dims,
                         const double *theta, int64_t nsamples,
                         const double *X, const double *Y, const double *M,
                         double lambda, double *grad, double *pred)
{
    int64_t off[64], width = 0, nparams = 0, total_act = 0;
    for (int l = 0; l < nlayers; ++l) {
        off[l] = nparams;
        nparams += (int64_t)dims[l + 1] * dims[l] + dims[l + 1];
    }
    for (int l = 0; l <= nlayers; ++l) {
        if (dims[l] > width) width = dims[l];
        total_act += dims[l];
    }
    int32_t C = dims[nlayers];
    double msum = 0.0;
    for (int64_t i = 0; i < nsamples * C; ++i) msum += M[i];
    double *h = malloc((size_t)total_act * sizeof(double));   /* pre-activations */
    double *a = malloc((size_t)total_act * sizeof(double));   /* activations */
    double *da = malloc((size_t)width * sizeof(double));
    double *dh = malloc((size_t)width * sizeof(double));
    if (grad) for (int64_t j = 0; j < nparams; ++j) grad[j] = 0.0;
    double data = 0.0;
    for (int64_t s = 0; s < nsamples; ++s) {
        int64_t ao = 0;
        for (int j = 0; j < dims[0]; ++j) a[j] = X[s * dims[0] + j];
        for (int l = 0; l < nlayers; ++l) {
            const double *W = theta + off[l];
            const double *bb = W + (int64_t)dims[l + 1] * dims[l];
            int64_t no = ao + dims[l];
            for (int o = 0; o < dims[l + 1]; ++o) {
                double acc = bb[o];
                for (int j = 0; j < dims[l]; ++j) acc += W[(int64_t)o * dims[l] + j] * a[ao + j];
                h[no + o] = acc;
                a[no + o] = (l < nlayers - 1) ? (acc > 0.0 ? acc : 0.0) : acc;
            }
            ao = no;
        }
        for (int c = 0; c < C; ++c) {
            double e = a[ao + c] - Y[s * C + c];
            double m = M[s * C + c];
            data += m * e * e;
            if (pred) pred[s * C + c] = a[ao + c];
            dh[c] = msum > 0.0 ? 2.0 * m * e / msum : 0.0;
        }
        if (!grad) continue;
        /* backward: dh holds d loss / d h for layer l's outputs */
        for (int l = nlayers - 1; l >= 0; --l) {
            const double *W = theta + off[l];
            double *gW = grad + off[l];
            double *gb = gW + (int64_t)dims[l + 1] * dims[l];
            int64_t in_o = ao - dims[l];
            for (int o = 0; o < dims[l + 1]; ++o) {
                gb[o] += dh[o];
                for (int j = 0; j < dims[l]; ++j)
                    gW[(int64_t)o * dims[l] + j] += dh[o] * a[in_o + j];
            }
            if (l == 0) break;
            for (int j = 0; j < dims[l]; ++j) {
                double acc = 0.0;
                for (int o = 0; o < dims[l + 1]; ++o) acc += W[(int64_t)o * dims[l] + j] * dh[o];
                da[j] = acc;
            }
            for (int j = 0; j < dims[l]; ++j) dh[j] = h[in_o + j] > 0.0 ? da[j] : 0.0;
            ao = in_o;
        }
    }
    double loss = msum > 0.0 ? data / msum : 0.0;
    for (int l = 0; l < nlayers; ++l) {
        const double *W = theta + off[l];
        int64_t nw = (int64_t)dims[l + 1] * dims[l];
        for (int64_t j = 0; j < nw; ++j) {
            loss += lambda * W[j] * W[j];
            if (grad) grad[off[l] + j] += 2.0 * lambda * W[j];
        }
    }
    free(h); free(a); free(da); free(dh);
    return loss;
}

/* Adam (Kingma & Ba) with bias correction; t is the 1-based step count. */
void orc_adam_step(int64_t nparams, double *theta, const double *grad,
                   double *m, double *v, int64_t t, double lr, double beta1,
                   double beta2, double eps)
{
    double c1 = 1.0 - pow(beta1, (double)t), c2 = 1.0 - pow(beta2, (double)t);
    for (int64_t j = 0; j < nparams; ++j) {
        m[j] = beta1 * m[j] + (1.0 - beta1) * grad[j];
        v[j] = beta2 * v[j] + (1.0 - beta2) * grad[j] * grad[j];
        double mh = m[j] / c1, vh = v[j] / c2;
        theta[j] -= lr * mh / (sqrt(vh) + eps);
    }
}

/* ------------------------------------------------------ block Jacobi */

/* Block-Jacobi (Sec. 3.2): the diagonal blocks of A over consecutive row
 * ranges [bptr[b], bptr[b+1]) are inverted (Gauss-Jordan elimination with
 * partial pivoting, as the paper's generation does) and, in the adaptive
 * mode, each inverse is stored in the lowest precision its conditioning
 * and exponent range allow (memory precision decoupled from the FP64
 * arithmetic).  Readings (the paper names the ingredients, not the rule):
 *   cond_b = ||D_b||_1 ||D_b^{-1}||_1;
 *   binary16 if cond_b * 2^-11 <= accuracy and every nonzero |inverse
 *   entry| lies in [2^-14, 65504]; else binary32 if cond_b * 2^-24 <=
 *   accuracy and they lie in [2^-126, FLT_MAX]; else binary64.
 * Stored values are the inverse entries rounded to nearest-even in that
 * precision; the product z_b = D_b^{-1} r_b sums over ascending columns in
 * FP64. */

/* Nearest-even rounding to IEEE binary16 written from the format's
 * definition (11-bit significand, exponents -14..15, subnormal quantum
 * 2^-24, overflow to infinity at 65520). */
double orc_round_f16(double x)
{
    if (x == 0.0 || !isfinite(x)) return x;
    double a = fabs(x);
    if (a >= 65520.0) return copysign(INFINITY, x);
    int e2;
    frexp(a, &e2);             /* a = m 2^e2, m in [0.5, 1): exponent e2 - 1 */
    int e = e2 - 1;
    if (e < -14) e = -14;      /* subnormal range shares the quantum 2^-24 */
    double quantum = ldexp(1.0, e - 10);
    double r = nearbyint(a / quantum) * quantum;  /* exact scaling, RNE */
    return copysign(r, x);
}

static double round_to(double x, int prec)
{
    if (prec == ORC_P32) return (double)(float)x;
    if (prec == ORC_P16) return orc_round_f16(x);
    return x;
}

/* Gauss-Jordan inversion of the m x m row-major matrix D (overwritten)
 * into Dinv, with partial pivoting.  Returns 0, or 1 if D is singular. */
static int gauss_jordan(int m, double *D, double *Dinv)
{
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < m; ++j) Dinv[i * m + j] = (i == j) ? 1.0 : 0.0;
    for (int c = 0; c < m; ++c) {
        int piv = c;
        for (int r = c + 1; r < m; ++r)
            if (fabs(D[r * m + c]) > fabs(D[piv * m + c])) piv = r;
        if (D[piv * m + c] == 0.0) return 1;
        if (piv != c)
            for (int j = 0; j < m; ++j) {
                double t = D[c * m + j]; D[c * m + j] = D[piv * m + j]; D[piv * m + j] = t;
                t = Dinv[c * m + j]; Dinv[c * m + j] = Dinv[piv * m + j]; Dinv[piv * m + j] = t;
            }
        double d = D[c * m + c];
        for (int j = 0; j < m; ++j) { D[c * m + j] /= d; Dinv[c * m + j] /= d; }
        for (int r = 0; r < m; ++r) {
            if (r == c) continue;
            double f = D[r * m + c];
            if (f == 0.0) continue;
            for (int j = 0; j < m; ++j) {
                D[r * m + j] -= f * D[c * m + j];
                Dinv[r * m + j] -= f * Dinv[c * m + j];
            }
        }
    }
    return 0;
}

static double norm1(int m, const double *M)
{
    double best = 0.0;
    for (int j = 0; j < m; ++j) {
        double s = 0.0;
        for (int i = 0; i < m; ++i) s += fabs(M[i * m + j]);
        if (s > best) best = s;
    }
    return best;
}

int orc_bj_choose_precision(int m, const double *inv, double cond, double accuracy)
{
    double lo = INFINITY, hi = 0.0;
    for (int k = 0; k < m * m; ++k) {
        double a = fabs(inv[k]);
        if (a == 0.0) continue;
        if (a < lo) lo = a;
        if (a > hi) hi = a;
    }
    if (hi == 0.0) lo = hi = 1.0;
    if (cond * ldexp(1.0, -11) <= accuracy && lo >= ldexp(1.0, -14) && hi <= 65504.0) return ORC_P16;
    if (cond * ldexp(1.0, -24) <= accuracy && lo >= ldexp(1.0, -126) && hi <= 3.4028234663852886e38)
        return ORC_P32;
    return ORC_P64;
}

/* Variable block boundaries for block-Jacobi (Sec. 3.2 names batched
 * variable-size Gauss-Jordan generation but no rule for the sizes).
 * Reading: supervariable agglomeration.  A supervariable is a maximal run of
 * consecutive rows whose column index sets are identical; one longer than
 * max_bs is cut into pieces of max_bs rows from its first row on (the last
 * piece may be shorter), and every piece counts as a unit.  Walking the
 * units in row order, a unit joins the current block when the block then
 * has at most max_bs rows, and starts a new block otherwise.  bptr (room
 * for n + 1 entries) receives the block boundaries; returns the number of
 * blocks. */
static int same_pattern(const int32_t *row_ptr, const int32_t *col, int64_t a, int64_t b)
{
    const int32_t la = row_ptr[a + 1] - row_ptr[a], lb = row_ptr[b + 1] - row_ptr[b];
    if (la != lb) return 0;
    for (int32_t k = 0; k < la; ++k)
        if (col[row_ptr[a] + k] != col[row_ptr[b] + k]) return 0;
    return 1;
}

int64_t orc_bj_supervariable_blocks(int64_t n, const int32_t *row_ptr, const int32_t *col, int max_bs,
                                    int32_t *bptr)
{
    int64_t nb = 0;
    bptr[0] = 0;
    int64_t block_rows = 0;
    int64_t i = 0;
    while (i < n) {
        /* the supervariable starting at row i */
        int64_t e = i + 1;
        while (e < n && same_pattern(row_ptr, col, e, i)) ++e;
        /* its pieces of at most max_bs rows */
        for (int64_t p = i; p < e; p += max_bs) {
            const int64_t len = (e - p < max_bs) ? e - p : max_bs;
            if (block_rows > 0 && block_rows + len > max_bs) {
                bptr[++nb] = (int32_t)p;
                block_rows = 0;
            }
            block_rows += len;
        }
        i = e;
    }
    if (n > 0) bptr[++nb] = (int32_t)n;
    return nb;
}

int64_t orc_bj_generate(int64_t n, const int32_t *row_ptr, const int32_t *col, const double *val,
                        int64_t nblocks, const int32_t *bptr, int adaptive, double accuracy,
                        double *inv, double *cond, int32_t *prec_out)
{
    int64_t off = 0;
    int mmax = 0;
    for (int64_t b = 0; b < nblocks; ++b)
        if (bptr[b + 1] - bptr[b] > mmax) mmax = bptr[b + 1] - bptr[b];
    double *D = (double *)malloc((size_t)mmax * mmax * sizeof(double) + 8);
    double *Dk = (double *)malloc((size_t)mmax * mmax * sizeof(double) + 8);
    int64_t bad = -1;
    (void)n;
    for (int64_t b = 0; b < nblocks && bad < 0; ++b) {
        const int r0 = bptr[b], m = bptr[b + 1] - bptr[b];
        for (int k = 0; k < m * m; ++k) D[k] = 0.0;
        for (int i = 0; i < m; ++i)
            for (int32_t k = row_ptr[r0 + i]; k < row_ptr[r0 + i + 1]; ++k) {
                const int j = col[k] - r0;
                if (j >= 0 && j < m) D[i * m + j] = val[k];
            }
        const double nD = norm1(m, D);
        for (int k = 0; k < m * m; ++k) Dk[k] = D[k];
        if (gauss_jordan(m, Dk, inv + off)) { bad = b; break; }
        const double c = nD * norm1(m, inv + off);
        const int p = adaptive ? orc_bj_choose_precision(m, inv + off, c, accuracy) : ORC_P64;
        for (int k = 0; k < m * m; ++k) inv[off + k] = round_to(inv[off + k], p);
        cond[b] = c;
        prec_out[b] = p;
        off += (int64_t)m * m;
    }
    free(D);
    free(Dk);
    return bad;
}

static void orc_bj_apply_impl(int64_t nb, const int32_t *bptr, const double *inv,
                              const double *r, double *z)
{
    int64_t off = 0;
    for (int64_t b = 0; b < nb; ++b) {
        const int r0 = bptr[b], m = bptr[b + 1] - bptr[b];
        for (int i = 0; i < m; ++i) {
            double s = 0.0;
            for (int j = 0; j < m; ++j) s += inv[off + (int64_t)i * m + j] * r[r0 + j];
            z[r0 + i] = s;
        }
        off += (int64_t)m * m;
    }
}

void orc_bj_apply(int64_t nb, const int32_t *bptr, const double *inv, const double *r, double *z)
{
    orc_bj_apply_impl(nb, bptr, inv, r, z);
}

/* ------------------------------------------------------ incomplete LU */

/* Incomplete LU factors are held in A's CSR pattern: the strictly lower
 * entries are L (unit diagonal implied), the diagonal and upper entries U
 * (the ILU-type preconditioners of Sec. 3.2). */

static int64_t find_col(const int32_t *row_ptr, const int32_t *col, int64_t row, int64_t c)
{
    int64_t lo = row_ptr[row], hi = row_ptr[row + 1] - 1;
    while (lo <= hi) {
        const int64_t mid = lo + (hi - lo) / 2;
        if (col[mid] == c) return mid;
        if (col[mid] < c) lo = mid + 1;
        else hi = mid - 1;
    }
    return -1;
}

static int64_t diag_pos(const int32_t *row_ptr, const int32_t *col, int64_t i)
{
    return find_col(row_ptr, col, i, i);
}

/* ILU(0): the factors with L U = A on A's pattern, by the row-wise
 * elimination of Saad's book (IKJ order): for each row i and each of its
 * lower entries k < i in ascending order, a_ik /= u_kk, then
 * a_ij -= a_ik u_kj for every later entry j of row i that row k also holds.
 * Returns -1, or the first row whose pivot is missing or zero. */
int64_t orc_ilu0(int64_t n, const int32_t *row_ptr, const int32_t *col, const double *val, double *lu)
{
    const int64_t nnz = row_ptr[n];
    for (int64_t q = 0; q < nnz; ++q) lu[q] = val[q];
    for (int64_t i = 0; i < n; ++i) {
        const int64_t di = diag_pos(row_ptr, col, i);
        if (di < 0) return i;
        for (int64_t q = row_ptr[i]; q < row_ptr[i + 1] && col[q] < i; ++q) {
            const int64_t k = col[q];
            const int64_t dk = diag_pos(row_ptr, col, k);
            lu[q] = lu[q] / lu[dk];
            for (int64_t t = q + 1; t < row_ptr[i + 1]; ++t) {
                const int64_t p = find_col(row_ptr, col, k, col[t]);
                if (p >= 0) lu[t] = lu[t] - lu[q] * lu[p];
            }
        }
        if (lu[di] == 0.0) return i;
    }
    return -1;
}

/* ParILU (the fine-grained fixed-point ILU the paper cites for its ILU
 * generation), synchronous form: every entry (i, j) of the pattern is
 * recomputed from the previous sweep's factors,
 *   s = a_ij - sum_{k < min(i,j)} l_ik u_kj   (ascending k, pattern entries)
 *   l_ij = s / u_jj (i > j),  u_ij = s (i <= j),
 * starting from l_ij = a_ij / a_jj and u_ij = a_ij.  The fixed point is
 * ILU(0).  Returns -1, or the first row with a missing or zero diagonal. */
int64_t orc_parilu(int64_t n, const int32_t *row_ptr, const int32_t *col, const double *val,
                   int32_t sweeps, double *lu)
{
    const int64_t nnz = row_ptr[n];
    int64_t *dg = (int64_t *)malloc((size_t)(n + 1) * sizeof(int64_t));
    double *old = (double *)malloc((size_t)(nnz + 1) * sizeof(double));
    for (int64_t i = 0; i < n; ++i) {
        dg[i] = diag_pos(row_ptr, col, i);
        if (dg[i] < 0 || val[dg[i]] == 0.0) {
            free(dg);
            free(old);
            return i;
        }
    }
    for (int64_t i = 0; i < n; ++i)
        for (int64_t q = row_ptr[i]; q < row_ptr[i + 1]; ++q)
            lu[q] = col[q] < i ? val[q] / val[dg[col[q]]] : val[q];
    for (int32_t sw = 0; sw < sweeps; ++sw) {
        for (int64_t q = 0; q < nnz; ++q) old[q] = lu[q];
        for (int64_t i = 0; i < n; ++i)
            for (int64_t q = row_ptr[i]; q < row_ptr[i + 1]; ++q) {
                const int64_t j = col[q];
                const int64_t m = i < j ? i : j;
                double s = val[q];
                for (int64_t t = row_ptr[i]; t < row_ptr[i + 1] && col[t] < m; ++t) {
                    const int64_t p = find_col(row_ptr, col, col[t], j);
                    if (p >= 0) s = s - old[t] * old[p];
                }
                lu[q] = i > j ? s / old[dg[j]] : s;
            }
    }
    free(dg);
    free(old);
    return -1;
}

/* Triangular solves with the factors in lu.  mode 0: exact forward and
 * backward substitution (ascending column order inside each row sum);
 * mode 1: `sweeps` Jacobi sweeps on each triangular system from
 * y = r (unit L) and z = y / u_ii (U):
 *   y_i <- r_i - sum_{k<i} l_ik y_k,   z_i <- (y_i - sum_{k>i} u_ik z_k) / u_ii
 * each sweep using only the previous sweep's vector.  z = U^{-1} L^{-1} r. */
void orc_ilu_apply(int64_t n, const int32_t *row_ptr, const int32_t *col, const double *lu,
                   int32_t mode, int32_t sweeps, const double *r, double *z)
{
    double *y = (double *)malloc((size_t)(n + 1) * sizeof(double));
    double *t = (double *)malloc((size_t)(n + 1) * sizeof(double));
    if (mode == 0) {
        for (int64_t i = 0; i < n; ++i) {
            double s = r[i];
            for (int64_t q = row_ptr[i]; q < row_ptr[i + 1] && col[q] < i; ++q) s -= lu[q] * y[col[q]];
            y[i] = s;
        }
        for (int64_t i = n - 1; i >= 0; --i) {
            double s = y[i], d = 0.0;
            for (int64_t q = row_ptr[i]; q < row_ptr[i + 1]; ++q) {
                if (col[q] > i) s -= lu[q] * z[col[q]];
                else if (col[q] == i) d = lu[q];
            }
            z[i] = s / d;
        }
    } else {
        for (int64_t i = 0; i < n; ++i) y[i] = r[i];
        for (int32_t sw = 0; sw < sweeps; ++sw) {
            for (int64_t i = 0; i < n; ++i) {
                double s = r[i];
                for (int64_t q = row_ptr[i]; q < row_ptr[i + 1] && col[q] < i; ++q) s -= lu[q] * y[col[q]];
                t[i] = s;
            }
            for (int64_t i = 0; i < n; ++i) y[i] = t[i];
        }
        for (int64_t i = 0; i < n; ++i) z[i] = y[i] / lu[diag_pos(row_ptr, col, i)];
        for (int32_t sw = 0; sw < sweeps; ++sw) {
            for (int64_t i = 0; i < n; ++i) {
                double s = y[i], d = 0.0;
                for (int64_t q = row_ptr[i]; q < row_ptr[i + 1]; ++q) {
                    if (col[q] > i) s -= lu[q] * z[col[q]];
                    else if (col[q] == i) d = lu[q];
                }
                t[i] = s / d;
            }
            for (int64_t i = 0; i < n; ++i) z[i] = t[i];
        }
    }
    free(y);
    free(t);
}

int orc_gmres_ilu(int64_t n, const int32_t *row_ptr, const int32_t *col, const double *val,
                  const double *lu, int32_t trs_mode, int32_t trs_sweeps, const double *b,
                  double *x, int32_t krylov_dim, orc_criteria crit, orc_info *info, double *history)
{
    orc_prec M = {NULL, 0, NULL, NULL, row_ptr, col, lu, trs_mode, trs_sweeps};
    return gmres_core(n, row_ptr, col, val, &M, b, x, krylov_dim, crit, info, history);
}
