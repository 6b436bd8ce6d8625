// batched.hip -- thousands of independent small Jacobi-PCG solves in one
// persistent launch (per-system stopping status: the per-right-hand-side
// stopping status of the criteria in Sec. 2.5 of the paper, applied to
// independent systems).
//
// Design (gfx950): a grid of wgs_per_cu x num_CU workgroups stays resident;
// each workgroup pulls a system id from an atomic queue, runs the whole CG
// for that system with its vectors r, p, q, x in LDS (or in a per-workgroup
// global scratch slice when the system is too large for LDS), reduces dot
// products inside the workgroup (fixed tree: deterministic), writes x, the
// iteration count, the recurrence residual and the stop reason, and pulls
// the next id.  Every workgroup exits when the queue is drained.  The
// schedule (workgroup size, residency, order) is chosen by an autotuner
// that times the candidates on the actual batch.
#include <algorithm>
#include <chrono>
#include <climits>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <numeric>
#include <string>
#include <vector>

#include "device_common.hpp"
#include "internal.hpp"

namespace mxl {

struct BatchImpl {
    CtxRef ctx;
    int64_t nsys = 0, rows = 0, nnz = 0;
    std::vector<int32_t> sys_ptr_h;
    int max_n = 0;
    BufPtr sys_ptr, row_ptr, col, val;
    BufPtr dinv;             // FP64 1/a_ii of every row
    BufPtr order_input, order_big;  // processing orders
    BufPtr queue;            // uint32 work counter
    BufPtr scratch;          // per-workgroup vectors for systems larger than LDS
    int64_t scratch_elems = 0;
    bool tuned = false;
    mxl_tuning best{};
    int small_shape = -1;    // single-system register-cached shape (-1: not chosen)
    int small_bi_shape = -1; // the same for the one-workgroup BiCGSTAB
    // Per-system slot-major ELL copy (built when it is compact): system s has
    // w_s = its longest row; slot e of local row i is at off_s + e*n_s + i,
    // columns as int16 local indices, -1 for padding.
    bool ell = false;
    int w_max = 0;
    int64_t ell_slots = 0;
    BufPtr ell_val, ell_col, ell_off, ell_w;
};

template <int B>
__device__ __forceinline__ double wg_sum(double v, double *red) {
    constexpr int NW = B / kWave;
    v = wave_sum(v);
    if (NW == 1) return v;
    const int lane = threadIdx.x % kWave, wid = threadIdx.x / kWave;
    __syncthreads();
    if (lane == 0) red[wid] = v;
    __syncthreads();
    double a = red[0];
#pragma unroll
    for (int w = 1; w < NW; ++w) a += red[w];
    return a;
}

template <int B>
__device__ __forceinline__ void wg_sum2(double &u, double &v, double *red) {
    constexpr int NW = B / kWave;
    u = wave_sum(u);
    v = wave_sum(v);
    if (NW == 1) return;
    const int lane = threadIdx.x % kWave, wid = threadIdx.x / kWave;
    __syncthreads();
    if (lane == 0) {
        red[wid] = u;
        red[NW + wid] = v;
    }
    __syncthreads();
    double a = red[0], c = red[NW];
#pragma unroll
    for (int w = 1; w < NW; ++w) {
        a += red[w];
        c += red[NW + w];
    }
    u = a;
    v = c;
}

template <int B>
__global__ __launch_bounds__(B) void k_batch_pcg(
    int64_t nsys, const int *__restrict__ sys_ptr, const int *__restrict__ rp,
    const int *__restrict__ col, const double *__restrict__ val, const double *__restrict__ dinv,
    const double *__restrict__ bvec, double *__restrict__ xout, int *__restrict__ iters_out,
    double *__restrict__ rel_out, uint8_t *__restrict__ status_out, const int *__restrict__ order,
    unsigned *__restrict__ queue, double red_factor, int64_t max_iters_fixed, int iter_factor,
    int chk, int lds_cap, double *__restrict__ scratch, int64_t scratch_stride, int use_x0) {
    extern __shared__ double smem[];
    __shared__ double red[2 * (B / kWave)];
    __shared__ int s_q;
    const int tid = threadIdx.x;
    for (;;) {
        if (tid == 0) s_q = (int)atomicAdd(queue, 1u);
        __syncthreads();
        const int qi = s_q;
        __syncthreads();
        if ((int64_t)qi >= nsys) break;
        const int s = order[qi];
        const int r0 = sys_ptr[s];
        const int n = sys_ptr[s + 1] - r0;
        const bool in_lds = n <= lds_cap;
        double *base = in_lds ? smem : scratch + (int64_t)blockIdx.x * scratch_stride;
        double *x = base, *r = base + n, *p = base + 2 * n, *q = base + 3 * n;
        const double *b = bvec + r0;
        const double *di = dinv + r0;
        const int *rps = rp + r0;
        // x = x0 (or 0), r = b - A x, p = z = D^{-1} r
        for (int i = tid; i < n; i += B) x[i] = use_x0 ? xout[r0 + i] : 0.0;
        if (use_x0) __syncthreads();
        double rz = 0.0, rr0 = 0.0, bb = 0.0;
        for (int i = tid; i < n; i += B) {
            const double bi = b[i];
            double ax = 0.0;
            if (use_x0)
                for (int e = rps[i]; e < rps[i + 1]; ++e) ax += val[e] * x[col[e]];
            const double ri = bi - ax;
            const double zi = di[i] * ri;
            r[i] = ri;
            p[i] = zi;
            rz += ri * zi;
            rr0 += ri * ri;
            bb += bi * bi;
        }
        wg_sum2<B>(rz, bb, red);
        rr0 = wg_sum<B>(rr0, red);
        const double nb = sqrt(bb);
        const int64_t maxit = max_iters_fixed > 0 ? max_iters_fixed : (int64_t)iter_factor * n;
        int stop = ST_RUN;
        int64_t k = 0;
        double rr = rr0;
        if (bb == 0.0) {  // zero right-hand side: x = 0
            for (int i = tid; i < n; i += B) x[i] = 0.0;
            stop = ST_CONVERGED;
        } else if (sqrt(rr) <= red_factor * nb) {
            stop = ST_CONVERGED;
        }
        double rho = rz;
        while (stop == ST_RUN && k < maxit) {
            __syncthreads();  // p complete
            double pq = 0.0;
            for (int i = tid; i < n; i += B) {
                const int e0 = rps[i], e1 = rps[i + 1];
                double acc = 0.0;
                for (int e = e0; e < e1; ++e) acc += val[e] * p[col[e]];
                q[i] = acc;
                pq += p[i] * acc;
            }
            const double eta = wg_sum<B>(pq, red);
            if (chk && !finite_d(eta)) { stop = ST_NONFINITE; break; }
            if (eta <= 0.0) { stop = ST_BREAKDOWN; break; }
            const double alpha = rho / eta;
            double rzn = 0.0, rrn = 0.0;
            for (int i = tid; i < n; i += B) {
                x[i] += alpha * p[i];
                const double ri = r[i] - alpha * q[i];
                r[i] = ri;
                rzn += ri * (di[i] * ri);
                rrn += ri * ri;
            }
            wg_sum2<B>(rzn, rrn, red);
            ++k;
            rr = rrn;
            if (chk && !finite_d(rr)) { stop = ST_NONFINITE; break; }
            if (sqrt(rr) <= red_factor * nb) { stop = ST_CONVERGED; break; }
            if (chk && !finite_d(rzn)) { stop = ST_NONFINITE; break; }
            if (rzn == 0.0) { stop = ST_BREAKDOWN; break; }
            const double beta = rzn / rho;
            rho = rzn;
            for (int i = tid; i < n; i += B) p[i] = di[i] * r[i] + beta * p[i];
        }
        if (stop == ST_RUN) stop = ST_MAX_ITERS;
        __syncthreads();
        for (int i = tid; i < n; i += B) xout[r0 + i] = x[i];
        if (tid == 0) {
            iters_out[s] = (int)k;
            rel_out[s] = nb > 0.0 ? sqrt(rr) / nb : 0.0;
            status_out[s] = (uint8_t)stop;
        }
        __syncthreads();
    }
}

// The same persistent Jacobi-PCG on the per-system ELL copy.  A system
// whose five vectors (x, r, p, q, dinv) fit the workgroup's LDS budget keeps
// them there, and its matrix too when that also fits, so every iteration
// after the first reads only LDS; the product walks slot-major entries
// (consecutive rows at consecutive addresses) in each row's stored order,
// so q and every scalar equal k_batch_pcg's at the same workgroup size.
// Larger systems keep their vectors in a global scratch slice and read the
// matrix from the global ELL copy.
template <int B>
__global__ __launch_bounds__(B) void k_batch_pcg_ell(
    int64_t nsys, const int *__restrict__ sys_ptr, const int64_t *__restrict__ ell_off,
    const int *__restrict__ ell_w, const double *__restrict__ ell_val, const short *__restrict__ ell_col,
    const double *__restrict__ dinv, const double *__restrict__ bvec, double *__restrict__ xout,
    int *__restrict__ iters_out, double *__restrict__ rel_out, uint8_t *__restrict__ status_out,
    const int *__restrict__ order, unsigned *__restrict__ queue, double red_factor, int64_t max_iters_fixed,
    int iter_factor, int chk, int64_t lds_budget, double *__restrict__ scratch, int64_t scratch_stride,
    int use_x0) {
    extern __shared__ double smem[];
    __shared__ double red[2 * (B / kWave)];
    __shared__ int s_q;
    const int tid = threadIdx.x;
    for (;;) {
        if (tid == 0) s_q = (int)atomicAdd(queue, 1u);
        __syncthreads();
        const int qi = s_q;
        __syncthreads();
        if ((int64_t)qi >= nsys) break;
        const int s = order[qi];
        const int r0 = sys_ptr[s];
        const int n = sys_ptr[s + 1] - r0;
        const int w = ell_w[s];
        const int64_t off = ell_off[s];
        const int64_t vec_bytes = (int64_t)40 * n, mat_bytes = (int64_t)10 * w * n;
        const bool in_lds = vec_bytes <= lds_budget;
        const bool mat_lds = in_lds && vec_bytes + mat_bytes <= lds_budget;
        double *base = in_lds ? smem : scratch + (int64_t)blockIdx.x * scratch_stride;
        double *x = base, *r = base + n, *p = base + 2 * n, *q = base + 3 * n, *di = base + 4 * n;
        const double *Vm = mat_lds ? base + 5 * n : ell_val + off;
        const short *Cm = mat_lds ? (const short *)(base + 5 * n + (int64_t)w * n) : ell_col + off;
        if (mat_lds) {
            double *vl = base + 5 * n;
            short *cl = (short *)(base + 5 * n + (int64_t)w * n);
            for (int64_t j = tid; j < (int64_t)w * n; j += B) {
                vl[j] = ell_val[off + j];
                cl[j] = ell_col[off + j];
            }
        }
        const double *b = bvec + r0;
        for (int i = tid; i < n; i += B) {
            x[i] = use_x0 ? xout[r0 + i] : 0.0;
            di[i] = dinv[r0 + i];
        }
        __syncthreads();
        // r = b - A x, p = z = D^{-1} r
        double rz = 0.0, rr0 = 0.0, bb = 0.0;
        for (int i = tid; i < n; i += B) {
            const double bi = b[i];
            double ax = 0.0;
            if (use_x0)
                for (int e = 0; e < w; ++e) {
                    const int c = Cm[(int64_t)e * n + i];
                    if (c >= 0) ax += Vm[(int64_t)e * n + i] * x[c];
                }
            const double ri = bi - ax;
            const double zi = di[i] * ri;
            r[i] = ri;
            p[i] = zi;
            rz += ri * zi;
            rr0 += ri * ri;
            bb += bi * bi;
        }
        wg_sum2<B>(rz, bb, red);
        rr0 = wg_sum<B>(rr0, red);
        const double nb = sqrt(bb);
        const int64_t maxit = max_iters_fixed > 0 ? max_iters_fixed : (int64_t)iter_factor * n;
        int stop = ST_RUN;
        int64_t k = 0;
        double rr = rr0;
        if (bb == 0.0) {  // zero right-hand side: x = 0
            for (int i = tid; i < n; i += B) x[i] = 0.0;
            stop = ST_CONVERGED;
        } else if (sqrt(rr) <= red_factor * nb) {
            stop = ST_CONVERGED;
        }
        double rho = rz;
        while (stop == ST_RUN && k < maxit) {
            __syncthreads();  // p complete
            double pq = 0.0;
            for (int i = tid; i < n; i += B) {
                double acc = 0.0;
#pragma unroll 4
                for (int e = 0; e < w; ++e) {
                    const int c = Cm[(int64_t)e * n + i];
                    if (c >= 0) acc += Vm[(int64_t)e * n + i] * p[c];
                }
                q[i] = acc;
                pq += p[i] * acc;
            }
            const double eta = wg_sum<B>(pq, red);
            if (chk && !finite_d(eta)) { stop = ST_NONFINITE; break; }
            if (eta <= 0.0) { stop = ST_BREAKDOWN; break; }
            const double alpha = rho / eta;
            double rzn = 0.0, rrn = 0.0;
            for (int i = tid; i < n; i += B) {
                x[i] += alpha * p[i];
                const double ri = r[i] - alpha * q[i];
                r[i] = ri;
                rzn += ri * (di[i] * ri);
                rrn += ri * ri;
            }
            wg_sum2<B>(rzn, rrn, red);
            ++k;
            rr = rrn;
            if (chk && !finite_d(rr)) { stop = ST_NONFINITE; break; }
            if (sqrt(rr) <= red_factor * nb) { stop = ST_CONVERGED; break; }
            if (chk && !finite_d(rzn)) { stop = ST_NONFINITE; break; }
            if (rzn == 0.0) { stop = ST_BREAKDOWN; break; }
            const double beta = rzn / rho;
            rho = rzn;
            for (int i = tid; i < n; i += B) p[i] = di[i] * r[i] + beta * p[i];
        }
        if (stop == ST_RUN) stop = ST_MAX_ITERS;
        __syncthreads();
        for (int i = tid; i < n; i += B) xout[r0 + i] = x[i];
        if (tid == 0) {
            iters_out[s] = (int)k;
            rel_out[s] = nb > 0.0 ? sqrt(rr) / nb : 0.0;
            status_out[s] = (uint8_t)stop;
        }
        __syncthreads();
    }
}

// One workgroup per system: checks 0 <= col < n_s for every stored entry
// (lowest bad row into *bad) and, when ev is not null, writes the system's
// slot-major ELL copy (padding: value 0, column -1).
__global__ void k_batch_to_ell(const int *__restrict__ sys_ptr, const int *__restrict__ rp,
                               const int *__restrict__ col, const double *__restrict__ val,
                               const int64_t *__restrict__ ell_off, const int *__restrict__ ell_w,
                               double *__restrict__ ev, short *__restrict__ ec, int *__restrict__ bad) {
    const int s = blockIdx.x;
    const int r0 = sys_ptr[s], n = sys_ptr[s + 1] - r0;
    const int w = ev ? ell_w[s] : 0;
    const int64_t off = ev ? ell_off[s] : 0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        const int e0 = rp[r0 + i], len = rp[r0 + i + 1] - e0;
        bool ok = true;
        for (int e = 0; e < len; ++e) {
            const int c = col[e0 + e];
            if (c < 0 || c >= n) ok = false;
        }
        if (!ok) atomicMin(bad, r0 + i);
        if (ev)
            for (int e = 0; e < w; ++e) {
                const bool in = e < len;
                ev[off + (int64_t)e * n + i] = in ? val[e0 + e] : 0.0;
                ec[off + (int64_t)e * n + i] = in ? (short)col[e0 + e] : (short)-1;
            }
    }
}

// Whole Jacobi-PCG of one small system in one workgroup with the matrix
// held in registers: thread t owns rows t + j*B (j < RPT) and keeps their
// (at most W) entries, r and p in registers; p, which the product gathers,
// is mirrored in LDS.  x and dinv stay in global memory for the large
// shapes (register budget) and in registers when REG; a one-wave shape
// (B = 64) reduces with lane shuffles only.  An iteration is the product,
// two reductions and the updates.
template <int B, int RPT, int W, bool REG>
__global__ __launch_bounds__(B) void k_small_pcg(int n, const int *__restrict__ rp,
                                                 const int *__restrict__ col,
                                                 const double *__restrict__ val,
                                                 const double *__restrict__ dinv,
                                                 const double *__restrict__ b,
                                                 double *__restrict__ xio, double red_factor,
                                                 int64_t maxit, int chk, int use_x0,
                                                 void *__restrict__ out3) {
    extern __shared__ double p_lds[];
    constexpr int NW = B / kWave;
    __shared__ double redA[NW], redB[2 * NW], redC[3 * NW];
    const int tid = threadIdx.x, lane = tid % kWave, wid = tid / kWave;
    int c[RPT][W];
    double v[RPT][W];
    double r[RPT], pr[RPT];
    double xr[REG ? RPT : 1], dv[REG ? RPT : 1];
#pragma unroll
    for (int j = 0; j < RPT; ++j) {
        const int i = tid + j * B;
        const bool own = i < n;
        if constexpr (REG) {
            dv[j] = own ? dinv[i] : 0.0;
            xr[j] = own && use_x0 ? xio[i] : 0.0;
        }
        const int e0 = own ? rp[i] : 0, e1 = own ? rp[i + 1] : 0;
#pragma unroll
        for (int e = 0; e < W; ++e) {
            const bool in = e0 + e < e1;
            // padding points at the thread's own row (value 0): SPD systems
            // store their diagonal, so padding adds no new dependency
            c[j][e] = in ? col[e0 + e] : (own ? i : 0);
            v[j][e] = in ? val[e0 + e] : 0.0;
        }
        if (own) p_lds[i] = use_x0 ? xio[i] : 0.0;
    }
    __syncthreads();
    double rz = 0.0, rr = 0.0, bb = 0.0;
#pragma unroll
    for (int j = 0; j < RPT; ++j) {
        const int i = tid + j * B;
        double ax = 0.0;
        if (use_x0) {
#pragma unroll
            for (int e = 0; e < W; ++e) ax += v[j][e] * p_lds[c[j][e]];
        }
        const bool own = i < n;
        const double bi = own ? b[i] : 0.0;
        r[j] = bi - ax;
        if constexpr (REG) pr[j] = dv[j] * r[j];
        else pr[j] = own ? dinv[i] * r[j] : 0.0;
        rz += r[j] * pr[j];
        rr += r[j] * r[j];
        bb += bi * bi;
    }
    __syncthreads();  // the initial guess in p_lds is consumed
#pragma unroll
    for (int j = 0; j < RPT; ++j) {
        const int i = tid + j * B;
        if (i < n) {
            p_lds[i] = pr[j];
            if (!REG && !use_x0) xio[i] = 0.0;
        }
    }
    rz = wave_sum(rz);
    rr = wave_sum(rr);
    bb = wave_sum(bb);
    if constexpr (NW > 1) {
        if (lane == 0) { redC[wid] = rz; redC[NW + wid] = rr; redC[2 * NW + wid] = bb; }
        __syncthreads();
        rz = rr = bb = 0.0;
#pragma unroll
        for (int w = 0; w < NW; ++w) { rz += redC[w]; rr += redC[NW + w]; bb += redC[2 * NW + w]; }
    } else {
        __syncthreads();  // p_lds complete before the first product
    }
    const double nb = sqrt(bb);
    int stop = ST_RUN;
    int64_t k = 0;
    if (bb == 0.0) {
#pragma unroll
        for (int j = 0; j < RPT; ++j) {
            if constexpr (REG) xr[j] = 0.0;
            else if (tid + j * B < n) xio[tid + j * B] = 0.0;
        }
        stop = ST_CONVERGED;
    } else if (sqrt(rr) <= red_factor * nb) {
        stop = ST_CONVERGED;
    }
    double rho = rz;
    while (stop == ST_RUN && k < maxit) {
        double q[RPT];
        double pq = 0.0;
#pragma unroll
        for (int j = 0; j < RPT; ++j) {
            double a = 0.0;
#pragma unroll
            for (int e = 0; e < W; ++e) a += v[j][e] * p_lds[c[j][e]];
            q[j] = a;
            pq += pr[j] * a;
        }
        pq = wave_sum(pq);
        double eta = 0.0;
        if constexpr (NW > 1) {
            if (lane == 0) redA[wid] = pq;
            __syncthreads();
#pragma unroll
            for (int w = 0; w < NW; ++w) eta += redA[w];
        } else {
            eta = pq;
        }
        if (chk && !finite_d(eta)) { stop = ST_NONFINITE; break; }
        if (eta <= 0.0) { stop = ST_BREAKDOWN; break; }
        const double alpha = rho / eta;
        double rzn = 0.0, rrn = 0.0;
        double z[RPT];
#pragma unroll
        for (int j = 0; j < RPT; ++j) {
            const int i = tid + j * B;
            const bool own = i < n;
            r[j] -= alpha * q[j];
            if constexpr (REG) {
                xr[j] += alpha * pr[j];
                z[j] = dv[j] * r[j];
            } else {
                if (own) xio[i] += alpha * pr[j];
                z[j] = own ? dinv[i] * r[j] : 0.0;
            }
            rzn += r[j] * z[j];
            rrn += r[j] * r[j];
        }
        rzn = wave_sum(rzn);
        rrn = wave_sum(rrn);
        if constexpr (NW > 1) {
            if (lane == 0) { redB[wid] = rzn; redB[NW + wid] = rrn; }
            __syncthreads();
            rzn = rrn = 0.0;
#pragma unroll
            for (int w = 0; w < NW; ++w) { rzn += redB[w]; rrn += redB[NW + w]; }
        }
        ++k;
        rr = rrn;
        if (chk && !finite_d(rr)) { stop = ST_NONFINITE; break; }
        if (sqrt(rr) <= red_factor * nb) { stop = ST_CONVERGED; break; }
        if (chk && !finite_d(rzn)) { stop = ST_NONFINITE; break; }
        if (rzn == 0.0) { stop = ST_BREAKDOWN; break; }
        const double beta = rzn / rho;
        rho = rzn;
#pragma unroll
        for (int j = 0; j < RPT; ++j) {
            pr[j] = z[j] + beta * pr[j];
            if (tid + j * B < n) p_lds[tid + j * B] = pr[j];
        }
        __syncthreads();
    }
    if (stop == ST_RUN) stop = ST_MAX_ITERS;
    if constexpr (REG) {
#pragma unroll
        for (int j = 0; j < RPT; ++j)
            if (tid + j * B < n) xio[tid + j * B] = xr[j];
    }
    if (tid == 0) {
        *(int32_t *)out3 = (int32_t)k;
        *(double *)((char *)out3 + 8) = nb > 0.0 ? sqrt(rr) / nb : 0.0;
        *((uint8_t *)out3 + 16) = (uint8_t)stop;
    }
}

// Whole Jacobi-BiCGSTAB of one small system in one workgroup, the steps
// and checks of the per-step solver in its order (right preconditioning,
// half-step exit x += alpha p_hat when ||s|| meets the criterion).  Thread t
// owns rows t + j*B (j < RPT): their entries and r, r_hat, p, v, x and dinv
// stay in registers; the vector the product gathers (p_hat, then s_hat) is
// mirrored in LDS.  out3: iterations (int32 at 0), relative residual
// (double at 8), status (byte 16), half step (byte 17).
template <int B, int RPT, int W>
__global__ __launch_bounds__(B) void k_small_bicgstab(int n, const int *__restrict__ rp,
                                                      const int *__restrict__ col,
                                                      const double *__restrict__ val,
                                                      const double *__restrict__ dinv,
                                                      const double *__restrict__ b,
                                                      double *__restrict__ xio, double red_factor,
                                                      int64_t maxit, int chk, void *__restrict__ out3) {
    extern __shared__ double pl[];
    __shared__ double red[2 * (B / kWave)];
    const int tid = threadIdx.x;
    int c[RPT][W];
    double a[RPT][W];
    double r[RPT], rh[RPT], p[RPT], v[RPT], x[RPT], dv[RPT];
#pragma unroll
    for (int j = 0; j < RPT; ++j) {
        const int i = tid + j * B;
        const bool own = i < n;
        dv[j] = own ? dinv[i] : 0.0;
        x[j] = own ? xio[i] : 0.0;
        const int e0 = own ? rp[i] : 0, e1 = own ? rp[i + 1] : 0;
#pragma unroll
        for (int e = 0; e < W; ++e) {
            const bool in = e0 + e < e1;
            c[j][e] = in ? col[e0 + e] : (own ? i : 0);  // padding: own row, value 0
            a[j][e] = in ? val[e0 + e] : 0.0;
        }
        if (own) pl[i] = x[j];
    }
    __syncthreads();
    double rr = 0.0, bb = 0.0;
#pragma unroll
    for (int j = 0; j < RPT; ++j) {
        const int i = tid + j * B;
        double ax = 0.0;
#pragma unroll
        for (int e = 0; e < W; ++e) ax += a[j][e] * pl[c[j][e]];
        const double bi = i < n ? b[i] : 0.0;
        r[j] = bi - ax;
        rh[j] = r[j];
        p[j] = 0.0;
        v[j] = 0.0;
        rr += r[j] * r[j];
        bb += bi * bi;
    }
    wg_sum2<B>(rr, bb, red);
    const double nb = sqrt(bb);
    const double tol = red_factor * nb;
    int stop = ST_RUN, half = 0;
    int64_t k = 0;
    if (bb == 0.0) {
#pragma unroll
        for (int j = 0; j < RPT; ++j) x[j] = 0.0;
        stop = ST_CONVERGED;
    } else if (sqrt(rr) <= tol) {
        stop = ST_CONVERGED;
    }
    double rho_old = 1.0, alpha = 1.0, omega = 1.0;
    while (stop == ST_RUN && k < maxit) {
        double rho = 0.0;
#pragma unroll
        for (int j = 0; j < RPT; ++j) rho += rh[j] * r[j];
        rho = wg_sum<B>(rho, red);
        if (chk && !finite_d(rho)) { stop = ST_NONFINITE; break; }
        if (rho == 0.0) { stop = ST_BREAKDOWN; break; }
        const double beta = (rho / rho_old) * (alpha / omega);
        __syncthreads();  // the previous product's reads of pl are done
#pragma unroll
        for (int j = 0; j < RPT; ++j) {
            p[j] = r[j] + beta * (p[j] - omega * v[j]);
            if (tid + j * B < n) pl[tid + j * B] = dv[j] * p[j];
        }
        __syncthreads();
        double rv = 0.0;
#pragma unroll
        for (int j = 0; j < RPT; ++j) {
            double q = 0.0;
#pragma unroll
            for (int e = 0; e < W; ++e) q += a[j][e] * pl[c[j][e]];
            v[j] = q;
            rv += rh[j] * q;
        }
        rv = wg_sum<B>(rv, red);
        if (chk && !finite_d(rv)) { stop = ST_NONFINITE; break; }
        if (rv == 0.0) { stop = ST_BREAKDOWN; break; }
        alpha = rho / rv;
        double ss = 0.0;
#pragma unroll
        for (int j = 0; j < RPT; ++j) {
            r[j] = r[j] - alpha * v[j];  // s
            ss += r[j] * r[j];
        }
        ++k;
        ss = wg_sum<B>(ss, red);
        if (sqrt(ss) <= tol) {
#pragma unroll
            for (int j = 0; j < RPT; ++j) x[j] += alpha * (dv[j] * p[j]);
            rr = ss;
            half = 1;
            stop = ST_CONVERGED;
            break;
        }
        __syncthreads();  // all reads of p_hat done
#pragma unroll
        for (int j = 0; j < RPT; ++j)
            if (tid + j * B < n) pl[tid + j * B] = dv[j] * r[j];
        __syncthreads();
        double tt = 0.0, ts = 0.0, t[RPT];
#pragma unroll
        for (int j = 0; j < RPT; ++j) {
            double q = 0.0;
#pragma unroll
            for (int e = 0; e < W; ++e) q += a[j][e] * pl[c[j][e]];
            t[j] = q;
            tt += q * q;
            ts += q * r[j];
        }
        wg_sum2<B>(tt, ts, red);
        if (chk && (!finite_d(tt) || !finite_d(ts))) { stop = ST_NONFINITE; break; }
        if (tt == 0.0) { stop = ST_BREAKDOWN; break; }
        omega = ts / tt;
        double rn = 0.0;
#pragma unroll
        for (int j = 0; j < RPT; ++j) {
            x[j] += alpha * (dv[j] * p[j]) + omega * (dv[j] * r[j]);
            r[j] = r[j] - omega * t[j];
            rn += r[j] * r[j];
        }
        rn = wg_sum<B>(rn, red);
        rr = rn;
        if (chk && !finite_d(rn)) { stop = ST_NONFINITE; break; }
        if (sqrt(rn) <= tol) { stop = ST_CONVERGED; break; }
        if (omega == 0.0) { stop = ST_BREAKDOWN; break; }
        rho_old = rho;
    }
    if (stop == ST_RUN) stop = ST_MAX_ITERS;
#pragma unroll
    for (int j = 0; j < RPT; ++j)
        if (tid + j * B < n) xio[tid + j * B] = x[j];
    if (tid == 0) {
        *(int32_t *)out3 = (int32_t)k;
        *(double *)((char *)out3 + 8) = nb > 0.0 ? sqrt(rr) / nb : 0.0;
        *((uint8_t *)out3 + 16) = (uint8_t)stop;
        *((uint8_t *)out3 + 17) = (uint8_t)half;
    }
}

__global__ void k_batch_jacobi(int64_t rows, const int *__restrict__ rows_sys_local_unused,
                               const int *__restrict__ rp, const int *__restrict__ col,
                               const double *__restrict__ val, const int *__restrict__ row_local,
                               double *__restrict__ dinv, int *__restrict__ bad) {
    (void)rows_sys_local_unused;
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= rows) return;
    const int li = row_local[i];
    double d = 0.0;
    bool found = false;
    for (int e = rp[i]; e < rp[i + 1]; ++e)
        if (col[e] == li) { d = val[e]; found = true; }
    if (found && d != 0.0) dinv[i] = 1.0 / d;
    else { dinv[i] = 0.0; atomicMin(bad, (int)i); }
}

__global__ void k_zero_u32(unsigned *p) { *p = 0u; }

// Fixed device scratch of mxl_batch_solve_noalloc: the work counter in the
// first 256 bytes, the spill region after it.  Each GPU that loads the
// library holds its own copy until the process ends.  Host code must not
// pass `noalloc_scratch` itself to a kernel (on the host it names a stand-in,
// not the device copy); it uses the address noalloc_scratch_init looked up.
constexpr size_t kNoAllocQueueBytes = 256;
__device__ __align__(256) unsigned char noalloc_scratch[kNoAllocScratchBytes];

namespace {
std::mutex g_noalloc_mu;
std::map<int, void *> g_noalloc_ptr;  // device -> address of that device's copy
}  // namespace

hipError_t noalloc_scratch_init(int device, void **out) {
    std::lock_guard<std::mutex> lk(g_noalloc_mu);
    auto it = g_noalloc_ptr.find(device);
    if (it != g_noalloc_ptr.end()) {
        *out = it->second;
        return hipSuccess;
    }
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(noalloc_scratch));
    if (e != hipSuccess || !ptr) {
        *out = nullptr;
        return e != hipSuccess ? e : hipErrorInvalidSymbol;
    }
    g_noalloc_ptr[device] = ptr;
    *out = ptr;
    return hipSuccess;
}

mxl_ctx *batch_ctx(const BatchImpl &B) { return B.ctx; }

}  // namespace mxl

using namespace mxl;

namespace {

size_t lds_bytes_for(int n) { return (size_t)4 * n * sizeof(double); }

// LDS bytes one workgroup of a schedule may use: all resident workgroups of
// a CU share its LDS.
int64_t lds_budget_for(const mxl_ctx *ctx, int wpc) {
    hipDeviceProp_t prop;
    size_t per_cu = 160 * 1024, per_wg = 64 * 1024;
    if (hipGetDeviceProperties(&prop, ctx->device) == hipSuccess) {
        if (prop.maxSharedMemoryPerMultiProcessor > 0) per_cu = prop.maxSharedMemoryPerMultiProcessor;
        if (prop.sharedMemPerBlock > 0) per_wg = prop.sharedMemPerBlock;
    }
    return (int64_t)std::min(per_wg, per_cu / (size_t)std::max(1, wpc)) - 2048;  // static LDS headroom
}

// Vector length of the CSR kernel's LDS vectors (x, r, p, q) for a schedule.
int lds_cap_for(const mxl_ctx *ctx, const BatchImpl &Bt, int wpc) {
    const int64_t budget = lds_budget_for(ctx, wpc);
    int cap = (int)(budget / (int64_t)(4 * sizeof(double)));
    return std::min(cap, Bt.max_n);
}

// The kernel a schedule runs: its format field, 0 choosing ELL when built.
bool use_ell(const BatchImpl &Bt, const mxl_tuning &t) { return t.format == 2 || (t.format == 0 && Bt.ell); }

// queue: the work counter (zeroed here by a kernel, not a memset, so the
// launch sequence can be captured); scr: the spill region, at least
// wgs_per_cu * num_cu * 5 * max_n doubles when any system spills, else NULL.
hipError_t launch_batch_on(const BatchImpl &Bt, const mxl_tuning &t, const mxl_criteria &c,
                           const double *b, double *x, int32_t *iters, double *rel, uint8_t *status,
                           int lds_cap, int64_t ell_budget, hipStream_t s, unsigned *queue, double *scr,
                           int use_x0 = 0) {
    const int G = t.wgs_per_cu * Bt.ctx->num_cu;
    const int *order = (const int *)(t.order ? Bt.order_big->p : Bt.order_input->p);
    hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(1), 0, s, queue);
    const int chk = c.nonfinite_check;
    const double red = c.reduction;
    const int64_t mif = c.max_iters;
    if (use_ell(Bt, t)) {
        const size_t shm = (size_t)ell_budget;
        const int64_t stride = scr ? (int64_t)5 * Bt.max_n : 0;
#define MXL_BATCH_ELL_CASE(BB)                                                                       \
    case BB:                                                                                         \
        hipLaunchKernelGGL(k_batch_pcg_ell<BB>, dim3(G), dim3(BB), shm, s, Bt.nsys,                  \
                           (const int *)Bt.sys_ptr->p, (const int64_t *)Bt.ell_off->p,              \
                           (const int *)Bt.ell_w->p, (const double *)Bt.ell_val->p,                 \
                           (const short *)Bt.ell_col->p, (const double *)Bt.dinv->p, b, x, iters,   \
                           rel, status, order, queue, red, mif, 10, chk,                            \
                           ell_budget, scr, stride, use_x0);                                        \
        break;
        switch (t.wg_size) {
            MXL_BATCH_ELL_CASE(64) MXL_BATCH_ELL_CASE(128) MXL_BATCH_ELL_CASE(256) MXL_BATCH_ELL_CASE(512)
            MXL_BATCH_ELL_CASE(1024)
        default: return hipErrorInvalidValue;
        }
#undef MXL_BATCH_ELL_CASE
        return hipGetLastError();
    }
    const size_t shm = lds_bytes_for(lds_cap);
    const int64_t stride = scr ? (int64_t)4 * Bt.max_n : 0;
#define MXL_BATCH_CASE(BB)                                                                          \
    case BB:                                                                                        \
        hipLaunchKernelGGL(k_batch_pcg<BB>, dim3(G), dim3(BB), shm, s, Bt.nsys,                     \
                           (const int *)Bt.sys_ptr->p, (const int *)Bt.row_ptr->p,                 \
                           (const int *)Bt.col->p, (const double *)Bt.val->p,                      \
                           (const double *)Bt.dinv->p, b, x, iters, rel, status, order,            \
                           queue, red, mif, 10, chk, lds_cap, scr, stride, use_x0);                \
        break;
    switch (t.wg_size) {
        MXL_BATCH_CASE(64) MXL_BATCH_CASE(128) MXL_BATCH_CASE(256) MXL_BATCH_CASE(512) MXL_BATCH_CASE(1024)
    default: return hipErrorInvalidValue;
    }
#undef MXL_BATCH_CASE
    return hipGetLastError();
}

// The handle's own queue counter and (lazily allocated) spill region.
hipError_t launch_batch(const BatchImpl &Bt, const mxl_tuning &t, const mxl_criteria &c,
                        const double *b, double *x, int32_t *iters, double *rel, uint8_t *status,
                        int lds_cap, int64_t ell_budget, hipStream_t s, int use_x0 = 0) {
    return launch_batch_on(Bt, t, c, b, x, iters, rel, status, lds_cap, ell_budget, s,
                           (unsigned *)Bt.queue->p, Bt.scratch ? (double *)Bt.scratch->p : nullptr,
                           use_x0);
}

}  // namespace

extern "C" mxl_status mxl_batch_csr_create(mxl_ctx *ctx, int64_t nsys, const int32_t *sys_ptr_host,
                                           const int32_t *sys_ptr, const int32_t *row_ptr,
                                           const int32_t *col, const double *val, int flags,
                                           mxl_op **out) try {
    (void)flags;
    if (!ctx || !out || !sys_ptr_host || nsys <= 0 || !sys_ptr || !row_ptr || !col || !val)
        return set_error(MXL_ERR_INVALID_ARG, "batch: NULL argument or nsys <= 0");
    *out = nullptr;
    auto Bt = std::make_shared<BatchImpl>();
    Bt->ctx = ctx;
    Bt->nsys = nsys;
    Bt->sys_ptr_h.assign(sys_ptr_host, sys_ptr_host + nsys + 1);
    if (Bt->sys_ptr_h[0] != 0) return set_error(MXL_ERR_INVALID_MATRIX, "sys_ptr[0] != 0");
    int max_n = 0;
    for (int64_t s = 0; s < nsys; ++s) {
        int n = Bt->sys_ptr_h[s + 1] - Bt->sys_ptr_h[s];
        if (n <= 0) return set_error(MXL_ERR_INVALID_MATRIX, "every system needs at least one row");
        max_n = std::max(max_n, n);
    }
    Bt->max_n = max_n;
    Bt->rows = Bt->sys_ptr_h[nsys];
    hipStream_t s = ctx->stream;
    int32_t nnz_h = 0;
    if (hipMemcpyAsync(&nnz_h, row_ptr + Bt->rows, 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return set_error(MXL_ERR_INVALID_ARG, "row_ptr is not readable device memory");
    Bt->nnz = nnz_h;
    mxl_status st;
    if ((st = check_device_ptr(ctx, sys_ptr, (nsys + 1) * 4, "sys_ptr")) != MXL_OK) return st;
    if ((st = check_device_ptr(ctx, row_ptr, (Bt->rows + 1) * 4, "row_ptr")) != MXL_OK) return st;
    if ((st = check_device_ptr(ctx, col, Bt->nnz * 4, "col")) != MXL_OK) return st;
    if ((st = check_device_ptr(ctx, val, Bt->nnz * 8, "val")) != MXL_OK) return st;
    auto borrow = [](const void *p, size_t b) {
        auto d = std::make_shared<DevBuf>();
        d->p = const_cast<void *>(p);
        d->bytes = b;
        return d;
    };
    Bt->sys_ptr = borrow(sys_ptr, (nsys + 1) * 4);
    Bt->row_ptr = borrow(row_ptr, (Bt->rows + 1) * 4);
    Bt->col = borrow(col, Bt->nnz * 4);
    Bt->val = borrow(val, Bt->nnz * 8);
    auto alloc = [](size_t bytes) -> BufPtr {
        auto d = std::make_shared<DevBuf>();
        if (hipMalloc(&d->p, bytes ? bytes : 16) != hipSuccess) return nullptr;
        d->bytes = bytes;
        d->owned = true;
        return d;
    };
    Bt->dinv = alloc(Bt->rows * 8);
    Bt->order_input = alloc(nsys * 4);
    Bt->order_big = alloc(nsys * 4);
    Bt->queue = alloc(64);
    auto rowloc = alloc(Bt->rows * 4);
    auto bad = alloc(4);
    if (!Bt->dinv || !Bt->order_input || !Bt->order_big || !Bt->queue || !rowloc || !bad)
        return set_error(MXL_ERR_OUT_OF_MEMORY, "batch workspace");
    std::vector<int32_t> ord(nsys), loc(Bt->rows);
    std::iota(ord.begin(), ord.end(), 0);
    if (hipMemcpyAsync(Bt->order_input->p, ord.data(), nsys * 4, hipMemcpyHostToDevice, s) != hipSuccess)
        return set_error(MXL_ERR_DEVICE, "upload order");
    std::vector<int32_t> big(ord);
    std::stable_sort(big.begin(), big.end(), [&](int a, int b) {
        return Bt->sys_ptr_h[a + 1] - Bt->sys_ptr_h[a] > Bt->sys_ptr_h[b + 1] - Bt->sys_ptr_h[b];
    });
    for (int64_t sy = 0; sy < nsys; ++sy)
        for (int32_t r = Bt->sys_ptr_h[sy]; r < Bt->sys_ptr_h[sy + 1]; ++r) loc[r] = r - Bt->sys_ptr_h[sy];
    int init = INT_MAX;
    if (hipMemcpyAsync(Bt->order_big->p, big.data(), nsys * 4, hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(rowloc->p, loc.data(), Bt->rows * 4, hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(bad->p, &init, 4, hipMemcpyHostToDevice, s) != hipSuccess)
        return set_error(MXL_ERR_DEVICE, "upload batch tables");
    hipLaunchKernelGGL(k_batch_jacobi, dim3((unsigned)((Bt->rows + 255) / 256)), dim3(256), 0, s, Bt->rows,
                       nullptr, (const int *)row_ptr, col, val, (const int *)rowloc->p,
                       (double *)Bt->dinv->p, (int *)bad->p);
    int badh = INT_MAX;
    if (hipMemcpyAsync(&badh, bad->p, 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return set_error(MXL_ERR_DEVICE, "batch jacobi");
    if (badh != INT_MAX)
        return set_error(MXL_ERR_ZERO_DIAG, "row " + std::to_string(badh) + " has a missing or zero diagonal");
    // Row lengths on the host: canonical row_ptr, and the per-system ELL
    // layout when it stays compact (<= 1.5 x the stored entries) and local
    // columns fit int16.
    std::vector<int32_t> rp_h((size_t)Bt->rows + 1);
    if (hipMemcpyAsync(rp_h.data(), row_ptr, ((size_t)Bt->rows + 1) * 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return set_error(MXL_ERR_DEVICE, "read row_ptr");
    if (rp_h[0] != 0) return set_error(MXL_ERR_INVALID_MATRIX, "row_ptr[0] != 0");
    for (int64_t r = 0; r < Bt->rows; ++r)
        if (rp_h[r + 1] < rp_h[r]) return set_error(MXL_ERR_INVALID_MATRIX, "row_ptr decreases at row " + std::to_string(r));
    std::vector<int32_t> w_h(nsys);
    std::vector<int64_t> off_h(nsys);
    int64_t slots = 0;
    int w_max = 0;
    for (int64_t sy = 0; sy < nsys; ++sy) {
        int w = 0;
        for (int32_t r = Bt->sys_ptr_h[sy]; r < Bt->sys_ptr_h[sy + 1]; ++r) w = std::max(w, rp_h[r + 1] - rp_h[r]);
        w_h[sy] = w;
        w_max = std::max(w_max, w);
        off_h[sy] = slots;
        slots += ((int64_t)w * (Bt->sys_ptr_h[sy + 1] - Bt->sys_ptr_h[sy]) + 1) / 2 * 2;
    }
    const bool ell = max_n <= 32767 && (double)slots <= 1.5 * (double)Bt->nnz + 64.0 * (double)nsys;
    if (ell) {
        Bt->ell_val = alloc((size_t)slots * 8);
        Bt->ell_col = alloc((size_t)slots * 2);
        Bt->ell_off = alloc((size_t)nsys * 8);
        Bt->ell_w = alloc((size_t)nsys * 4);
        if (!Bt->ell_val || !Bt->ell_col || !Bt->ell_off || !Bt->ell_w)
            return set_error(MXL_ERR_OUT_OF_MEMORY, "batch ELL copy");
        if (hipMemcpyAsync(Bt->ell_off->p, off_h.data(), (size_t)nsys * 8, hipMemcpyHostToDevice, s) != hipSuccess ||
            hipMemcpyAsync(Bt->ell_w->p, w_h.data(), (size_t)nsys * 4, hipMemcpyHostToDevice, s) != hipSuccess)
            return set_error(MXL_ERR_DEVICE, "upload ELL tables");
        Bt->ell = true;
        Bt->w_max = w_max;
        Bt->ell_slots = slots;
    }
    badh = INT_MAX;
    if (hipMemcpyAsync(bad->p, &badh, 4, hipMemcpyHostToDevice, s) != hipSuccess)
        return set_error(MXL_ERR_DEVICE, "upload flag");
    hipLaunchKernelGGL(k_batch_to_ell, dim3((unsigned)nsys), dim3(256), 0, s, sys_ptr, row_ptr, col, val,
                       ell ? (const int64_t *)Bt->ell_off->p : nullptr, ell ? (const int *)Bt->ell_w->p : nullptr,
                       ell ? (double *)Bt->ell_val->p : nullptr, ell ? (short *)Bt->ell_col->p : nullptr,
                       (int *)bad->p);
    if (hipMemcpyAsync(&badh, bad->p, 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return set_error(MXL_ERR_DEVICE, "batch column check");
    if (badh != INT_MAX)
        return set_error(MXL_ERR_INVALID_MATRIX, "row " + std::to_string(badh) + " has a column outside its system");
    auto *op = new mxl_op;
    op->kind = MXL_OP_BATCH;
    op->bat = Bt;
    *out = op;
    return MXL_OK;
} catch (...) {
    return mxl::abi_exception(__func__);
}

static const BatchImpl *batch_of(const mxl_op *op) {
    return op && op->kind == MXL_OP_BATCH ? op->bat.get() : nullptr;
}

static mxl_status batch_args(const BatchImpl &Bt, const double *b, double *x, const int32_t *iters,
                             const double *rel, const uint8_t *status) {
    mxl_status st;
    const mxl_ctx *c = Bt.ctx;
    if ((st = check_device_ptr(c, b, Bt.rows * 8, "b")) != MXL_OK) return st;
    if ((st = check_device_ptr(c, x, Bt.rows * 8, "x")) != MXL_OK) return st;
    if ((st = check_device_ptr(c, iters, Bt.nsys * 4, "iters")) != MXL_OK) return st;
    if ((st = check_device_ptr(c, rel, Bt.nsys * 8, "rel_res")) != MXL_OK) return st;
    if ((st = check_device_ptr(c, status, Bt.nsys, "status")) != MXL_OK) return st;
    if ((const void *)b == (const void *)x) return set_error(MXL_ERR_INVALID_ARG, "b and x alias");
    return MXL_OK;
}

// Dynamic LDS above 64 KB needs the kernel's attribute raised first.
#define MXL_ALLOW_LDS(KERN, WG, SHM)                                                                    \
    [&]() -> hipError_t {                                                                               \
        if ((SHM) <= 64 * 1024) return hipSuccess;                                                      \
        const int v_ = (int)(SHM);                                                                      \
        switch (WG) {                                                                                   \
        case 64: return hipFuncSetAttribute((const void *)KERN<64>, hipFuncAttributeMaxDynamicSharedMemorySize, v_);   \
        case 128: return hipFuncSetAttribute((const void *)KERN<128>, hipFuncAttributeMaxDynamicSharedMemorySize, v_); \
        case 256: return hipFuncSetAttribute((const void *)KERN<256>, hipFuncAttributeMaxDynamicSharedMemorySize, v_); \
        case 512: return hipFuncSetAttribute((const void *)KERN<512>, hipFuncAttributeMaxDynamicSharedMemorySize, v_); \
        default: return hipFuncSetAttribute((const void *)KERN<1024>, hipFuncAttributeMaxDynamicSharedMemorySize, v_); \
        }                                                                                               \
    }()

// What a schedule needs: its kernel, that kernel's LDS, and the spill region
// (doubles) when the largest system does not fit in LDS.
struct SchedPlan {
    bool ell = false;
    int cap = 0;
    int64_t ell_budget = 0;
    int64_t spill_elems = 0;
};

static mxl_status plan_schedule(const BatchImpl &Bt, const mxl_tuning &t, SchedPlan &p) {
    if (t.wg_size != 64 && t.wg_size != 128 && t.wg_size != 256 && t.wg_size != 512 && t.wg_size != 1024)
        return set_error(MXL_ERR_INVALID_ARG, "wg_size must be 64, 128, 256, 512 or 1024");
    if (t.wgs_per_cu < 1 || t.wgs_per_cu > 32 || (t.order != 0 && t.order != 1))
        return set_error(MXL_ERR_INVALID_ARG, "wgs_per_cu in 1..32, order 0 or 1");
    if (t.format < 0 || t.format > 2) return set_error(MXL_ERR_INVALID_ARG, "format must be 0, 1 or 2");
    if (t.format == 2 && !Bt.ell)
        return set_error(MXL_ERR_NOT_IMPLEMENTED, "this batch has no compact ELL copy (format 2)");
    p.ell = use_ell(Bt, t);
    p.cap = lds_cap_for(Bt.ctx, Bt, t.wgs_per_cu);
    // the ELL kernel's LDS: at most what the largest system can use
    p.ell_budget = std::min(lds_budget_for(Bt.ctx, t.wgs_per_cu),
                            (int64_t)Bt.max_n * (40 + 10 * (int64_t)Bt.w_max));
    if (p.cap < 1 || p.ell_budget < 40) return set_error(MXL_ERR_INVALID_ARG, "schedule leaves no LDS per workgroup");
    const bool spill = p.ell ? (int64_t)40 * Bt.max_n > p.ell_budget : p.cap < Bt.max_n;
    // systems above the LDS capacity run from a global scratch slice per workgroup
    p.spill_elems = spill ? (int64_t)t.wgs_per_cu * Bt.ctx->num_cu * 5 * Bt.max_n : 0;
    return MXL_OK;
}

static mxl_status allow_lds(const SchedPlan &p, const mxl_tuning &t) {
    hipError_t e = p.ell ? MXL_ALLOW_LDS(k_batch_pcg_ell, t.wg_size, (size_t)p.ell_budget)
                         : MXL_ALLOW_LDS(k_batch_pcg, t.wg_size, lds_bytes_for(p.cap));
    if (e != hipSuccess) return set_error(MXL_ERR_DEVICE, std::string("LDS attribute: ") + hipGetErrorString(e));
    return MXL_OK;
}

static mxl_status run_schedule(BatchImpl &Bt, const mxl_tuning &t, const mxl_criteria &c,
                               const double *b, double *x, int32_t *iters, double *rel,
                               uint8_t *status) {
    SchedPlan p;
    mxl_status st;
    if ((st = plan_schedule(Bt, t, p)) != MXL_OK) return st;
    if (p.spill_elems > 0 && Bt.scratch_elems < p.spill_elems) {
        auto d = std::make_shared<DevBuf>();
        if (hipMalloc(&d->p, p.spill_elems * 8) != hipSuccess)
            return set_error(MXL_ERR_OUT_OF_MEMORY, "batch scratch");
        d->bytes = p.spill_elems * 8;
        d->owned = true;
        Bt.scratch = d;
        Bt.scratch_elems = p.spill_elems;
    }
    if ((st = allow_lds(p, t)) != MXL_OK) return st;
    hipError_t e = launch_batch(Bt, t, c, b, x, iters, rel, status, p.cap, p.ell_budget, Bt.ctx->stream);
    if (e != hipSuccess) return set_error(MXL_ERR_DEVICE, std::string("batched launch: ") + hipGetErrorString(e));
    return MXL_OK;
}

static mxl_tuning default_tuning() {
    mxl_tuning t;
    t.wg_size = 256;
    t.wgs_per_cu = 2;
    t.order = 0;
    t.format = 0;
    return t;
}

extern "C" mxl_status mxl_batch_solve(const mxl_op *Bop, const mxl_criteria *crit, const mxl_tuning *tuning,
                                      const double *b, double *x, int32_t *iters, double *rel_res,
                                      uint8_t *status) try {
    BatchImpl *Bt = const_cast<BatchImpl *>(batch_of(Bop));
    if (!Bt || !crit) return set_error(MXL_ERR_INVALID_ARG, "batch operator and criteria required");
    if (!(crit->reduction >= 0.0)) return set_error(MXL_ERR_INVALID_ARG, "reduction must be >= 0");
    mxl_status st;
    if ((st = batch_args(*Bt, b, x, iters, rel_res, status)) != MXL_OK) return st;
    mxl_tuning t = tuning ? *tuning : (Bt->tuned ? Bt->best : default_tuning());
    if ((st = run_schedule(*Bt, t, *crit, b, x, iters, rel_res, status)) != MXL_OK) return st;
    if (hipStreamSynchronize(Bt->ctx->stream) != hipSuccess)
        return set_error(MXL_ERR_DEVICE, "batched solve");
    return MXL_OK;
} catch (...) {
    return mxl::abi_exception(__func__);
}

extern "C" mxl_status mxl_batch_solve_noalloc(const mxl_op *Bop, const mxl_criteria *crit,
                                              const mxl_tuning *tuning, const double *b, double *x,
                                              int32_t *iters, double *rel_res, uint8_t *status) try {
    BatchImpl *Bt = const_cast<BatchImpl *>(batch_of(Bop));
    if (!Bt || !crit) return set_error(MXL_ERR_INVALID_ARG, "batch operator and criteria required");
    if (!(crit->reduction >= 0.0)) return set_error(MXL_ERR_INVALID_ARG, "reduction must be >= 0");
    mxl_status st;
    if ((st = batch_args(*Bt, b, x, iters, rel_res, status)) != MXL_OK) return st;
    const mxl_tuning t = tuning ? *tuning : (Bt->tuned ? Bt->best : default_tuning());
    SchedPlan p;
    if ((st = plan_schedule(*Bt, t, p)) != MXL_OK) return st;
    const size_t need = kNoAllocQueueBytes + (size_t)p.spill_elems * 8;
    if (need > kNoAllocScratchBytes)
        return set_error(MXL_ERR_INVALID_ARG,
                         "schedule needs " + std::to_string(need) + " bytes of scratch; the static limit is " +
                             std::to_string(kNoAllocScratchBytes) + " (fewer workgroups per CU spill less)");
    char *base = (char *)Bt->ctx->noalloc_scratch;
    if (!base) return set_error(MXL_ERR_DEVICE, "static scratch address not available on this device");
    if ((st = allow_lds(p, t)) != MXL_OK) return st;
    double *spill = p.spill_elems > 0 ? (double *)(base + kNoAllocQueueBytes) : nullptr;
    hipError_t e = launch_batch_on(*Bt, t, *crit, b, x, iters, rel_res, status, p.cap, p.ell_budget,
                                   Bt->ctx->stream, (unsigned *)base, spill);
    if (e != hipSuccess) return set_error(MXL_ERR_DEVICE, std::string("batched launch: ") + hipGetErrorString(e));
    return MXL_OK;
} catch (...) {
    return mxl::abi_exception(__func__);
}

extern "C" mxl_status mxl_batch_autotune(const mxl_op *Bop, const mxl_criteria *crit, const double *b,
                                         double *x_scratch, int reps, mxl_tuning *best_out,
                                         double *best_ms) try {
    BatchImpl *Bt = const_cast<BatchImpl *>(batch_of(Bop));
    if (!Bt || !crit || reps < 1) return set_error(MXL_ERR_INVALID_ARG, "batch operator, criteria, reps >= 1");
    mxl_status st;
    if ((st = check_device_ptr(Bt->ctx, b, Bt->rows * 8, "b")) != MXL_OK) return st;
    if ((st = check_device_ptr(Bt->ctx, x_scratch, Bt->rows * 8, "x_scratch")) != MXL_OK) return st;
    hipStream_t s = Bt->ctx->stream;
    void *it = nullptr, *rl = nullptr, *stt = nullptr;
    if (hipMalloc(&it, Bt->nsys * 4) != hipSuccess || hipMalloc(&rl, Bt->nsys * 8) != hipSuccess ||
        hipMalloc(&stt, Bt->nsys) != hipSuccess) {
        (void)hipFree(it); (void)hipFree(rl); (void)hipFree(stt);
        return set_error(MXL_ERR_OUT_OF_MEMORY, "autotune buffers");
    }
    hipEvent_t e0, e1;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    double best = 1e300;
    mxl_tuning bt = default_tuning();
    st = MXL_OK;
    std::vector<int> fmts{1};
    if (Bt->ell) fmts.push_back(2);
    for (int fmt : fmts) {
    if (st != MXL_OK) break;
    for (int B : {64, 128, 256, 512}) {
        for (int wpc : {1, 2, 4, 8}) {
            if (B * wpc > 2048) continue;  // at most 32 waves per CU
            for (int ord : {0, 1}) {
                mxl_tuning t{B, wpc, ord, fmt};
                std::vector<float> ts;
                for (int r = 0; r < reps + 1 && st == MXL_OK; ++r) {
                    (void)hipEventRecord(e0, s);
                    st = run_schedule(*Bt, t, *crit, b, x_scratch, (int32_t *)it, (double *)rl, (uint8_t *)stt);
                    (void)hipEventRecord(e1, s);
                    (void)hipEventSynchronize(e1);
                    float ms = 0.f;
                    (void)hipEventElapsedTime(&ms, e0, e1);
                    if (r > 0) ts.push_back(ms);  // the first run warms caches
                }
                if (st != MXL_OK) break;
                std::sort(ts.begin(), ts.end());
                double med = ts[ts.size() / 2];
                if (med < best) { best = med; bt = t; }
            }
            if (st != MXL_OK) break;
        }
        if (st != MXL_OK) break;
    }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipFree(it); (void)hipFree(rl); (void)hipFree(stt);
    if (st != MXL_OK) return st;
    Bt->best = bt;
    Bt->tuned = true;
    if (best_out) *best_out = bt;
    if (best_ms) *best_ms = best;
    return MXL_OK;
} catch (...) {
    return mxl::abi_exception(__func__);
}

namespace mxl {

// A single system (a solver's matrix) viewed as a batch of one, for the
// one-launch CG path of small systems.
std::shared_ptr<BatchImpl> batch_from_matrix(const MatrixImpl &A, const void *dinv) {
    auto Bt = std::make_shared<BatchImpl>();
    Bt->ctx = A.ctx;
    Bt->nsys = 1;
    Bt->rows = A.nrows;
    Bt->nnz = A.nnz;
    Bt->sys_ptr_h = {0, (int32_t)A.nrows};
    Bt->max_n = (int)A.nrows;
    Bt->row_ptr = A.row_ptr;
    Bt->col = A.col;
    Bt->val = A.val;
    auto alloc = [](size_t bytes) -> BufPtr {
        auto d = std::make_shared<DevBuf>();
        if (hipMalloc(&d->p, bytes ? bytes : 16) != hipSuccess) return nullptr;
        d->bytes = bytes;
        d->owned = true;
        return d;
    };
    Bt->sys_ptr = alloc(8);
    Bt->order_input = alloc(4);
    Bt->order_big = Bt->order_input;
    Bt->queue = alloc(64);
    Bt->scratch = nullptr;
    if (!Bt->sys_ptr || !Bt->order_input || !Bt->queue) return nullptr;
    if (dinv) {
        Bt->dinv = std::make_shared<DevBuf>();
        Bt->dinv->p = const_cast<void *>(dinv);
        Bt->dinv->bytes = A.nrows * 8;
    } else {
        Bt->dinv = alloc(A.nrows * 8);
        if (!Bt->dinv || launch_fill(MXL_F64, A.nrows, 1.0, Bt->dinv->p, A.ctx->stream) != hipSuccess) return nullptr;
    }
    int32_t sp[2] = {0, (int32_t)A.nrows}, z = 0;
    if (hipMemcpyAsync(Bt->sys_ptr->p, sp, 8, hipMemcpyHostToDevice, A.ctx->stream) != hipSuccess ||
        hipMemcpyAsync(Bt->order_input->p, &z, 4, hipMemcpyHostToDevice, A.ctx->stream) != hipSuccess ||
        hipStreamSynchronize(A.ctx->stream) != hipSuccess)
        return nullptr;
    return Bt;
}

// The whole CG of one system in one workgroup (x holds the initial guess).
// Register-cached single-workgroup shapes: (threads, rows per thread,
// entries per row).  The first that holds the system is used.
struct SmallShape {
    int B, RPT, W;
};
static const SmallShape kSmallShapes[] = {{64, 2, 8}, {512, 8, 5}, {512, 4, 8}, {256, 4, 32}};

static hipError_t launch_small(const SmallShape &sh, int n, const BatchImpl &Bt, const mxl_criteria &c,
                               const double *b, double *x, void *out3) {
    const size_t shm = (size_t)n * sizeof(double);
    hipStream_t s = Bt.ctx->stream;
#define MXL_SMALL(BB, RR, WW)                                                                        \
    if (sh.B == BB && sh.RPT == RR && sh.W == WW) {                                                  \
        hipLaunchKernelGGL((k_small_pcg<BB, RR, WW, (BB == 64)>), dim3(1), dim3(BB), shm, s, n,       \
                           (const int *)Bt.row_ptr->p, (const int *)Bt.col->p,                       \
                           (const double *)Bt.val->p, (const double *)Bt.dinv->p, b, x,              \
                           c.reduction, c.max_iters, c.nonfinite_check, 1, out3);                    \
        return hipGetLastError();                                                                    \
    }
    MXL_SMALL(64, 2, 8)
    MXL_SMALL(512, 8, 5)
    MXL_SMALL(512, 4, 8)
    MXL_SMALL(256, 4, 32)
#undef MXL_SMALL
    return hipErrorInvalidValue;
}

// The whole BiCGSTAB of one system in one workgroup, when a register shape
// holds it (returns false otherwise; the caller then runs the per-step
// solver).  x holds the initial guess.
static const SmallShape kSmallBiShapes[] = {{64, 2, 8}, {256, 4, 8}, {512, 8, 5}};

bool batch_single_bicgstab(BatchImpl &Bt, const mxl_criteria &c, const double *b, double *x, void *out3,
                           int64_t *iters, double *rel, int *stop, int *half, mxl_status *st) {
    *st = MXL_OK;
    const int n = (int)Bt.rows;
    constexpr int NS = (int)(sizeof(kSmallBiShapes) / sizeof(kSmallBiShapes[0]));
    if (Bt.small_bi_shape < 0) {
        std::vector<int32_t> rp(n + 1);
        if (hipMemcpyAsync(rp.data(), Bt.row_ptr->p, (n + 1) * 4, hipMemcpyDeviceToHost, Bt.ctx->stream) != hipSuccess ||
            hipStreamSynchronize(Bt.ctx->stream) != hipSuccess) {
            *st = set_error(MXL_ERR_DEVICE, "row pointer read");
            return true;
        }
        int maxlen = 0;
        for (int i = 0; i < n; ++i) maxlen = std::max(maxlen, rp[i + 1] - rp[i]);
        Bt.small_bi_shape = NS;
        for (int k = 0; k < NS; ++k)
            if (n <= kSmallBiShapes[k].B * kSmallBiShapes[k].RPT && maxlen <= kSmallBiShapes[k].W &&
                (size_t)n * 8 <= 60 * 1024) {
                Bt.small_bi_shape = k;
                break;
            }
    }
    if (Bt.small_bi_shape >= NS) return false;
    const SmallShape &sh = kSmallBiShapes[Bt.small_bi_shape];
    const size_t shm = (size_t)n * sizeof(double);
    hipStream_t s = Bt.ctx->stream;
#define MXL_SMALL_BI(BB, RR, WW)                                                                     \
    if (sh.B == BB && sh.RPT == RR && sh.W == WW)                                                    \
        hipLaunchKernelGGL((k_small_bicgstab<BB, RR, WW>), dim3(1), dim3(BB), shm, s, n,              \
                           (const int *)Bt.row_ptr->p, (const int *)Bt.col->p,                       \
                           (const double *)Bt.val->p, (const double *)Bt.dinv->p, b, x,              \
                           c.reduction, c.max_iters, c.nonfinite_check, out3);
    MXL_SMALL_BI(64, 2, 8)
    MXL_SMALL_BI(256, 4, 8)
    MXL_SMALL_BI(512, 8, 5)
#undef MXL_SMALL_BI
    hipError_t e = hipGetLastError();
    char h[24];
    if (e == hipSuccess) e = hipMemcpyAsync(h, out3, 24, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        *st = set_error(MXL_ERR_DEVICE, std::string("small BiCGSTAB: ") + hipGetErrorString(e));
        return true;
    }
    int32_t it;
    memcpy(&it, h, 4);
    memcpy(rel, h + 8, 8);
    *iters = it;
    *stop = (uint8_t)h[16];
    *half = (uint8_t)h[17];
    return true;
}

mxl_status batch_single_solve(BatchImpl &Bt, const mxl_criteria &c, const double *b, double *x,
                              void *out3, int64_t *iters, double *rel, int *stop) {
    const int n = (int)Bt.rows;
    if (Bt.small_shape < 0) {  // pick once: the maximum row length needs the row pointers
        std::vector<int32_t> rp(n + 1);
        if (hipMemcpyAsync(rp.data(), Bt.row_ptr->p, (n + 1) * 4, hipMemcpyDeviceToHost, Bt.ctx->stream) != hipSuccess ||
            hipStreamSynchronize(Bt.ctx->stream) != hipSuccess)
            return set_error(MXL_ERR_DEVICE, "row pointer read");
        int maxlen = 0;
        for (int i = 0; i < n; ++i) maxlen = std::max(maxlen, rp[i + 1] - rp[i]);
        Bt.small_shape = (int)(sizeof(kSmallShapes) / sizeof(kSmallShapes[0]));
        for (int k = 0; k < (int)(sizeof(kSmallShapes) / sizeof(kSmallShapes[0])); ++k)
            if (n <= kSmallShapes[k].B * kSmallShapes[k].RPT && maxlen <= kSmallShapes[k].W &&
                (size_t)n * 8 <= 60 * 1024) {
                Bt.small_shape = k;
                break;
            }
    }
    if (Bt.small_shape < (int)(sizeof(kSmallShapes) / sizeof(kSmallShapes[0]))) {
        hipError_t e = launch_small(kSmallShapes[Bt.small_shape], n, Bt, c, b, x, out3);
        if (e != hipSuccess) return set_error(MXL_ERR_DEVICE, std::string("small CG: ") + hipGetErrorString(e));
        char h[24];
        if (hipMemcpyAsync(h, out3, 24, hipMemcpyDeviceToHost, Bt.ctx->stream) != hipSuccess ||
            hipStreamSynchronize(Bt.ctx->stream) != hipSuccess)
            return set_error(MXL_ERR_DEVICE, "small CG read-back");
        int32_t it;
        memcpy(&it, h, 4);
        memcpy(rel, h + 8, 8);
        *iters = it;
        *stop = (uint8_t)h[16];
        return MXL_OK;
    }
    mxl_tuning t{1024, 1, 0, 1};
    const int cap = lds_cap_for(Bt.ctx, Bt, 1);
    if (cap < Bt.max_n && !Bt.scratch) {
        auto d = std::make_shared<DevBuf>();
        if (hipMalloc(&d->p, (size_t)Bt.ctx->num_cu * 4 * Bt.max_n * 8) != hipSuccess)
            return set_error(MXL_ERR_OUT_OF_MEMORY, "single-launch scratch");
        d->bytes = (size_t)Bt.ctx->num_cu * 4 * Bt.max_n * 8;
        d->owned = true;
        Bt.scratch = d;
        Bt.scratch_elems = (int64_t)Bt.ctx->num_cu * 4 * Bt.max_n;
    }
    const size_t shm = lds_bytes_for(cap);
    if (shm > 64 * 1024 &&
        hipFuncSetAttribute((const void *)k_batch_pcg<1024>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm) != hipSuccess)
        return set_error(MXL_ERR_DEVICE, "LDS attribute");
    int32_t *dit = (int32_t *)out3;
    double *drel = (double *)((char *)out3 + 8);
    uint8_t *dst = (uint8_t *)((char *)out3 + 16);
    hipError_t e = launch_batch(Bt, t, c, b, x, dit, drel, dst, cap, 0, Bt.ctx->stream, 1);
    if (e != hipSuccess) return set_error(MXL_ERR_DEVICE, std::string("single-launch CG: ") + hipGetErrorString(e));
    char h[24];
    if (hipMemcpyAsync(h, out3, 24, hipMemcpyDeviceToHost, Bt.ctx->stream) != hipSuccess ||
        hipStreamSynchronize(Bt.ctx->stream) != hipSuccess)
        return set_error(MXL_ERR_DEVICE, "single-launch read-back");
    int32_t it;
    memcpy(&it, h, 4);
    memcpy(rel, h + 8, 8);
    *iters = it;
    *stop = (uint8_t)h[16];
    return MXL_OK;
}

}  // namespace mxl
