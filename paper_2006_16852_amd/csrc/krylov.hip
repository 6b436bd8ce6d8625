// krylov.hip -- fused vector kernels of the Krylov solvers: the CG step
// (x += alpha p, r -= alpha q, z = D^{-1} r with r.z and r.r in the same
// pass), the search-direction update, the BiCGSTAB steps, point-Jacobi
// application, the iterative-refinement scaling/correction and utilities.
//
// Every reduction is deterministic: each workgroup reduces a contiguous
// range in a fixed tree and publishes one partial; the kernel that needs
// the scalar reduces the partials in its prologue, identically in every
// workgroup (device_common.hpp).  Dot products of FP32 vectors multiply
// exactly in FP64 and accumulate in FP64.
#include <initializer_list>

#include "device_common.hpp"
#include "internal.hpp"

namespace mxl {

// Contiguous [i0, i1) range of logical workgroup L, walked 256 at a time so
// each wave's accesses are coalesced.
#define MXL_RANGE(n)                                                 \
    const int L = blockIdx.x;                                        \
    int64_t tb_, te_;                                                \
    int ts_;                                                         \
    band_walk(((n) + kWG - 1) / kWG, blockIdx.x, gridDim.x, tb_, te_, ts_);

// Element loop of one workgroup over its tiles of 256 (see band_walk).
#define MXL_FOR(i, n)                                   \
    for (int64_t t_ = tb_; t_ < te_; t_ += ts_)         \
        if (const int64_t i = t_ * kWG + threadIdx.x; i < (n))

#define MXL_LEAD (blockIdx.x == 0 && threadIdx.x == 0)

// The same walk for B-thread workgroups (tiles of B elements or chunks).
#define MXL_RANGE_B(n, B)                                            \
    const int L = blockIdx.x;                                        \
    int64_t tb_, te_;                                                \
    int ts_;                                                         \
    band_walk(((n) + (B) - 1) / (B), blockIdx.x, gridDim.x, tb_, te_, ts_);

template <typename V>
__device__ __forceinline__ double prec_z(const V *dinv, int64_t i, V r) {
    return dinv ? (double)dinv[i] * (double)r : (double)r;
}

// ------------------------------------------------------- one-shot finalise
template <int NV>
__global__ __launch_bounds__(kWG) void k_finalize(const double *__restrict__ partials, int nslots,
                                                  SolverState *st, int op, int k, int max_iters,
                                                  double *hist) {
    double tot[NV];
    gather_all<NV>(partials, nslots, tot, op == FIN_NORMS ? 0x2u : 0u);
    if (threadIdx.x == 0) {
        double s4[4] = {0, 0, 0, 0};
#pragma unroll
        for (int j = 0; j < NV && j < 4; ++j) s4[j] = tot[j];
        finalize(op, st, s4, k, max_iters, hist);
    }
}

// ---------------------------------------------------------------- CG
template <typename V>
__global__ __launch_bounds__(kWG) void k_cg_init(int64_t n, const V *__restrict__ b,
                                                 const V *__restrict__ r, V *__restrict__ p,
                                                 const V *__restrict__ dinv,
                                                 double *__restrict__ parts) {
    MXL_RANGE(n)
    double rz = 0.0, rr = 0.0, bb = 0.0;
    MXL_FOR(i, n) {
        V ri = r[i];
        double z = prec_z(dinv, i, ri);
        p[i] = (V)z;
        rz += (double)ri * z;
        rr += (double)ri * (double)ri;
        bb += (double)b[i] * (double)b[i];
    }
    double v[3] = {rz, rr, bb};
    publish<3>(v, parts, L);
}

// The update kernels first load their operands for the workgroup's first
// kPf tiles, then reduce the partials of the previous kernel (gather_all):
// the loads do not depend on that scalar, so their latency overlaps the
// reduction instead of every workgroup paying the two in sequence.
constexpr int kPf = 2;

#define MXL_PF_INDEX_B(u, cnt, B)                               \
    const int64_t t_##u = tb_ + (int64_t)(u) * ts_;             \
    const int64_t i_##u = t_##u * (B) + threadIdx.x;            \
    const bool in_##u = t_##u < te_ && i_##u < (cnt);
#define MXL_PF_INDEX(u, cnt) MXL_PF_INDEX_B(u, cnt, kWG)

// The CG update kernels run B = kCgWG threads per workgroup: every workgroup
// of a consumer reduces all partials of the kernel before it, so fewer,
// larger workgroups read fewer partials in all (half of the 256-thread
// workgroups' traffic, and the gather of 4,096 partials costs each launch
// about 4 us less on the 128^3 system).
constexpr int kCgWG = 512;

// A thread of the CG update kernels owns chunks of E consecutive elements:
// E = 2 for FP32 vectors (one 8-byte load per array, as wide as an FP64
// element), E = 1 for FP64.  Chunk c holds elements cE .. cE + E - 1; the
// last chunk may run past n and is then loaded and stored element-wise.
template <typename V, int E>
struct Chunk {
    V v[E];
};

template <typename V, int E>
__device__ __forceinline__ Chunk<V, E> fill_chunk(V a) {
    Chunk<V, E> o;
#pragma unroll
    for (int e = 0; e < E; ++e) o.v[e] = a;
    return o;
}

template <typename V, int E>
__device__ __forceinline__ Chunk<V, E> ld_chunk(const V *__restrict__ p, int64_t c, int64_t n) {
    Chunk<V, E> o;
    const int64_t i0 = c * E;
    if constexpr (E == 1) {
        o.v[0] = p[i0];
    } else {
        typedef V VE __attribute__((ext_vector_type(E)));
        if (i0 + E <= n) {
            const VE t = *(const VE *)(p + i0);
#pragma unroll
            for (int e = 0; e < E; ++e) o.v[e] = t[e];
        } else {
#pragma unroll
            for (int e = 0; e < E; ++e) o.v[e] = i0 + e < n ? p[i0 + e] : (V)0;
        }
    }
    return o;
}

template <typename V, int E>
__device__ __forceinline__ void st_chunk(V *__restrict__ p, int64_t c, int64_t n, const Chunk<V, E> &o) {
    const int64_t i0 = c * E;
    if constexpr (E == 1) {
        p[i0] = o.v[0];
    } else {
        typedef V VE __attribute__((ext_vector_type(E)));
        if (i0 + E <= n) {
            VE t;
#pragma unroll
            for (int e = 0; e < E; ++e) t[e] = o.v[e];
            *(VE *)(p + i0) = t;
        } else {
#pragma unroll
            for (int e = 0; e < E; ++e)
                if (i0 + e < n) p[i0 + e] = o.v[e];
        }
    }
}

// Consumes p.q (fused into the SpMV): alpha = rho_{k-1} / p.q, then
// r -= alpha q and the reductions r.z, r.r.  The matching x += alpha p is
// applied by k_cg_pupdate, which reads p anyway, so p is read once less.
template <typename V, int E>
__global__ __launch_bounds__(kCgWG) void k_cg_update(int64_t n, V *__restrict__ r, const V *__restrict__ q,
                                                   const V *__restrict__ dinv, SolverState *st,
                                                   const double *__restrict__ pq_parts, int pq_slots,
                                                   double *__restrict__ parts, int k) {
    if (st->stop) {
        if (MXL_LEAD) st->ustop = 1;
        return;
    }
    typedef Chunk<V, E> CV;
    const int64_t nc = (n + E - 1) / E;
    MXL_RANGE_B(nc, kCgWG)
    CV rv[kPf], qv[kPf], dv[kPf];
#pragma unroll
    for (int u = 0; u < kPf; ++u) {
        MXL_PF_INDEX_B(u, nc, kCgWG)
        rv[u] = in_u ? ld_chunk<V, E>(r, i_u, n) : fill_chunk<V, E>(0);
        qv[u] = in_u ? ld_chunk<V, E>(q, i_u, n) : fill_chunk<V, E>(0);
        dv[u] = in_u && dinv ? ld_chunk<V, E>(dinv, i_u, n) : fill_chunk<V, E>(1);
    }
    double eta[1];
    gather_all<1, kCgWG>(pq_parts, pq_slots, eta);
    const bool chk = st->nonfinite_check != 0;
    const bool nonfin = chk && !finite_d(eta[0]);
    if (nonfin || eta[0] <= 0.0) {  // not positive definite along p
        if (MXL_LEAD) {
            st->stop = nonfin ? ST_NONFINITE : ST_BREAKDOWN;
            st->ustop = 1;
            st->iters = k - 1;
            st->eta = eta[0];
        }
        return;
    }
    const double alpha = st->rho2[(k - 1) & 1] / eta[0];
    if (MXL_LEAD) {
        st->alpha = alpha;
        st->eta = eta[0];
        st->ustop = 0;
    }
    double rz = 0.0, rr = 0.0;
    auto step = [&](int64_t c, const CV &r0, const CV &q0, const CV &d0) {
        CV ro;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            V ri;
            if constexpr (sizeof(V) == 8) ri = r0.v[e] - alpha * q0.v[e];
            else ri = (V)((double)r0.v[e] - alpha * (double)q0.v[e]);
            ro.v[e] = ri;
            if (E == 1 || c * E + e < n) {
                const double z = dinv ? (double)d0.v[e] * (double)ri : (double)ri;
                rz += (double)ri * z;
                rr += (double)ri * (double)ri;
            }
        }
        st_chunk<V, E>(r, c, n, ro);
    };
#pragma unroll
    for (int u = 0; u < kPf; ++u) {
        MXL_PF_INDEX_B(u, nc, kCgWG)
        if (in_u) step(i_u, rv[u], qv[u], dv[u]);
    }
    for (int64_t t_ = tb_ + (int64_t)kPf * ts_; t_ < te_; t_ += ts_)
        if (const int64_t c = t_ * kCgWG + threadIdx.x; c < nc)
            step(c, ld_chunk<V, E>(r, c, n), ld_chunk<V, E>(q, c, n),
                 dinv ? ld_chunk<V, E>(dinv, c, n) : fill_chunk<V, E>(1));
    double v[2] = {rz, rr};
    publish<2, kCgWG>(v, parts, L);
}

// Consumes r.z and r.r: x += alpha p (alpha from k_cg_update), the
// criterion of iteration k, then p = z + beta p unless the solve stops.
template <typename V, int E>
__global__ __launch_bounds__(kCgWG) void k_cg_pupdate(int64_t n, V *__restrict__ x, const V *__restrict__ r,
                                                    V *__restrict__ p, const V *__restrict__ dinv,
                                                    SolverState *st, const double *__restrict__ parts,
                                                    int slots, int k, double *hist) {
    // k_cg_update saw an earlier stop or broke down: x is not advanced.  The
    // stop this kernel decides goes to st->stop, which it never reads.
    if (st->ustop) return;
    typedef Chunk<V, E> CV;
    const int64_t nc = (n + E - 1) / E;
    MXL_RANGE_B(nc, kCgWG)
    (void)L;
    CV xv[kPf], rv[kPf], pv[kPf], dv[kPf];
#pragma unroll
    for (int u = 0; u < kPf; ++u) {
        MXL_PF_INDEX_B(u, nc, kCgWG)
        xv[u] = in_u ? ld_chunk<V, E>(x, i_u, n) : fill_chunk<V, E>(0);
        rv[u] = in_u ? ld_chunk<V, E>(r, i_u, n) : fill_chunk<V, E>(0);
        pv[u] = in_u ? ld_chunk<V, E>(p, i_u, n) : fill_chunk<V, E>(0);
        dv[u] = in_u && dinv ? ld_chunk<V, E>(dinv, i_u, n) : fill_chunk<V, E>(1);
    }
    double t[2];
    gather_all<2, kCgWG>(parts, slots, t);
    const double rz = t[0], rr = t[1];
    const double alpha = st->alpha;
    const bool chk = st->nonfinite_check != 0;
    const double nb = sqrt(st->nb2);
    int stop = ST_RUN;
    if (chk && !finite_d(rr)) stop = ST_NONFINITE;
    else if (sqrt(rr) <= st->red * nb) stop = ST_CONVERGED;
    else if (chk && !finite_d(rz)) stop = ST_NONFINITE;
    else if (rz == 0.0) stop = ST_BREAKDOWN;
    const double beta = rz / st->rho2[(k - 1) & 1];
    const bool run = stop == ST_RUN;
    auto step = [&](int64_t c, const CV &x0, const CV &r0, const CV &p0, const CV &d0) {
        CV xo, po;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            if constexpr (sizeof(V) == 8) xo.v[e] = x0.v[e] + alpha * p0.v[e];
            else xo.v[e] = (V)((double)x0.v[e] + alpha * (double)p0.v[e]);
            po.v[e] = (V)((dinv ? (double)d0.v[e] * (double)r0.v[e] : (double)r0.v[e]) + beta * (double)p0.v[e]);
        }
        st_chunk<V, E>(x, c, n, xo);
        if (run) st_chunk<V, E>(p, c, n, po);
    };
#pragma unroll
    for (int u = 0; u < kPf; ++u) {
        MXL_PF_INDEX_B(u, nc, kCgWG)
        if (in_u) step(i_u, xv[u], rv[u], pv[u], dv[u]);
    }
    for (int64_t t_ = tb_ + (int64_t)kPf * ts_; t_ < te_; t_ += ts_)
        if (const int64_t c = t_ * kCgWG + threadIdx.x; c < nc)
            step(c, ld_chunk<V, E>(x, c, n), run ? ld_chunk<V, E>(r, c, n) : fill_chunk<V, E>(0),
                 ld_chunk<V, E>(p, c, n),
                 run && dinv ? ld_chunk<V, E>(dinv, c, n) : fill_chunk<V, E>(1));
    if (MXL_LEAD) {
        st->rr = rr;
        st->iters = k;
        if (hist) hist[k] = sqrt(rr) / nb;
        if (stop != ST_RUN) st->stop = stop;
        else {
            st->rho2[k & 1] = rz;
            st->beta = beta;
        }
    }
}

// ---------------------------------------------------------------- BiCGSTAB
template <typename V>
__global__ __launch_bounds__(kWG) void k_bi_init(int64_t n, const V *__restrict__ b,
                                                 const V *__restrict__ r, V *__restrict__ rhat,
                                                 V *__restrict__ p, V *__restrict__ v,
                                                 double *__restrict__ parts) {
    MXL_RANGE(n)
    double rr = 0.0, bb = 0.0;
    MXL_FOR(i, n) {
        V ri = r[i];
        rhat[i] = ri;
        p[i] = (V)0;
        v[i] = (V)0;
        rr += (double)ri * (double)ri;
        bb += (double)b[i] * (double)b[i];
    }
    double s[3] = {rr, rr, bb};  // rhat = r, so rhat.r = r.r
    publish<3>(s, parts, L);
}

// Consumes [r.r, rhat.r] of iteration k-1: its criterion (k >= 2), then the
// loop head of iteration k: rho_k, beta, p = r + beta (p - omega v),
// p_hat = D^{-1} p (not stored when phat is NULL: block Jacobi forms it).
template <typename V>
__global__ __launch_bounds__(kWG) void k_bi_pupdate(int64_t n, const V *__restrict__ r,
                                                    V *__restrict__ p, const V *__restrict__ v,
                                                    V *__restrict__ phat, const V *__restrict__ dinv,
                                                    SolverState *st, const double *__restrict__ parts,
                                                    int slots, int k, double *hist) {
    if (st->stop) return;
    MXL_RANGE(n)
    V rv[kPf], pv[kPf], vv[kPf], dv[kPf];
#pragma unroll
    for (int u = 0; u < kPf; ++u) {
        MXL_PF_INDEX(u, n)
        rv[u] = in_u ? r[i_u] : (V)0;
        pv[u] = in_u ? p[i_u] : (V)0;
        vv[u] = in_u ? v[i_u] : (V)0;
        dv[u] = in_u && dinv ? dinv[i_u] : (V)1;
    }
    double t[3];
    gather_all<3>(parts, slots, t);
    const double rr = t[0], rho = t[1];
    const bool chk = st->nonfinite_check != 0;
    const double nb = sqrt(st->nb2);
    const double omega_prev = st->omega, alpha_prev = st->alpha;
    int stop = ST_RUN;
    if (k >= 2) {
        if (chk && !finite_d(rr)) stop = ST_NONFINITE;
        else if (sqrt(rr) <= st->red * nb) stop = ST_CONVERGED;
        else if (omega_prev == 0.0) stop = ST_BREAKDOWN;
    }
    if (stop == ST_RUN) {
        if (chk && !finite_d(rho)) stop = ST_NONFINITE;
        else if (rho == 0.0) stop = ST_BREAKDOWN;
    }
    const double beta = (rho / st->rho2[(k - 1) & 1]) * (alpha_prev / omega_prev);
    if (MXL_LEAD) {
        if (k >= 2) {
            st->rr = rr;
            if (hist) hist[k - 1] = sqrt(rr) / nb;
        }
        if (stop != ST_RUN) {
            st->stop = stop;
            st->iters = k - 1;
        } else {
            st->rho2[k & 1] = rho;
            st->beta = beta;
        }
    }
    if (stop != ST_RUN) return;
    auto step = [&](int64_t i, V r0, V p0, V v0, V d0) {
        const V pi = (V)((double)r0 + beta * ((double)p0 - omega_prev * (double)v0));
        p[i] = pi;
        if (phat) phat[i] = (V)(dinv ? (double)d0 * (double)pi : (double)pi);
    };
#pragma unroll
    for (int u = 0; u < kPf; ++u) {
        MXL_PF_INDEX(u, n)
        if (in_u) step(i_u, rv[u], pv[u], vv[u], dv[u]);
    }
    for (int64_t t_ = tb_ + (int64_t)kPf * ts_; t_ < te_; t_ += ts_)
        if (const int64_t i = t_ * kWG + threadIdx.x; i < n) step(i, r[i], p[i], v[i], dinv ? dinv[i] : (V)1);
}

// Consumes rhat.v (fused into the SpMV): alpha = rho_k / rhat.v; s = r - alpha v
// and s_hat = D^{-1} s (not stored when shat is NULL).
template <typename V>
__global__ __launch_bounds__(kWG) void k_bi_supdate(int64_t n, const V *__restrict__ r,
                                                    const V *__restrict__ v, V *__restrict__ s,
                                                    V *__restrict__ shat,
                                                    const V *__restrict__ dinv, SolverState *st,
                                                    const double *__restrict__ rv_parts, int rv_slots,
                                                    double *__restrict__ parts, int k) {
    if (st->stop) return;
    MXL_RANGE(n)
    V r_[kPf], v_[kPf], d_[kPf];
#pragma unroll
    for (int u = 0; u < kPf; ++u) {
        MXL_PF_INDEX(u, n)
        r_[u] = in_u ? r[i_u] : (V)0;
        v_[u] = in_u ? v[i_u] : (V)0;
        d_[u] = in_u && dinv ? dinv[i_u] : (V)1;
    }
    double rv[1];
    gather_all<1>(rv_parts, rv_slots, rv);
    const bool chk = st->nonfinite_check != 0;
    const bool nonfin = chk && !finite_d(rv[0]);
    if (nonfin || rv[0] == 0.0) {
        if (MXL_LEAD) {
            st->stop = nonfin ? ST_NONFINITE : ST_BREAKDOWN;
            st->iters = k - 1;
        }
        return;
    }
    const double alpha = st->rho2[k & 1] / rv[0];
    if (MXL_LEAD) st->alpha = alpha;
    double ss = 0.0;
    auto step = [&](int64_t i, V r0, V v0, V d0) {
        const V si = (V)((double)r0 - alpha * (double)v0);
        s[i] = si;
        if (shat) shat[i] = (V)(dinv ? (double)d0 * (double)si : (double)si);
        ss += (double)si * (double)si;
    };
#pragma unroll
    for (int u = 0; u < kPf; ++u) {
        MXL_PF_INDEX(u, n)
        if (in_u) step(i_u, r_[u], v_[u], d_[u]);
    }
    for (int64_t t_ = tb_ + (int64_t)kPf * ts_; t_ < te_; t_ += ts_)
        if (const int64_t i = t_ * kWG + threadIdx.x; i < n) step(i, r[i], v[i], dinv ? dinv[i] : (V)1);
    double a[1] = {ss};
    publish<1>(a, parts, L);
}

// Consumes s.s: half-step criterion; otherwise t.s and t.t.
template <typename V>
__global__ __launch_bounds__(kWG) void k_bi_tdots(int64_t n, const V *__restrict__ t,
                                                  const V *__restrict__ s, SolverState *st,
                                                  const double *__restrict__ ss_parts, int ss_slots,
                                                  double *__restrict__ parts, int k, double *hist) {
    if (st->stop) return;
    MXL_RANGE(n)
    V t_v[kPf], s_v[kPf];
#pragma unroll
    for (int u = 0; u < kPf; ++u) {
        MXL_PF_INDEX(u, n)
        t_v[u] = in_u ? t[i_u] : (V)0;
        s_v[u] = in_u ? s[i_u] : (V)0;
    }
    double ss[1];
    gather_all<1>(ss_parts, ss_slots, ss);
    const double nb = sqrt(st->nb2);
    if (sqrt(ss[0]) <= st->red * nb) {
        if (MXL_LEAD) {
            st->stop = ST_HALF;
            st->half = 1;
            st->iters = k;
            st->rr = ss[0];
            if (hist) hist[k] = sqrt(ss[0]) / nb;
        }
        return;
    }
    double ts = 0.0, tt = 0.0;
    auto step = [&](V t0, V s0) {
        const double ti = (double)t0;
        ts += ti * (double)s0;
        tt += ti * ti;
    };
#pragma unroll
    for (int u = 0; u < kPf; ++u) {
        MXL_PF_INDEX(u, n)
        if (in_u) step(t_v[u], s_v[u]);
    }
    for (int64_t t_ = tb_ + (int64_t)kPf * ts_; t_ < te_; t_ += ts_)
        if (const int64_t i = t_ * kWG + threadIdx.x; i < n) step(t[i], s[i]);
    double a[2] = {ts, tt};
    publish<2>(a, parts, L);
}

// Consumes t.s and t.t: omega; x += alpha p_hat + omega s_hat, r = s - omega t,
// then [r.r, rhat.r] for the next loop head.  At a half-step stop of this
// iteration it applies x += alpha p_hat only.
template <typename V>
__global__ __launch_bounds__(kWG) void k_bi_xupdate(int64_t n, V *__restrict__ x, V *__restrict__ r,
                                                    const V *__restrict__ phat,
                                                    const V *__restrict__ shat,
                                                    const V *__restrict__ s, const V *__restrict__ t,
                                                    const V *__restrict__ rhat, SolverState *st,
                                                    const double *__restrict__ ts_parts, int ts_slots,
                                                    double *__restrict__ parts, int k) {
    const int mode = st->stop;
    const double alpha = st->alpha;
    if (mode == ST_HALF) {
        if (st->iters != k) return;
        MXL_RANGE(n)
        MXL_FOR(i, n)
            x[i] = (V)((double)x[i] + alpha * (double)phat[i]);
        return;
    }
    if (mode != ST_RUN) return;
    MXL_RANGE(n)
    V xv[kPf], ph[kPf], sh[kPf], sv[kPf], tv[kPf], rh[kPf];
#pragma unroll
    for (int u = 0; u < kPf; ++u) {
        MXL_PF_INDEX(u, n)
        xv[u] = in_u ? x[i_u] : (V)0;
        ph[u] = in_u ? phat[i_u] : (V)0;
        sh[u] = in_u ? shat[i_u] : (V)0;
        sv[u] = in_u ? s[i_u] : (V)0;
        tv[u] = in_u ? t[i_u] : (V)0;
        rh[u] = in_u ? rhat[i_u] : (V)0;
    }
    double d[2];
    gather_all<2>(ts_parts, ts_slots, d);
    const double ts = d[0], tt = d[1];
    const bool chk = st->nonfinite_check != 0;
    const bool nonfin = chk && (!finite_d(tt) || !finite_d(ts));
    if (nonfin || tt == 0.0) {
        if (MXL_LEAD) {
            st->stop = nonfin ? ST_NONFINITE : ST_BREAKDOWN;
            st->iters = k;
        }
        return;
    }
    const double omega = ts / tt;
    if (MXL_LEAD) st->omega = omega;
    double rr = 0.0, rhr = 0.0;
    auto step = [&](int64_t i, V x0, V ph0, V sh0, V s0, V t0, V rh0) {
        x[i] = (V)((double)x0 + alpha * (double)ph0 + omega * (double)sh0);
        const V ri = (V)((double)s0 - omega * (double)t0);
        r[i] = ri;
        rr += (double)ri * (double)ri;
        rhr += (double)rh0 * (double)ri;
    };
#pragma unroll
    for (int u = 0; u < kPf; ++u) {
        MXL_PF_INDEX(u, n)
        if (in_u) step(i_u, xv[u], ph[u], sh[u], sv[u], tv[u], rh[u]);
    }
    for (int64_t t_ = tb_ + (int64_t)kPf * ts_; t_ < te_; t_ += ts_)
        if (const int64_t i = t_ * kWG + threadIdx.x; i < n) step(i, x[i], phat[i], shat[i], s[i], t[i], rhat[i]);
    double a[3] = {rr, rhr, 0.0};
    publish<3>(a, parts, L);
}

// ----------------------------------------------------- small utilities
template <typename V>
__global__ void k_jacobi_apply(int64_t n, V alpha, const V *__restrict__ dinv,
                               const V *__restrict__ b, V beta, V *__restrict__ x) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        V v = alpha * (dinv[i] * b[i]);
        x[i] = beta == (V)0 ? v : v + beta * x[i];
    }
}

template <typename V>
__global__ void k_copy(int64_t n, const V *__restrict__ a, V *__restrict__ b) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        b[i] = a[i];
}

template <typename V>
__global__ void k_fill(int64_t n, V v, V *__restrict__ b) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        b[i] = v;
}

__global__ void k_state_init(SolverState *st, double red, int chk) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    st->rho2[0] = st->rho2[1] = 0.0;
    st->alpha = st->omega = st->beta = st->eta = 0.0;
    st->rr = st->nb2 = 0.0;
    st->red = red;
    for (int j = 0; j < 4; ++j) st->sums[j] = 0.0;
    st->stop = ST_RUN;
    st->iters = 0;
    st->nonfinite_check = chk;
    st->half = 0;
    st->ustop = 0;
}

// ||r||_2^2 and ||r||_inf in one pass (iterative refinement outer step).
__global__ __launch_bounds__(kWG) void k_ir_norms(int64_t n, const double *__restrict__ r,
                                                  double *__restrict__ parts) {
    MXL_RANGE(n)
    double rr = 0.0, mx = 0.0;
    MXL_FOR(i, n) {
        double v = r[i];
        rr += v * v;
        double a = fabs(v);
        mx = a > mx ? a : mx;
    }
    double a[2] = {rr, mx};
    publish<2>(a, parts, L, 0x2u);
}

__global__ void k_ir_scale(int64_t n, const double *__restrict__ r,
                           const SolverState *__restrict__ st, float *__restrict__ r32) {
    const double s = st->sums[1];
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        r32[i] = (float)(r[i] / s);
}

__global__ void k_ir_correct(int64_t n, double *__restrict__ x, const float *__restrict__ d,
                             const SolverState *__restrict__ st) {
    const double s = st->sums[1];
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        x[i] += s * (double)d[i];
}

// STREAM-style reference kernels: b = a, c = a + alpha*b, and a.b, with
// 16-byte accesses, walked like every other streaming kernel (band_walk).
typedef double dvec2 __attribute__((ext_vector_type(2)));
__global__ __launch_bounds__(kWG) void k_stream_copy(int64_t n2, const dvec2 *__restrict__ a,
                                                     dvec2 *__restrict__ b) {
    MXL_RANGE(n2)
    MXL_FOR(i, n2) b[i] = __builtin_nontemporal_load(a + i);
}

__global__ __launch_bounds__(kWG) void k_stream_triad(int64_t n2, const dvec2 *__restrict__ a,
                                                      const dvec2 *__restrict__ b, double alpha,
                                                      dvec2 *__restrict__ c) {
    MXL_RANGE(n2)
    MXL_FOR(i, n2) {
        dvec2 x = __builtin_nontemporal_load(a + i), y = __builtin_nontemporal_load(b + i);
        c[i] = x + alpha * y;
    }
}

__global__ __launch_bounds__(kWG) void k_stream_dot(int64_t n2, const dvec2 *__restrict__ a,
                                                    const dvec2 *__restrict__ b,
                                                    double *__restrict__ parts) {
    MXL_RANGE(n2)
    double acc = 0.0;
    MXL_FOR(i, n2) {
        dvec2 x = __builtin_nontemporal_load(a + i), y = __builtin_nontemporal_load(b + i);
        acc += x.x * y.x + x.y * y.y;
    }
    double v[1] = {acc};
    publish<1>(v, parts, L);
}

// Read-only sum of a with ordinary (temporal) loads, `sweeps` times over the
// array in one launch.  Ordinary loads allocate in L2 and the last-level
// cache, and each workgroup re-reads its own band, so over an array whose
// per-XCD band fits L2 (or whose whole fits the last-level cache) every
// sweep after the first measures that cache's read bandwidth; one sweep over
// a large array calibrates the fetch counters for ordinary loads (the other
// stream kernels stream with nontemporal loads).
__global__ __launch_bounds__(kWG) void k_stream_read(int64_t n2, const dvec2 *__restrict__ a, int sweeps,
                                                     double *__restrict__ parts) {
    MXL_RANGE(n2)
    double acc = 0.0;
    for (int sw = 0; sw < sweeps; ++sw) {
        MXL_FOR(i, n2) {
            const dvec2 x = a[i];
            acc += x.x + x.y;
        }
    }
    double v[1] = {acc};
    publish<1>(v, parts, L);
}

// Sweeps of the cached read: enough to read 2^28 values in one launch.
int stream_read_sweeps(int64_t n) {
    const int64_t target = (int64_t)1 << 28;
    return n >= target ? 1 : (int)((target + n - 1) / n);
}

hipError_t launch_stream(const mxl_ctx *ctx, int op, int64_t n, const double *a, const double *b,
                         double *c, hipStream_t s) {
    const int64_t n2 = n / 2;
    const int G = ctx->num_cu * 8;
    switch (op) {
    case 0: hipLaunchKernelGGL(k_stream_copy, dim3(G), dim3(kWG), 0, s, n2, (const dvec2 *)a, (dvec2 *)c); break;
    case 1: hipLaunchKernelGGL(k_stream_triad, dim3(G), dim3(kWG), 0, s, n2, (const dvec2 *)a, (const dvec2 *)b, 0.5, (dvec2 *)c); break;
    case 2: hipLaunchKernelGGL(k_stream_dot, dim3(G), dim3(kWG), 0, s, n2, (const dvec2 *)a, (const dvec2 *)b, c); break;
    case 3: hipLaunchKernelGGL(k_stream_read, dim3(G), dim3(kWG), 0, s, n2, (const dvec2 *)a,
                               stream_read_sweeps(n), c);
        break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// Evicts the caches by reading a buffer larger than the last-level cache.
// Reading leaves clean lines behind, so the timed kernel that follows does
// not pay for writing back the flush's own data.  The store happens only if
// the XOR of a thread's words equals `key`, which keeps the loads alive; it
// writes into the buffer itself, whose contents never matter.
__global__ void k_flush(int4 *buf, int64_t n, int key) {
    int acc = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int4 v = buf[i];
        acc ^= v.x ^ v.y ^ v.z ^ v.w;
    }
    if (acc == key) buf[(int64_t)blockIdx.x * blockDim.x + threadIdx.x] = make_int4(acc, 0, 0, 0);
}

// ============================================================ host side
int vec_grid(const mxl_ctx *ctx, int64_t n) {
    int64_t want = (n + kWG * 4 - 1) / (kWG * 4);
    int cap = ctx->num_cu * 8 < kMaxGrid ? ctx->num_cu * 8 : kMaxGrid;
    if (want < 1) want = 1;
    return (int)(want < cap ? want : cap);
}

static unsigned gs(int64_t n) {
    int64_t g = (n + 255) / 256;
    if (g < 1) g = 1;
    if (g > 8192) g = 8192;
    return (unsigned)g;
}

// Launch KERNEL<double> or KERNEL<float>; arguments of type `VP` are cast.
#define MXL_LAUNCH_V(dtype, KERNEL, GRID, ...)                                                     \
    do {                                                                                           \
        if ((dtype) == MXL_F64) {                                                                  \
            using V = double;                                                                      \
            hipLaunchKernelGGL(KERNEL<V>, dim3(GRID), dim3(kWG), 0, s, __VA_ARGS__);               \
        } else {                                                                                   \
            using V = float;                                                                       \
            hipLaunchKernelGGL(KERNEL<V>, dim3(GRID), dim3(kWG), 0, s, __VA_ARGS__);               \
        }                                                                                          \
    } while (0)

hipError_t launch_finalize(int nv, const double *parts, int slots, SolverState *st, int op, int k,
                           int max_iters, double *hist, hipStream_t s) {
    if (nv == 2)
        hipLaunchKernelGGL(k_finalize<2>, dim3(1), dim3(kWG), 0, s, parts, slots, st, op, k, max_iters, hist);
    else
        hipLaunchKernelGGL(k_finalize<3>, dim3(1), dim3(kWG), 0, s, parts, slots, st, op, k, max_iters, hist);
    return hipGetLastError();
}

hipError_t launch_jacobi_apply(int dtype, int64_t n, double alpha, const void *dinv, const void *b,
                               double beta, void *x, hipStream_t s) {
    if (n == 0) return hipSuccess;
    if (dtype == MXL_F64)
        hipLaunchKernelGGL(k_jacobi_apply<double>, dim3(gs(n)), dim3(256), 0, s, n, alpha,
                           (const double *)dinv, (const double *)b, beta, (double *)x);
    else
        hipLaunchKernelGGL(k_jacobi_apply<float>, dim3(gs(n)), dim3(256), 0, s, n, (float)alpha,
                           (const float *)dinv, (const float *)b, (float)beta, (float *)x);
    return hipGetLastError();
}

hipError_t launch_copy(int dtype, int64_t n, const void *src, void *dst, hipStream_t s) {
    if (n == 0) return hipSuccess;
    if (dtype == MXL_F64)
        hipLaunchKernelGGL(k_copy<double>, dim3(gs(n)), dim3(256), 0, s, n, (const double *)src, (double *)dst);
    else
        hipLaunchKernelGGL(k_copy<float>, dim3(gs(n)), dim3(256), 0, s, n, (const float *)src, (float *)dst);
    return hipGetLastError();
}

hipError_t launch_fill(int dtype, int64_t n, double v, void *dst, hipStream_t s) {
    if (n == 0) return hipSuccess;
    if (dtype == MXL_F64)
        hipLaunchKernelGGL(k_fill<double>, dim3(gs(n)), dim3(256), 0, s, n, v, (double *)dst);
    else
        hipLaunchKernelGGL(k_fill<float>, dim3(gs(n)), dim3(256), 0, s, n, (float)v, (float *)dst);
    return hipGetLastError();
}

hipError_t launch_state_init(SolverState *st, double red, int nonfinite_check, hipStream_t s) {
    hipLaunchKernelGGL(k_state_init, dim3(1), dim3(64), 0, s, st, red, nonfinite_check);
    return hipGetLastError();
}

hipError_t cg_init(const mxl_ctx *ctx, int dtype, int64_t n, const void *b, const void *r, void *p,
                   const void *dinv, double *parts, hipStream_t s) {
    MXL_LAUNCH_V(dtype, k_cg_init, vec_grid(ctx, n), n, (const V *)b, (const V *)r, (V *)p,
                 (const V *)dinv, parts);
    return hipGetLastError();
}

// FP32 vectors move two elements per thread when every vector the kernel
// touches is 8-byte aligned (a caller's x may be an odd offset view).
static bool aligned8(std::initializer_list<const void *> ps) {
    for (const void *p : ps)
        if (p && ((uintptr_t)p & 7u)) return false;
    return true;
}

// Grid of the CG update kernels (kCgWG threads): four tiles per workgroup,
// at most four workgroups per CU.  k_cg_update publishes this many partials.
int cg_update_grid(const mxl_ctx *ctx, int64_t n) {
    int64_t want = (n + (int64_t)kCgWG * 4 - 1) / ((int64_t)kCgWG * 4);
    const int cap = ctx->num_cu * 4;
    if (want < 1) want = 1;
    return (int)(want < cap ? want : cap);
}

hipError_t cg_update(const mxl_ctx *ctx, int dtype, int64_t n, void *r, const void *q, const void *dinv,
                     SolverState *st, const double *pq_parts, int pq_slots, double *parts, int k,
                     hipStream_t s) {
    const dim3 g(cg_update_grid(ctx, n)), b(kCgWG);
    if (dtype == MXL_F64)
        hipLaunchKernelGGL((k_cg_update<double, 1>), g, b, 0, s, n, (double *)r, (const double *)q,
                           (const double *)dinv, st, pq_parts, pq_slots, parts, k);
    else if (aligned8({r, q, dinv}))
        hipLaunchKernelGGL((k_cg_update<float, 2>), g, b, 0, s, n, (float *)r, (const float *)q,
                           (const float *)dinv, st, pq_parts, pq_slots, parts, k);
    else
        hipLaunchKernelGGL((k_cg_update<float, 1>), g, b, 0, s, n, (float *)r, (const float *)q,
                           (const float *)dinv, st, pq_parts, pq_slots, parts, k);
    return hipGetLastError();
}

hipError_t cg_pupdate(const mxl_ctx *ctx, int dtype, int64_t n, void *x, const void *r, void *p,
                      const void *dinv, SolverState *st, const double *parts, int slots, int k,
                      double *hist, hipStream_t s) {
    const dim3 g(cg_update_grid(ctx, n)), b(kCgWG);
    if (dtype == MXL_F64)
        hipLaunchKernelGGL((k_cg_pupdate<double, 1>), g, b, 0, s, n, (double *)x, (const double *)r,
                           (double *)p, (const double *)dinv, st, parts, slots, k, hist);
    else if (aligned8({x, r, p, dinv}))
        hipLaunchKernelGGL((k_cg_pupdate<float, 2>), g, b, 0, s, n, (float *)x, (const float *)r,
                           (float *)p, (const float *)dinv, st, parts, slots, k, hist);
    else
        hipLaunchKernelGGL((k_cg_pupdate<float, 1>), g, b, 0, s, n, (float *)x, (const float *)r,
                           (float *)p, (const float *)dinv, st, parts, slots, k, hist);
    return hipGetLastError();
}

hipError_t bi_init(const mxl_ctx *ctx, int dtype, int64_t n, const void *b, const void *r,
                   void *rhat, void *p, void *v, double *parts, hipStream_t s) {
    MXL_LAUNCH_V(dtype, k_bi_init, vec_grid(ctx, n), n, (const V *)b, (const V *)r, (V *)rhat, (V *)p,
                 (V *)v, parts);
    return hipGetLastError();
}

hipError_t bi_pupdate(const mxl_ctx *ctx, int dtype, int64_t n, const void *r, void *p,
                      const void *v, void *phat, const void *dinv, SolverState *st,
                      const double *parts, int slots, int k, double *hist, hipStream_t s) {
    MXL_LAUNCH_V(dtype, k_bi_pupdate, vec_grid(ctx, n), n, (const V *)r, (V *)p, (const V *)v,
                 (V *)phat, (const V *)dinv, st, parts, slots, k, hist);
    return hipGetLastError();
}

hipError_t bi_supdate(const mxl_ctx *ctx, int dtype, int64_t n, const void *r, const void *v,
                      void *sv, void *shat, const void *dinv, SolverState *st,
                      const double *rv_parts, int rv_slots, double *parts, int k, hipStream_t s) {
    MXL_LAUNCH_V(dtype, k_bi_supdate, vec_grid(ctx, n), n, (const V *)r, (const V *)v, (V *)sv,
                 (V *)shat, (const V *)dinv, st, rv_parts, rv_slots, parts, k);
    return hipGetLastError();
}

hipError_t bi_tdots(const mxl_ctx *ctx, int dtype, int64_t n, const void *t, const void *sv,
                    SolverState *st, const double *ss_parts, int ss_slots, double *parts, int k,
                    double *hist, hipStream_t s) {
    MXL_LAUNCH_V(dtype, k_bi_tdots, vec_grid(ctx, n), n, (const V *)t, (const V *)sv, st, ss_parts,
                 ss_slots, parts, k, hist);
    return hipGetLastError();
}

hipError_t bi_xupdate(const mxl_ctx *ctx, int dtype, int64_t n, void *x, void *r, const void *phat,
                      const void *shat, const void *sv, const void *t, const void *rhat,
                      SolverState *st, const double *ts_parts, int ts_slots, double *parts, int k,
                      hipStream_t s) {
    MXL_LAUNCH_V(dtype, k_bi_xupdate, vec_grid(ctx, n), n, (V *)x, (V *)r, (const V *)phat,
                 (const V *)shat, (const V *)sv, (const V *)t, (const V *)rhat, st, ts_parts, ts_slots,
                 parts, k);
    return hipGetLastError();
}

hipError_t ir_norms(const mxl_ctx *ctx, int64_t n, const double *r, SolverState *st, double *parts,
                    hipStream_t s) {
    int G = vec_grid(ctx, n);
    hipLaunchKernelGGL(k_ir_norms, dim3(G), dim3(kWG), 0, s, n, r, parts);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_finalize(2, parts, G, st, FIN_NORMS, 0, 0, nullptr, s);
}

hipError_t ir_scale_to_f32(int64_t n, const double *r, const SolverState *st, float *r32,
                           hipStream_t s) {
    hipLaunchKernelGGL(k_ir_scale, dim3(gs(n)), dim3(256), 0, s, n, r, st, r32);
    return hipGetLastError();
}

hipError_t ir_correct(int64_t n, double *x, const float *d, const SolverState *st, hipStream_t s) {
    hipLaunchKernelGGL(k_ir_correct, dim3(gs(n)), dim3(256), 0, s, n, x, d, st);
    return hipGetLastError();
}

hipError_t launch_flush(void *buf, size_t bytes, hipStream_t s) {
    static int v = 0;
    ++v;
    int64_t n = (int64_t)(bytes / sizeof(int4));
    hipLaunchKernelGGL(k_flush, dim3(8192), dim3(256), 0, s, (int4 *)buf, n, v);
    return hipGetLastError();
}

}  // namespace mxl
