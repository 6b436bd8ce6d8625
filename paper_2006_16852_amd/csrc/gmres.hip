// gmres.hip -- restarted GMRES(m) preconditioned from the right (Krylov
// solvers of Sec. 3.1; the restart parameter and memory model of Table 2).
//
// The Arnoldi basis V (m+1 vectors of ld >= n doubles, vector after vector)
// stays resident.  Orthogonalisation is classical Gram-Schmidt with the
// re-orthogonalisation of each vector delayed by one step (the "DCGS2"
// scheme of Bielich, Langou, Thomas, Swirydowicz, Yamazaki and Boman):
// step j holds the final v_0..v_{j-1}, the candidate t_j (projected once,
// not normalised) in slot j, and u = A M^{-1} t_j.  One pass over the basis
// gives s_k = v_k . t_j, c_k = v_k . u (k < j), sigma = t_j . t_j and
// tau = t_j . u; then
//   beta = sqrt(sigma - |s|^2)      v_j = (t_j - sum s_k v_k) / beta
//   column j-1 of H += s, h_{j,j-1} = beta   (column j-1 is now final)
//   A M^{-1} v_j = (u - V (H s)) / beta      (Arnoldi relation of columns < j)
//   h_kj = (c_k - (Hs)_k) / beta,  h_jj = ((tau - s.c) / beta - (Hs)_j) / beta
//   t_{j+1} = u / beta - sum_{k<j} ((Hs)_k / beta + h_kj) v_k
//             - ((Hs)_j / beta + h_jj) v_j
// and one more pass writes v_j over t_j and t_{j+1} into slot j+1.  So every
// step reads the basis twice (a multi-dot and a multi-axpy) and still
// orthogonalises every vector twice; a modified Gram-Schmidt step reads it
// five times.  Column j-1 becomes final during step j, so the Givens
// rotation, the residual estimate and the criteria of step j-1 run there;
// a cycle ends with one more multi-dot that finalises its last column.
//
// Kernels of a step: SpMV, k_gm_dots (partials), k_gm_reduce (one
// workgroup per value), k_gm_finish (one workgroup: column update, Givens,
// criteria, coefficients), k_gm_update.  Every step kernel returns at once
// when the solve has stopped, so the host enqueues steps without reading
// the state after each one.
#include <cmath>
#include <cstring>

#include "device_common.hpp"
#include "internal.hpp"

namespace mxl {

constexpr int kGmRows = 8;              // rows per thread in the basis kernels
constexpr int kGmTile = kWG * kGmRows;  // rows per workgroup
constexpr int kGmKC = 4;                // basis vectors per multi-dot chunk (2 dots each)

// Device scalars of a GMRES solve besides SolverState.
struct GmresState {
    int32_t j;      // final columns in the current cycle
    int32_t k;      // final columns in the solve (the iteration count)
    int32_t jx;     // basis vectors combined by the cycle's closing update
    int32_t pad;
    double beta;    // norm of the current candidate after re-orthogonalisation
    double bcoef;   // coefficient of v_j in t_{j+1}
    int64_t nspmv;  // products A M^{-1} t_j of the steps (each step's finish counts its own)
};

struct GmPtrs {
    double *H;    // (m+1) x m Hessenberg matrix, column j at H + (m+1) j (final columns)
    double *Ht;   // the tentative column j of step j (before its re-orthogonalisation)
    double *R;    // the final columns after the Givens rotations
    double *cs, *sn;
    double *g;    // m+1: rotated right-hand side beta e_1
    double *sv;   // m+1: re-orthogonalisation coefficients s_k
    double *av;   // m+1: coefficients of v_k in t_{j+1}; closing combination y
    double *red;  // 2m+2: reduced dots of the current step
    GmresState *gs;
    int m;
};

size_t gm_ws_bytes(int m) {
    const size_t d = 3 * (size_t)(m + 1) * m + 2 * (size_t)m + 3 * (size_t)(m + 1) + 2 * (size_t)(m + 1);
    return d * sizeof(double) + 256;
}

static GmPtrs gm_ptrs(void *ws, int m) {
    GmPtrs P;
    P.gs = (GmresState *)ws;
    P.m = m;
    double *d = (double *)((char *)ws + 256);
    P.H = d;
    d += (size_t)(m + 1) * m;
    P.Ht = d;
    d += (size_t)(m + 1) * m;
    P.R = d;
    d += (size_t)(m + 1) * m;
    P.cs = d;
    d += m;
    P.sn = d;
    d += m;
    P.g = d;
    d += m + 1;
    P.sv = d;
    d += m + 1;
    P.av = d;
    d += m + 1;
    P.red = d;
    return P;
}

int gm_grid(int64_t n) {
    const int64_t g = (n + kGmTile - 1) / kGmTile;
    return (int)(g < 1 ? 1 : g);
}

// Thread t of a workgroup owns the row pairs (p, p+1), p = tile start +
// 512 q + 2 t, q = 0..3: one 16-byte load per pair and vector (a 1 KB
// contiguous request per wave; 8-byte loads reach only about 60% of the
// bandwidth on this access pattern).
typedef double d2 __attribute__((ext_vector_type(2)));
constexpr int kGmPairs = kGmRows / 2;
__device__ __forceinline__ int64_t gm_pair(int g, int t, int q) {
    return (int64_t)g * kGmTile + (int64_t)q * (2 * kWG) + 2 * t;
}
// Pair (i, i+1) of a vector, zeros past n; 16-byte aligned when both exist.
__device__ __forceinline__ d2 ld2(const double *p, int64_t i, int64_t n) {
    if (i + 1 < n) return *(const d2 *)(p + i);
    d2 v = {i < n ? p[i] : 0.0, 0.0};
    return v;
}
__device__ __forceinline__ d2 ld2_nt(const double *p, int64_t i, int64_t n) {
    if (i + 1 < n) return __builtin_nontemporal_load((const d2 *)(p + i));
    d2 v = {i < n ? p[i] : 0.0, 0.0};
    return v;
}
__device__ __forceinline__ void st2(double *p, int64_t i, int64_t n, d2 v) {
    if (i + 1 < n) *(d2 *)(p + i) = v;
    else if (i < n) p[i] = v[0];
}

// [v.v, b.b] partials (b optional) and z = dinv .* v (when z is given).
__global__ __launch_bounds__(kWG) void k_gm_prep(int64_t n, const double *__restrict__ v,
                                                 const double *__restrict__ b,
                                                 const double *__restrict__ dinv, double *__restrict__ z,
                                                 double *__restrict__ parts) {
    double vv = 0.0, bb = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x; i < n; i += (int64_t)gridDim.x * kWG) {
        const double vi = v[i];
        vv += vi * vi;
        if (b) bb += b[i] * b[i];
        if (z) z[i] = dinv ? dinv[i] * vi : vi;
    }
    double t[2] = {vv, bb};
    publish<2>(t, parts, blockIdx.x);
}

// Start of a cycle from the residual r held (unnormalised) in slot 0:
// g = 0, the criteria on ||r||.  first: also ||b||^2 and history[0].  Step 0
// normalises r with its own norm and sets g_0.
__global__ void k_gm_start(const double *__restrict__ parts, int slots, SolverState *st, GmPtrs P,
                           double *hist, int first) {
    double t[2];
    gather_all<2>(parts, slots, t);
    if (threadIdx.x != 0) return;
    GmresState *gs = P.gs;
    const double nb2 = first ? t[1] : st->nb2;
    if (first) {
        st->nb2 = nb2;
        st->iters = 0;
        gs->k = 0;
        gs->nspmv = 0;
    }
    const double beta = sqrt(t[0]);
    st->rr = t[0];
    gs->j = 0;
    gs->jx = 0;
    for (int i = 0; i <= P.m; ++i) P.g[i] = 0.0;
    const double nb = sqrt(nb2);
    if (first && hist) hist[0] = nb > 0.0 ? beta / nb : 0.0;
    const bool chk = st->nonfinite_check != 0;
    if (nb2 == 0.0) st->stop = ST_CONVERGED;
    else if (chk && !finite_d(beta)) st->stop = ST_NONFINITE;
    else if (beta <= st->red * nb) st->stop = ST_CONVERGED;
}

// Partials (one tile of kGmTile rows per workgroup) of s_k = V_k . t and,
// with u, c_k = V_k . u for k < j, then t.t and t.u, t = slot j.  Value
// layout: s_k at 2k, c_k at 2k+1, t.t at 2j, t.u at 2j+1; partial (v, g) at
// parts[v * G + g].
__global__ __launch_bounds__(kWG) void k_gm_dots(int64_t n, int64_t ld, const double *__restrict__ V, int j,
                                                 const double *__restrict__ u, double *__restrict__ parts,
                                                 const SolverState *st) {
    if (st->stop) return;
    __shared__ double red[2 * kGmKC][kWG];
    const int G = gridDim.x, g = blockIdx.x, t = threadIdx.x;
    const double *tj = V + (int64_t)j * ld;
    d2 tr[kGmPairs], ur[kGmPairs];
    double tt = 0.0, tu = 0.0;
#pragma unroll
    for (int q = 0; q < kGmPairs; ++q) {
        const int64_t i = gm_pair(g, t, q);
        tr[q] = ld2(tj, i, n);
        ur[q] = u ? ld2(u, i, n) : (d2)0.0;
        tt += tr[q][0] * tr[q][0] + tr[q][1] * tr[q][1];
        tu += tr[q][0] * ur[q][0] + tr[q][1] * ur[q][1];
    }
    for (int k0 = 0; k0 < j; k0 += kGmKC) {
        double acc[2 * kGmKC];
#pragma unroll
        for (int kk = 0; kk < kGmKC; ++kk) {
            acc[2 * kk] = 0.0;
            acc[2 * kk + 1] = 0.0;
            if (k0 + kk < j) {
                const double *vk = V + (int64_t)(k0 + kk) * ld;
#pragma unroll
                for (int q = 0; q < kGmPairs; ++q) {
                    const d2 v = ld2_nt(vk, gm_pair(g, t, q), n);
                    acc[2 * kk] += v[0] * tr[q][0] + v[1] * tr[q][1];
                    acc[2 * kk + 1] += v[0] * ur[q][0] + v[1] * ur[q][1];
                }
            }
        }
#pragma unroll
        for (int e = 0; e < 2 * kGmKC; ++e) red[e][t] = acc[e];
        __syncthreads();
        // thread t sums 8 of the 256 partials of value e = t / 32, then the
        // 32 lanes of that group combine by shuffles (fixed order)
        const int e = t / 32, q = t % 32;
        double s = 0.0;
#pragma unroll
        for (int f = 0; f < 8; ++f) s += red[e][q * 8 + f];
#pragma unroll
        for (int off = 16; off > 0; off >>= 1) s += __shfl_xor(s, off, kWave);
        if (q == 0 && k0 + e / 2 < j) parts[(int64_t)(2 * k0 + e) * G + g] = s;
        __syncthreads();
    }
    double v2[2] = {tt, tu};
    block_reduce<2>(v2);
    if (t == 0) {
        parts[(int64_t)(2 * j) * G + g] = v2[0];
        parts[(int64_t)(2 * j + 1) * G + g] = v2[1];
    }
}

// One workgroup per value v: the total of its G partials in a fixed order.
__global__ __launch_bounds__(kWG) void k_gm_reduce(const double *__restrict__ parts, int G, const SolverState *st,
                                                   double *__restrict__ red) {
    if (st->stop) return;
    const int v = blockIdx.x;
    double s[1] = {0.0};
    for (int g = threadIdx.x; g < G; g += kWG) s[0] += parts[(int64_t)v * G + g];
    block_reduce<1>(s);
    if (threadIdx.x == 0) red[v] = s[0];
}

// Step j's scalar work, one launch of j+2 workgroups (1 for the closing
// pass).  Workgroups l = 0..j form (Hs)_l = sum_{k<j} h_lk s_k over the
// final columns (column j-1 = its tentative values + s, h_{j,j-1} = beta)
// and the tentative column j: h_lj = (c_l - (Hs)_l) / beta (l < j),
// h_jj = ((tau - s.c) / beta - (Hs)_j) / beta, with the update's
// coefficients.  The last workgroup writes the final column j-1, rotates it
// (the earlier rotations and a new one), and applies the residual estimate
// and the criteria in the oracle's order; for j = 0 it sets g_0 = beta.
// Every workgroup recomputes beta = sqrt(t.t - |s|^2) itself.  No workgroup
// reads what another one writes: final columns go to H, tentative ones to
// Ht, and column j-1 is read from Ht.
__global__ __launch_bounds__(kWG) void k_gm_finish(int j, int last, SolverState *st, GmPtrs P, double *hist) {
    if (st->stop) return;
    __shared__ double col[kGmMaxKrylov + 1], rc[kGmMaxKrylov], rs[kGmMaxKrylov];
    GmresState *gs = P.gs;
    const int64_t ldh = P.m + 1;
    const int t = threadIdx.x;
    const bool givens = last || (int)blockIdx.x == j + 1;
    double part[2] = {0.0, 0.0};  // |s|^2, s.c
    for (int k = t; k < j; k += kWG) {
        const double sk = P.red[2 * k];
        part[0] += sk * sk;
        if (!givens) part[1] += sk * P.red[2 * k + 1];
    }
    block_reduce<2>(part);
    __shared__ double bsh[2];
    if (t == 0) {
        const double b2 = P.red[2 * j] - part[0];
        // b2 <= 0: the candidate lies in the span (happy breakdown); NaN stays NaN
        bsh[0] = b2 <= 0.0 ? 0.0 : sqrt(b2);
        bsh[1] = part[1];
    }
    __syncthreads();
    const double beta = bsh[0];
    if (givens) {
        if (j == 0) {
            if (t == 0) {
                P.g[0] = beta;
                if (!last) gs->nspmv += 1;
            }
            return;
        }
        // final column j-1 and the earlier rotations, staged in LDS
        const double *ht = P.Ht + ldh * (j - 1);
        for (int k = t; k < j; k += kWG) {
            col[k] = ht[k] + P.red[2 * k];
            if (k < j - 1) {
                rc[k] = P.cs[k];
                rs[k] = P.sn[k];
            }
        }
        if (t == 0) col[j] = beta;
        __syncthreads();
        double *h = P.H + ldh * (j - 1), *r = P.R + ldh * (j - 1);
        for (int k = t; k <= j; k += kWG) h[k] = col[k];
        if (t != 0) return;
        if (!last) gs->nspmv += 1;  // this step's SpMV ran (the solve had not stopped)
        const int c0 = j - 1;
        for (int i = 0; i < c0; ++i) {
            const double a = col[i], c = col[i + 1];
            col[i] = rc[i] * a + rs[i] * c;
            col[i + 1] = -rs[i] * a + rc[i] * c;
        }
        const double a = col[c0];
        const double d = hypot(a, beta);
        const double cc = d == 0.0 ? 1.0 : a / d, ss = d == 0.0 ? 0.0 : beta / d;
        P.cs[c0] = cc;
        P.sn[c0] = ss;
        col[c0] = d;
        col[c0 + 1] = 0.0;
        for (int k = 0; k <= j; ++k) r[k] = col[k];
        const double gj = P.g[c0];
        const double gn = -ss * gj;
        P.g[c0 + 1] = gn;
        P.g[c0] = cc * gj;
        const int k = gs->k + 1;
        gs->k = k;
        gs->j = j;
        st->iters = k;
        st->rr = gn * gn;
        const double nb = sqrt(st->nb2);
        const double rel = fabs(gn) / nb;
        if (hist) hist[k] = rel;
        const bool chk = st->nonfinite_check != 0;
        if (chk && (!finite_d(rel) || !finite_d(d))) st->stop = ST_NONFINITE;
        else if (fabs(gn) <= st->red * nb) st->stop = ST_CONVERGED;
        else if (beta == 0.0 || d == 0.0) st->stop = ST_BREAKDOWN;
        return;
    }
    // workgroup l: (Hs)_l over columns max(l-1, 0) .. j-1
    const int l = blockIdx.x;
    double hsl[1] = {0.0};
    for (int k = (l > 0 ? l - 1 : 0) + t; k < j; k += kWG) {
        double hlk;
        if (k < j - 1) hlk = P.H[l + ldh * k];
        else hlk = l < j ? P.Ht[l + ldh * k] + P.red[2 * l] : beta;  // column j-1
        hsl[0] += hlk * P.red[2 * k];
    }
    block_reduce<1>(hsl);
    if (t != 0) return;
    const double hs = hsl[0];
    const double ib = 1.0 / beta;
    double *hc = P.Ht + ldh * j;
    if (l < j) {
        const double h = (P.red[2 * l + 1] - hs) * ib;
        hc[l] = h;
        P.sv[l] = P.red[2 * l];
        P.av[l] = hs * ib + h;
    } else {
        const double hjj = ((P.red[2 * j + 1] - bsh[1]) * ib - hs) * ib;
        hc[j] = hjj;
        gs->beta = beta;
        gs->bcoef = hs * ib + hjj;
    }
}

// v_j = (t_j - sum_{k<j} s_k v_k) / beta over slot j, and
// t_{j+1} = u / beta - sum_{k<j} a_k v_k - bcoef v_j into slot j+1, with
// z = dinv .* t_{j+1} (or t_{j+1}) when z is given.
__global__ __launch_bounds__(kWG) void k_gm_update(int64_t n, int64_t ld, double *V, int j,
                                                   const double *__restrict__ u, const double *__restrict__ dinv,
                                                   double *__restrict__ z, const SolverState *st, GmPtrs P) {
    if (st->stop) return;
    const int g = blockIdx.x, t = threadIdx.x;
    double *tj = V + (int64_t)j * ld, *tn = V + (int64_t)(j + 1) * ld;
    const double ib = 1.0 / P.gs->beta, bc = P.gs->bcoef;
    d2 a[kGmPairs], b[kGmPairs];
#pragma unroll
    for (int q = 0; q < kGmPairs; ++q) {
        const int64_t i = gm_pair(g, t, q);
        a[q] = ld2(tj, i, n);
        b[q] = ld2(u, i, n) * ib;
    }
    for (int k = 0; k < j; ++k) {
        const double s = P.sv[k], c = P.av[k];
        const double *vk = V + (int64_t)k * ld;
#pragma unroll
        for (int q = 0; q < kGmPairs; ++q) {
            const d2 v = ld2_nt(vk, gm_pair(g, t, q), n);
            a[q] -= s * v;
            b[q] -= c * v;
        }
    }
#pragma unroll
    for (int q = 0; q < kGmPairs; ++q) {
        const int64_t i = gm_pair(g, t, q);
        if (i >= n) continue;
        const d2 vj = a[q] * ib;
        const d2 tn2 = b[q] - bc * vj;
        st2(tj, i, n, vj);
        st2(tn, i, n, tn2);
        if (z) st2(z, i, n, dinv ? ld2(dinv, i, n) * tn2 : tn2);
    }
}

// R y = g over the cycle's final columns (one wave; column sweep, g kept
// in LDS); y goes to av for the closing update.  Nothing is combined after
// a non-finite stop.
__global__ __launch_bounds__(kWave) void k_gm_backsub(const SolverState *st, GmPtrs P) {
    __shared__ double gl[kGmMaxKrylov];
    GmresState *gs = P.gs;
    const int jj = st->stop == ST_NONFINITE ? 0 : gs->j;
    const int lane = threadIdx.x;
    const int64_t ldh = P.m + 1;
    for (int l = lane; l < jj; l += kWave) gl[l] = P.g[l];
    __syncthreads();
    for (int i = jj - 1; i >= 0; --i) {
        const double yi = gl[i] / P.R[i + ldh * i];
        __syncthreads();
        for (int l = lane; l < i; l += kWave) gl[l] -= P.R[l + ldh * i] * yi;
        if (lane == 0) P.av[i] = yi;
        __syncthreads();
    }
    if (lane == 0) gs->jx = jj;
}

// s = sum_{k < jx} y_k v_k; x += dinv .* s (or s), or t = s for a block
// preconditioner applied afterwards (t = 0 when nothing is combined).
__global__ __launch_bounds__(kWG) void k_gm_xupdate(int64_t n, int64_t ld, const double *__restrict__ V,
                                                    GmPtrs P, const double *__restrict__ dinv,
                                                    double *__restrict__ x, double *__restrict__ tout) {
    const int jx = P.gs->jx;
    if (jx == 0 && !tout) return;
    const int g = blockIdx.x, t = threadIdx.x;
    d2 s[kGmPairs];
#pragma unroll
    for (int q = 0; q < kGmPairs; ++q) s[q] = (d2)0.0;
    for (int k = 0; k < jx; ++k) {
        const double c = P.av[k];
        const double *vk = V + (int64_t)k * ld;
#pragma unroll
        for (int q = 0; q < kGmPairs; ++q) s[q] += c * ld2_nt(vk, gm_pair(g, t, q), n);
    }
#pragma unroll
    for (int q = 0; q < kGmPairs; ++q) {
        const int64_t i = gm_pair(g, t, q);
        if (i >= n) continue;
        if (tout) {
            st2(tout, i, n, s[q]);
        } else {  // x is the caller's vector: element accesses, no alignment assumed
            for (int e = 0; e < 2 && i + e < n; ++e) x[i + e] += dinv ? dinv[i + e] * s[q][e] : s[q][e];
        }
    }
}

// The whole restarted GMRES of a small system (n <= 1024 rows, Krylov
// dimension <= 128, point Jacobi or none) in one workgroup of 1024 threads:
// thread i owns row i (its CSR entries are read from global memory, the
// vector a product gathers is staged in LDS), the basis V and H live in the
// solver's buffers (L2-resident at these sizes).  Each step orthogonalises
// twice by classical Gram-Schmidt: the j+1 dot products run side by side,
// T threads per basis vector (a power of two <= 64, so a group stays in one
// wave) reducing by shuffles.  The criteria, history and stop reasons are
// those of the per-step solver.  out: iterations, products, restarts
// (int64 at 0, 8, 16), status (int32 at 24), relative residual (double at 32).
constexpr int kSmallGmN = 1024, kSmallGmM = 128;
__global__ __launch_bounds__(kSmallGmN) void k_small_gmres(int n, int m, const int *__restrict__ rp,
                                                           const int *__restrict__ col,
                                                           const double *__restrict__ val,
                                                           const double *__restrict__ dinv,
                                                           const double *__restrict__ b, double *__restrict__ x,
                                                           double *__restrict__ V, int64_t ld, GmPtrs P,
                                                           double red_factor, int64_t maxit, int chk,
                                                           double *hist, char *out) {
    __shared__ double zl[kSmallGmN], wl[kSmallGmN], hk[kSmallGmM + 2], yv[kSmallGmM];
    // rotations and the rotated right-hand side stay in LDS for the solve
    __shared__ double csl[kSmallGmM], snl[kSmallGmM], gl[kSmallGmM + 1], colj[kSmallGmM + 2];
    __shared__ double red2[2][kSmallGmN / kWave];
    __shared__ int flag[1];
    const int t = threadIdx.x, lane = t % kWave, wid = t / kWave;
    constexpr int NW = kSmallGmN / kWave;
    const bool own = t < n;
    const int64_t ldh = m + 1;
    // deterministic workgroup sums of two values (result in every thread)
    auto sum2 = [&](double &u, double &v) {
        u = wave_sum(u);
        v = wave_sum(v);
        __syncthreads();
        if (lane == 0) {
            red2[0][wid] = u;
            red2[1][wid] = v;
        }
        __syncthreads();
        double a = 0.0, c = 0.0;
        for (int w = 0; w < NW; ++w) {
            a += red2[0][w];
            c += red2[1][w];
        }
        u = a;
        v = c;
    };
    auto spmv_row = [&]() {  // (A zl)_t for the thread's row
        double s = 0.0;
        if (own)
            for (int q = rp[t]; q < rp[t + 1]; ++q) s += val[q] * zl[col[q]];
        return s;
    };
    const double di = own && dinv ? dinv[t] : 1.0;
    const double bi = own ? b[t] : 0.0;
    double xi = own ? x[t] : 0.0;
    if (own) zl[t] = xi;
    __syncthreads();
    double ri = bi - spmv_row();
    double rr = ri * ri, bb = bi * bi;
    sum2(rr, bb);
    int64_t k = 0, nspmv = 1, restarts = 0;
    int stop = ST_RUN;
    const double nb = sqrt(bb);
    double rel = nb > 0.0 ? sqrt(rr) / nb : 0.0;
    if (t == 0 && hist) hist[0] = rel;
    if (bb == 0.0) {
        xi = 0.0;
        rel = 0.0;
        stop = ST_CONVERGED;
    } else if (chk && !finite_d(sqrt(rr))) {
        stop = ST_NONFINITE;
    } else if (sqrt(rr) <= red_factor * nb) {
        stop = ST_CONVERGED;
    }
    while (stop == ST_RUN) {
        const double beta = sqrt(rr);
        if (own) V[t] = ri / beta;
        if (t <= m) gl[t] = t == 0 ? beta : 0.0;
        int j = 0;
        while (j < m && k < maxit) {
            __syncthreads();  // V column j and the previous products complete
            if (own) zl[t] = di * V[(int64_t)j * ld + t];
            __syncthreads();
            double wi = spmv_row();
            ++nspmv;
            const int nv = j + 1;
            int T = 64;
            while (T > 1 && T * nv > kSmallGmN) T >>= 1;
            for (int pass = 0; pass < 2; ++pass) {
                if (own) wl[t] = wi;
                __syncthreads();
                const int kk = t / T, part = t % T;
                double sdot = 0.0;
                if (kk < nv)
                    for (int i = part; i < n; i += T) sdot += V[(int64_t)kk * ld + i] * wl[i];
                for (int off = T / 2; off > 0; off >>= 1) sdot += __shfl_xor(sdot, off, kWave);
                if (kk < nv && part == 0) {
                    hk[kk] = sdot;
                    colj[kk] = pass == 0 ? sdot : colj[kk] + sdot;
                }
                __syncthreads();
                if (own) {
#pragma unroll 8
                    for (int q = 0; q < nv; ++q) wi -= hk[q] * V[(int64_t)q * ld + t];
                }
                __syncthreads();  // hk consumed before the next pass writes it
            }
            double ww = own ? wi * wi : 0.0, dummy = 0.0;
            sum2(ww, dummy);
            const double hn = sqrt(ww);
            if (t == 0) {  // column j: earlier rotations, a new one, the criteria (oracle order)
                double *h = colj;
                h[j + 1] = hn;
                for (int i2 = 0; i2 < j; ++i2) {
                    const double a = h[i2], c = h[i2 + 1];
                    h[i2] = csl[i2] * a + snl[i2] * c;
                    h[i2 + 1] = -snl[i2] * a + csl[i2] * c;
                }
                const double a = h[j];
                const double d = hypot(a, hn);
                const double cc = d == 0.0 ? 1.0 : a / d, ss = d == 0.0 ? 0.0 : hn / d;
                csl[j] = cc;
                snl[j] = ss;
                h[j] = d;
                h[j + 1] = 0.0;
                const double gj = gl[j];
                gl[j + 1] = -ss * gj;
                gl[j] = cc * gj;
                const double r2 = fabs(gl[j + 1]) / nb;
                if (hist) hist[k + 1] = r2;
                int st2 = ST_RUN;
                if (chk && (!finite_d(r2) || !finite_d(d))) st2 = ST_NONFINITE;
                else if (fabs(gl[j + 1]) <= red_factor * nb) st2 = ST_CONVERGED;
                else if (hn == 0.0 || d == 0.0) st2 = ST_BREAKDOWN;
                flag[0] = st2;
                hk[kSmallGmM + 1] = r2;
            }
            __syncthreads();
            if (t <= j) P.H[t + ldh * j] = colj[t];  // rotated column j (R) for the back substitution
            __syncthreads();
            stop = flag[0];
            rel = hk[kSmallGmM + 1];
            ++j;
            ++k;
            if (stop != ST_RUN) break;
            if (j < m && own) V[(int64_t)j * ld + t] = wi / hn;
        }
        __syncthreads();
        if (stop == ST_NONFINITE) break;
        // x += M^{-1} V y with R y = g over the j steps of this cycle
        // (column sweep: y_i = g_i / r_ii, then g_l -= r_li y_i for l < i)
        for (int i2 = j - 1; i2 >= 0; --i2) {
            if (t == 0) yv[i2] = gl[i2] / P.H[i2 + ldh * i2];
            __syncthreads();
            if (t < i2) gl[t] -= P.H[t + ldh * i2] * yv[i2];
            __syncthreads();
        }
        if (own) {
            double sacc = 0.0;
#pragma unroll 8
            for (int l = 0; l < j; ++l) sacc += V[(int64_t)l * ld + t] * yv[l];
            xi += di * sacc;
        }
        if (stop != ST_RUN) break;
        if (k >= maxit) {
            stop = ST_MAX_ITERS;
            break;
        }
        // restart from the recomputed residual
        __syncthreads();
        if (own) zl[t] = xi;
        __syncthreads();
        ri = bi - spmv_row();
        ++nspmv;
        ++restarts;
        rr = ri * ri;
        double dummy = 0.0;
        sum2(rr, dummy);
        rel = sqrt(rr) / nb;
        if (chk && !finite_d(sqrt(rr))) stop = ST_NONFINITE;
        else if (sqrt(rr) <= red_factor * nb) stop = ST_CONVERGED;
    }
    if (stop == ST_RUN) stop = ST_MAX_ITERS;
    if (own) x[t] = xi;
    if (t == 0) {
        ((int64_t *)out)[0] = k;
        ((int64_t *)out)[1] = nspmv;
        ((int64_t *)out)[2] = restarts;
        ((int32_t *)out)[6] = stop;
        ((double *)out)[4] = rel;
    }
}

hipError_t gm_small(int n, int m, const int *rp, const int *col, const double *val, const double *dinv,
                    const double *b, double *x, double *V, int64_t ld, void *ws, double red, int64_t maxit, int chk,
                    double *hist, void *out, hipStream_t s) {
    hipLaunchKernelGGL(k_small_gmres, dim3(1), dim3(kSmallGmN), 0, s, n, m, rp, col, val, dinv, b, x, V, ld,
                       gm_ptrs(ws, m), red, maxit, chk, hist, (char *)out);
    return hipGetLastError();
}

// ------------------------------------------------------------ launchers
hipError_t gm_prep(const mxl_ctx *ctx, int64_t n, const double *v, const double *b, const double *dinv,
                   double *z, double *parts, int *slots, hipStream_t s) {
    const int g = vec_grid(ctx, n);
    *slots = g;
    hipLaunchKernelGGL(k_gm_prep, dim3(g), dim3(kWG), 0, s, n, v, b, dinv, z, parts);
    return hipGetLastError();
}

hipError_t gm_start(const double *parts, int slots, SolverState *st, void *ws, int m, double *hist, int first,
                    hipStream_t s) {
    hipLaunchKernelGGL(k_gm_start, dim3(1), dim3(kWG), 0, s, parts, slots, st, gm_ptrs(ws, m), hist, first);
    return hipGetLastError();
}

// Step j after the SpMV u = A M^{-1} t_j (u == nullptr: the cycle's closing
// pass, which only finalises column j-1).
hipError_t gm_step(int64_t n, int64_t ld, double *V, int j, const double *u, const double *dinv, double *z,
                   double *dparts, SolverState *st, void *ws, int m, double *hist, hipStream_t s) {
    const int G = gm_grid(n);
    const GmPtrs P = gm_ptrs(ws, m);
    const int last = u == nullptr;
    hipLaunchKernelGGL(k_gm_dots, dim3(G), dim3(kWG), 0, s, n, ld, (const double *)V, j, u, dparts,
                       (const SolverState *)st);
    hipLaunchKernelGGL(k_gm_reduce, dim3(2 * j + 2), dim3(kWG), 0, s, (const double *)dparts, G,
                       (const SolverState *)st, P.red);
    hipLaunchKernelGGL(k_gm_finish, dim3(last ? 1 : j + 2), dim3(kWG), 0, s, j, last, st, P, hist);
    if (!last)
        hipLaunchKernelGGL(k_gm_update, dim3(G), dim3(kWG), 0, s, n, ld, V, j, u, dinv, z, (const SolverState *)st,
                           P);
    return hipGetLastError();
}

hipError_t gm_close(int64_t n, int64_t ld, const double *V, const double *dinv, double *x, double *t,
                    const SolverState *st, void *ws, int m, hipStream_t s) {
    const GmPtrs P = gm_ptrs(ws, m);
    hipLaunchKernelGGL(k_gm_backsub, dim3(1), dim3(kWave), 0, s, st, P);
    hipLaunchKernelGGL(k_gm_xupdate, dim3(gm_grid(n)), dim3(kWG), 0, s, n, ld, V, P, dinv, x, t);
    return hipGetLastError();
}

hipError_t gm_read(const void *ws, int64_t *nspmv, hipStream_t s) {
    GmresState h;
    hipError_t e = hipMemcpyAsync(&h, ws, sizeof(h), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e == hipSuccess) *nspmv = h.nspmv;
    return e;
}

}  // namespace mxl
