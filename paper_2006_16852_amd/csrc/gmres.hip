// gmres.hip -- restarted GMRES(m) preconditioned from the right (Krylov
// solvers of Sec. 3.1; the restart parameter and memory model of Table 2).
//
// The Arnoldi basis V (m+1 vectors of ld >= n doubles, vector after vector)
// stays resident.  Basis vectors are stored unnormalised: v_k = scl[k] V_k,
// so no pass rewrites a vector to normalise it.  One Arnoldi step is
//
//   u = A z_j, z_j = M^{-1} V_j                          (SpMV)
//   h_kj = scl_k scl_j (V_k . u), ||w||^2 = scl_j^2 u.u  (k_gm_dots + k_gm_h)
//   w' = scl_j u - sum_k h_kj scl_k V_k -> V_{j+1}, z    (k_gm_update)
//   second pass only when ||w'|| < ||w|| / sqrt(2)        (k_gm_norm1, then
//     k_gm_dots/k_gm_h/k_gm_update again on V_{j+1})
//   Givens rotations, residual estimate, criteria         (k_gm_givens)
//
// i.e. classical Gram-Schmidt, whose projections are one skinny multi-dot
// and one multi-axpy over the basis (two passes over V instead of the five
// of a modified Gram-Schmidt step), with the Daniel-Gragg-Kaufman-Stewart
// test deciding the re-orthogonalisation that keeps the basis orthogonal to
// working precision.  A cycle ends with the back substitution R y = g
// (k_gm_backsub) and x += M^{-1} V (scl .* y) (k_gm_xupdate).
//
// Every step kernel returns at once when the solve has stopped, so the host
// can enqueue steps without reading the state after each one.
#include <cmath>
#include <cstring>

#include "device_common.hpp"
#include "internal.hpp"

namespace mxl {

constexpr int kGmRows = 8;              // rows per thread in the basis kernels
constexpr int kGmTile = kWG * kGmRows;  // rows per workgroup
constexpr int kGmKC = 8;                // basis vectors per multi-dot chunk

// Device scalars of a GMRES solve besides SolverState.
struct GmresState {
    int32_t j;        // steps completed in the current cycle
    int32_t k;        // steps completed in the solve
    int32_t reorth;   // 1: the current step takes the second Gram-Schmidt pass
    int32_t nreorth;  // second passes taken in the solve
    int32_t jx;       // basis vectors combined by the cycle's closing update
    int32_t pad;
    double wn2;       // ||w||^2 before orthogonalisation
    double hn2;       // ||w||^2 after the first pass
};

struct GmPtrs {
    double *H;     // (m+1) x m Hessenberg matrix, column j at H + (m+1) j
    double *cs, *sn;
    double *g;     // m+1: rotated right-hand side beta e_1
    double *scl;   // m+1: v_k = scl[k] V_k
    double *coef;  // m+1: projection coefficients / closing combination
    double *y;     // m
    GmresState *gs;
    int m;
};

size_t gm_ws_bytes(int m) {
    const size_t d = (size_t)(m + 1) * m + 2 * (size_t)m + 3 * (size_t)(m + 1) + (size_t)m;
    return d * sizeof(double) + 256;
}

static GmPtrs gm_ptrs(void *ws, int m) {
    GmPtrs P;
    auto *gs = (GmresState *)ws;
    double *d = (double *)((char *)ws + 256);
    P.gs = gs;
    P.m = m;
    P.H = d;
    d += (size_t)(m + 1) * m;
    P.cs = d;
    d += m;
    P.sn = d;
    d += m;
    P.g = d;
    d += m + 1;
    P.scl = d;
    d += m + 1;
    P.coef = d;
    d += m + 1;
    P.y = d;
    return P;
}

int gm_grid(int64_t n) {
    const int64_t g = (n + kGmTile - 1) / kGmTile;
    return (int)(g < 1 ? 1 : g);
}

__device__ __forceinline__ double nt_ld(const double *p) { return __builtin_nontemporal_load(p); }

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

// Start of a cycle from the residual held in V_0: beta = ||V_0||,
// scl_0 = 1/beta, g = beta e_1, and the criteria on beta.  first: also
// ||b||^2 and history[0].
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
        gs->nreorth = 0;
    }
    const double beta = sqrt(t[0]);
    st->rr = t[0];
    gs->j = 0;
    gs->jx = 0;
    gs->reorth = 0;
    for (int i = 0; i <= P.m; ++i) P.g[i] = 0.0;
    P.g[0] = beta;
    P.scl[0] = 1.0 / beta;
    const double nb = sqrt(nb2);
    if (first && hist) hist[0] = nb > 0.0 ? beta / nb : 0.0;
    const bool chk = st->nonfinite_check != 0;
    if (nb2 == 0.0) st->stop = ST_CONVERGED;
    else if (chk && !finite_d(beta)) st->stop = ST_NONFINITE;
    else if (beta <= st->red * nb) st->stop = ST_CONVERGED;
}

// Partials of V_k . u for k = 0..nv-1 and of u.u (slot nv), one tile of
// kGmTile rows per workgroup; partial (k, g) at parts[k * G + g].  u may be
// V_nv itself (second pass).
__global__ __launch_bounds__(kWG) void k_gm_dots(int64_t n, int64_t ld, const double *__restrict__ V,
                                                 int nv, const double *u, double *__restrict__ parts,
                                                 const SolverState *st, const GmresState *gs, int pass) {
    if (st->stop) return;
    if (pass == 2 && !gs->reorth) return;
    __shared__ double red[kGmKC][kWG];
    const int G = gridDim.x, g = blockIdx.x, t = threadIdx.x;
    const int64_t row0 = (int64_t)g * kGmTile + t;
    double ur[kGmRows];
    double uu = 0.0;
#pragma unroll
    for (int r = 0; r < kGmRows; ++r) {
        const int64_t i = row0 + (int64_t)r * kWG;
        ur[r] = i < n ? u[i] : 0.0;
        uu += ur[r] * ur[r];
    }
    for (int k0 = 0; k0 < nv; k0 += kGmKC) {
        double acc[kGmKC];
#pragma unroll
        for (int kk = 0; kk < kGmKC; ++kk) {
            acc[kk] = 0.0;
            if (k0 + kk < nv) {
                const double *vk = V + (int64_t)(k0 + kk) * ld;
#pragma unroll
                for (int r = 0; r < kGmRows; ++r) {
                    const int64_t i = row0 + (int64_t)r * kWG;
                    if (i < n) acc[kk] += nt_ld(vk + i) * ur[r];
                }
            }
        }
#pragma unroll
        for (int kk = 0; kk < kGmKC; ++kk) red[kk][t] = acc[kk];
        __syncthreads();
        // thread t sums 8 of the 256 values of vector kk = t / 32, then the
        // 32 lanes of that group combine by shuffles (fixed order)
        const int kk = t / 32, q = t % 32;
        double s = 0.0;
#pragma unroll
        for (int e = 0; e < 8; ++e) s += red[kk][q * 8 + e];
#pragma unroll
        for (int off = 16; off > 0; off >>= 1) s += __shfl_xor(s, off, kWave);
        if (q == 0 && k0 + kk < nv) parts[(int64_t)(k0 + kk) * G + g] = s;
        __syncthreads();
    }
    double v1[1] = {uu};
    block_reduce<1>(v1);
    if (t == 0) parts[(int64_t)nv * G + g] = v1[0];
}

// One workgroup per value k = 0..j+1 of a multi-dot: the total of its G
// partials (fixed order), then pass 1: h_kj = scl_k scl_j s and
// ||w||^2 = scl_j^2 s at k = j+1; pass 2: h_kj += scl_k s.  coef_k = h scl_k
// is the coefficient of V_k in the following update.
__global__ __launch_bounds__(kWG) void k_gm_h(const double *__restrict__ parts, int G, int j,
                                              const SolverState *st, GmPtrs P, int pass) {
    if (st->stop) return;
    if (pass == 2 && !P.gs->reorth) return;
    const int kk = blockIdx.x;
    double s[1] = {0.0};
    for (int g = threadIdx.x; g < G; g += kWG) s[0] += parts[(int64_t)kk * G + g];
    block_reduce<1>(s);
    if (threadIdx.x != 0) return;
    const int64_t ldh = P.m + 1;
    if (kk <= j) {
        if (pass == 1) {
            const double h = P.scl[kk] * P.scl[j] * s[0];
            P.H[kk + ldh * j] = h;
            P.coef[kk] = h * P.scl[kk];
        } else {
            const double c = P.scl[kk] * s[0];
            P.H[kk + ldh * j] += c;
            P.coef[kk] = c * P.scl[kk];
        }
    } else if (pass == 1) {
        P.gs->wn2 = P.scl[j] * P.scl[j] * s[0];
    }
}

// w = a u - sum_{k<=j} coef_k V_k into V_{j+1} (a = scl_j in pass 1, 1 in
// pass 2 where u is V_{j+1} itself), z = dinv .* w when z is given, and
// partials of w.w (one per workgroup).
__global__ __launch_bounds__(kWG) void k_gm_update(int64_t n, int64_t ld, double *V, int j, const double *u,
                                                   const double *__restrict__ dinv, double *__restrict__ z,
                                                   double *__restrict__ parts, const SolverState *st,
                                                   GmPtrs P, int pass) {
    if (st->stop) return;
    if (pass == 2 && !P.gs->reorth) return;
    const int g = blockIdx.x, t = threadIdx.x;
    const int64_t row0 = (int64_t)g * kGmTile + t;
    const double a = pass == 1 ? P.scl[j] : 1.0;
    double w[kGmRows];
#pragma unroll
    for (int r = 0; r < kGmRows; ++r) {
        const int64_t i = row0 + (int64_t)r * kWG;
        w[r] = i < n ? a * u[i] : 0.0;
    }
    for (int k = 0; k <= j; ++k) {
        const double c = P.coef[k];
        const double *vk = V + (int64_t)k * ld;
#pragma unroll
        for (int r = 0; r < kGmRows; ++r) {
            const int64_t i = row0 + (int64_t)r * kWG;
            if (i < n) w[r] -= c * nt_ld(vk + i);
        }
    }
    double *vn = V + (int64_t)(j + 1) * ld;
    double ww = 0.0;
#pragma unroll
    for (int r = 0; r < kGmRows; ++r) {
        const int64_t i = row0 + (int64_t)r * kWG;
        if (i < n) {
            vn[i] = w[r];
            if (z) z[i] = dinv ? dinv[i] * w[r] : w[r];
            ww += w[r] * w[r];
        }
    }
    double v1[1] = {ww};
    publish<1>(v1, parts, g);
}

// ||w'||^2 after the first pass and the re-orthogonalisation test.
__global__ __launch_bounds__(kWG) void k_gm_norm1(const double *__restrict__ parts, int G,
                                                  const SolverState *st, GmresState *gs) {
    if (st->stop) return;
    double t[1];
    gather_all<1>(parts, G, t);
    if (threadIdx.x != 0) return;
    gs->hn2 = t[0];
    const int re = t[0] < 0.5 * gs->wn2 ? 1 : 0;
    gs->reorth = re;
    gs->nreorth += re;
}

// Closes Arnoldi step j: h_{j+1,j} = ||w||, the earlier rotations and a new
// one on column j, g, the residual estimate |g_{j+1}| and the criteria (in
// the oracle's order), scl_{j+1} = 1 / h_{j+1,j}.
__global__ __launch_bounds__(kWG) void k_gm_givens(const double *__restrict__ parts, int G, int j,
                                                   SolverState *st, GmPtrs P, double *hist) {
    if (st->stop) return;
    GmresState *gs = P.gs;
    double hn2 = gs->hn2;
    if (gs->reorth) {
        double t[1];
        gather_all<1>(parts, G, t);
        hn2 = t[0];
    }
    if (threadIdx.x != 0) return;
    const int64_t ldh = P.m + 1;
    double *h = P.H + ldh * j;
    const double hn = sqrt(hn2);
    for (int i = 0; i < j; ++i) {
        const double a = h[i], c = h[i + 1];
        h[i] = P.cs[i] * a + P.sn[i] * c;
        h[i + 1] = -P.sn[i] * a + P.cs[i] * c;
    }
    const double a = h[j];
    const double d = hypot(a, hn);
    const double c = d == 0.0 ? 1.0 : a / d, s = d == 0.0 ? 0.0 : hn / d;
    P.cs[j] = c;
    P.sn[j] = s;
    h[j] = d;
    h[j + 1] = 0.0;
    const double gj = P.g[j];
    const double gn = -s * gj;
    P.g[j + 1] = gn;
    P.g[j] = c * gj;
    const int k = gs->k + 1;
    gs->k = k;
    gs->j = j + 1;
    st->iters = k;
    st->rr = gn * gn;
    const double nb = sqrt(st->nb2);
    const double rel = fabs(gn) / nb;
    if (hist) hist[k] = rel;
    P.scl[j + 1] = 1.0 / hn;
    const bool chk = st->nonfinite_check != 0;
    if (chk && (!finite_d(rel) || !finite_d(d))) st->stop = ST_NONFINITE;
    else if (fabs(gn) <= st->red * nb) st->stop = ST_CONVERGED;
    else if (hn == 0.0 || d == 0.0) st->stop = ST_BREAKDOWN;
}

// R y = g over the cycle's steps (one wave; column sweep, g kept in LDS),
// then coef_k = scl_k y_k for the closing update.  Nothing is combined
// after a non-finite stop.
__global__ __launch_bounds__(kWave) void k_gm_backsub(const SolverState *st, GmPtrs P) {
    __shared__ double gl[kGmMaxKrylov];
    GmresState *gs = P.gs;
    const int jj = st->stop == ST_NONFINITE ? 0 : gs->j;
    const int lane = threadIdx.x;
    const int64_t ldh = P.m + 1;
    for (int l = lane; l < jj; l += kWave) gl[l] = P.g[l];
    __syncthreads();
    for (int i = jj - 1; i >= 0; --i) {
        const double yi = gl[i] / P.H[i + ldh * i];
        __syncthreads();
        for (int l = lane; l < i; l += kWave) gl[l] -= P.H[l + ldh * i] * yi;
        if (lane == 0) P.y[i] = yi;
        __syncthreads();
    }
    __syncthreads();
    for (int l = lane; l < jj; l += kWave) P.coef[l] = P.y[l] * P.scl[l];
    if (lane == 0) gs->jx = jj;
}

// s = sum_{k < jx} coef_k V_k; x += dinv .* s (or s), or t = s for a block
// preconditioner applied afterwards (t = 0 when nothing is combined).
__global__ __launch_bounds__(kWG) void k_gm_xupdate(int64_t n, int64_t ld, const double *__restrict__ V,
                                                    GmPtrs P, const double *__restrict__ dinv,
                                                    double *__restrict__ x, double *__restrict__ tout) {
    const int jx = P.gs->jx;
    if (jx == 0 && !tout) return;
    const int64_t row0 = (int64_t)blockIdx.x * kGmTile + threadIdx.x;
    double s[kGmRows];
#pragma unroll
    for (int r = 0; r < kGmRows; ++r) s[r] = 0.0;
    for (int k = 0; k < jx; ++k) {
        const double c = P.coef[k];
        const double *vk = V + (int64_t)k * ld;
#pragma unroll
        for (int r = 0; r < kGmRows; ++r) {
            const int64_t i = row0 + (int64_t)r * kWG;
            if (i < n) s[r] += c * nt_ld(vk + i);
        }
    }
#pragma unroll
    for (int r = 0; r < kGmRows; ++r) {
        const int64_t i = row0 + (int64_t)r * kWG;
        if (i >= n) continue;
        if (tout) tout[i] = s[r];
        else x[i] += dinv ? dinv[i] * s[r] : s[r];
    }
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

hipError_t gm_step(int64_t n, int64_t ld, double *V, int j, const double *u, const double *dinv, double *z,
                   double *dparts, double *nparts, SolverState *st, void *ws, int m, double *hist,
                   hipStream_t s) {
    const int G = gm_grid(n);
    const GmPtrs P = gm_ptrs(ws, m);
    double *vn = V + (int64_t)(j + 1) * ld;
    hipLaunchKernelGGL(k_gm_dots, dim3(G), dim3(kWG), 0, s, n, ld, (const double *)V, j + 1, u, dparts,
                       (const SolverState *)st, (const GmresState *)P.gs, 1);
    hipLaunchKernelGGL(k_gm_h, dim3(j + 2), dim3(kWG), 0, s, (const double *)dparts, G, j,
                       (const SolverState *)st, P, 1);
    hipLaunchKernelGGL(k_gm_update, dim3(G), dim3(kWG), 0, s, n, ld, V, j, u, dinv, z, nparts,
                       (const SolverState *)st, P, 1);
    hipLaunchKernelGGL(k_gm_norm1, dim3(1), dim3(kWG), 0, s, (const double *)nparts, G,
                       (const SolverState *)st, P.gs);
    hipLaunchKernelGGL(k_gm_dots, dim3(G), dim3(kWG), 0, s, n, ld, (const double *)V, j + 1,
                       (const double *)vn, dparts, (const SolverState *)st, (const GmresState *)P.gs, 2);
    hipLaunchKernelGGL(k_gm_h, dim3(j + 1), dim3(kWG), 0, s, (const double *)dparts, G, j,
                       (const SolverState *)st, P, 2);
    hipLaunchKernelGGL(k_gm_update, dim3(G), dim3(kWG), 0, s, n, ld, V, j, (const double *)vn, dinv, z,
                       nparts, (const SolverState *)st, P, 2);
    hipLaunchKernelGGL(k_gm_givens, dim3(1), dim3(kWG), 0, s, (const double *)nparts, G, j, st, P, hist);
    return hipGetLastError();
}

hipError_t gm_close(int64_t n, int64_t ld, const double *V, const double *dinv, double *x, double *t,
                    const SolverState *st, void *ws, int m, hipStream_t s) {
    const GmPtrs P = gm_ptrs(ws, m);
    hipLaunchKernelGGL(k_gm_backsub, dim3(1), dim3(kWave), 0, s, st, P);
    hipLaunchKernelGGL(k_gm_xupdate, dim3(gm_grid(n)), dim3(kWG), 0, s, n, ld, V, P, dinv, x, t);
    return hipGetLastError();
}

hipError_t gm_read(const void *ws, int64_t *reorth, hipStream_t s) {
    GmresState h;
    hipError_t e = hipMemcpyAsync(&h, ws, sizeof(h), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e == hipSuccess) *reorth = h.nreorth;
    return e;
}

}  // namespace mxl
