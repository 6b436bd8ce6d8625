// device_common.hpp -- wave64 reductions, XCD-aware workgroup mapping and
// the device-resident solver state shared by the SpMV and Krylov kernels
// (gfx950 / CDNA4).
//
// Reduction protocol: a producing kernel publishes one partial per
// workgroup with plain stores; the kernel that consumes the scalar reduces
// all partials in its prologue, identically in every workgroup (fixed
// order), and takes its decisions from that value.  Scalars that later
// kernels need are written by workgroup 0 into SolverState.  No kernel reads
// a SolverState field that the same kernel writes (rho is double-buffered by
// iteration parity), so there is no intra-kernel race.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mxl {

constexpr int kWG = 256;        // threads per workgroup (4 wave64s)
constexpr int kWave = 64;
constexpr int kNumXcd = 8;      // MI355X: 8 accelerator complex dies, one L2 each
constexpr int kMaxGrid = 2048;  // upper bound on workgroups of a reducing kernel

// Device-side status codes (the stopping_status of the criteria).  ST_HALF:
// BiCGSTAB met the criterion at its half step of iteration `iters`.
enum : int {
    ST_RUN = 0, ST_CONVERGED = 1, ST_MAX_ITERS = 2, ST_TIME = 3,
    ST_BREAKDOWN = 4, ST_NONFINITE = 5, ST_HALF = 16
};

// One-shot finalisations run by the single-workgroup k_finalize kernel.
enum FinOp : int {
    FIN_NORMS = 1,      // [r.r, max|r|]        -> sums[0..1]
    FIN_CG_INIT = 2,    // [r.z, r.r, b.b]
    FIN_BI_INIT = 3,    // [r.r, rhat.r, b.b]
    FIN_BI_LAST = 4     // [r.r, rhat.r, -] of the last executed iteration
};

// Scalars of one Krylov solve, resident in device memory.
struct SolverState {
    double rho2[2];   // r.z (CG) or rhat.r (BiCGSTAB) of iteration k in rho2[k & 1]
    double alpha, omega, beta, eta;
    double rr;        // latest squared residual norm
    double nb2;       // ||b||^2
    double red;       // ResidualNormReduction factor
    double sums[4];
    int32_t stop;     // ST_*
    int32_t iters;    // iteration count when stop was set
    int32_t nonfinite_check;
    int32_t half;     // BiCGSTAB: 1 if it stopped at a half step
    int32_t ustop;    // CG: set by k_cg_update for k_cg_pupdate (1 = do nothing),
                      // so that k_cg_pupdate never reads the stop it writes
};

// Tile walk of workgroup `bid` of G over T tiles.  Workgroups are
// dispatched round-robin over the 8 XCDs (bid % 8); XCD x owns one
// contiguous band of tiles, proportional to its workgroup count, and its
// workgroups walk that band interleaved (first = band start + bid / 8,
// step = workgroups on the XCD).  Each XCD's resident workgroups therefore
// sweep one compact region at a time: the x window they gather stays in that
// XCD's L2 and the streamed matrix arrays are read as a few dense fronts.
// Every tile is visited exactly once.
__device__ __forceinline__ void band_walk(int64_t T, int bid, int G, int64_t &first, int64_t &end,
                                          int &step) {
    const int x = bid % kNumXcd, j = bid / kNumXcd;
    const int q = G / kNumXcd, rem = G % kNumXcd;
    const int cnt = q + (x < rem ? 1 : 0);
    const int before = x * q + (x < rem ? x : rem);
    const int64_t lo = T * before / G, hi = T * (before + cnt) / G;
    first = lo + j;
    end = hi;
    step = cnt;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

template <typename T>
__device__ __forceinline__ T wave_max(T v) {
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) {
        T o = __shfl_xor(v, off, kWave);
        v = o > v ? o : v;
    }
    return v;
}

// Reduce NV doubles over the B-thread workgroup (fixed tree: shuffle within
// each wave, then the wave results in order).  Result valid in thread 0.
// mask selects which values are max-reductions instead of sums.
template <int NV, int B = kWG>
__device__ __forceinline__ void block_reduce(double (&v)[NV], unsigned max_mask = 0) {
    __shared__ double red_smem[B / kWave][NV > 0 ? NV : 1];
    const int lane = threadIdx.x % kWave, wid = threadIdx.x / kWave;
#pragma unroll
    for (int j = 0; j < NV; ++j) v[j] = (max_mask >> j & 1) ? wave_max(v[j]) : wave_sum(v[j]);
    __syncthreads();
    if (lane == 0) {
#pragma unroll
        for (int j = 0; j < NV; ++j) red_smem[wid][j] = v[j];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int j = 0; j < NV; ++j) {
            double a = red_smem[0][j];
            for (int w = 1; w < B / kWave; ++w) {
                double b = red_smem[w][j];
                a = (max_mask >> j & 1) ? (b > a ? b : a) : a + b;
            }
            v[j] = a;
        }
    }
    __syncthreads();
}

// Publish one workgroup's NV partial values (thread 0 after the block
// reduction) to slot `slot` of an NV-interleaved partial array.  Plain
// stores: the consumer is a later kernel, and the kernel boundary makes them
// visible on every XCD.  (A per-workgroup device-scope fence would write
// back the whole L2 of the XCD for every workgroup.)
template <int NV, int B = kWG>
__device__ __forceinline__ void publish(double (&v)[NV], double *partials, int slot,
                                        unsigned max_mask = 0) {
    block_reduce<NV, B>(v, max_mask);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int j = 0; j < NV; ++j) partials[(int64_t)slot * NV + j] = v[j];
    }
}

// Every thread of every workgroup obtains the same deterministic total of
// slots [0, nslots) (fixed striding, fixed tree), so a consumer kernel can
// take the same scalar decisions in all of its workgroups without any
// inter-workgroup communication.
// A thread's slots are t, t + B, t + 2B, ...; a batch of U rounds of
// them is loaded before any is added, so one round trip to L2 serves U slots
// (a loop that adds each value as it arrives waits once per slot), and the
// values are added in slot order, so the sum does not depend on U.  Whether
// a batch is complete depends only on nslots, so the branch is uniform and
// complete batches load without per-slot predicates.  U shrinks as NV grows
// to keep the batch at 8 doubles per thread: the update kernels hold their
// prefetched operands in registers at the same time.
template <int NV, int B = kWG>
__device__ __forceinline__ void gather_all(const double *__restrict__ partials, int nslots,
                                           double (&tot)[NV], unsigned max_mask = 0) {
    constexpr int U = NV <= 1 ? 8 : (NV == 2 ? 4 : 2);
    __shared__ double bc[NV > 0 ? NV : 1];
#pragma unroll
    for (int j = 0; j < NV; ++j) tot[j] = 0.0;
    auto add = [&](int j, double v) {
        tot[j] = (max_mask >> j & 1) ? (v > tot[j] ? v : tot[j]) : tot[j] + v;
    };
    const int full = nslots / B;  // rounds in which every thread has a slot
    for (int r0 = 0; r0 * B < nslots; r0 += U) {
        if (r0 + U <= full) {
            double buf[U][NV > 0 ? NV : 1];
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
                for (int j = 0; j < NV; ++j) buf[u][j] = partials[(int64_t)((r0 + u) * B + threadIdx.x) * NV + j];
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
                for (int j = 0; j < NV; ++j) add(j, buf[u][j]);
        } else {
            for (int u = 0; u < U; ++u) {
                const int s = (r0 + u) * B + threadIdx.x;
                if (s < nslots) {
#pragma unroll
                    for (int j = 0; j < NV; ++j) add(j, partials[(int64_t)s * NV + j]);
                }
            }
        }
    }
    block_reduce<NV, B>(tot, max_mask);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int j = 0; j < NV; ++j) bc[j] = tot[j];
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < NV; ++j) tot[j] = bc[j];
    __syncthreads();
}

__device__ __forceinline__ bool finite_d(double v) { return __builtin_isfinite(v); }

// One-shot scalar logic of k_finalize (thread 0 only).
__device__ inline void finalize(int op, SolverState *st, const double *s, int k, int max_iters,
                                double *hist) {
    const bool chk = st->nonfinite_check != 0;
    switch (op) {
    case FIN_NORMS:
        st->sums[0] = s[0];
        st->sums[1] = s[1];
        break;
    case FIN_CG_INIT: {
        st->rho2[0] = s[0];
        st->rr = s[1];
        st->nb2 = s[2];
        st->iters = 0;
        st->stop = ST_RUN;
        double nb = sqrt(s[2]);
        if (hist) hist[0] = nb > 0.0 ? sqrt(s[1]) / nb : 0.0;
        if (s[2] == 0.0 || sqrt(s[1]) <= st->red * nb) st->stop = ST_CONVERGED;
        break;
    }
    case FIN_BI_INIT: {
        st->rr = s[0];
        st->nb2 = s[2];
        st->iters = 0;
        st->stop = ST_RUN;
        st->rho2[0] = 1.0;  // rho_0 = alpha_0 = omega_0 = 1
        st->alpha = 1.0;
        st->omega = 1.0;
        double nb = sqrt(s[2]);
        if (hist) hist[0] = nb > 0.0 ? sqrt(s[0]) / nb : 0.0;
        if (s[2] == 0.0 || sqrt(s[0]) <= st->red * nb) st->stop = ST_CONVERGED;
        break;
    }
    case FIN_BI_LAST: {  // criterion of the final iteration k (no next iteration)
        if (st->stop != ST_RUN) break;
        double rr = s[0];
        st->rr = rr;
        double nb = sqrt(st->nb2);
        if (hist) hist[k] = sqrt(rr) / nb;
        st->iters = k;
        if (chk && !finite_d(rr)) st->stop = ST_NONFINITE;
        else if (sqrt(rr) <= st->red * nb) st->stop = ST_CONVERGED;
        else if (st->omega == 0.0) st->stop = ST_BREAKDOWN;
        break;
    }
    default:
        break;
    }
}

}  // namespace mxl
